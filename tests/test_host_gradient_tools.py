"""The host references of the gradient pieces (include/qedx_tools.h) against
the oracle's reverse-mode autodiff, on the CPU.

qed_graph_grad_interpret: log of the helicity-summed |M|^2 of the library's
graph and its derivative with respect to every momentum component, by the
graph's reverse sweep in float64 (the sweep the adjoint kernels run).
qed_rambo_vjp_host: the final-state momenta of RAMBO and the vector-Jacobian
product (dk/du)^T g, including the implicit derivative of the massive
rescale.  The oracle differentiates its own per-diagram amplitude and its own
RAMBO (Newton iterations included) with torch autograd.
"""
import numpy as np
import pytest
import torch

from oracle import qed_oracle as O
from paper_2511_19456_amd import inputs
from paper_2511_19456_amd._lib import check, lib


@pytest.mark.parametrize("n,sqrt_s,reduced", [(1, 4.0, 1), (2, 6.0, 1), (3, 10.0, 1), (3, 10.0, 0),
                                              (4, 15.0, 1), (3, 10.0, 2)])
def test_graph_grad_interpret_matches_oracle_autodiff(n, sqrt_s, reduced):
    """The momentum gradient itself is not unique: off the mass shells and the
    momentum-conservation surface the graph and the oracle are different
    functions (the graph forms Q^2 - m^2 from whichever electron side has
    fewer photons), so their partial derivatives may differ along the normals
    of those constraints.  Pulled back through the RAMBO map, whose image lies
    on them, the gradient with respect to the uniforms is unique: that is
    compared, together with the value."""
    N = 24 if n < 4 else 8
    u, _ = inputs.rambo_inputs(50 + n, n, N)
    nf = n + 1
    pts = O.momenta_from_uniforms(u, sqrt_s, n).numpy()          # [N, n+3, 4]
    flat = np.ascontiguousarray(pts.reshape(N, -1))
    val = np.zeros(N)
    gm = np.zeros_like(flat)
    check(lib().qed_graph_grad_interpret(n, (n + 1) // 2, reduced, flat.ctypes.data, N, val.ctypes.data,
                                         gm.ctypes.data))
    v_o, g_o = O.logm2_and_grad(u, sqrt_s, n)
    assert np.abs(val - v_o.numpy()).max() < 1e-12 * max(1.0, np.abs(v_o.numpy()).max())
    assert np.all(gm[:, :8] == 0.0)          # incoming momenta are fixed by sqrt(s)
    gk = np.ascontiguousarray(gm[:, 8:])
    mom = np.zeros((N, 4 * nf))
    gu = np.zeros((N, 4 * nf))
    u_pm = np.ascontiguousarray(u.T)                              # point-major [N, 4 nf]
    check(lib().qed_rambo_vjp_host(n, u_pm.ctypes.data, sqrt_s, gk.ctypes.data, N, mom.ctypes.data,
                                   gu.ctypes.data))
    go = g_o.numpy().T
    err = np.linalg.norm(gu - go, axis=1) / np.linalg.norm(go, axis=1)
    assert err.max() < 1e-10, err.max()


@pytest.mark.parametrize("n,sqrt_s", [(1, 3.0), (2, 6.0), (3, 10.0), (4, 15.0), (6, 25.0)])
def test_rambo_vjp_host_matches_oracle_autodiff(n, sqrt_s):
    N = 32
    nf = n + 1
    u, _ = inputs.rambo_inputs(60 + n, n, N)                      # [4 nf, N]
    gk = np.ascontiguousarray(inputs.rng_for(70 + n).standard_normal((N, 4 * nf)))
    u_pm = np.ascontiguousarray(u.T)                              # point-major [N, 4 nf]
    mom = np.zeros((N, 4 * nf))
    gu = np.zeros((N, 4 * nf))
    check(lib().qed_rambo_vjp_host(n, u_pm.ctypes.data, sqrt_s, gk.ctypes.data, N, mom.ctypes.data,
                                   gu.ctypes.data))
    ut = torch.as_tensor(u, dtype=torch.float64).clone().requires_grad_(True)
    fin = O.rambo(ut, sqrt_s, [1.0] + [0.0] * n)                  # [N, nf, 4]
    assert np.abs(mom - fin.detach().numpy().reshape(N, -1)).max() < 1e-12 * sqrt_s
    (g,) = torch.autograd.grad((fin.reshape(N, -1) * torch.as_tensor(gk)).sum(), ut)
    g = g.numpy().T                                               # [N, 4 nf]
    err = np.linalg.norm(gu - g, axis=1) / np.linalg.norm(g, axis=1)
    assert err.max() < 1e-11, err.max()


def test_host_gradient_tools_reject_bad_arguments():
    L = lib()
    assert L.qed_graph_grad_interpret(0, 1, 1, None, 0, None, None) != 0
    assert L.qed_graph_grad_interpret(3, 4, 1, None, 0, None, None) != 0
    assert L.qed_rambo_vjp_host(7, None, 10.0, None, 0, None, None) != 0
    assert L.qed_rambo_vjp_host(2, None, 10.0, None, -1, None, None) != 0
