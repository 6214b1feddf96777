"""The allocation-free gradient entry point (qed_eval_grad_noalloc) against
qed_eval_grad with a caller-owned workspace, through the C ABI, on two calls
in a row (the second smaller, so it runs on the scratch the first one left
behind), and against the oracle's stored gradient (tests/golden/)."""
import ctypes
import os

import numpy as np
import pytest
import torch

from paper_2511_19456_amd import inputs

pytestmark = pytest.mark.gpu

DEV = "cuda:0"
HERE = os.path.dirname(os.path.abspath(__file__))


def _grad_ws(lib, h, u, rs):
    N = u.shape[1]
    val = torch.full((N,), float("nan"), dtype=torch.float64, device=DEV)
    grad = torch.full((u.shape[0], N), float("nan"), dtype=torch.float64, device=DEV)
    nb = ctypes.c_int64()
    assert lib.qed_eval_grad_workspace_size(h, N, ctypes.byref(nb)) == 0
    ws = torch.empty(max(nb.value, 1), dtype=torch.uint8, device=DEV)
    st = ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    rc = lib.qed_eval_grad(h, ctypes.c_void_p(u.data_ptr()), rs, None, N, ctypes.c_void_p(val.data_ptr()),
                           ctypes.c_void_p(grad.data_ptr()), ctypes.c_void_p(ws.data_ptr()), nb.value, st)
    assert rc == 0, lib.qed_last_error()
    torch.cuda.synchronize()
    return val, grad


def _grad_noalloc(lib, h, u, rs):
    N = u.shape[1]
    val = torch.full((N,), float("nan"), dtype=torch.float64, device=DEV)
    grad = torch.full((u.shape[0], N), float("nan"), dtype=torch.float64, device=DEV)
    st = ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    rc = lib.qed_eval_grad_noalloc(h, ctypes.c_void_p(u.data_ptr()), rs, None, N, ctypes.c_void_p(val.data_ptr()),
                                   ctypes.c_void_p(grad.data_ptr()), st)
    assert rc == 0, lib.qed_last_error()
    torch.cuda.synchronize()
    return val, grad


def _same(a, b):
    a, b = a.cpu().numpy(), b.cpu().numpy()
    assert np.all(np.isfinite(a)) and np.all(np.isfinite(b))
    return float(np.max(np.abs(a - b) / np.maximum(np.abs(b), 1e-300)))


@pytest.mark.parametrize("n", [4, 2])
def test_noalloc_gradient_matches_workspace_gradient(n):
    from paper_2511_19456_amd._lib import lib
    from paper_2511_19456_amd.qedx import QedProcess
    L = lib()
    wl = inputs.WORKLOADS["grad_n4_sum_rs15_2p18"]
    rs = wl["sqrt_s"]
    u_all, _ = inputs.rambo_inputs(wl["seed"] if n == 4 else 52, n, wl["N"])
    p = QedProcess(n, "sum")
    # first call: 150,000 points (more than one scratch chunk at n = 4)
    u1 = torch.as_tensor(np.ascontiguousarray(u_all[:, :150000]), device=DEV)
    print(f"noalloc n={n} call 1: N={u1.shape[1]}", flush=True)
    v1, g1 = _grad_noalloc(L, p.handle, u1, rs)
    w1, h1 = _grad_ws(L, p.handle, u1, rs)
    assert _same(v1, w1) <= 1e-12 and _same(g1, h1) <= 1e-12
    if n == 4:
        gold = np.load(os.path.join(HERE, "golden", "grad_n4_rs15_seed5_first1024.npz"))
        K = gold["logm2"].shape[0]
        assert np.abs(v1[:K].cpu().numpy() - gold["logm2"]).max() < 1e-10 * max(1.0, np.abs(gold["logm2"]).max())
        gg = g1[:, :K].cpu().numpy()
        err = np.linalg.norm(gg - gold["grad"], axis=0) / np.linalg.norm(gold["grad"], axis=0)
        assert err.max() < 1e-10, err.max()
    # second call, smaller and on other points: runs on what the first left in the scratch
    u2 = torch.as_tensor(np.ascontiguousarray(u_all[:, 200000:203001]), device=DEV)
    print(f"noalloc n={n} call 2: N={u2.shape[1]}", flush=True)
    v2, g2 = _grad_noalloc(L, p.handle, u2, rs)
    w2, h2 = _grad_ws(L, p.handle, u2, rs)
    assert _same(v2, w2) <= 1e-12 and _same(g2, h2) <= 1e-12
    # N = 0 is a no-op; NULL outputs are rejected before anything runs
    st = ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    assert L.qed_eval_grad_noalloc(p.handle, ctypes.c_void_p(u2.data_ptr()), rs, None, 0, None, None, st) == 0
    assert L.qed_eval_grad_noalloc(p.handle, ctypes.c_void_p(u2.data_ptr()), rs, None, 10, None, None, st) == 1
