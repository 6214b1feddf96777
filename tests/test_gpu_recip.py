"""Accuracy of the kernels' reciprocal and reciprocal square root.

The generated kernels divide by propagator denominators and take 1/sqrt for
spinor normalisations and polarisation vectors through qx::rcp and
qx::rsqrt of the device header: the hardware estimate refined by two
Newton-Raphson steps, not correctly rounded.  This checks, through the
measurement library's reciprocal probe, that both stay within one ulp of
the exact values (computed in x86 extended precision) over the range of
magnitudes the kernels see, with both signs for the reciprocal.
"""
import ctypes

import numpy as np
import pytest

from paper_2511_19456_amd import _lib

def _ulps(got, exact):
    e = exact.astype(np.float64)
    return np.abs(got.astype(np.longdouble) - exact) / np.spacing(np.abs(e)).astype(np.longdouble)


@pytest.mark.gpu
def test_device_reciprocals_accuracy():
    import torch

    rng = np.random.default_rng(11)
    n = 1 << 20
    x = rng.uniform(1.0, 2.0, n) * np.exp2(np.floor(rng.uniform(-12.0, 12.0, n)))
    x[1::2] *= -1.0
    print(f"reciprocal probe: {n} inputs, seed 11", flush=True)
    xd = torch.as_tensor(x, device="cuda:0")
    r = torch.empty_like(xd)
    q = torch.empty_like(xd)
    stream = ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    _lib.check(_lib.probe_lib().qed_recip_probe(ctypes.c_void_p(xd.data_ptr()), n, ctypes.c_void_p(r.data_ptr()),
                                                 ctypes.c_void_p(q.data_ptr()), stream))
    torch.cuda.synchronize()
    xl = x.astype(np.longdouble)
    ur = _ulps(r.cpu().numpy(), 1.0 / xl)
    uq = _ulps(q.cpu().numpy(), 1.0 / np.sqrt(np.abs(xl)))
    print(f"rcp max {ur.max():.3f} ulp, rsqrt max {uq.max():.3f} ulp", flush=True)
    assert float(ur.max()) <= 1.0
    assert float(uq.max()) <= 1.0


def test_recip_probe_rejects_bad_arguments():
    # argument checks run before any HIP call (no GPU needed)
    P = _lib.probe_lib()
    assert P.qed_recip_probe(None, 0, None, None, None) == _lib.QED_ERR_INVALID_ARG
    assert P.qed_recip_probe(None, 16, None, None, None) == _lib.QED_ERR_INVALID_ARG
