"""Parity bounds for per-configuration values, from the oracle's own terms.

One spin/polarisation configuration of a point can be much smaller than the
diagrams that sum to it (Sec. III-A: the amplitude is the sum over all photon
orderings).  Rounding then costs digits in any evaluation, the oracle's and
the kernels' alike, in proportion to the cancellation
kappa = sum_sigma |term_sigma| / |A_h| over the orderings sigma.  The per-point
tests therefore allow

    |got - ref| <= (REL + 2 C eps kappa) |ref|,        eps = 2^-53,

for float64 (REL = 1e-10, the stated tolerance; the factor 2 takes the error
of A to |A|^2), with C = C_FP64 roundings per term: every term is a chain of
at most 2P - 1 sparse 4x4 products (P photons), each entry of which takes at
most 8 rounded operations, plus the external states; C = 64 covers P <= 7 with
room, and the tests fail if a point needs more.  Where kappa is of order one
this is the plain 1e-10 relative tolerance.
"""
from __future__ import annotations

import numpy as np
import torch

from oracle import qed_oracle as O

REL_FP64 = 1e-10
C_FP64 = 64.0
EPS64 = 2.0 ** -53


def per_point_ref(mom_soa, n: int, hel, n_in: int = 1, chunk: int = 1024):
    """Oracle |A_h|^2 for one configuration per point and kappa (float64)."""
    pts = O.soa_to_points(mom_soa)
    proc = O.Process(n, n_in=n_in)
    hh = torch.as_tensor(np.asarray(hel).astype(np.int64))
    vals, kaps = [], []
    for s in range(0, pts.shape[0], chunk):
        A, absterms = O.amplitudes(pts[s:s + chunk], hh[s:s + chunk].reshape(-1, 1), proc, want_abs_terms=True)
        a = A[:, 0].abs()
        vals.append((A.real ** 2 + A.imag ** 2)[:, 0])
        kaps.append(absterms[:, 0] / a)
    if not vals:
        return np.zeros(0), np.zeros(0)
    return torch.cat(vals).numpy(), torch.cat(kaps).numpy()


def fp64_allowed(ref, kappa, rel: float = REL_FP64):
    """Allowed |got - ref| per point for float64 parity."""
    return (rel + 2.0 * C_FP64 * EPS64 * np.asarray(kappa)) * np.abs(ref)


def check_fp64(got, ref, kappa, what: str = "", rel: float = REL_FP64):
    """Assert float64 parity point by point; report the worst point."""
    got, ref, kappa = np.asarray(got), np.asarray(ref), np.asarray(kappa)
    err = np.abs(got - ref)
    ok = err <= fp64_allowed(ref, kappa, rel)
    if not ok.all():
        i = int(np.argmax(err / fp64_allowed(ref, kappa, rel)))
        raise AssertionError(f"{what}: {int((~ok).sum())} of {len(ok)} points outside the bound; worst point {i}: "
                             f"got {got[i]!r} ref {ref[i]!r} rel {err[i] / abs(ref[i]):.3e} kappa {kappa[i]:.3e}")
    return float((err / np.abs(ref)).max()) if len(ref) else 0.0


def rambo_boost_gamma(u, n: int):
    """Per point, the boost factor gamma = Q^0 / M of RAMBO's massless stage
    (the isotropic momenta q_j drawn from the uniforms sum to Q, M^2 = Q.Q).

    RAMBO forms M from Q^0^2 - |Q|^2, which cancels by ~gamma^2, and its
    boost adds terms each ~gamma^2 larger than their sum; rounding in any
    float64 evaluation of the map (the device's and the oracle's alike) is
    therefore amplified by up to ~gamma^4.  Used only to scale tolerances."""
    u = np.asarray(u, dtype=np.float64)
    Q = np.zeros((4, u.shape[1]))
    for j in range(n + 1):
        c = 2.0 * u[4 * j] - 1.0
        ph = 2.0 * np.pi * u[4 * j + 1]
        q0 = -np.log(u[4 * j + 2] * u[4 * j + 3])
        st = np.sqrt(np.maximum(0.0, 1.0 - c * c))
        Q += np.stack([q0, q0 * st * np.cos(ph), q0 * st * np.sin(ph), q0 * c])
    M = np.sqrt(np.maximum(Q[0] ** 2 - (Q[1:] ** 2).sum(0), 1e-300))
    return Q[0] / M


def rambo_allowed(u, n: int, sqrt_s: float):
    """Allowed |device - oracle| per point for RAMBO momenta: 1e-12 sqrt(s),
    or 16 eps gamma^4 sqrt(s) where the massless boost is large."""
    g = rambo_boost_gamma(u, n)
    return sqrt_s * np.maximum(1e-12, 16.0 * EPS64 * g ** 4)


def check_rambo(mom_dev, ref_mom, u, n: int, sqrt_s: float, what: str = ""):
    """Assert device RAMBO momenta [rows][N] against the oracle's, per point."""
    d = np.abs(np.asarray(mom_dev) - np.asarray(ref_mom)).max(axis=0)
    lim = rambo_allowed(u, n, sqrt_s)
    ok = d <= lim
    if not ok.all():
        i = int(np.argmax(d / lim))
        raise AssertionError(f"{what}: RAMBO momenta off at {int((~ok).sum())} points; worst {i}: "
                             f"diff {d[i]:.3e} allowed {lim[i]:.3e} gamma {rambo_boost_gamma(u[:, i:i + 1], n)[0]:.2f}")
