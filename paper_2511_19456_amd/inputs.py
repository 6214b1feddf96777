"""Seeded synthetic inputs shared by the oracle side and the HIP side.

This module draws random numbers and lays out kinematic inputs; it holds none
of the matrix-element arithmetic and none of the phase-space map.  Both the
CPU oracle (under ``oracle/``) and the HIP path consume exactly these arrays.

Generators
----------
* ``uniforms(seed, dims, N)``: float64 ``[dims][N]`` (C order) from numpy's
  PCG64 stream seeded with ``seed``.  These are the RAMBO inputs: particle ``i``
  of the final state uses rows ``4i .. 4i+3``.
* ``helicities(rng, n, N)``: one helicity configuration per point, drawn from
  the same stream after the uniforms (bit ``i`` belongs to external particle
  ``i`` in the order [e-_in, gamma_in, e-_out, gamma_out_1..n]; 0 means spin
  +1/2 or linear polarisation x, 1 means spin -1/2 or polarisation y).
* ``compton_lab_momenta(seed, N, omega)``: the one-photon workload with the
  electron at rest (m = 1) and the photon along +z; the outgoing photon angle is
  cos(theta) ~ U(-1,1), phi ~ U(0, 2 pi).  The outgoing photon energy follows
  from two-body kinematics, and the outgoing electron from momentum
  conservation.  Returned SoA ``[16][N]`` (row = 4 * particle + mu).
* ``crossed_inputs(seed, n_in, N)``: e- gamma^n_in -> e- gamma, electron at
  rest, incoming photons with random energies and directions, the outgoing
  photon isotropic in the centre-of-mass frame (two-body kinematics).
* ``mixed_batch_spec(seed)``: per-process point counts ``round(10**U(3,6))`` and
  centre-of-mass energies ``sqrt(s) ~ U(5,30)`` for n = 1..6.

The paper's own workloads (Sec. III: n-photon Compton processes) are
synthetic by nature; no dataset is involved.
"""
from __future__ import annotations

import math

import numpy as np

ELECTRON_MASS = 1.0


def rng_for(seed: int) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(seed))


def uniforms(seed: int, dims: int, n_points: int, rng: np.random.Generator | None = None) -> np.ndarray:
    """Float64 uniforms in (0,1), shape ``[dims][n_points]``, C order."""
    g = rng if rng is not None else rng_for(seed)
    u = g.random((dims, n_points), dtype=np.float64)
    # RAMBO takes logs of u; an exact 0 has probability 2^-53 per draw but
    # would give an infinite energy, so it is mapped to the smallest normal.
    np.maximum(u, np.finfo(np.float64).tiny, out=u)
    return np.ascontiguousarray(u)


def helicities(rng: np.random.Generator, n_photons_out: int, n_points: int) -> np.ndarray:
    """Random helicity configurations, uint32 ``[n_points]``, values < 2^(n+3)."""
    h = rng.integers(0, 1 << (n_photons_out + 3), size=n_points, dtype=np.int64)
    return h.astype(np.uint32)


def rambo_inputs(seed: int, n_photons_out: int, n_points: int, with_helicities: bool = False):
    """Uniforms for an (n+1)-body final state, then (optionally) helicities.

    Returns ``(u, hel)`` with ``u`` of shape ``[4(n+1)][N]`` and ``hel`` None
    unless requested.
    """
    g = rng_for(seed)
    u = uniforms(seed, 4 * (n_photons_out + 1), n_points, rng=g)
    hel = helicities(g, n_photons_out, n_points) if with_helicities else None
    return u, hel


def compton_lab_momenta(seed: int, n_points: int, omega: float = 1.0) -> np.ndarray:
    """One-photon Compton momenta in the electron rest frame, SoA [16][N].

    Particle order: e-_in, gamma_in, e-_out, gamma_out.  The photon comes in
    along +z with energy ``omega``; the outgoing photon direction is drawn as
    cos(theta) = 2u-1, phi = 2 pi u'.  Two-body kinematics fix its energy to
    omega' = omega / (1 + omega (1 - cos(theta))) (m = 1).
    """
    u = uniforms(seed, 2, n_points)
    m = ELECTRON_MASS
    ct = 2.0 * u[0] - 1.0
    st = np.sqrt(np.maximum(0.0, 1.0 - ct * ct))
    ph = 2.0 * math.pi * u[1]
    w2 = omega / (1.0 + (omega / m) * (1.0 - ct))
    mom = np.zeros((16, n_points), dtype=np.float64)
    # e-_in at rest
    mom[0] = m
    # gamma_in along +z
    mom[4] = omega
    mom[7] = omega
    # gamma_out
    mom[12] = w2
    mom[13] = w2 * st * np.cos(ph)
    mom[14] = w2 * st * np.sin(ph)
    mom[15] = w2 * ct
    # e-_out = p + k - k'
    mom[8:12] = mom[0:4] + mom[4:8] - mom[12:16]
    return np.ascontiguousarray(mom)


def compton_lab_angles(theta: np.ndarray, phi: np.ndarray, omega: float = 1.0) -> np.ndarray:
    """Same kinematics as :func:`compton_lab_momenta` at given angles (fixtures)."""
    theta = np.asarray(theta, dtype=np.float64)
    phi = np.asarray(phi, dtype=np.float64)
    m = ELECTRON_MASS
    ct, st = np.cos(theta), np.sin(theta)
    w2 = omega / (1.0 + (omega / m) * (1.0 - ct))
    n = theta.shape[0]
    mom = np.zeros((16, n), dtype=np.float64)
    mom[0] = m
    mom[4] = omega
    mom[7] = omega
    mom[12] = w2
    mom[13] = w2 * st * np.cos(phi)
    mom[14] = w2 * st * np.sin(phi)
    mom[15] = w2 * ct
    mom[8:12] = mom[0:4] + mom[4:8] - mom[12:16]
    return np.ascontiguousarray(mom)


def crossed_inputs(seed: int, n_in: int, n_points: int, with_helicities: bool = False,
                   omega_lo: float = 0.5, omega_hi: float = 2.0):
    """Momenta of e- gamma^n_in -> e- gamma (the Table I orientation), SoA
    ``[4(n_in+3)][N]`` in the order [e-_in, gamma_in_1..n_in, e-_out, gamma_out].

    The electron is at rest (m = 1).  Incoming photon i has energy
    omega_i ~ U(omega_lo, omega_hi) and an isotropic direction.  The outgoing
    photon is isotropic in the centre-of-mass frame of the total momentum P,
    with energy (s - m^2) / (2 sqrt(s)) there, and is boosted back along
    P/P^0; the outgoing electron is P minus that photon.  Draws 3 n_in + 2
    uniform rows, then (optionally) one helicity code < 2^(n_in+3) per point.
    Returns ``(mom, hel)``.
    """
    g = rng_for(seed)
    u = uniforms(seed, 3 * n_in + 2, n_points, rng=g)
    m = ELECTRON_MASS
    npart = n_in + 3
    mom = np.zeros((4 * npart, n_points), dtype=np.float64)
    mom[0] = m
    for i in range(n_in):
        w = omega_lo + (omega_hi - omega_lo) * u[3 * i]
        ct = 2.0 * u[3 * i + 1] - 1.0
        st = np.sqrt(np.maximum(0.0, 1.0 - ct * ct))
        ph = 2.0 * math.pi * u[3 * i + 2]
        r = 4 * (1 + i)
        mom[r] = w
        mom[r + 1] = w * st * np.cos(ph)
        mom[r + 2] = w * st * np.sin(ph)
        mom[r + 3] = w * ct
    P = mom[0:4 * (n_in + 1)].reshape(n_in + 1, 4, n_points).sum(axis=0)
    s = P[0] ** 2 - P[1] ** 2 - P[2] ** 2 - P[3] ** 2
    rs = np.sqrt(s)
    q = (s - m * m) / (2.0 * rs)
    ct = 2.0 * u[3 * n_in] - 1.0
    st = np.sqrt(np.maximum(0.0, 1.0 - ct * ct))
    ph = 2.0 * math.pi * u[3 * n_in + 1]
    kc = np.stack([q * st * np.cos(ph), q * st * np.sin(ph), q * ct])
    beta = P[1:] / P[0]
    gam = P[0] / rs
    bk = (beta * kc).sum(axis=0)
    k0 = gam * (q + bk)
    kv = kc + beta * gam * (gam / (gam + 1.0) * bk + q)
    ro = 4 * (n_in + 2)
    mom[ro] = k0
    mom[ro + 1:ro + 4] = kv
    re = 4 * (n_in + 1)
    mom[re:re + 4] = P - mom[ro:ro + 4]
    hel = None
    if with_helicities:
        hel = g.integers(0, 1 << npart, size=n_points, dtype=np.int64).astype(np.uint32)
    return np.ascontiguousarray(mom), hel


def mixed_batch_spec(seed: int, n_values=(1, 2, 3, 4, 5, 6)):
    """Per-process point counts and sqrt(s) for the mixed-process batch.

    N_n = round(10**U(3,6)); sqrt(s)_n ~ U(5, 30).  Returns a list of
    ``(n, N, sqrt_s, sub_seed)`` tuples; ``sub_seed`` seeds that process's
    uniforms and helicities.
    """
    g = rng_for(seed)
    out = []
    for n in n_values:
        npts = int(round(10.0 ** g.uniform(3.0, 6.0)))
        rs = float(g.uniform(5.0, 30.0))
        out.append((n, npts, rs, 1000 * seed + n))
    return out


# Workload table: (name, n, mode, N, sqrt_s, seed).  mode "sum" sums all
# 2^(n+3) helicity configurations; "per_point" takes one per point.
WORKLOADS = {
    "compton_n1_sum_65536": dict(n=1, mode="sum", N=65536, sqrt_s=None, seed=1),
    "n3_sum_rs10_2p20": dict(n=3, mode="sum", N=1 << 20, sqrt_s=10.0, seed=2),
    "n5_perpoint_rs20_2p20": dict(n=5, mode="per_point", N=1 << 20, sqrt_s=20.0, seed=3),
    "mixed_n1to6": dict(n=None, mode="per_point", N=None, sqrt_s=None, seed=4),
    "grad_n4_sum_rs15_2p18": dict(n=4, mode="sum", N=1 << 18, sqrt_s=15.0, seed=5),
}
