"""Extended-precision CPU oracle for tree-level multi-photon Compton |M|^2 -- TEST INFRASTRUCTURE ONLY.

Only ``tests/``, ``__graft_entry__.smoke()`` and the ``cpu_baseline`` leg of
``bench.py`` (and the committed scripts under ``tests/golden/`` that write
stored expected values) may import this module.  The HIP library never calls
it and shares no code with it.

What it computes
----------------
The same plain definition as ``qed_oracle`` -- the sum over all orderings in
which the photons attach to the single electron line (Sec. III-A), each
ordering written out with the Feynman rules of Sec. I-D (external bispinors,
polarisation vectors, a vertex gamma^mu per photon, the electron propagator
(Qslash + m)/(Q^2 - m^2) on every inner line; Eq. (1) for one photon) with
explicit 4x4 Dirac matrices -- but in x86 80-bit extended precision
(numpy ``longdouble`` / ``clongdouble``, unit roundoff 5.4e-20) and with
numpy instead of torch.  Its purpose is the oracle's own error estimate: the
float64 oracle forms Q.Q - m^2 plainly and loses digits where a photon goes
soft or collinear; this evaluation of the same formulas carries 11 more bits,
so its difference from the float64 oracle estimates that oracle's error, and
it serves as the reference where the float64 oracle's error is not small.

It also returns two conditioning numbers of every amplitude A_h (a measure of
how much rounding in any evaluation of the diagram sum is amplified):
  kappa_terms = sum_sigma |term_sigma| / |A_h|   (cancellation between diagrams)
  kappa_chain = sum_sigma ||ubar|| prod_j ||S(Q_j)|| ||u|| / |A_h|
with ||S(Q)|| bounded by (m + |Q^0| + |Qvec|) / |Q^2 - m^2| and the vertex
factors of norm 1 (real unit polarisation vectors with eps^0 = 0).
kappa_chain >= kappa_terms; it also sees cancellation inside a diagram's
chain of spinor products (a propagator acting on a spinor it nearly
annihilates), which the per-diagram magnitudes do not show.

Conventions (readings of the paper) are those of ``qed_oracle``: reduced
amplitude (e = 1, overall phase dropped), no spin average, i*epsilon = 0,
Dirac representation, rest-frame z spin boosted to p, linear polarisations in
the theta/phi basis of k-hat (k_T = 0: phi = 0, cos theta = sign k_z),
outgoing photons carry eps* (= eps), helicity bit i belongs to particle i of
[e-_in, gamma_in..., e-_out, gamma_out...] with 0 = spin +1/2 / pol x.
"""
from __future__ import annotations

import itertools

import numpy as np

LD = np.longdouble
CLD = np.clongdouble
M_E = LD(1)


def _pauli():
    s = np.zeros((3, 2, 2), dtype=CLD)
    s[0, 0, 1] = s[0, 1, 0] = 1
    s[1, 0, 1] = -1j
    s[1, 1, 0] = 1j
    s[2, 0, 0] = 1
    s[2, 1, 1] = -1
    return s


def _gammas():
    """gamma^mu in the Dirac representation (Sec. I-D slash notation)."""
    g = np.zeros((4, 4, 4), dtype=CLD)
    g[0, 0, 0] = g[0, 1, 1] = 1
    g[0, 2, 2] = g[0, 3, 3] = -1
    s = _pauli()
    for i in range(3):
        g[i + 1, :2, 2:] = s[i]
        g[i + 1, 2:, :2] = -s[i]
    return g


PAULI = _pauli()
GAMMA = _gammas()
METRIC = np.array([1, -1, -1, -1], dtype=LD)


def mdot(a, b):
    """Minkowski product with metric (+,-,-,-) over the last axis."""
    return a[..., 0] * b[..., 0] - a[..., 1] * b[..., 1] - a[..., 2] * b[..., 2] - a[..., 3] * b[..., 3]


def slash(a):
    """a-slash = gamma^mu a_mu for contravariant a[..., 4]."""
    return np.einsum("...m,mij->...ij", (a * METRIC).astype(CLD), GAMMA)


def spinor_u(p, s):
    """u(p, s) = [sqrt(E+m) chi_s ; (sigma.p) chi_s / sqrt(E+m)], [N, 4]."""
    E = p[:, 0]
    nrm = np.sqrt(E + M_E)
    chi = np.zeros((p.shape[0], 2), dtype=CLD)
    chi[:, s] = 1
    sp = np.einsum("ni,ijk->njk", p[:, 1:4].astype(CLD), PAULI)
    lower = np.einsum("njk,nk->nj", sp, chi) / nrm[:, None]
    return np.concatenate([chi * nrm[:, None], lower], axis=1)


def spinor_ubar(p, s):
    """u-bar = u^dagger gamma^0 as a row, [N, 4]."""
    return np.einsum("ni,ij->nj", np.conj(spinor_u(p, s)), GAMMA[0])


def photon_pol(k, lam):
    """Real linear polarisation eps(k, lam), lam 0 = x, 1 = y, [N, 4]."""
    kx, ky, kz = k[:, 1], k[:, 2], k[:, 3]
    kt = np.sqrt(kx * kx + ky * ky)
    kk = np.sqrt(kx * kx + ky * ky + kz * kz)
    flat = kt == 0
    one = np.ones_like(kt)
    safe = np.where(flat, one, kt)
    cphi = np.where(flat, one, kx / safe)
    sphi = np.where(flat, 0 * one, ky / safe)
    cth = np.where(flat, np.sign(kz), kz / np.where(kk == 0, one, kk))
    sth = np.where(flat, 0 * one, kt / np.where(kk == 0, one, kk))
    z = np.zeros_like(kx)
    if lam == 0:
        return np.stack([z, cth * cphi, cth * sphi, -sth], axis=1)
    return np.stack([z, -sphi, cphi, z], axis=1)


def amplitudes(mom, hel, n_out, n_in=1):
    """A_h for one helicity code per point, with both conditioning numbers.

    mom: [N, n_in + n_out + 2, 4] (promoted to long double exactly);
    hel: [N] integer codes.  Returns (A [N] complex, kappa_terms [N],
    kappa_chain [N]).  A = sum over photon orderings sigma of
    ubar(p') w_sig(P) S(Q_{P-1}) ... S(Q_1) w_sig(1) u(p) with
    Q_j = p + sum_{i<=j} ktilde_sig(i), ktilde = +k (incoming), -k' (outgoing).
    """
    mom = np.asarray(mom).astype(LD)
    hel = np.asarray(hel).astype(np.int64)
    N = mom.shape[0]
    P = n_in + n_out
    i_ein, i_eout = 0, 1 + n_in
    photon_idx = list(range(1, 1 + n_in)) + list(range(2 + n_in, 2 + n_in + n_out))
    sign = [LD(1)] * n_in + [LD(-1)] * n_out
    p_in, p_out = mom[:, i_ein], mom[:, i_eout]
    u = np.where(((hel >> i_ein) & 1)[:, None] == 0, spinor_u(p_in, 0), spinor_u(p_in, 1))
    ub = np.where(((hel >> i_eout) & 1)[:, None] == 0, spinor_ubar(p_out, 0), spinor_ubar(p_out, 1))
    nu = np.sqrt(2 * p_in[:, 0]) * np.sqrt(2 * p_out[:, 0])   # ||u|| ||ubar||
    ws, kt = [], []
    for j, pi in enumerate(photon_idx):
        k = mom[:, pi]
        kt.append(sign[j] * k)
        lam = (hel >> pi) & 1
        e = np.where(lam[:, None] == 0, photon_pol(k, 0), photon_pol(k, 1))
        ws.append(slash(e))
    A = np.zeros(N, dtype=CLD)
    l1 = np.zeros(N, dtype=LD)
    ch = np.zeros(N, dtype=LD)
    for sigma in itertools.permutations(range(P)):
        v = u
        Q = p_in
        bound = np.ones(N, dtype=LD)
        for i, a in enumerate(sigma):
            v = np.einsum("nij,nj->ni", ws[a], v)
            if i < P - 1:
                Q = Q + kt[a]
                den = mdot(Q, Q) - M_E * M_E
                S = (slash(Q) + M_E * np.eye(4, dtype=CLD)) / den[:, None, None]
                v = np.einsum("nij,nj->ni", S, v)
                bound = bound * (M_E + np.abs(Q[:, 0]) + np.sqrt((Q[:, 1:] ** 2).sum(1))) / np.abs(den)
        term = (ub * v).sum(1)
        A = A + term
        l1 = l1 + np.abs(term)
        ch = ch + bound
    aa = np.abs(A)
    with np.errstate(divide="ignore", invalid="ignore"):   # an amplitude can vanish exactly
        return A, l1 / aa, ch * nu / aa


def m2_per_point(mom, hel, n_out, n_in=1):
    """(|A_h|^2 [N], kappa_terms [N], kappa_chain [N]) in long double."""
    A, kt, kc = amplitudes(mom, hel, n_out, n_in)
    return (A.real ** 2 + A.imag ** 2), kt, kc


def m2_sum(mom, n_out, n_in=1):
    """sum over all 2^(n_in+n_out+2) configurations of |A_h|^2, [N] long double."""
    mom = np.asarray(mom).astype(LD)
    N = mom.shape[0]
    tot = np.zeros(N, dtype=LD)
    for h in range(1 << (n_in + n_out + 2)):
        A, _, _ = amplitudes(mom, np.full(N, h), n_out, n_in)
        tot = tot + A.real ** 2 + A.imag ** 2
    return tot


def soa_to_points(m_soa):
    """SoA [4 npart][N] -> [N, npart, 4] (long double)."""
    t = np.asarray(m_soa).astype(LD)
    npart = t.shape[0] // 4
    return np.ascontiguousarray(t.reshape(npart, 4, -1).transpose(2, 0, 1))
