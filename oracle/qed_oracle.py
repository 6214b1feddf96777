"""CPU oracle for tree-level multi-photon Compton |M|^2 -- TEST INFRASTRUCTURE ONLY.

Only ``tests/``, ``__graft_entry__.smoke()`` and the ``cpu_baseline`` leg of
``bench.py`` may import this module.  The HIP library never calls it, shares no
code with it, and must fail loudly when its own extension is missing.

What it computes
----------------
The squared matrix element of e-(p) gamma(k) -> e-(p') gamma(k'_1) .. gamma(k'_n)
at tree level, written out as the plain definition: the sum over all (n+1)!
orderings in which the photons attach to the single electron line (Sec. III-A),
each ordering evaluated with the QED Feynman rules of Sec. I-D -- external
bispinors u, u-bar, photon polarisation vectors, a vertex gamma^mu per photon and
the electron propagator S(Q) = (Qslash + m)/(Q^2 - m^2) on every inner line --
with explicit 4x4 Dirac matrices in complex128.  For one photon this is Eq. (1).
All arithmetic is float64 / complex128; the only library primitives are small
matrix products, and automatic differentiation for the gradient.

Readings where the paper is silent:
* Reduced amplitude: the coupling and the overall phase (-ie)^(n+1) i^n are
  dropped, i.e. e = 1; |M|^2 reported is sum |A_h|^2 with no spin average.
* iepsilon in S(Q) is set to 0 (no inner line can go on shell for this process
  with m > 0).
* Dirac representation; electron spin states are rest-frame z spin boosted to
  p: u = [sqrt(E+m) chi ; (sigma.p) chi / sqrt(E+m)], chi_+ = (1,0), chi_- = (0,1).
* Linear photon polarisations in the frame the momenta are given in:
  eps_x = (0; cos t cos f, cos t sin f, -sin t), eps_y = (0; -sin f, cos f, 0),
  with k-hat = (sin t cos f, sin t sin f, cos t); for k_T = 0 take f = 0 and
  cos t = sign(k_z).  Outgoing photons carry eps* (= eps, real).
* Helicity code: bit i belongs to external particle i in the order
  [e-_in, gamma_in..., e-_out, gamma_out...]; 0 = spin +1/2 or pol x,
  1 = spin -1/2 or pol y.
* Phase space: RAMBO (Kleiss, Stirling, Ellis 1986), massless momenta rescaled
  to the final-state masses by a Newton solve for the common factor xi.  The
  incoming pair is in its CM frame with the photon along +z.

Parity pins (tests/test_oracle_*.py): Klein-Nishina (unpolarised and
polarised), Ward identity, Lorentz invariance of the helicity sum, Bose
symmetry of the outgoing photons, the (n+1)! diagram count, the soft-photon
(eikonal) limit relating n to n-1 photons, Dirac algebra identities, RAMBO
momentum conservation / mass shells / two-body closed form, and central finite
differences for the gradient.
"""
from __future__ import annotations

import itertools
import math
from typing import Iterable, Sequence

import torch

M_E = 1.0
F64 = torch.float64
C128 = torch.complex128

# ---------------------------------------------------------------------------
# Dirac algebra (Sec. I-D: slash notation a-slash = gamma^mu a_mu)
# ---------------------------------------------------------------------------
METRIC = torch.tensor([1.0, -1.0, -1.0, -1.0], dtype=F64)


def pauli() -> torch.Tensor:
    s1 = torch.tensor([[0, 1], [1, 0]], dtype=C128)
    s2 = torch.tensor([[0, -1j], [1j, 0]], dtype=C128)
    s3 = torch.tensor([[1, 0], [0, -1]], dtype=C128)
    return torch.stack([s1, s2, s3])


def gamma_dirac() -> torch.Tensor:
    """gamma^mu, mu = 0..3, in the Dirac representation, shape [4,4,4]."""
    g = torch.zeros(4, 4, 4, dtype=C128)
    eye2 = torch.eye(2, dtype=C128)
    g[0, :2, :2] = eye2
    g[0, 2:, 2:] = -eye2
    s = pauli()
    for i in range(3):
        g[i + 1, :2, 2:] = s[i]
        g[i + 1, 2:, :2] = -s[i]
    return g


GAMMA = gamma_dirac()
EYE4 = torch.eye(4, dtype=C128)


def mdot(a: torch.Tensor, b: torch.Tensor) -> torch.Tensor:
    """Minkowski product a.b with metric (+,-,-,-) over the last axis."""
    return a[..., 0] * b[..., 0] - a[..., 1] * b[..., 1] - a[..., 2] * b[..., 2] - a[..., 3] * b[..., 3]


def slash(a: torch.Tensor) -> torch.Tensor:
    """a-slash = gamma^mu a_mu for contravariant a[..., 4] (real or complex)."""
    a = a.to(C128)
    low = a * METRIC.to(C128)
    return torch.einsum("...m,mij->...ij", low, GAMMA)


# ---------------------------------------------------------------------------
# External states (Sec. II-B: base_state per species and spin/polarisation)
# ---------------------------------------------------------------------------
def spinor_u(p: torch.Tensor, s: int) -> torch.Tensor:
    """Dirac spinor u(p, s) for momentum p[..., 4]; s = 0 (+1/2) or 1 (-1/2)."""
    E = p[..., 0]
    nrm = torch.sqrt(E + M_E)
    chi = torch.zeros(p.shape[:-1] + (2,), dtype=C128)
    chi[..., s] = 1.0
    sig = pauli()
    pvec = p[..., 1:4].to(C128)
    sp = torch.einsum("...i,ijk->...jk", pvec, sig)  # sigma . p
    lower = torch.einsum("...jk,...k->...j", sp, chi) / nrm[..., None]
    upper = chi * nrm[..., None]
    return torch.cat([upper, lower], dim=-1)


def spinor_ubar(p: torch.Tensor, s: int) -> torch.Tensor:
    """u-bar = u^dagger gamma^0, returned as a row vector [..., 4]."""
    u = spinor_u(p, s)
    return torch.einsum("...i,ij->...j", u.conj(), GAMMA[0])


def photon_pol(k: torch.Tensor, lam: int) -> torch.Tensor:
    """Linear polarisation vector eps(k, lam), lam = 0 (x) or 1 (y), real, [..., 4]."""
    kx, ky, kz = k[..., 1], k[..., 2], k[..., 3]
    kt = torch.sqrt(kx * kx + ky * ky)
    kk = torch.sqrt(kx * kx + ky * ky + kz * kz)
    flat = kt == 0
    safe_kt = torch.where(flat, torch.ones_like(kt), kt)
    cphi = torch.where(flat, torch.ones_like(kt), kx / safe_kt)
    sphi = torch.where(flat, torch.zeros_like(kt), ky / safe_kt)
    cth = torch.where(flat, torch.sign(kz), kz / kk)
    sth = torch.where(flat, torch.zeros_like(kt), kt / kk)
    zero = torch.zeros_like(kx)
    if lam == 0:
        return torch.stack([zero, cth * cphi, cth * sphi, -sth], dim=-1)
    return torch.stack([zero, -sphi, cphi, zero], dim=-1)


# ---------------------------------------------------------------------------
# Process description
# ---------------------------------------------------------------------------
class Process:
    """e-(p) + n_in photons -> e-(p') + n_out photons, one electron line.

    Particle order: [e-_in, gamma_in_1..n_in, e-_out, gamma_out_1..n_out].
    The workloads here use n_in = 1; the paper's Table I processes use
    n_out = 1 (Sec. III); both have (n_in + n_out)! diagrams.
    """

    def __init__(self, n_out: int, n_in: int = 1):
        self.n_in = n_in
        self.n_out = n_out
        self.n_photons = n_in + n_out
        self.n_particles = n_in + n_out + 2
        self.i_ein = 0
        self.i_eout = 1 + n_in
        self.photon_idx = list(range(1, 1 + n_in)) + list(range(2 + n_in, 2 + n_in + n_out))
        # +1 for momentum flowing into the electron line (incoming photon)
        self.photon_sign = [1.0] * n_in + [-1.0] * n_out
        self.n_hel = 1 << self.n_particles

    def n_diagrams(self) -> int:
        return sum(1 for _ in self.orderings())

    def orderings(self) -> Iterable[tuple]:
        """All orders in which the photons attach to the electron line (Sec. III-A)."""
        return itertools.permutations(range(self.n_photons))


# ---------------------------------------------------------------------------
# Amplitude: plain per-diagram Feynman rules (Sec. I-D Eq. (1), Sec. II-B)
# ---------------------------------------------------------------------------
def _gather_bits(states2: torch.Tensor, hel: torch.Tensor, bit: int) -> torch.Tensor:
    """states2 [N,2,...] -> [N,K,...] picking state ((hel >> bit) & 1)."""
    idx = (hel >> bit) & 1  # [N,K]
    shape = idx.shape + states2.shape[2:]
    ix = idx.reshape(idx.shape + (1,) * (states2.dim() - 2)).expand(shape)
    return torch.gather(states2, 1, ix)


def amplitudes(mom: torch.Tensor, hel: torch.Tensor, proc: Process,
               photon_override: dict | None = None, want_abs_terms: bool = False):
    """Reduced amplitudes A_h for each point and requested helicity code.

    mom: float64 [N, n_particles, 4]; hel: int64 [N, K] helicity codes.
    photon_override: optional {photon number j: complex [N,K,4]} replacing the
    polarisation vector of photon j (used for the Ward identity).
    Returns A [N, K] complex128 (and sum_sigma |A_sigma| if requested).

    A_h = sum over orderings sigma of
          ubar(p') w_sig(P) S(Q_{P-1}) ... S(Q_1) w_sig(1) u(p),
    Q_j = p + sum_{i<=j} ktilde_sig(i), ktilde = +k (incoming), -k' (outgoing),
    w = eps (incoming) or eps* (outgoing).
    """
    N, K = hel.shape
    p_in = mom[:, proc.i_ein, :]
    p_out = mom[:, proc.i_eout, :]
    u2 = torch.stack([spinor_u(p_in, 0), spinor_u(p_in, 1)], dim=1)          # [N,2,4]
    ub2 = torch.stack([spinor_ubar(p_out, 0), spinor_ubar(p_out, 1)], dim=1)  # [N,2,4]
    u = _gather_bits(u2, hel, proc.i_ein)       # [N,K,4]
    ub = _gather_bits(ub2, hel, proc.i_eout)    # [N,K,4]

    P = proc.n_photons
    wslash = []
    ktil = []
    for j, pi in enumerate(proc.photon_idx):
        k = mom[:, pi, :]
        ktil.append(proc.photon_sign[j] * k)
        if photon_override is not None and j in photon_override:
            w = photon_override[j]
        else:
            e2 = torch.stack([photon_pol(k, 0), photon_pol(k, 1)], dim=1).to(C128)
            if proc.photon_sign[j] < 0:
                e2 = e2.conj()
            w = _gather_bits(e2, hel, pi)
        wslash.append(slash(w))                   # [N,K,4,4]

    A = torch.zeros(N, K, dtype=C128)
    absterms = torch.zeros(N, K, dtype=F64) if want_abs_terms else None
    for sigma in proc.orderings():
        v = u
        Q = p_in
        for i, a in enumerate(sigma):
            v = torch.matmul(wslash[a], v[..., None])[..., 0]
            if i < P - 1:
                Q = Q + ktil[a]
                den = mdot(Q, Q) - M_E * M_E
                S = (slash(Q) + M_E * EYE4) / den[:, None, None].to(C128)
                v = torch.matmul(S[:, None, :, :], v[..., None])[..., 0]
        term = (ub * v).sum(-1)
        A = A + term
        if want_abs_terms:
            absterms = absterms + term.abs()
    if want_abs_terms:
        return A, absterms
    return A


def all_helicities(N: int, proc: Process) -> torch.Tensor:
    return torch.arange(proc.n_hel, dtype=torch.int64)[None, :].expand(N, proc.n_hel).contiguous()


def m2_sum(mom: torch.Tensor, proc: Process) -> torch.Tensor:
    """sum over all 2^(n+3) spin/polarisation configurations of |A_h|^2, [N]."""
    A = amplitudes(mom, all_helicities(mom.shape[0], proc), proc)
    return (A.real ** 2 + A.imag ** 2).sum(-1)


def m2_per_point(mom: torch.Tensor, hel: torch.Tensor, proc: Process) -> torch.Tensor:
    """|A_{h_i}|^2 for one helicity code per point, [N]."""
    A = amplitudes(mom, hel.to(torch.int64).reshape(-1, 1), proc)[:, 0]
    return A.real ** 2 + A.imag ** 2


# ---------------------------------------------------------------------------
# Layout helpers (SoA [4 * particle + mu][N] <-> [N, particle, 4])
# ---------------------------------------------------------------------------
def soa_to_points(m_soa) -> torch.Tensor:
    t = torch.as_tensor(m_soa, dtype=F64)
    npart = t.shape[0] // 4
    return t.reshape(npart, 4, -1).permute(2, 0, 1).contiguous()


def points_to_soa(mom: torch.Tensor) -> torch.Tensor:
    N, npart, _ = mom.shape
    return mom.permute(1, 2, 0).reshape(4 * npart, N).contiguous()


def m2(m_soa, n: int, mode: str, hel=None, chunk: int = 2048, n_in: int = 1) -> torch.Tensor:
    """|M|^2 in reduced units for SoA momenta ``[4(n+n_in+2)][N]`` of
    e- gamma^n_in -> e- gamma^n; mode 'sum' or 'per_point'."""
    mom = soa_to_points(m_soa)
    proc = Process(n, n_in=n_in)
    outs = []
    for s in range(0, mom.shape[0], chunk):
        mm = mom[s:s + chunk]
        if mode == "sum":
            outs.append(m2_sum(mm, proc))
        else:
            hh = torch.as_tensor(hel[s:s + chunk].astype("int64"))
            outs.append(m2_per_point(mm, hh, proc))
    return torch.cat(outs) if outs else torch.zeros(0, dtype=F64)


# ---------------------------------------------------------------------------
# Phase space: RAMBO (Kleiss, Stirling, Ellis, Comput. Phys. Commun. 40 (1986) 359)
# ---------------------------------------------------------------------------
def incoming_cm(sqrt_s: float, N: int):
    """e-_in and gamma_in in their CM frame, photon along +z (m = 1)."""
    s = sqrt_s * sqrt_s
    kap = (s - M_E * M_E) / (2.0 * sqrt_s)
    E = (s + M_E * M_E) / (2.0 * sqrt_s)
    p = torch.tensor([E, 0.0, 0.0, -kap], dtype=F64).expand(N, 4)
    k = torch.tensor([kap, 0.0, 0.0, kap], dtype=F64).expand(N, 4)
    return p, k


def rambo(u: torch.Tensor, sqrt_s: float, masses: Sequence[float], max_iter: int = 50) -> torch.Tensor:
    """Final-state momenta [N, nf, 4] from uniforms u[4 nf, N] (differentiable).

    Steps: isotropic massless q_i with q0 = -ln(u2 u3); a Lorentz boost and
    scaling that bring sum q to (sqrt_s, 0); then a common rescale xi of the
    three-momenta solving sum sqrt(m_i^2 + xi^2 |p_i|^2) = sqrt_s by Newton.
    """
    nf = len(masses)
    u = u.reshape(nf, 4, -1)
    c = 2.0 * u[:, 0] - 1.0
    phi = 2.0 * math.pi * u[:, 1]
    q0 = -torch.log(u[:, 2] * u[:, 3])
    st = torch.sqrt(1.0 - c * c)
    q = torch.stack([q0, q0 * st * torch.cos(phi), q0 * st * torch.sin(phi), q0 * c], dim=-1)  # [nf,N,4]
    Qs = q.sum(0)  # [N,4]
    Mq = torch.sqrt(mdot(Qs, Qs))
    b = -Qs[:, 1:] / Mq[:, None]
    gam = Qs[:, 0] / Mq
    a = 1.0 / (1.0 + gam)
    x = sqrt_s / Mq
    bq = (b[None] * q[..., 1:]).sum(-1)  # [nf,N]
    p0 = x[None] * (gam[None] * q[..., 0] + bq)
    pv = x[None, :, None] * (q[..., 1:] + b[None] * q[..., 0:1] + a[None, :, None] * bq[..., None] * b[None])
    m = torch.tensor(list(masses), dtype=F64)[:, None]
    if float(m.abs().sum()) == 0.0:
        return torch.cat([p0[..., None], pv], dim=-1).permute(1, 0, 2)
    msum = float(m.sum())
    xi = torch.full_like(p0[0], math.sqrt(1.0 - (msum / sqrt_s) ** 2))
    for _ in range(max_iter):
        e = torch.sqrt(m * m + (xi[None] * p0) ** 2)
        f = e.sum(0) - sqrt_s
        fp = (xi[None] * p0 * p0 / e).sum(0)
        dxi = f / fp
        xi = xi - dxi
        if bool((dxi.detach().abs() <= 4.0 * torch.finfo(F64).eps * xi.detach().abs()).all()):
            break
    E = torch.sqrt(m * m + (xi[None] * p0) ** 2)
    out = torch.cat([E[..., None], xi[None, :, None] * pv], dim=-1)  # [nf,N,4]
    return out.permute(1, 0, 2)


def momenta_from_uniforms(u, sqrt_s: float, n: int) -> torch.Tensor:
    """Full momenta [N, n+3, 4]: CM incoming pair + RAMBO final state [e-, n gamma]."""
    ut = torch.as_tensor(u, dtype=F64)
    N = ut.shape[-1]
    p, k = incoming_cm(sqrt_s, N)
    fin = rambo(ut, sqrt_s, [M_E] + [0.0] * n)
    return torch.cat([p[:, None, :], k[:, None, :], fin], dim=1)


def momenta_soa_from_uniforms(u, sqrt_s: float, n: int) -> torch.Tensor:
    return points_to_soa(momenta_from_uniforms(u, sqrt_s, n))


# ---------------------------------------------------------------------------
# Gradient of log |M|^2 (helicity sum) with respect to the RAMBO uniforms
# ---------------------------------------------------------------------------
def logm2_and_grad(u, sqrt_s: float, n: int, chunk: int = 256):
    """(log sum_h |A_h|^2 [N], d/du [4(n+1), N]) by reverse-mode autodiff in float64."""
    ut = torch.as_tensor(u, dtype=F64)
    proc = Process(n)
    vals, grads = [], []
    for s in range(0, ut.shape[1], chunk):
        uc = ut[:, s:s + chunk].clone().requires_grad_(True)
        mom = momenta_from_uniforms(uc, sqrt_s, n)
        f = torch.log(m2_sum(mom, proc))
        (g,) = torch.autograd.grad(f.sum(), uc)
        vals.append(f.detach())
        grads.append(g.detach())
    return torch.cat(vals), torch.cat(grads, dim=1)


def logm2_value(u, sqrt_s: float, n: int) -> torch.Tensor:
    with torch.no_grad():
        mom = momenta_from_uniforms(torch.as_tensor(u, dtype=F64), sqrt_s, n)
        return torch.log(m2_sum(mom, Process(n)))
