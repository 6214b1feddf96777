"""Writes the stored expected values under tests/golden/ from the CPU oracle.

Calls only ``oracle/`` (and the seeded input generators, which hold none of
the method's arithmetic); nothing here touches the HIP library.  Run from the
repository root:

    python tests/golden/make_golden.py            # every file
    python tests/golden/make_golden.py near_soft  # one of them

Files
-----
near_soft_n2.txt
    e- gamma -> e- 2 gamma with the first final-state photon nearly soft, at
    kinematics that are exact in binary: every component is a dyadic
    rational, every momentum is exactly on its mass shell and momentum is
    exactly conserved (electron at rest, a one-photon Compton configuration
    with the incoming photon's energy raised by delta, the extra energy
    carried off by a photon of energy ~delta along the incoming one).  The
    float64 momenta (hex), one helicity code per point, and from the
    extended-precision oracle the helicity sum, the per-configuration value
    and both conditioning numbers (sum |term| / |A| and the chain-norm bound).
    Rounded inputs would not do here: near the propagator's pole (Sec. I-D,
    Eq. 1) the value moves by ~eps |Q|^2 / |Q^2 - m^2| under a last-bit
    change of the momenta, and the kernels' cancellation-free Q^2 - m^2
    assumes on-shell, conserving momenta.  The float64 oracle forms
    Q.Q - m^2 plainly and loses digits there; the long-double evaluation of
    the same definition does not.
grad_n4_rs15_seed5_first1024.npz
    The gradient workload (e- gamma -> e- 4 gamma, helicity sum, sqrt(s) = 15,
    uniforms of seed 5 drawn for 2^18 points): log|M|^2 and its gradient with
    respect to the 20 RAMBO uniforms for the first 1,024 points, by reverse
    autodiff through the oracle's RAMBO and per-diagram amplitude.
"""
from __future__ import annotations

import os
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

import numpy as np  # noqa: E402

from oracle import qed_oracle as O  # noqa: E402
from oracle import qed_oracle_ld as L  # noqa: E402
from paper_2511_19456_amd import inputs  # noqa: E402

NEAR_SOFT = os.path.join(HERE, "near_soft_n2.txt")
GRAD = os.path.join(HERE, "grad_n4_rs15_seed5_first1024.npz")


SOFT_SHIFTS = (13, 23)   # delta = 2^-13 and 2^-23


def exact_compton_bases(count: int = 8):
    """One-photon Compton configurations e-(p) gamma(k) -> e-(p') gamma(k') with
    every component dyadic and every relation exact: p = (1, 0, 0, 0); the
    incoming direction n = (1 + a^2 + b^2, 2a, 2b, 1 - a^2 - b^2) (lightlike
    for any a, b); p' = (A, X, Y, Z) / 4 with A^2 - X^2 - Y^2 - Z^2 = 16 (on
    shell, m = 1); k = w n with w = (E' - 1) / (n^0 (1 - E') + nvec.pvec'),
    the energy that makes k' = p + k - p' lightlike.  Deterministic order;
    keeps configurations with a, b != 0, 1/2 <= w <= 4, w dyadic and k' off
    the z axis, the first one for each |p'| quadruple (X <= Y <= Z), so the
    points differ in their invariants.  Returns [(n, w, p', k')] as Fractions."""
    from fractions import Fraction as Fr
    import itertools
    vals = [Fr(k, 4) for k in (-3, -2, -1, 1, 2, 3)]
    out = []
    for A in range(5, 40):
        for X, Y, Z in itertools.combinations_with_replacement(range(A), 3):
            if A * A - X * X - Y * Y - Z * Z != 16:
                continue
            E = Fr(A, 4)
            hit = None
            for (sx, sy, sz), perm in itertools.product(itertools.product((1, -1), repeat=3),
                                                        sorted(set(itertools.permutations((X, Y, Z))))):
                pv = (Fr(sx * perm[0], 4), Fr(sy * perm[1], 4), Fr(sz * perm[2], 4))
                for a, b in itertools.product(vals, repeat=2):
                    n = (1 + a * a + b * b, 2 * a, 2 * b, 1 - a * a - b * b)
                    den = n[0] * (1 - E) + n[1] * pv[0] + n[2] * pv[1] + n[3] * pv[2]
                    if den <= 0:
                        continue
                    w = (E - 1) / den
                    dd = w.denominator
                    if dd & (dd - 1) or dd > 256 or not (Fr(1, 2) <= w <= 4):
                        continue
                    kp = (1 + w * n[0] - E,) + tuple(w * n[i + 1] - pv[i] for i in range(3))
                    if kp[1] == 0 and kp[2] == 0:
                        continue
                    assert kp[0] ** 2 == kp[1] ** 2 + kp[2] ** 2 + kp[3] ** 2
                    hit = (n, w, (E,) + pv, kp)
                    break
                if hit:
                    break
            if hit:
                out.append(hit)
                if len(out) == count:
                    return out
    return out


def near_soft_points(shift: int, N: int = 8, seed: int = 77):
    """float64 SoA momenta [20][N] of e- gamma -> e- 2 gamma, order
    [e-_in, gamma_in, e-_out, gamma_out_1 (soft), gamma_out_2], and one helicity
    code per point.  From each exact Compton base: k -> k + delta n, the soft
    photon delta n, delta = 2^-shift (all exact in float64)."""
    from fractions import Fraction as Fr
    delta = Fr(1, 1 << shift)
    mom = np.zeros((20, N))
    for i, (n, w, pp, kp) in enumerate(exact_compton_bases(N)):
        parts = [(Fr(1), Fr(0), Fr(0), Fr(0)), tuple((w + delta) * c for c in n), pp,
                 tuple(delta * c for c in n), kp]
        tot = [sum(parts[j][mu] for j in (0, 1)) - sum(parts[j][mu] for j in (2, 3, 4)) for mu in range(4)]
        assert all(t == 0 for t in tot)
        for j, q in enumerate(parts):
            assert q[0] ** 2 - q[1] ** 2 - q[2] ** 2 - q[3] ** 2 == (1 if j in (0, 2) else 0)
            for mu in range(4):
                mom[4 * j + mu, i] = float(q[mu])
                assert Fr(mom[4 * j + mu, i]) == q[mu]     # exactly representable
    h = inputs.rng_for(seed).integers(0, 32, size=N).astype(np.uint32)
    return np.ascontiguousarray(mom), h


def write_near_soft() -> None:
    n = 2
    lines = ["# e- gamma -> e- 2 gamma at exact (dyadic, on-shell, conserving) kinematics, first final-state",
             "# photon nearly soft (energy ~2^-shift along the incoming photon, electron at rest).",
             "# Written by tests/golden/make_golden.py from the extended-precision oracle.",
             "# One record per point: shift, point index, helicity code, then",
             "#   sum_h |A_h|^2, |A_hel|^2, kappa_terms, kappa_chain (decimal, long double),",
             "#   then the 20 float64 momenta of [e-_in, gamma_in, e-_out, gamma_out_1, gamma_out_2]",
             "#   (E, px, py, pz each) as hex floats."]
    for shift in SOFT_SHIFTS:
        mom, h = near_soft_points(shift)
        pts = L.soa_to_points(mom)
        tot = L.m2_sum(pts, n)
        pp, kt, kc = L.m2_per_point(pts, h, n)
        for i in range(mom.shape[1]):
            rec = [str(shift), str(i), str(int(h[i])),
                   np.format_float_scientific(tot[i], precision=20),
                   np.format_float_scientific(pp[i], precision=20),
                   np.format_float_scientific(kt[i], precision=6),
                   np.format_float_scientific(kc[i], precision=6)]
            rec += [float(x).hex() for x in mom[:, i]]
            lines.append(" ".join(rec))
    with open(NEAR_SOFT, "w") as f:
        f.write("\n".join(lines) + "\n")


def read_near_soft(path: str = NEAR_SOFT):
    """{shift: dict(mom [20][N] float64, hel [N], sum, pp, kappa_terms, kappa_chain)} (values as float64)."""
    out = {}
    for line in open(path):
        if line.startswith("#") or not line.strip():
            continue
        t = line.split()
        shift = int(t[0])
        d = out.setdefault(shift, {"mom": [], "hel": [], "sum": [], "pp": [], "kappa_terms": [], "kappa_chain": []})
        d["hel"].append(int(t[2]))
        d["sum"].append(float(t[3]))
        d["pp"].append(float(t[4]))
        d["kappa_terms"].append(float(t[5]))
        d["kappa_chain"].append(float(t[6]))
        d["mom"].append([float.fromhex(x) for x in t[7:]])
    for d in out.values():
        d["mom"] = np.ascontiguousarray(np.array(d["mom"], dtype=np.float64).T)
        d["hel"] = np.array(d["hel"], dtype=np.uint32)
        for k in ("sum", "pp", "kappa_terms", "kappa_chain"):
            d[k] = np.array(d[k], dtype=np.float64)
    return out


def grad_inputs(count: int = 1024):
    """The first `count` points of the 2^18-point gradient workload (seed 5)."""
    wl = inputs.WORKLOADS["grad_n4_sum_rs15_2p18"]
    u, _ = inputs.rambo_inputs(wl["seed"], wl["n"], wl["N"])
    return np.ascontiguousarray(u[:, :count]), wl["sqrt_s"], wl["n"]


def write_grad() -> None:
    u, rs, n = grad_inputs()
    v, g = O.logm2_and_grad(u, rs, n, chunk=128)
    np.savez_compressed(GRAD, logm2=v.numpy(), grad=g.numpy())


def main(argv) -> None:
    want = set(argv) or {"near_soft", "grad"}
    if "near_soft" in want:
        write_near_soft()
    if "grad" in want:
        write_grad()


if __name__ == "__main__":
    main(sys.argv[1:])
