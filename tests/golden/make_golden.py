"""Writes the stored expected values under tests/golden/ from the CPU oracle.

Calls only ``oracle/`` (and the seeded input generators, which hold none of
the method's arithmetic); nothing here touches the HIP library.  Run from the
repository root:

    python tests/golden/make_golden.py            # every file
    python tests/golden/make_golden.py near_soft  # one of them

Files
-----
near_soft_n2.txt
    e- gamma -> e- 2 gamma at sqrt(s) = 6 with the first final-state photon
    nearly soft (its RAMBO energy -ln(u2 u3) -> 0 as u2, u3 -> 1): the exact
    float64 momenta (hex), one helicity code per point, and from the
    extended-precision oracle the helicity sum, the per-configuration value
    and both conditioning numbers (sum |term| / |A| and the chain-norm bound).
    The float64 oracle forms Q.Q - m^2 plainly and loses digits there; the
    long-double evaluation of the same definition does not (Sec. I-D, Eq. 1;
    the soft limit of the propagator).
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


def near_soft_points(eps: float, n: int = 2, rs: float = 6.0, N: int = 8, seed: int = 77):
    """Seeded RAMBO points with the first final-state photon's u2 = u3 = 1 - eps."""
    u, h = inputs.rambo_inputs(seed, n, N, with_helicities=True)
    u[4 + 2] = 1.0 - eps
    u[4 + 3] = 1.0 - eps
    mom = O.momenta_soa_from_uniforms(u, rs, n).numpy()
    return mom, h


def write_near_soft() -> None:
    n = 2
    lines = ["# e- gamma -> e- 2 gamma, sqrt(s) = 6, first final-state photon nearly soft.",
             "# Written by tests/golden/make_golden.py from the extended-precision oracle.",
             "# One record per point: eps, point index, helicity code, then",
             "#   sum_h |A_h|^2, |A_hel|^2, kappa_terms, kappa_chain (decimal, long double),",
             "#   then the 20 float64 momenta of [e-_in, gamma_in, e-_out, gamma_out_1, gamma_out_2]",
             "#   (E, px, py, pz each) as hex floats."]
    for eps in (1e-4, 1e-7):
        mom, h = near_soft_points(eps)
        pts = L.soa_to_points(mom)
        tot = L.m2_sum(pts, n)
        pp, kt, kc = L.m2_per_point(pts, h, n)
        for i in range(mom.shape[1]):
            rec = [repr(eps), str(i), str(int(h[i])),
                   np.format_float_scientific(tot[i], precision=20),
                   np.format_float_scientific(pp[i], precision=20),
                   np.format_float_scientific(kt[i], precision=6),
                   np.format_float_scientific(kc[i], precision=6)]
            rec += [float(x).hex() for x in mom[:, i]]
            lines.append(" ".join(rec))
    with open(NEAR_SOFT, "w") as f:
        f.write("\n".join(lines) + "\n")


def read_near_soft(path: str = NEAR_SOFT):
    """{eps: dict(mom [20][N] float64, hel [N], sum, pp, kappa_terms, kappa_chain)} (values as float64)."""
    out = {}
    for line in open(path):
        if line.startswith("#") or not line.strip():
            continue
        t = line.split()
        eps = float(t[0])
        d = out.setdefault(eps, {"mom": [], "hel": [], "sum": [], "pp": [], "kappa_terms": [], "kappa_chain": []})
        d["hel"].append(int(t[2]))
        d["sum"].append(float(t[3]))
        d["pp"].append(float(t[4]))
        d["kappa_terms"].append(float(t[5]))
        d["kappa_chain"].append(float(t[6]))
        d["mom"].append([float.fromhex(x) for x in t[7:]])
    for d in out.values():
        d["mom"] = np.ascontiguousarray(np.array(d["mom"], dtype=np.float64).T)
        for k in ("hel",):
            d[k] = np.array(d[k], dtype=np.uint32)
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
