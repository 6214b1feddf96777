"""Host-side tests of the CDAG generator, node reduction and cost model.

Pins: Table I node counts (golden file, the paper's printed values), the App. D
wiring of the one-photon graph, computational equivalence of the reduced graph
(App. B-C) against the unreduced one and against the CPU oracle, and the
uniqueness of the reduction fixpoint (Sec. III-D).
"""
import math
import os

import numpy as np
import pytest
import torch

from oracle import qed_oracle as O
from paper_2511_19456_amd import inputs
from paper_2511_19456_amd import qedx as Q

GOLD = os.path.join(os.path.dirname(__file__), "golden")


def _table1():
    rows = {}
    for line in open(os.path.join(GOLD, "table1_node_counts.txt")):
        if line.startswith("#") or not line.strip():
            continue
        n, c = line.split()
        rows[int(n)] = int(c)
    return rows


@pytest.mark.parametrize("n", [1, 2, 3, 4, 5, 6, 7])
def test_table1_node_counts_paper_orientation(n):
    """e- gamma^n -> e- gamma: n incoming photons, one outgoing (the paper's process)."""
    c = Q.graph_counts(1, n_in=n, split=(n + 1) // 2, reduced=False)
    assert c["total"] == _table1()[n]
    P = n + 1
    assert c["V"] == P * math.factorial(P)
    assert c["S1"] == (P - 2) * math.factorial(P)
    assert c["S2"] == math.factorial(P)
    assert c["U"] == n + 3 and c["Sum"] == 1
    assert c["data"] == c["compute"] + (n + 3)


@pytest.mark.parametrize("n", [1, 2, 3, 4, 5, 6])
def test_node_counts_workload_orientation(n):
    """e- gamma -> e- n gamma has the same graph size (crossing)."""
    c = Q.graph_counts(n, n_in=1, reduced=False)
    assert c["total"] == _table1()[n]


def test_appD_one_photon_graph():
    want = {}
    for line in open(os.path.join(GOLD, "appD_n1_graph.txt")):
        if line.startswith("count"):
            _, k, v = line.split()
            want[k] = int(v)
    c = Q.graph_counts(1, reduced=False, split=1)
    for k in ("U", "V", "S2", "Sum", "data", "total"):
        assert c[k] == want[k]
    # nothing is shared in the one-photon graph: reduction leaves it as is
    r = Q.graph_counts(1, reduced=True, split=1)
    assert r["V"] == 4 and r["Dot"] == 2


@pytest.mark.parametrize("n", [2, 3, 4, 5])
def test_reduced_counts_are_prefix_tries(n):
    """After reduction the vertices of each side form the trie of ordered photon
    prefixes: sum over levels i of P!/(P-i)!."""
    P = n + 1
    j = P // 2
    c = Q.graph_counts(n, reduced=True, split=j)
    levels = lambda m: sum(math.factorial(P) // math.factorial(P - i) for i in range(1, m + 1))
    assert c["V"] == levels(j) + levels(P - j)
    assert c["Dot"] == math.factorial(P)
    # chain propagators on both sides plus one join propagator per right leaf
    assert c["S1"] == levels(j - 1) + levels(P - j - 1) + math.factorial(P) // math.factorial(j)


@pytest.mark.parametrize("n,sqrt_s,mask", [(1, 3.0, 0), (2, 5.0, 0b11111), (3, 8.0, 0), (3, 8.0, 0b111111)])
def test_reduced_equals_unreduced_and_oracle(n, sqrt_s, mask):
    N = 40
    u, hel = inputs.rambo_inputs(17, n, N, with_helicities=True)
    mom = O.momenta_from_uniforms(u, sqrt_s, n).numpy()
    a = Q.graph_interpret(n, mom, hel, enum_mask=mask, reduced=False)
    b = Q.graph_interpret(n, mom, hel, enum_mask=mask, reduced=True)
    assert np.max(np.abs(a / b - 1)) < 1e-13
    proc = O.Process(n)
    if mask == (1 << (n + 3)) - 1:
        ref = O.m2_sum(O.torch.as_tensor(mom), proc).numpy()
    else:
        # bits outside mask come from hel; bits inside are summed
        tot = np.zeros(N)
        for sub in range(1 << bin(mask).count("1")):
            h = hel.astype(np.int64) & ~mask
            k = 0
            for b_ in range(n + 3):
                if (mask >> b_) & 1:
                    h |= ((sub >> k) & 1) << b_
                    k += 1
            A = O.amplitudes(O.torch.as_tensor(mom), O.torch.as_tensor(h).reshape(-1, 1), proc)[:, 0].numpy()
            tot += np.abs(A) ** 2
        ref = tot
    scale = O.m2_sum(O.torch.as_tensor(mom), proc).numpy() / (1 << (n + 3))
    assert np.max(np.abs(b - ref) / np.maximum(ref, 1e-3 * scale)) < 1e-11


@pytest.mark.parametrize("n,seed", [(2, 1), (2, 7), (3, 3), (3, 11)])
def test_reduction_fixpoint_is_order_independent(n, seed):
    a, b, steps = Q.reduction_check(n, seed)
    assert a == b and len(a) > 0
    assert steps > 0


def test_reduction_lowers_compute_effort():
    """C(DAG) drops by node reduction; the drop grows with n (Sec. III-D/E)."""
    ratios = []
    for n in (2, 3, 4, 5):
        cu, du = Q.graph_metrics(n, reduced=False)
        cr, dr = Q.graph_metrics(n, reduced=True)
        assert cr < cu
        ratios.append(cu / cr)
    assert all(b > a for a, b in zip(ratios, ratios[1:]))
    c1, _ = Q.graph_metrics(1, reduced=False, split=1)
    c1r, _ = Q.graph_metrics(1, reduced=True, split=1)
    assert abs(c1 / c1r - 1) < 1e-12


def test_invalid_arguments_are_rejected():
    from paper_2511_19456_amd._lib import QedError
    with pytest.raises(QedError):
        Q.graph_counts(0)
    with pytest.raises(QedError):
        Q.graph_counts(3, split=4)
    with pytest.raises(QedError):
        Q.graph_counts(2, enum_mask=1 << 9)


# ---------------------------------------------------------------------------
# distributive rewrite (term rewriting proposed in Sec. IV / App. C)
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("n", [2, 3, 4, 5, 6])
def test_distributed_counts_are_subset_currents(n):
    """After the rewrite each side holds one current per photon subset: a
    subset S of size k is the sum over its k possible last photons of that
    vertex applied to the propagated current of S minus that photon
    (Berends-Giele recursion), and the diagram sum is one join per partition."""
    P = n + 1
    j = P // 2
    C = math.comb
    c = Q.graph_counts(n, reduced=2, split=j)
    assert c["Dot"] == C(P, j)
    assert c["V"] == sum(C(P, k) * k for k in range(1, j + 1)) + sum(C(P, k) * k for k in range(1, P - j + 1))
    # propagated subsets below the join on both sides, plus the join propagator
    assert c["S1"] == sum(C(P, k) for k in range(1, j)) + sum(C(P, k) for k in range(1, P - j)) + C(P, P - j)
    assert c["S2"] == 0 and c["Sum"] == 1


@pytest.mark.parametrize("n,sqrt_s,mask", [(1, 3.0, 0), (2, 5.0, 0b11111), (3, 8.0, 0), (3, 8.0, 0b111111),
                                           (4, 12.0, 0), (5, 20.0, 0)])
def test_distributed_equals_unreduced_and_oracle(n, sqrt_s, mask):
    N = 24
    u, hel = inputs.rambo_inputs(19, n, N, with_helicities=True)
    mom = O.momenta_from_uniforms(u, sqrt_s, n).numpy()
    d = Q.graph_interpret(n, mom, hel, enum_mask=mask, reduced=2)
    r = Q.graph_interpret(n, mom, hel, enum_mask=mask, reduced=True)
    proc = O.Process(n)
    tot = O.m2_sum(O.torch.as_tensor(mom), proc).numpy()
    scale = tot / (1 << (n + 3))
    if mask == (1 << (n + 3)) - 1:
        ref = tot
    else:
        ref = O.m2(O.points_to_soa(O.torch.as_tensor(mom)), n, "per_point", hel).numpy()
    assert np.max(np.abs(d - r) / np.maximum(np.abs(r), 1e-3 * scale)) < 1e-12
    assert np.max(np.abs(d - ref) / np.maximum(np.abs(ref), 1e-3 * scale)) < 1e-11


def test_distributive_rewrite_lowers_compute_effort():
    """The rewrite turns the factorial diagram sum into subset currents: the
    gain over node reduction alone grows with n."""
    gains = []
    for n in (2, 3, 4, 5, 6):
        cr, _ = Q.graph_metrics(n, reduced=True)
        cd, _ = Q.graph_metrics(n, reduced=2)
        assert cd < cr
        gains.append(cr / cd)
    assert all(b > a for a, b in zip(gains, gains[1:]))
    # one photon: nothing to factor
    c1r, _ = Q.graph_metrics(1, reduced=True, split=1)
    c1d, _ = Q.graph_metrics(1, reduced=2, split=1)
    assert c1r == c1d


@pytest.mark.parametrize("steps", [0, 35, 140, 280])
def test_partial_reduction_keeps_the_computation(steps):
    """The reduction experiment's graphs (Sec. III-D): after any number of
    single node reductions the graph computes the same amplitude (App. B-C);
    0 steps is the unreduced graph of Table I and all 280 steps (n = 4, seed 1)
    reach the fixpoint of the one-pass reduction."""
    n, N = 4, 12
    u, hel = inputs.rambo_inputs(29, n, N, with_helicities=True)
    mom = O.momenta_from_uniforms(u, 15.0, n).numpy().reshape(N, -1)
    c, got = Q.graph_partial(n, steps, 1, mom, hel)
    ref = Q.graph_interpret(n, mom, hel, reduced=False)
    tot = O.m2_sum(O.torch.as_tensor(mom.reshape(N, n + 3, 4)), O.Process(n)).numpy()
    assert np.max(np.abs(got - ref) / np.maximum(np.abs(ref), 1e-3 * tot / (1 << (n + 3)))) < 1e-12
    if steps == 0:
        assert c["total"] == _table1()[n]
    a, b, total = Q.reduction_check(n, 1, enum_mask=0, split=2)
    assert total == 280
    if steps == total:
        fix = Q.graph_counts(n, split=2, reduced=False)
        assert c["total"] < fix["total"] and c["S2"] == 120


@pytest.mark.parametrize("n_in,n_out,reduced", [(2, 1, False), (2, 1, True), (3, 1, True), (3, 1, 2),
                                                (2, 2, True), (4, 1, True)])
def test_crossed_graph_equals_oracle(n_in, n_out, reduced):
    """The graph of e- gamma^n_in -> e- gamma^n_out (the Table I orientation)
    evaluates to the oracle's |M|^2, per configuration and summed."""
    N = 16
    if n_out == 1:
        mom, hel = inputs.crossed_inputs(41 + n_in, n_in, N, with_helicities=True)
        pts = O.soa_to_points(mom)
    else:
        # physical e- gamma -> e- 3gamma points with one outgoing photon crossed in
        u, _ = inputs.rambo_inputs(43, 3, N)
        m3 = O.momenta_from_uniforms(u, 9.0, 3)
        pts = torch.cat([m3[:, :2], -m3[:, 3:4], m3[:, 2:3], m3[:, 4:]], dim=1)
        hel = inputs.rng_for(44).integers(0, 1 << 6, size=N).astype(np.uint32)
    npart = n_in + n_out + 2
    flat = pts.numpy().reshape(N, 4 * npart)
    proc = O.Process(n_out, n_in=n_in)
    tot = O.m2_sum(pts, proc).numpy()
    scale = tot / (1 << npart)
    got = Q.graph_interpret(n_out, flat, hel, n_in=n_in, reduced=reduced)
    ref = O.m2_per_point(pts, torch.as_tensor(hel.astype(np.int64)), proc).numpy()
    assert np.max(np.abs(got - ref) / np.maximum(ref, 1e-3 * scale)) < 1e-11
    all_mask = (1 << npart) - 1
    got_s = Q.graph_interpret(n_out, flat, None, n_in=n_in, enum_mask=all_mask, reduced=reduced)
    assert np.max(np.abs(got_s / tot - 1)) < 1e-11


def test_adjoint_cost_model():
    """The gradient's algorithmic FLOPs (forward C(DAG) plus the reverse-mode
    cost of the same graph): the forward part equals C(DAG); by node, the
    adjoint of a vertex costs 2.5x its forward (3.5x for the y polarisation),
    of a propagator 2.2x, and the dots of one amplitude in one photon
    partition take their adjoint from the two leaf sums, so the ratio of the
    total to the forward lies between 2 and 4.5 (lower for larger n, where
    dots dominate the forward count); node reduction lowers both."""
    for n in (1, 2, 3, 4):
        m = (1 << (n + 3)) - 1
        f, a = Q.graph_adjoint_metrics(n, enum_mask=m)
        assert f == Q.graph_metrics(n, enum_mask=m, split=(n + 1) // 2)[0]
        assert 2.0 < (f + a) / f < 4.5, (n, f, a)
        fu, au = Q.graph_adjoint_metrics(n, enum_mask=0, reduced=False)
        fr, ar = Q.graph_adjoint_metrics(n, enum_mask=0, reduced=True)
        assert fr <= fu and (n == 1 or ar < au)
    from paper_2511_19456_amd._lib import QedError
    with pytest.raises(QedError):
        Q.graph_adjoint_metrics(0)
