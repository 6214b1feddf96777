"""GPU parity: generated HIP kernels through the C ABI vs the CPU oracle.

Inputs are the seeded synthetic workloads (inputs.py); the oracle computes its
own momenta from the same uniforms with its own RAMBO.  Tolerances: 1e-10
relative for FP64 (stated target), widened per configuration only by the
rounding its own cancellation costs (tests/parity.py: 2 C eps kappa with
kappa = sum |term| / |A| from the oracle); plain 1e-4 relative on every point
for the compensated FP32 path.
"""
import math

import numpy as np
import pytest
import torch

from oracle import qed_oracle as O
from paper_2511_19456_amd import inputs
from parity import check_fp64, check_rambo, per_point_ref

pytestmark = pytest.mark.gpu

DEV = "cuda:0"


def _proc(n, mode="sum", prec="fp64", variant=None):
    from paper_2511_19456_amd.qedx import QedProcess
    return QedProcess(n, mode, prec, variant)


def _rel(a, b):
    return np.abs(a / b - 1.0)


def test_compton_n1_sum_matches_oracle_and_klein_nishina():
    N = 4099
    mom = inputs.compton_lab_momenta(1, N)
    p = _proc(1)
    got = p.eval(torch.as_tensor(mom, device=DEV)).cpu().numpy()
    ref = O.m2(mom, 1, "sum").numpy()
    assert _rel(got, ref).max() < 1e-10
    ct = mom[15] / mom[12]
    wp = mom[12]
    kn = 8.0 * (wp + 1.0 / wp - (1.0 - ct * ct))
    assert _rel(got, kn).max() < 1e-12


@pytest.mark.parametrize("n,sqrt_s", [(1, 3.0), (2, 6.0), (3, 10.0)])
def test_sum_mode_fp64(n, sqrt_s):
    N = 1000 + 37
    u, _ = inputs.rambo_inputs(2, n, N)
    p = _proc(n)
    ud = torch.as_tensor(u, device=DEV)
    mom_gpu = p.rambo(ud, sqrt_s)
    ref_mom = O.momenta_soa_from_uniforms(u, sqrt_s, n)
    # RAMBO parity
    check_rambo(mom_gpu.cpu().numpy(), ref_mom.numpy(), u, n, sqrt_s, f"n={n}")
    # |M|^2 on the oracle's momenta and on the device's own momenta
    got = p.eval(torch.as_tensor(ref_mom.numpy(), device=DEV)).cpu().numpy()
    got2 = p.eval(mom_gpu).cpu().numpy()
    ref = O.m2(ref_mom, n, "sum").numpy()
    assert _rel(got, ref).max() < 1e-10
    assert _rel(got2, ref).max() < 1e-10


@pytest.mark.parametrize("n,sqrt_s", [(1, 4.0), (3, 10.0), (5, 20.0)])
def test_per_point_fp64(n, sqrt_s):
    N = 700 + 13
    u, hel = inputs.rambo_inputs(3, n, N, with_helicities=True)
    ref_mom = O.momenta_soa_from_uniforms(u, sqrt_s, n)
    p = _proc(n, "per_point")
    got = p.eval(torch.as_tensor(ref_mom.numpy(), device=DEV),
                 torch.as_tensor(hel.astype(np.int32), device=DEV)).cpu().numpy()
    ref, kap = per_point_ref(ref_mom, n, hel)
    check_fp64(got, ref, kap, f"per point n={n}")


def test_per_point_sums_to_sum_mode():
    n, sqrt_s, N = 2, 7.0, 300
    u, _ = inputs.rambo_inputs(8, n, N)
    ps = _proc(n)
    pp = _proc(n, "per_point")
    mom = ps.rambo(torch.as_tensor(u, device=DEV), sqrt_s)
    tot = ps.eval(mom)
    acc = torch.zeros_like(tot)
    for h in range(1 << (n + 3)):
        acc += pp.eval(mom, torch.full((N,), h, dtype=torch.int32, device=DEV))
    assert ((acc / tot - 1).abs().max().item()) < 1e-13


def test_empty_and_single_point():
    p = _proc(1)
    mom = torch.zeros(16, 0, dtype=torch.float64, device=DEV)
    assert p.eval(mom).shape == (0,)
    m1 = inputs.compton_lab_momenta(4, 1)
    got = p.eval(torch.as_tensor(m1, device=DEV)).cpu().numpy()
    assert _rel(got, O.m2(m1, 1, "sum").numpy()).max() < 1e-10


# ---------------------------------------------------------------------------
# schedule variants must not change results
# ---------------------------------------------------------------------------
# order flags: 4 partition-local blocks, 8 partition loop, 16 LDS staging of
# the held side, 32 momenta reloaded per loop iteration
@pytest.mark.parametrize("mode,lanes,order,loop", [("sum", 7, 0, 0), ("sum", 5, 4, 0), ("sum", 63, 4, 0),
                                                   ("per_point", 0, 4, 0), ("sum", 5, 16, 0), ("sum", 5, 32, 2),
                                                   ("per_point", 0, 24, 0)])
def test_schedule_variants_n3(mode, lanes, order, loop):
    from paper_2511_19456_amd.qedx import make_variant
    n, sqrt_s, N = 3, 10.0, 517
    u, hel = inputs.rambo_inputs(21, n, N, with_helicities=True)
    ref_mom = O.momenta_soa_from_uniforms(u, sqrt_s, n)
    p = _proc(n, mode, "fp64", make_variant(lane_bits=lanes, loop_bits=loop, order=order))
    h = torch.as_tensor(hel.astype(np.int32), device=DEV) if mode == "per_point" else None
    got = p.eval(torch.as_tensor(ref_mom.numpy(), device=DEV), h).cpu().numpy()
    if mode == "sum":
        assert _rel(got, O.m2(ref_mom, n, "sum").numpy()).max() < 1e-10
    else:
        ref, kap = per_point_ref(ref_mom, n, hel)
        check_fp64(got, ref, kap, f"schedule {order}")


def test_per_point_n4_and_sum_n4():
    n, sqrt_s, N = 4, 15.0, 300
    u, hel = inputs.rambo_inputs(22, n, N, with_helicities=True)
    ref_mom = O.momenta_soa_from_uniforms(u, sqrt_s, n)
    md = torch.as_tensor(ref_mom.numpy(), device=DEV)
    pp = _proc(n, "per_point")
    got = pp.eval(md, torch.as_tensor(hel.astype(np.int32), device=DEV)).cpu().numpy()
    ref, kap = per_point_ref(ref_mom, n, hel)
    check_fp64(got, ref, kap, "per point n=4")
    tot = O.m2(ref_mom, n, "sum").numpy()
    ps = _proc(n, "sum")
    assert _rel(ps.eval(md).cpu().numpy(), tot).max() < 1e-10


# ---------------------------------------------------------------------------
# FP32 path with compensated diagram sum: stated bound 1e-4 relative
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("n,mode,sqrt_s", [(3, "sum", 10.0), (5, "per_point", 20.0)])
def test_fp32c_error_bound(n, mode, sqrt_s):
    N = 4096
    u, hel = inputs.rambo_inputs(3, n, N, with_helicities=True)
    ref_mom = O.momenta_soa_from_uniforms(u, sqrt_s, n)
    p = _proc(n, mode, "fp32c")
    h = torch.as_tensor(hel.astype(np.int32), device=DEV) if mode == "per_point" else None
    got = p.eval(torch.as_tensor(ref_mom.numpy(), device=DEV), h).cpu().numpy()
    ref = O.m2(ref_mom, n, mode, hel).numpy()
    err = _rel(got, ref)   # plain relative error on every point, no floor
    print(f"fp32c n={n} {mode}: max {err.max():.2e} p99 {np.quantile(err, 0.99):.2e} median {np.median(err):.2e}")
    assert err.max() < 1e-4
    assert np.median(err) < 1e-5


# ---------------------------------------------------------------------------
# gradient of log|M|^2 through RAMBO (adjoint kernel)
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("n,sqrt_s,N,rewrite", [(1, 4.0, 200, 0), (2, 6.0, 200, 0), (3, 10.0, 128, 0),
                                                 (4, 15.0, 96, 0), (4, 15.0, 96, 1)])
def test_gradient_vs_oracle(n, sqrt_s, N, rewrite):
    from paper_2511_19456_amd.qedx import make_variant
    u, _ = inputs.rambo_inputs(5, n, N)
    p = _proc(n, "sum", "fp64", make_variant(rewrite=1) if rewrite else None)
    val, g = p.eval_grad(torch.as_tensor(u, device=DEV), sqrt_s)
    v_o, g_o = O.logm2_and_grad(u, sqrt_s, n)
    assert np.abs(val.cpu().numpy() - v_o.numpy()).max() < 1e-10 * max(1.0, np.abs(v_o.numpy()).max())
    gg, go = g.cpu().numpy(), g_o.numpy()
    err = np.linalg.norm(gg - go, axis=0) / np.linalg.norm(go, axis=0)
    assert err.max() < 1e-10


def test_gradient_vs_central_differences_and_autograd():
    """Central differences with h = 1e-6 on the uniforms, at points whose
    uniforms all lie at least 1e-5 from the ends of (0,1).  The difference
    quotient has its own truncation error (h^2/6 times the third derivative,
    large where the kinematics approach a soft or collinear photon); it is
    estimated per point from the quotients at h and h/2 (Richardson:
    4/3 |D(h) - D(h/2)|) and added to the 1e-6 normwise tolerance.  Most points
    must also agree to 1e-6 with no allowance at all."""
    from paper_2511_19456_amd.qedx import QedLogM2
    n, sqrt_s, N = 4, 15.0, 1024
    u, _ = inputs.rambo_inputs(5, n, N)
    p = _proc(n, "sum")
    ud = torch.as_tensor(u, device=DEV)
    _, g = p.eval_grad(ud, sqrt_s)

    def fdiff(h):
        fd = torch.zeros_like(ud)
        for r in range(ud.shape[0]):
            up, um = ud.clone(), ud.clone()
            up[r] += h
            um[r] -= h
            fd[r] = (torch.log(p.eval(p.rambo(up, sqrt_s))) - torch.log(p.eval(p.rambo(um, sqrt_s)))) / (2 * h)
        return fd

    fd1, fd2 = fdiff(1e-6), fdiff(5e-7)
    gn = torch.linalg.norm(g, dim=0)
    trunc = (torch.linalg.norm(fd1 - fd2, dim=0) * 4.0 / 3.0 / gn).cpu().numpy()
    keep = np.all((u > 1e-5) & (u < 1 - 1e-5), axis=0)
    err = (torch.linalg.norm(g - fd1, dim=0) / gn).cpu().numpy()
    plain = err[keep] < 1e-6
    print(f"FD check: {keep.sum()} of {N} points away from the ends; {plain.sum()} within 1e-6 outright; "
          f"max err {err[keep].max():.2e}, median {np.median(err[keep]):.2e}, max FD error estimate "
          f"{trunc[keep].max():.2e}")
    assert keep.mean() > 0.95
    assert np.all(err[keep] < 1e-6 + 2.0 * trunc[keep])
    assert plain.mean() > 0.95 and np.median(err[keep]) < 1e-8
    # torch.autograd.Function wrapper
    x = ud.clone().requires_grad_(True)
    y = QedLogM2.apply(x, p, sqrt_s)
    (gx,) = torch.autograd.grad(y.sum(), x)
    assert torch.allclose(gx, g, rtol=1e-12, atol=0)


# ---------------------------------------------------------------------------
# mixed-process batch: one persistent launch over segments n = 1..6
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("n,sqrt_s,N", [(6, 25.0, 40)])
def test_per_point_n6_fp64(n, sqrt_s, N):
    u, hel = inputs.rambo_inputs(23, n, N, with_helicities=True)
    ref_mom = O.momenta_soa_from_uniforms(u, sqrt_s, n)
    p = _proc(n, "per_point")
    got = p.eval(torch.as_tensor(ref_mom.numpy(), device=DEV),
                 torch.as_tensor(hel.astype(np.int32), device=DEV)).cpu().numpy()
    ref, kap = per_point_ref(ref_mom, n, hel)
    check_fp64(got, ref, kap, "per point n=6")


# One-photon current cache of the per-point partition loop: each lane split
# and cached side, FP64 and FP32C, partition counts the lanes divide and ones
# they do not (the last round's spare lanes repeat a partition and drop it).
@pytest.mark.parametrize("n,sqrt_s,N,order,prec", [
    (4, 15.0, 333, 8, "fp64"),                # the loop without the cache
    (4, 15.0, 333, 8 | 256, "fp64"),          # 2 lanes, both sides cached
    (4, 15.0, 333, 8 | 512, "fp64"),          # 4 lanes over 10 partitions
    (5, 20.0, 257, 8 | 256 | 1024, "fp64"),   # 2 lanes, e-_in side only
    (6, 25.0, 67, 8 | 256, "fp64"),           # 35 partitions over 2 lanes
    (4, 15.0, 333, 8 | 512, "fp32c"),
    (6, 25.0, 67, 8 | 256 | 1024, "fp32c"),
])
def test_current_cache_shapes(n, sqrt_s, N, order, prec):
    from paper_2511_19456_amd.qedx import make_variant
    u, hel = inputs.rambo_inputs(29, n, N, with_helicities=True)
    ref_mom = O.momenta_soa_from_uniforms(u, sqrt_s, n)
    p = _proc(n, "per_point", prec, make_variant(order=order))
    assert p.info()["lanes_per_point"] == (4 if order & 512 else 2 if order & 256 else 1)
    got = p.eval(torch.as_tensor(ref_mom.numpy(), device=DEV),
                 torch.as_tensor(hel.astype(np.int32), device=DEV)).cpu().numpy()
    ref, kap = per_point_ref(ref_mom, n, hel)
    if prec == "fp64":
        check_fp64(got, ref, kap, f"per point n={n} order={order}")
    else:
        assert _rel(got, ref).max() < 1e-4


@pytest.mark.parametrize("prec,tile,rewrite", [("fp64", 128, 0), ("fp64", 0, 0), ("fp32c", 0, 0), ("fp64", 256, 1)])
def test_mixed_batch_matches_per_process_and_oracle(prec, tile, rewrite):
    from paper_2511_19456_amd.qedx import BatchPlan, make_variant
    spec = [(1, 1000, 6.0), (2, 3 * 64 + 5, 9.0), (3, 2500, 12.0), (4, 777, 15.0), (5, 301, 20.0),
            (6, 130, 25.0), (3, 0, 10.0)]
    segs, refs, checks = [], [], []
    for k, (n, N, rs) in enumerate(spec):
        u, hel = inputs.rambo_inputs(40 + k, n, N, with_helicities=True)
        p = _proc(n, "per_point", prec, make_variant(rewrite=1) if rewrite else None)
        mom = p.rambo(torch.as_tensor(u, device=DEV), rs)
        h = torch.as_tensor(hel.astype(np.int32), device=DEV)
        out = torch.full((N,), float("nan"), dtype=torch.float64, device=DEV)
        segs.append((p, mom, h, out))
        # reference: the plain per-process FP64 kernel on the same inputs
        refs.append(_proc(n, "per_point", "fp64").eval(mom, h) if N else out.clone())
        checks.append((n, u, hel, rs))
    # FP64: every point against the oracle (below); FP32C: every point within
    # the stated bound of the compensated FP32 path against the FP64 kernel
    plan = BatchPlan(segs, tile_points=tile)
    info = plan.info()
    print(f"batch {prec} tile={tile}: {info}")
    for rep in range(3):
        for s in segs:
            s[3].fill_(float("nan"))
        torch.cuda.synchronize()
        plan.launch()
        torch.cuda.synchronize()
        for (p, mom, h, out), ref, (n, u, hel, rs) in zip(segs, refs, checks):
            if out.numel() == 0:
                continue
            assert torch.isfinite(out).all(), (n, rep)
            if prec == "fp64":
                # the same generated body as the per-process kernel
                assert torch.equal(out, ref) or ((out - ref).abs() / ref.abs()).max().item() < 1e-12, (n, rep)
            else:
                assert ((out - ref).abs() / ref.abs()).max().item() < 1e-4, (n, rep)
    # every point of every FP64 segment against the oracle
    if prec == "fp64":
        for (p, mom, h, out), (n, u, hel, rs) in zip(segs, checks):
            N = out.numel()
            if N == 0:
                continue
            ref_mom = O.momenta_soa_from_uniforms(u, rs, n)
            # the batch ran on the device RAMBO's momenta; the oracle's agree
            # to 1e-12 sqrt(s) but where RAMBO's massless boost is large
            check_rambo(mom.cpu().numpy(), ref_mom.numpy(), u, n, rs, f"batch segment n={n}")
            ref, kap = per_point_ref(mom.cpu().numpy(), n, hel)
            check_fp64(out.cpu().numpy(), ref, kap, f"batch segment n={n}")


# ---------------------------------------------------------------------------
# distributive rewrite (rewrite = 1): same |M|^2 as the oracle
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("n,mode,sqrt_s,lanes,N", [(2, "sum", 6.0, 0, 333), (3, "sum", 10.0, 0, 517),
                                                   (3, "sum", 10.0, 7, 517), (4, "sum", 15.0, 0, 160),
                                                   (4, "per_point", 15.0, 0, 300), (5, "per_point", 20.0, 0, 200),
                                                   (6, "per_point", 25.0, 0, 40)])
def test_distributive_rewrite_fp64(n, mode, sqrt_s, lanes, N):
    from paper_2511_19456_amd.qedx import make_variant
    u, hel = inputs.rambo_inputs(31, n, N, with_helicities=True)
    ref_mom = O.momenta_soa_from_uniforms(u, sqrt_s, n)
    p = _proc(n, mode, "fp64", make_variant(lane_bits=lanes, rewrite=1))
    assert p.info()["kernel_tag"].endswith("_d1")
    h = torch.as_tensor(hel.astype(np.int32), device=DEV) if mode == "per_point" else None
    got = p.eval(torch.as_tensor(ref_mom.numpy(), device=DEV), h).cpu().numpy()
    ref = O.m2(ref_mom, n, mode, hel).numpy()
    if mode == "sum":
        assert _rel(got, ref).max() < 1e-10
    else:
        ref, kap = per_point_ref(ref_mom, n, hel)
        check_fp64(got, ref, kap, f"distributive n={n}")


@pytest.mark.parametrize("N", [517, 64 * 4 * 3 + 5, 1])
def test_distributive_join_on_matrix_cores(N):
    """The n = 3 helicity-sum distributive kernel with its joins on the FP64
    matrix cores (4 x 4 complex dot blocks by v_mfma_f64_4x4x4, lanes
    permuted per partition; the join task of Sec. II-B): against the oracle
    at 1e-10 and against the same graph's vector joins, on a ragged point
    count, several full waves and a single point."""
    from paper_2511_19456_amd.qedx import make_variant
    n, sqrt_s = 3, 10.0
    u, _ = inputs.rambo_inputs(33, n, N)
    ref_mom = O.momenta_soa_from_uniforms(u, sqrt_s, n)
    p = _proc(n, "sum", "fp64", make_variant(rewrite=1, order=128))
    assert p.info()["kernel_name"].endswith("_mfma")
    m = torch.as_tensor(ref_mom.numpy(), device=DEV)
    got = p.eval(m).cpu().numpy()
    ref = O.m2(ref_mom, n, "sum").numpy()
    assert _rel(got, ref).max() < 1e-10
    vec = _proc(n, "sum", "fp64", make_variant(rewrite=1)).eval(m).cpu().numpy()
    assert _rel(got, vec).max() < 1e-13


@pytest.mark.parametrize("n,mode,sqrt_s", [(3, "sum", 10.0), (5, "per_point", 20.0)])
def test_distributive_rewrite_fp32c(n, mode, sqrt_s):
    from paper_2511_19456_amd.qedx import make_variant
    N = 4096
    u, hel = inputs.rambo_inputs(3, n, N, with_helicities=True)
    ref_mom = O.momenta_soa_from_uniforms(u, sqrt_s, n)
    p = _proc(n, mode, "fp32c", make_variant(rewrite=1))
    h = torch.as_tensor(hel.astype(np.int32), device=DEV) if mode == "per_point" else None
    got = p.eval(torch.as_tensor(ref_mom.numpy(), device=DEV), h).cpu().numpy()
    ref = O.m2(ref_mom, n, mode, hel).numpy()
    err = _rel(got, ref)
    print(f"fp32c rewrite n={n} {mode}: max {err.max():.2e} p99 {np.quantile(err, 0.99):.2e} "
          f"median {np.median(err):.2e}")
    assert err.max() < 1e-4
    assert np.median(err) < 1e-5


# ---------------------------------------------------------------------------
# reduction experiment: partially reduced graphs of the paper's form
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("steps", [0, 140, 280])
def test_partially_reduced_kernels(steps):
    from paper_2511_19456_amd.qedx import make_variant
    n, sqrt_s, N = 4, 15.0, 300
    u, hel = inputs.rambo_inputs(33, n, N, with_helicities=True)
    ref_mom = O.momenta_soa_from_uniforms(u, sqrt_s, n)
    p = _proc(n, "per_point", "fp64", make_variant(partial_steps=steps, partial_seed=1))
    assert p.info()["kernel_tag"].endswith(f"_k{steps}s1")
    got = p.eval(torch.as_tensor(ref_mom.numpy(), device=DEV),
                 torch.as_tensor(hel.astype(np.int32), device=DEV)).cpu().numpy()
    ref, kap = per_point_ref(ref_mom, n, hel)
    check_fp64(got, ref, kap, f"partial {steps}")


# Table I orientation e- gamma^n_in -> e- gamma^n_out (crossed processes).
@pytest.mark.parametrize("n_in,n_out,mode,prec,rewrite,N", [
    (2, 1, "sum", "fp64", 0, 515), (3, 1, "sum", "fp64", 0, 389), (4, 1, "sum", "fp64", 0, 150),
    (3, 1, "sum", "fp32c", 0, 389), (2, 2, "sum", "fp64", 0, 300),
    (2, 1, "per_point", "fp64", 0, 777), (3, 1, "per_point", "fp64", 0, 601), (4, 1, "per_point", "fp64", 0, 300),
    (5, 1, "per_point", "fp64", 0, 120), (6, 1, "per_point", "fp64", 0, 40), (6, 1, "per_point", "fp64", 1, 40),
    (3, 1, "per_point", "fp32c", 0, 601), (6, 1, "per_point", "fp32c", 0, 40)])
def test_crossed_processes(n_in, n_out, mode, prec, rewrite, N):
    from paper_2511_19456_amd._lib import QedError
    from paper_2511_19456_amd.qedx import QedProcess, make_variant
    print(f"crossed n_in={n_in} n_out={n_out} {mode} {prec} rewrite={rewrite} N={N}", flush=True)
    if n_out == 1:
        mom, hel = inputs.crossed_inputs(200 + n_in, n_in, N, with_helicities=True)
        pts = O.soa_to_points(mom)
    else:
        u, _ = inputs.rambo_inputs(201, 3, N)
        m3 = O.momenta_from_uniforms(u, 9.0, 3)
        pts = torch.cat([m3[:, :2], -m3[:, 3:4], m3[:, 2:3], m3[:, 4:]], dim=1)
        mom = O.points_to_soa(pts).numpy()
        hel = inputs.rng_for(202).integers(0, 1 << 6, size=N).astype(np.uint32)
    npart = n_in + n_out + 2
    var = make_variant(rewrite=1) if rewrite else None
    p = QedProcess(n_out, mode, prec, var, n_in=n_in)
    assert p.info()["n_in"] == n_in
    md = torch.as_tensor(mom, device=DEV)
    tot = O.m2(mom, n_out, "sum", n_in=n_in).numpy()
    tol = 1e-10 if prec == "fp64" else 1e-4
    if mode == "sum":
        got = p.eval(md).cpu().numpy()
        assert _rel(got, tot).max() < tol
    else:
        got = p.eval(md, torch.as_tensor(hel.astype(np.int32), device=DEV)).cpu().numpy()
        ref, kap = per_point_ref(mom, n_out, hel, n_in=n_in)
        if prec == "fp64":
            check_fp64(got, ref, kap, f"crossed {n_in}->{n_out}")
        else:
            assert _rel(got, ref).max() < tol
    with pytest.raises(QedError):
        p.rambo(torch.zeros(4 * (n_out + 1), 4, dtype=torch.float64, device=DEV), 10.0)


def test_fp64_pipe_probe_closed_forms():
    """The pipe probe's kernels do the work they are timed for: the vector
    chains match the closed form of a <- a m + c, the matrix chains 4 iters A.B
    with the stated operand and result lane layouts (dyadic inputs: exact)."""
    from paper_2511_19456_amd._lib import check, probe_lib
    blocks, it_v, it_m = 3, 1000, 64
    mm, cc = 0.999, 0.001
    av = (torch.arange(64, dtype=torch.float64) + 1) / 64.0
    bv = (torch.arange(64, dtype=torch.float64) * 3 + 1) / 128.0
    a_d, b_d = av.to(DEV), bv.to(DEV)
    ov = torch.full((blocks * 256,), -1.0, dtype=torch.float64, device=DEV)
    om = torch.full((blocks * 1024,), -1.0, dtype=torch.float64, device=DEV)
    st = torch.cuda.current_stream().cuda_stream
    lane = np.arange(blocks * 256) % 64
    mn = mm ** it_v
    chains = sum(mn * (lane + j) + cc * (1 - mn) / (1 - mm) for j in range(8))
    A = av.numpy().reshape(4, 16).T          # A[i][k] = a[i + 16 k]
    B = bv.numpy().reshape(4, 16)            # B[k][j] = b[j + 16 k]
    C = 4 * it_m * (A @ B)
    lanes = np.arange(blocks * 256)
    expect_m = np.zeros(blocks * 1024)
    for r in range(4):
        # item r of lane l holds row l/16 + 4r, column l%16
        expect_m[4 * lanes + r] = C[(lanes % 64) // 16 + 4 * r, lanes % 16]
    check(probe_lib().qed_pipe_probe(0, blocks, it_v, 0, mm, cc, None, None, ov.data_ptr(), None, st))
    torch.cuda.synchronize()
    assert np.max(np.abs(ov.cpu().numpy() / chains - 1)) < 1e-12
    check(probe_lib().qed_pipe_probe(1, blocks, it_m, 0, mm, cc, a_d.data_ptr(), b_d.data_ptr(), om.data_ptr(),
                               None, st))
    torch.cuda.synchronize()
    assert np.array_equal(om.cpu().numpy(), expect_m)
    ov.fill_(-1.0)
    om.fill_(-1.0)
    check(probe_lib().qed_pipe_probe(2, blocks, it_v, it_m, mm, cc, a_d.data_ptr(), b_d.data_ptr(), ov.data_ptr(),
                               om.data_ptr(), st))
    torch.cuda.synchronize()
    even = ((lanes // 64) % 2) == 0
    got_v, got_m = ov.cpu().numpy(), om.cpu().numpy().reshape(-1, 4)
    assert np.max(np.abs(got_v[even] / chains[even] - 1)) < 1e-12
    assert np.array_equal(got_m[~even], expect_m.reshape(-1, 4)[~even])


@pytest.mark.parametrize("n,sqrt_s", [(3, 10.0), (5, 20.0)])
def test_fp32c_fp64_fixup(n, sqrt_s):
    """FP32C per-point kernels mark the points they cannot vouch for and the
    FP64 pass recomputes them in place.  Against the FP64 kernel (itself
    pinned to the oracle), over calls of growing and shrinking N (ragged
    tails of the fix-up pass's point ranges): plain relative error below 1e-4
    on every point."""
    from paper_2511_19456_amd.qedx import make_variant
    N = 1 << 16
    u, h = inputs.rambo_inputs(5 + n, n, N, with_helicities=True)
    p64 = _proc(n, "per_point", "fp64")
    mom = p64.rambo(torch.as_tensor(u, device=DEV), sqrt_s)
    hel = torch.as_tensor(h.astype(np.int32), device=DEV)
    ref = p64.eval(mom, hel).cpu().numpy()
    p = _proc(n, "per_point", "fp32c")
    assert p.info()["fixup"] == 1 and p.info()["fix_kappa"] > 0
    off = _proc(n, "per_point", "fp32c", make_variant(fixup=-1))
    assert off.info()["fixup"] == 0
    worst = 0.0
    for M in (N, 1000, 1, 4099, 4096, N):
        m = mom[:, :M].contiguous()
        got = p.eval(m, hel[:M].contiguous()).cpu().numpy()
        assert np.all(got >= 0), M          # no mark left behind
        rel = np.abs(got - ref[:M]) / np.abs(ref[:M])
        assert rel.max() < 1e-4, (M, rel.max(), int(np.argmax(rel)))
        worst = max(worst, rel.max())
    raw = off.eval(mom, hel).cpu().numpy()
    # the pass changes something: without it the worst point is worse
    assert np.abs(raw / ref - 1.0).max() > worst


def test_fp32c_two_streams_match_serial():
    """A process handle is read-only: the same FP32C per-point process
    evaluated on two streams at once gives bit for bit the results of
    serial calls (nothing is shared between the calls but the handle)."""
    n, sqrt_s, N = 5, 20.0, 1 << 17
    u, h = inputs.rambo_inputs(61, n, N, with_helicities=True)
    p = _proc(n, "per_point", "fp32c")
    mom = p.rambo(torch.as_tensor(u, device=DEV), sqrt_s)
    hel = torch.as_tensor(h.astype(np.int32), device=DEV)
    a_m, b_m = mom[:, : N // 2].contiguous(), mom[:, N // 2:].contiguous()
    a_h, b_h = hel[: N // 2].contiguous(), hel[N // 2:].contiguous()
    ser_a, ser_b = p.eval(a_m, a_h), p.eval(b_m, b_h)
    torch.cuda.synchronize()
    s1, s2 = torch.cuda.Stream(), torch.cuda.Stream()
    out_a = torch.full_like(ser_a, float("nan"))
    out_b = torch.full_like(ser_b, float("nan"))
    for _ in range(3):
        with torch.cuda.stream(s1):
            p.eval(a_m, a_h, out=out_a)
        with torch.cuda.stream(s2):
            p.eval(b_m, b_h, out=out_b)
        torch.cuda.synchronize()
        assert torch.equal(out_a, ser_a) and torch.equal(out_b, ser_b)


def test_batch_plan_rejections():
    """Plans refuse what their single module cannot serve: crossed processes,
    mixed precisions, mixed FP64 fix-up settings, helicity sums."""
    from paper_2511_19456_amd._lib import QedError
    from paper_2511_19456_amd.qedx import BatchPlan, QedProcess, make_variant
    N = 64

    def seg(p):
        mom = torch.zeros(4 * p.n_particles, N, dtype=torch.float64, device=DEV)
        hel = torch.zeros(N, dtype=torch.int32, device=DEV)
        return (p, mom, hel, torch.empty(N, dtype=torch.float64, device=DEV))
    a = QedProcess(2, "per_point", "fp32c")
    cases = [
        [seg(QedProcess(1, "per_point", "fp64", n_in=2))],
        [seg(QedProcess(2, "per_point", "fp64")), seg(a)],
        [seg(a), seg(QedProcess(3, "per_point", "fp32c", make_variant(fixup=-1)))],
    ]
    for segs in cases:
        with pytest.raises(QedError):
            BatchPlan(segs, tile_points=64)
    p_sum = QedProcess(2, "sum", "fp64")
    with pytest.raises(QedError):
        BatchPlan([(p_sum, torch.zeros(20, N, dtype=torch.float64, device=DEV),
                    torch.zeros(N, dtype=torch.int32, device=DEV), torch.empty(N, dtype=torch.float64, device=DEV))],
                  tile_points=64)


def test_degenerate_kinematics():
    """Edge cases of the kinematics: photons exactly along the z axis (the
    polarisation basis switches to its k_T = 0 branch), backward scattering,
    and a nearly soft photon (a propagator close to its pole)."""
    # one photon, exact angles: Klein-Nishina closed form at omega = 1
    theta = np.array([0.0, np.pi / 2, np.pi, np.pi, 0.0])
    phi = np.array([0.0, 0.0, 0.0, 1.3, 2.0])
    mom = inputs.compton_lab_angles(theta, phi)
    got = _proc(1).eval(torch.as_tensor(mom, device=DEV)).cpu().numpy()
    ct, wp = np.cos(theta), mom[12]
    kn = 8.0 * (wp + 1.0 / wp - (1.0 - ct * ct))
    assert np.abs(got / kn - 1).max() < 1e-12
    # every configuration at those points against the oracle
    N = len(theta)
    hel = np.tile(np.arange(16, dtype=np.uint32), N)
    mm = np.repeat(mom, 16, axis=1)
    pp = _proc(1, "per_point").eval(torch.as_tensor(mm, device=DEV),
                                    torch.as_tensor(hel.astype(np.int32), device=DEV)).cpu().numpy()
    ref, kap = per_point_ref(mm, 1, hel)
    nz = ref > 0          # exact zeros (forbidden configurations at theta = 0, pi) must come out tiny
    check_fp64(pp[nz], ref[nz], kap[nz], "n=1 along the axis")
    assert np.all(np.abs(pp[~nz]) <= 1e-20 * np.repeat(kn, 16)[~nz])
    # two photons, the first final-state photon nearly soft, at kinematics
    # exact in binary (dyadic components, exactly on shell and conserving;
    # tests/golden/near_soft_n2.txt, written by make_golden.py from oracle/
    # only): the extended-precision oracle's values are the reference.  The
    # kernels' cancellation-free Q^2 - m^2 is exact algebra for such inputs,
    # so they must agree to the stated tolerance however close the pole.
    import sys
    import os
    sys.path.insert(0, os.path.join(os.path.dirname(__file__), "golden"))
    from make_golden import SOFT_SHIFTS, read_near_soft
    n = 2
    gold = read_near_soft()
    assert sorted(gold) == sorted(SOFT_SHIFTS)
    for shift, d in sorted(gold.items()):
        m = torch.as_tensor(d["mom"], device=DEV)
        assert float(d["mom"][4 * 3].max()) < 4.0 * 2.0 ** -shift   # the soft photon's energy
        s_got = _proc(n).eval(m).cpu().numpy()
        p_got = _proc(n, "per_point").eval(m, torch.as_tensor(d["hel"].astype(np.int32), device=DEV)).cpu().numpy()
        assert _rel(s_got, d["sum"]).max() < 1e-10, (shift, _rel(s_got, d["sum"]).max())
        check_fp64(p_got, d["pp"], d["kappa_terms"], f"near soft 2^-{shift}")
        # FP32C at the same points: the FP64 first-step currents keep the
        # cancellation next to the resting electron out of FP32
        p32 = _proc(n, "per_point", "fp32c").eval(m, torch.as_tensor(d["hel"].astype(np.int32), device=DEV))
        assert _rel(p32.cpu().numpy(), d["pp"]).max() < 1e-4, (shift, _rel(p32.cpu().numpy(), d["pp"]).max())
