#!/usr/bin/env python3
"""Benchmark of the batched |M|^2 hot path on one MI355X.

Headline workload: e- gamma -> e- 3 gamma (24 diagrams), FP64, 2^20
phase-space points from RAMBO at sqrt(s) = 10 m (seeded uniforms), |M|^2 summed
over all 2^6 spin/polarisation configurations.  Inputs are generated on the
device and resident in HBM before the timed region.  One step = one evaluation
of the whole batch by qed_eval (momentum load, external states, vertices,
propagators, joins, diagram sum, |A|^2 and helicity sum).

Printed: one JSON line with the throughput, a roofline entry for the eval
kernel (algorithmic FLOPs = C(DAG) of the node-reduced helicity-summed graph
per point, against the FP64 vector peak; kernel time from HIP events on the
launch stream), the CPU oracle timed on a bounded sample on the host cores,
and further legs on the same GPU: the one-photon workload, the FP32-compensated
forms (with their error against the FP64 kernel), one random configuration per
point at n = 5, the mixed n = 1..6 batch in one persistent launch against the
six plain launches, and the gradient through RAMBO at n = 4.
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "|M|² phase-space points/s per process (FP64 vs FP32-comp, batched) + % of peak"
FP64_VECTOR_PEAK_TFLOPS = 78.6   # 256 CU x 4 SIMD x 16 lanes x 2 FLOP (FMA) x 2.4 GHz
FP32_VECTOR_PEAK_TFLOPS = 157.3  # packed FP32


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--no-legs", action="store_true", help="skip the extra legs")
    ap.add_argument("--legs", default="", help="comma-separated subset of legs to run")
    ap.add_argument("--cpu-seconds", type=float, default=12.0)
    ap.add_argument("--copy-calibration", action="store_true",
                    help="only run a plain device copy of 512 MiB three times (reference for HBM byte counters)")
    return ap.parse_args()


def copy_calibration():
    """A plain copy of known size: 512 MiB read and 512 MiB written per launch.
    rocprofv3's FETCH_SIZE / WRITE_SIZE on this kernel give the factor that
    turns those counters into bytes."""
    import torch
    n = 1 << 26
    src = torch.ones(n, dtype=torch.float64, device="cuda:0")
    dst = torch.empty_like(src)
    for _ in range(3):
        dst.copy_(src)
    torch.cuda.synchronize()
    print(json.dumps({"copy_bytes_read_per_launch": 8 * n, "copy_bytes_written_per_launch": 8 * n}), flush=True)


# Untimed calls after the warm-up steps, for at least this long: from idle
# the GPU's clocks take ~20 launches (~50 ms) of this path to settle (a
# kernel trace shows the headline kernel going from 2.29 to 1.85 ms over its
# first 20 launches); the timed steps measure the settled rate.
SETTLE_MS = 150.0


def time_launches(fn, steps, warmup, settle_ms=SETTLE_MS):
    """Average ms per call of fn (which launches on torch's current stream),
    from HIP events recorded on that stream around `steps` calls, after
    `warmup` calls and at least `settle_ms` of further untimed calls."""
    import torch
    for _ in range(warmup):
        fn()
    torch.cuda.synchronize()
    t0, k = time.perf_counter(), 0
    while (time.perf_counter() - t0) * 1e3 < settle_ms and k < 4000:
        fn()
        k += 1
        if k % 8 == 0:
            torch.cuda.synchronize()
    torch.cuda.synchronize()
    s = torch.cuda.Event(enable_timing=True)
    e = torch.cuda.Event(enable_timing=True)
    s.record()
    for _ in range(steps):
        fn()
    e.record()
    torch.cuda.synchronize()
    return s.elapsed_time(e) / steps


def _cpu_model():
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown CPU"


def _timed_oracle(step, chunk, total, budget_s):
    """Run step(lo, hi) over consecutive chunks of the sample until the time
    budget is spent; returns (points done, seconds)."""
    done, t_used = 0, 0.0
    while t_used < budget_s and done < total:
        hi = min(total, done + chunk)
        t0 = time.perf_counter()
        step(done, hi)
        t_used += time.perf_counter() - t0
        done = hi
    return done, t_used


def cpu_baseline(u, sqrt_s, n, budget_s, per_config=True):
    """The oracle (plain per-diagram |M|^2, explicit 4x4 Dirac matrices) on the
    host cores: the headline workload on every thread torch uses and on one
    thread, and bounded samples of the other workloads.  Momenta come from the
    oracle's own RAMBO outside the timed |M|^2 calls; the gradient row times
    the oracle's RAMBO and reverse-mode autodiff together, as the GPU path
    does."""
    import numpy as np
    import torch

    from oracle import qed_oracle as O
    from paper_2511_19456_amd import inputs
    threads = torch.get_num_threads()
    model = _cpu_model()

    def m2_rate(mom, nn, mode, hel, chunk, budget):
        def step(lo, hi):
            O.m2(mom[:, lo:hi], nn, mode, None if hel is None else hel[lo:hi])
        return _timed_oracle(step, chunk, mom.shape[1], budget)

    # headline: n = 3, helicity sum
    mom3 = O.momenta_soa_from_uniforms(u[:, :1 << 18], sqrt_s, n)
    done, t_used = m2_rate(mom3, n, "sum", None, 2048, budget_s)
    rec = {"value": done / t_used, "unit": "points/s", "cores": threads, "kind": "oracle",
           "sample": f"first {done} points of the workload (n=3, helicity sum), momenta from the oracle's RAMBO, "
                     f"{t_used:.1f} s of |M|^2 time on {threads} threads of {model} "
                     f"({os.cpu_count()} logical CPUs visible)"}
    if not per_config:
        return rec
    sub = max(2.0, budget_s / 4)
    torch.set_num_threads(1)
    try:
        d1, t1 = m2_rate(mom3, n, "sum", None, 256, sub)
    finally:
        torch.set_num_threads(threads)
    rec["one_thread"] = {"value": d1 / t1, "unit": "points/s", "cores": 1,
                         "sample": f"first {d1} points of the same workload, {t1:.1f} s on 1 thread"}
    rows = []
    # config 1: n = 1, helicity sum, electron at rest, omega = 1
    m1 = torch.as_tensor(inputs.compton_lab_momenta(1, 65536))
    d, t = m2_rate(m1, 1, "sum", None, 8192, sub)
    rows.append({"workload": "n=1 helicity sum, 65,536 points (electron at rest, omega = 1)", "value": d / t,
                 "unit": "points/s", "cores": threads, "sample": f"first {d} points, {t:.1f} s"})
    # config 3: n = 5, one configuration per point
    wl5 = inputs.WORKLOADS["n5_perpoint_rs20_2p20"]
    u5, h5 = inputs.rambo_inputs(wl5["seed"], 5, 4096, with_helicities=True)
    m5 = O.momenta_soa_from_uniforms(u5, wl5["sqrt_s"], 5)
    d, t = m2_rate(m5, 5, "per_point", h5, 128, sub)
    rows.append({"workload": "n=5 one configuration per point, sqrt(s)=20", "value": d / t, "unit": "points/s",
                 "cores": threads, "sample": f"first {d} points of a 4,096-point draw of seed 3, {t:.1f} s"})
    # config 5: gradient of log|M|^2 at n = 4 through RAMBO
    wlg = inputs.WORKLOADS["grad_n4_sum_rs15_2p18"]
    ug, _ = inputs.rambo_inputs(wlg["seed"], 4, 1024)

    def gstep(lo, hi):
        O.logm2_and_grad(np.ascontiguousarray(ug[:, lo:hi]), wlg["sqrt_s"], 4, chunk=hi - lo)
    d, t = _timed_oracle(gstep, 32, ug.shape[1], sub)
    rows.append({"workload": "n=4 helicity sum, log|M|^2 and its gradient w.r.t. the 20 RAMBO uniforms, "
                             "sqrt(s)=15", "value": d / t, "unit": "points/s", "cores": threads,
                 "sample": f"first {d} points of seed 5, {t:.1f} s (oracle RAMBO + reverse-mode autodiff)"})
    rec["per_config"] = rows
    return rec


def traffic_entry(code_hash):
    """HBM bytes per launch from the committed rocprofv3 FETCH_SIZE/WRITE_SIZE
    summary, if it was taken on this exact code object; else None."""
    path = os.path.join(ROOT, "profiles", "traffic.json")
    try:
        with open(path) as f:
            ent = json.load(f).get(code_hash)
        return ent["bytes_per_launch"] if ent else None
    except (OSError, ValueError, KeyError):
        return None


def alg_flops(n, mode, rewrite=0):
    """C(DAG) per point of the graph the kernel evaluates (node-reduced, or
    node-reduced then distributed when rewrite = 1)."""
    from paper_2511_19456_amd.qedx import graph_metrics
    mask = (1 << (n + 3)) - 1 if mode == "sum" else 0
    return graph_metrics(n, enum_mask=mask, reduced=2 if rewrite else True)[0]


def rel_err_stats(a, b, per_point=False):
    """Plain relative error |a - b| / |b| of a against b, point by point:
    max, p99, median, fraction and count above 1e-4."""
    import torch
    r = ((a - b).abs() / b.abs()).double()
    q = torch.quantile(r[: 1 << 20].float(), torch.tensor([0.5, 0.99], device=r.device)).tolist()
    return {"max": r.max().item(), "p99": q[1], "median": q[0], "frac_above_1e-4": (r > 1e-4).double().mean().item(),
            "points_above_1e-4": int((r > 1e-4).sum().item())}


def main():
    a = parse()
    if a.copy_calibration:
        copy_calibration()
        return
    if a.gpus != 1:
        print(f"bench.py: measures one GPU only (asked for --gpus {a.gpus}); points are independent, so "
              "running on several GPUs is a split of the point range with no communication", file=sys.stderr)
        sys.exit(2)
    import torch

    from paper_2511_19456_amd import inputs
    from paper_2511_19456_amd.qedx import QedProcess

    dev = torch.device("cuda:0")
    wl = inputs.WORKLOADS["n3_sum_rs10_2p20"]
    n, N, sqrt_s = wl["n"], wl["N"], wl["sqrt_s"]
    u, _ = inputs.rambo_inputs(wl["seed"], n, N)

    proc = QedProcess(n, "sum", "fp64")
    info = proc.info()
    ud = torch.as_tensor(u, device=dev)
    mom = proc.rambo(ud, sqrt_s)
    out = torch.empty(N, dtype=torch.float64, device=dev)
    torch.cuda.synchronize()

    ms = time_launches(lambda: proc.eval(mom, out=out), a.steps, a.warmup)
    value = N / (ms * 1e-3)
    flops_pt = alg_flops(n, "sum")
    achieved = flops_pt * N / (ms * 1e-3) / 1e12
    rec = {
        "metric": METRIC,
        "value": value,
        "unit": "points/s",
        "n_gpus": 1,
        "steps": a.steps,
        "warmup": a.warmup,
        "ms_per_step": ms,
        "clock_settle_ms": SETTLE_MS,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": "e- gamma -> e- 3gamma, FP64, 2^20 RAMBO points at sqrt(s)=10 m, "
                               "sum over 64 spin/polarisation configurations",
                   "n_photons_out": n, "points": N, "sqrt_s": sqrt_s, "helicity": "sum", "seed": wl["seed"],
                   "kernel": info["kernel_tag"], "code_hash": info["code_hash"]},
        "roofline": {"bound": "alu", "achieved": achieved, "peak": FP64_VECTOR_PEAK_TFLOPS, "unit": "TFLOP/s",
                     "frac": achieved / FP64_VECTOR_PEAK_TFLOPS, "traffic": traffic_entry(info["code_hash"]),
                     "flops_per_point": flops_pt, "kernel": info["kernel_name"],
                     "executed_flops_per_point": info["flops_per_point"]},
    }
    ref_n3 = out.clone()
    if not a.no_legs:
        want = set(x for x in a.legs.split(",") if x)
        rec["legs"] = extra_legs(torch, inputs, QedProcess, dev, a, want, ref_n3, mom)
    if not a.no_cpu:
        rec["cpu_baseline"] = cpu_baseline(u, sqrt_s, n, a.cpu_seconds)
    print(json.dumps(rec), flush=True)


def _leg(legs, key, want, fn):
    if want and key not in want:
        return
    try:
        legs[key] = fn()
    except Exception as ex:  # a leg that fails is reported in the line, not fatal
        legs[key] = {"error": f"{type(ex).__name__}: {str(ex)[:300]}"}
    print(f"[bench] leg {key}: {json.dumps(legs[key])}", file=sys.stderr, flush=True)


def extra_legs(torch, inputs, QedProcess, dev, a, want, ref_n3, mom_n3):
    import numpy as np
    legs = {}
    steps = max(5, a.steps // 2)

    def rate(ms, N, flops_pt, peak):
        t = flops_pt * N / (ms * 1e-3) / 1e12
        return {"ms": ms, "points_per_s": N / (ms * 1e-3), "alg_tflops": t, "frac": t / peak,
                "flops_per_point": flops_pt}

    def n1_sum():
        N = 65536
        m = torch.as_tensor(inputs.compton_lab_momenta(1, N), device=dev)
        p = QedProcess(1, "sum", "fp64")
        o = torch.empty(N, dtype=torch.float64, device=dev)
        ms = time_launches(lambda: p.eval(m, out=o), steps, 2)
        r = rate(ms, N, alg_flops(1, "sum"), FP64_VECTOR_PEAK_TFLOPS)
        r["note"] = "65,536 points fill ~1 wave per SIMD: launch/latency bound, roofline fraction not meaningful"
        return r
    _leg(legs, "n1_sum_fp64_65536", want, n1_sum)

    def n3_fp32c():
        N = ref_n3.numel()
        p = QedProcess(3, "sum", "fp32c")
        o = torch.empty(N, dtype=torch.float64, device=dev)
        ms = time_launches(lambda: p.eval(mom_n3, out=o), steps, 2)
        r = rate(ms, N, alg_flops(3, "sum"), FP32_VECTOR_PEAK_TFLOPS)
        r["err_vs_fp64_kernel"] = rel_err_stats(o, ref_n3)
        return r
    _leg(legs, "n3_sum_fp32c_2p20", want, n3_fp32c)

    def distributive(n, mode, rs, seed):
        def run():
            from paper_2511_19456_amd.qedx import make_variant
            N = 1 << 20
            u, h = inputs.rambo_inputs(seed, n, N, with_helicities=True)
            hd = torch.as_tensor(h.astype(np.int32), device=dev) if mode == "per_point" else None
            base = QedProcess(n, mode, "fp64")
            dist = QedProcess(n, mode, "fp64", make_variant(rewrite=1))
            m = base.rambo(torch.as_tensor(u, device=dev), rs)
            o0 = torch.empty(N, dtype=torch.float64, device=dev)
            o1 = torch.empty(N, dtype=torch.float64, device=dev)
            ms0 = time_launches(lambda: base.eval(m, hd, out=o0), steps, 2)
            ms1 = time_launches(lambda: dist.eval(m, hd, out=o1), steps, 2)
            r = rate(ms1, N, alg_flops(n, mode, rewrite=1), FP64_VECTOR_PEAK_TFLOPS)
            r.update({"ms_node_reduced_only": ms0, "speedup_vs_node_reduced": ms0 / ms1,
                      "rel_diff_vs_node_reduced": rel_err_stats(o1, o0, per_point=(mode == "per_point")),
                      "kernel": dist.info()["kernel_name"]})
            return r
        return run
    _leg(legs, "n3_sum_fp64_distributive_2p20", want, distributive(3, "sum", 10.0, 2))

    def mfma_join():
        """The same distributive n = 3 helicity-sum graph with its joins (4 x 4
        complex dot blocks per photon partition) on the FP64 matrix cores,
        against its vector joins, on the headline points."""
        from paper_2511_19456_amd.qedx import make_variant
        N = ref_n3.numel()
        vec = QedProcess(3, "sum", "fp64", make_variant(rewrite=1))
        mat = QedProcess(3, "sum", "fp64", make_variant(rewrite=1, order=128))
        o0 = torch.empty(N, dtype=torch.float64, device=dev)
        o1 = torch.empty(N, dtype=torch.float64, device=dev)
        ms0 = time_launches(lambda: vec.eval(mom_n3, out=o0), steps, 2)
        ms1 = time_launches(lambda: mat.eval(mom_n3, out=o1), steps, 2)
        fl = alg_flops(3, "sum", rewrite=1)
        r = rate(ms1, N, fl, FP64_VECTOR_PEAK_TFLOPS)
        i0, i1 = vec.info(), mat.info()
        r.update({"ms_vector_join": ms0, "speedup_vs_vector_join": ms0 / ms1,
                  "rel_diff_vs_vector_join": rel_err_stats(o1, o0), "kernel": i1["kernel_name"],
                  "vgpr_agpr_scratch": [i1["vgpr"], i1["agpr"], i1["scratch_bytes"]],
                  "vector_vgpr_agpr_scratch": [i0["vgpr"], i0["agpr"], i0["scratch_bytes"]]})
        return r
    _leg(legs, "n3_sum_fp64_distributive_mfma_join_2p20", want, mfma_join)
    _leg(legs, "n5_per_point_fp64_distributive_2p20", want, distributive(5, "per_point", 20.0, 3))
    _leg(legs, "n6_per_point_fp64_distributive_2p20", want, distributive(6, "per_point", 25.0, 3))

    wl5 = inputs.WORKLOADS["n5_perpoint_rs20_2p20"]
    u5, h5 = inputs.rambo_inputs(wl5["seed"], 5, wl5["N"], with_helicities=True)
    h5d = torch.as_tensor(h5.astype(np.int32), device=dev)
    p5 = {}

    def n5(prec):
        def run():
            p = QedProcess(5, "per_point", prec)
            p5[prec] = p
            m = p.rambo(torch.as_tensor(u5, device=dev), wl5["sqrt_s"])
            o = torch.empty(wl5["N"], dtype=torch.float64, device=dev)
            ms = time_launches(lambda: p.eval(m, h5d, out=o), steps, 2)
            r = rate(ms, wl5["N"], alg_flops(5, "per_point"),
                     FP64_VECTOR_PEAK_TFLOPS if prec == "fp64" else FP32_VECTOR_PEAK_TFLOPS)
            p5[prec + "_out"] = o
            info = p.info()
            r.update({"vgpr": info["vgpr"], "agpr": info["agpr"], "scratch": info["scratch_bytes"]})
            if prec == "fp32c" and "fp64_out" in p5:
                r["err_vs_fp64_kernel"] = rel_err_stats(o, p5["fp64_out"], per_point=True)
                r["speedup_vs_fp64"] = legs["n5_per_point_fp64_2p20"]["ms"] / ms
                # the same kernel without the FP64 pass over ill-conditioned points
                from paper_2511_19456_amd.qedx import make_variant
                q = QedProcess(5, "per_point", prec, make_variant(fixup=-1))
                o2 = torch.empty_like(o)
                r["ms_without_fixup"] = time_launches(lambda: q.eval(m, h5d, out=o2), steps, 2)
                r["err_without_fixup"] = rel_err_stats(o2, p5["fp64_out"], per_point=True)
                r["fix_kappa"] = info["fix_kappa"]
            return r
        return run
    _leg(legs, "n5_per_point_fp64_2p20", want, n5("fp64"))
    _leg(legs, "n5_per_point_fp32c_2p20", want, n5("fp32c"))

    def mixed(prec):
        def run():
            from paper_2511_19456_amd.qedx import BatchPlan
            spec = inputs.mixed_batch_spec(inputs.WORKLOADS["mixed_n1to6"]["seed"])
            segs, plain, tot_flops, tot_pts = [], [], 0.0, 0
            for (n, Np, rs, sub) in spec:
                u, h = inputs.rambo_inputs(sub, n, Np, with_helicities=True)
                p = QedProcess(n, "per_point", prec)
                m = p.rambo(torch.as_tensor(u, device=dev), rs)
                hd = torch.as_tensor(h.astype(np.int32), device=dev)
                o = torch.empty(Np, dtype=torch.float64, device=dev)
                segs.append((p, m, hd, o))
                tot_flops += alg_flops(n, "per_point") * Np
                tot_pts += Np
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            plan = BatchPlan(segs, tile_points=0)
            t_plan = time.perf_counter() - t0
            ms_b = time_launches(plan.launch, steps, 2)
            outs_b = [s[3].clone() for s in segs]
            # the same work as six plain per-process launches (FP64 eval kernels)
            plain_procs = [(QedProcess(s[0].n, "per_point", "fp64"), s[1], s[2],
                            torch.empty_like(s[3])) for s in segs]

            def six():
                for p, m, hd, o in plain_procs:
                    p.eval(m, hd, out=o)
            ms_p = time_launches(six, steps, 2)
            err = max(((ob - pp[3]).abs() / pp[3].abs().clamp_min(1e-300)).max().item()
                      for ob, pp in zip(outs_b, plain_procs)) if prec == "fp64" else None
            t = tot_flops / (ms_b * 1e-3) / 1e12
            peak = FP64_VECTOR_PEAK_TFLOPS if prec == "fp64" else FP32_VECTOR_PEAK_TFLOPS
            r = {"ms": ms_b, "points_per_s": tot_pts / (ms_b * 1e-3), "alg_tflops": t, "frac": t / peak,
                 "points": tot_pts, "segments": [(n, Np, round(rs, 3)) for (n, Np, rs, _) in spec],
                 "plan": plan.info(), "plan_create_s": t_plan, "ms_six_plain_fp64_launches": ms_p,
                 "speedup_vs_plain_fp64": ms_p / ms_b}
            if err is not None:
                r["max_rel_diff_vs_plain"] = err
            else:
                # FP32C batch against the plain FP64 kernels, over all points
                r["err_vs_fp64_kernel"] = rel_err_stats(torch.cat(outs_b), torch.cat([pp[3] for pp in plain_procs]),
                                                        per_point=True)
            return r
        return run
    def mixed_small():
        """Many small segments (48 segments, n cycling 1..6, N log-uniform in
        [10^3, 10^4]): the regime where one persistent graph launch replaces
        many short kernel launches."""
        from paper_2511_19456_amd.qedx import BatchPlan
        g = inputs.rng_for(41)
        procs = {n: QedProcess(n, "per_point", "fp64") for n in range(1, 7)}
        segs, tot_flops, tot_pts = [], 0.0, 0
        for i in range(48):
            n = 1 + i % 6
            Np = int(round(10.0 ** g.uniform(3.0, 4.0)))
            rs = float(g.uniform(5.0, 30.0))
            u, h = inputs.rambo_inputs(2000 + i, n, Np, with_helicities=True)
            p = procs[n]
            m = p.rambo(torch.as_tensor(u, device=dev), rs)
            segs.append((p, m, torch.as_tensor(h.astype(np.int32), device=dev),
                         torch.empty(Np, dtype=torch.float64, device=dev)))
            tot_flops += alg_flops(n, "per_point") * Np
            tot_pts += Np
        torch.cuda.synchronize()
        plan = BatchPlan(segs, tile_points=0)
        ms_b = time_launches(plan.launch, steps, 2)

        def plain():
            for p, m, hd, o in segs:
                p.eval(m, hd, out=o)
        ms_p = time_launches(plain, steps, 2)
        return {"segments": len(segs), "points": tot_pts, "ms": ms_b, "points_per_s": tot_pts / (ms_b * 1e-3),
                "alg_tflops": tot_flops / (ms_b * 1e-3) / 1e12, "plan": plan.info(),
                "ms_plain_launches": ms_p, "speedup_vs_plain_fp64": ms_p / ms_b}
    _leg(legs, "mixed_small_48seg_fp64", want, mixed_small)
    _leg(legs, "mixed_n1to6_fp64", want, mixed("fp64"))
    _leg(legs, "mixed_n1to6_fp32c", want, mixed("fp32c"))

    def reduction_sweep():
        """The paper's reduction experiment (Sec. III-D, III-E) on this GPU:
        n = 4, one configuration per point, the unsplit graph after k of the
        single node reductions (seeded random order), each emitted as one
        straight-line kernel; plus the full pipeline (reduction, join split,
        reduction, partition loop).  Speedup S(N) = t_e N / (t'_e N + t_o) and
        break-even N = t_o / (t_e - t'_e), t_o = host time of the reductions."""
        from paper_2511_19456_amd.qedx import graph_partial, make_variant, reduction_check
        n, seed = 4, 1
        total = reduction_check(n, seed, enum_mask=0, split=2)[2]
        t0 = time.perf_counter()
        graph_partial(n, total, seed)
        t_o = time.perf_counter() - t0
        ks = [0, total // 4, total // 2, 3 * total // 4, total]
        N = 1 << 20
        u, h = inputs.rambo_inputs(3, n, N, with_helicities=True)
        hd = torch.as_tensor(h.astype(np.int32), device=dev)
        rows = []
        base = {}
        for k in ks + ["full"]:
            v = None if k == "full" else make_variant(partial_steps=k, partial_seed=seed)
            p = QedProcess(n, "per_point", "fp64", v)
            m = p.rambo(torch.as_tensor(u, device=dev), 15.0)
            row = {"k": k, "nodes": p.info()["nodes_reduced"], "scratch": p.info()["scratch_bytes"]}
            for Nt in (1 << 14, N):
                mm, hh = m[:, :Nt].contiguous(), hd[:Nt].contiguous()
                o = torch.empty(Nt, dtype=torch.float64, device=dev)
                ms = time_launches(lambda: p.eval(mm, hh, out=o), steps, 2)
                row[f"ms_{Nt}"] = ms
                if k == 0:
                    base[Nt] = ms
                row[f"speedup_{Nt}"] = base[Nt] / ms
            te, tk = base[N] / N * 1e-3, row[f"ms_{N}"] / N * 1e-3
            row["break_even_N"] = t_o / (te - tk) if te > tk else None
            rows.append(row)
        return {"process": "e- gamma -> e- 4gamma, one configuration per point", "total_reductions": total,
                "t_o_s": t_o, "rows": rows}
    _leg(legs, "reduction_sweep_n4", want, reduction_sweep)

    def grad():
        wl = inputs.WORKLOADS["grad_n4_sum_rs15_2p18"]
        u, _ = inputs.rambo_inputs(wl["seed"], wl["n"], wl["N"])
        p = QedProcess(wl["n"], "sum", "fp64")
        ud = torch.as_tensor(u, device=dev)
        val = torch.empty(wl["N"], dtype=torch.float64, device=dev)
        g = torch.empty(4 * (wl["n"] + 1), wl["N"], dtype=torch.float64, device=dev)
        ms = time_launches(lambda: p.eval_grad(ud, wl["sqrt_s"], out=(val, g)), steps, 2)
        # forward only (RAMBO + |M|^2) on the same points, for the cost ratio
        m = torch.empty(4 * (wl["n"] + 3), wl["N"], dtype=torch.float64, device=dev)
        o = torch.empty(wl["N"], dtype=torch.float64, device=dev)

        def fwd():
            p.rambo(ud, wl["sqrt_s"], out=m)
            p.eval(m, out=o)
        ms_f = time_launches(fwd, steps, 2)
        # algorithmic FLOPs: forward C(DAG) of the node-reduced helicity-sum
        # graph plus the reverse-mode cost of the same graph (per-node
        # vector-Jacobian products); RAMBO and its adjoint are HBM-side and
        # not counted
        from paper_2511_19456_amd.qedx import graph_adjoint_metrics
        c_f, c_a = graph_adjoint_metrics(wl["n"], enum_mask=(1 << (wl["n"] + 3)) - 1)
        achieved = (c_f + c_a) * wl["N"] / (ms * 1e-3) / 1e12
        return {"ms": ms, "points_per_s": wl["N"] / (ms * 1e-3), "ms_forward_only": ms_f,
                "grad_over_forward": ms / ms_f,
                "roofline": {"bound": "alu", "achieved": achieved, "peak": FP64_VECTOR_PEAK_TFLOPS,
                             "unit": "TFLOP/s", "frac": achieved / FP64_VECTOR_PEAK_TFLOPS,
                             "flops_per_point": c_f + c_a, "forward_flops_per_point": c_f,
                             "adjoint_flops_per_point": c_a,
                             "note": "whole qed_eval_grad call (RAMBO, amplitudes, adjoint sweeps, RAMBO adjoint)"}}
    _leg(legs, "grad_n4_sum_fp64_2p18", want, grad)

    def table1_crossed():
        """The paper's Table I processes e- gamma^n -> e- gamma, one random
        configuration per point, FP64, 2^20 points each (crossed kinematics)."""
        N = 1 << 20
        rows = []
        for n_in in range(1, 7):
            mom, hel = inputs.crossed_inputs(300 + n_in, n_in, N, with_helicities=True)
            p = QedProcess(1, "per_point", "fp64", n_in=n_in)
            md = torch.as_tensor(mom, device=dev)
            hd = torch.as_tensor(hel.astype(np.int32), device=dev)
            o = torch.empty(N, dtype=torch.float64, device=dev)
            ms = time_launches(lambda: p.eval(md, hd, out=o), steps, 2)
            inf = p.info()
            from paper_2511_19456_amd.qedx import graph_metrics
            fl = graph_metrics(1, n_in=n_in, reduced=True)[0]   # C(DAG), one configuration
            t = fl * N / (ms * 1e-3) / 1e12
            rows.append({"n": n_in, "ms": ms, "ns_per_point": ms * 1e6 / N, "points_per_s": N / (ms * 1e-3),
                         "nodes_unreduced": inf["nodes_unreduced"], "nodes_reduced": inf["nodes_reduced"],
                         "flops_per_point": fl, "alg_tflops": t, "frac": t / FP64_VECTOR_PEAK_TFLOPS,
                         "executed_flops_per_point": inf["flops_per_point"]})
        return {"process": "e- gamma^n -> e- gamma, per point, FP64, 2^20 points", "rows": rows}
    _leg(legs, "table1_crossed_per_point_2p20", want, table1_crossed)

    def fp64_pipes():
        """FP64 vector pipe, FP64 matrix pipe (v_mfma_f64_16x16x4) and both at
        once: achievable rates on this chip, and whether the two overlap."""
        from paper_2511_19456_amd._lib import check, probe_lib
        blocks = 2048                      # 8 waves per SIMD
        it_v, it_m = 60000, 8000
        mm, cc = 0.999999, 1e-6
        av = torch.arange(64, dtype=torch.float64, device=dev) / 64.0
        bv = torch.arange(64, dtype=torch.float64, device=dev) / 128.0
        ov = torch.empty(blocks * 256, dtype=torch.float64, device=dev)
        om = torch.empty(blocks * 1024, dtype=torch.float64, device=dev)
        stream = torch.cuda.current_stream().cuda_stream

        def run(kind):
            if kind == 0:
                check(probe_lib().qed_pipe_probe(0, blocks, it_v, 0, mm, cc, None, None, ov.data_ptr(), None, stream))
            elif kind == 1:
                check(probe_lib().qed_pipe_probe(1, blocks, it_m, 0, mm, cc, av.data_ptr(), bv.data_ptr(),
                                           om.data_ptr(), None, stream))
            else:
                check(probe_lib().qed_pipe_probe(2, blocks, it_v, it_m, mm, cc, av.data_ptr(), bv.data_ptr(),
                                           ov.data_ptr(), om.data_ptr(), stream))
        waves = blocks * 4
        fl_v = waves * 64 * 16.0 * it_v            # 8 FMA chains per lane
        fl_m = waves * 4 * 2048.0 * it_m           # 4 MFMA per step per wave
        t0 = time_launches(lambda: run(0), 5, 1)
        t1 = time_launches(lambda: run(1), 5, 1)
        t2 = time_launches(lambda: run(2), 5, 1)
        half = 0.5 * (t0 + t1)                     # the mixed launch does half of each
        return {"vector_ms": t0, "vector_tflops": fl_v / (t0 * 1e-3) / 1e12,
                "matrix_ms": t1, "matrix_tflops": fl_m / (t1 * 1e-3) / 1e12,
                "mixed_ms": t2, "mixed_tflops": 0.5 * (fl_v + fl_m) / (t2 * 1e-3) / 1e12,
                "serial_estimate_ms": half, "overlap": half / t2,
                "peak_tflops": FP64_VECTOR_PEAK_TFLOPS}
    _leg(legs, "fp64_pipes", want, fp64_pipes)
    return legs


if __name__ == "__main__":
    main()
