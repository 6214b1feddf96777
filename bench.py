#!/usr/bin/env python3
"""Benchmark of the batched |M|^2 hot path on one MI355X.

Workload (the configuration the headline metric is quoted on): e- gamma ->
e- 3 gamma (24 diagrams), FP64, 2^20 phase-space points from RAMBO at
sqrt(s) = 10 m (seeded uniforms), |M|^2 summed over all 2^6 spin/polarisation
configurations.  Inputs are generated on the device and resident in HBM before
the timed region.  One step = one evaluation of the whole batch (qed_eval:
momentum load, external states, vertices, propagators, joins, diagram sum,
|A|^2 and helicity sum).

Printed: one JSON line with the throughput, a roofline entry for the eval
kernel (algorithmic FLOPs = C(DAG) of the node-reduced helicity-summed graph
per point, against the FP64 vector peak), and the CPU oracle timed on a
bounded sample on the host cores.  Extra legs (FP32-compensated, mixed batch,
gradient) are reported under "legs" when those kernels are available.
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "|M|² phase-space points/s per process (FP64 vs FP32-comp, batched) + % of peak"
FP64_VECTOR_PEAK_TFLOPS = 78.6  # 256 CU x 4 SIMD x 16 lanes x 2 FLOP x 2.4 GHz


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--no-legs", action="store_true", help="skip the extra legs")
    ap.add_argument("--cpu-seconds", type=float, default=12.0)
    return ap.parse_args()


def time_launches(fn, steps, warmup):
    import torch
    for _ in range(warmup):
        fn()
    torch.cuda.synchronize()
    s = torch.cuda.Event(enable_timing=True)
    e = torch.cuda.Event(enable_timing=True)
    s.record()
    for _ in range(steps):
        fn()
    e.record()
    torch.cuda.synchronize()
    return s.elapsed_time(e) / steps  # ms per launch (kernel-only stream time)


def cpu_baseline(u, sqrt_s, n, budget_s):
    import torch

    from oracle import qed_oracle as O
    chunk = 2048
    done, t_used = 0, 0.0
    while t_used < budget_s and done + chunk <= u.shape[1]:
        m = O.momenta_soa_from_uniforms(u[:, done:done + chunk], sqrt_s, n)
        t0 = time.perf_counter()
        O.m2(m, n, "sum")
        t_used += time.perf_counter() - t0
        done += chunk
    return {"value": done / t_used, "unit": "points/s", "cores": torch.get_num_threads(), "kind": "oracle",
            "sample": f"first {done} points of the workload (n=3, helicity sum), momenta from the oracle's RAMBO, "
                      f"{t_used:.1f} s of |M|^2 time"}


def traffic_entry(tag):
    path = os.path.join(ROOT, "profiles", "traffic.json")
    try:
        with open(path) as f:
            tab = json.load(f)
        ent = tab.get(tag)
        if ent:
            return ent["bytes_per_launch"]
    except (OSError, ValueError, KeyError):
        pass
    return None


def main():
    a = parse()
    if a.gpus != 1:
        print(f"bench.py: this build runs on one GPU only (asked for --gpus {a.gpus}); points are independent, "
              "so sharding is a split of the point range (see DESIGN.md)", file=sys.stderr)
        sys.exit(2)
    import numpy as np
    import torch

    from paper_2511_19456_amd import inputs
    from paper_2511_19456_amd.qedx import QedProcess, graph_metrics

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
    flops_pt, _ = graph_metrics(n, enum_mask=(1 << (n + 3)) - 1, reduced=True)
    achieved = flops_pt * N / (ms * 1e-3) / 1e12
    rec = {
        "metric": METRIC,
        "value": value,
        "unit": "points/s",
        "n_gpus": 1,
        "steps": a.steps,
        "warmup": a.warmup,
        "ms_per_step": ms,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": "e- gamma -> e- 3gamma, FP64, 2^20 RAMBO points at sqrt(s)=10 m, "
                               "sum over 64 spin/polarisation configurations",
                   "n_photons_out": n, "points": N, "sqrt_s": sqrt_s, "helicity": "sum", "seed": wl["seed"],
                   "kernel": info["kernel_tag"]},
        "roofline": {"bound": "alu", "achieved": achieved, "peak": FP64_VECTOR_PEAK_TFLOPS, "unit": "TFLOP/s",
                     "frac": achieved / FP64_VECTOR_PEAK_TFLOPS, "traffic": traffic_entry(info["kernel_tag"]),
                     "flops_per_point": flops_pt, "kernel": "qedx_eval"},
    }
    legs = {}
    if not a.no_legs:
        legs.update(extra_legs(torch, np, inputs, QedProcess, dev, a))
    if legs:
        rec["legs"] = legs
    if not a.no_cpu:
        rec["cpu_baseline"] = cpu_baseline(u, sqrt_s, n, a.cpu_seconds)
    print(json.dumps(rec), flush=True)


def extra_legs(torch, np, inputs, QedProcess, dev, a):
    """FP32-compensated and per-point forms on the same GPU (throughput only)."""
    legs = {}
    steps = max(3, a.steps // 4)
    try:
        n, N, rs = 3, 1 << 20, 10.0
        u, _ = inputs.rambo_inputs(2, n, N)
        p32 = QedProcess(n, "sum", "fp32c")
        mom = p32.rambo(torch.as_tensor(u, device=dev), rs)
        ms = time_launches(lambda: p32.eval(mom), steps, 1)
        legs["n3_sum_fp32c"] = {"points_per_s": N / (ms * 1e-3), "ms": ms}
    except Exception as ex:  # a leg that is not built is reported, not fatal
        legs["n3_sum_fp32c"] = {"error": str(ex)[:200]}
    for n, rs, prec in ((5, 20.0, "fp64"), (5, 20.0, "fp32c")):
        key = f"n{n}_per_point_{prec}"
        try:
            N = 1 << 20
            u, h = inputs.rambo_inputs(3, n, N, with_helicities=True)
            p = QedProcess(n, "per_point", prec)
            mom = p.rambo(torch.as_tensor(u, device=dev), rs)
            hel = torch.as_tensor(h.astype(np.int32), device=dev)
            ms = time_launches(lambda: p.eval(mom, hel), steps, 1)
            legs[key] = {"points_per_s": N / (ms * 1e-3), "ms": ms}
        except Exception as ex:
            legs[key] = {"error": str(ex)[:200]}
    return legs


if __name__ == "__main__":
    main()
