"""Build the qedx native library and prebuild its kernel cache.

Steps
1. Embed the device headers (qedx_device.h, qedx_rambo.h) as a raw string
   literal so generated kernels are self-contained translation units.
2. Compile the host library libqedx.so (graph builder, reducer, emitter,
   runtime) with the host C++ compiler against the HIP runtime.
3. Emit and compile (hipcc --genco, gfx950) the kernels of the default process
   variants into the code-object cache next to the library, in parallel.
   Cache entries are keyed by the hash of source + flags, so unchanged kernels
   are not recompiled.

Run as ``python -m paper_2511_19456_amd.build_ext [--no-kernels] [--jobs J]``.
"""
from __future__ import annotations

import argparse
import concurrent.futures as cf
import ctypes
import os
import subprocess
import sys
import time

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
CSRC = os.path.join(PKG, "csrc")
LIB = os.path.join(PKG, "libqedx.so")
ROCM = os.environ.get("ROCM_PATH", "/opt/rocm")

HOST_SOURCES = ["qedx_dag.cpp", "qedx_emit.cpp", "qedx_kernels.cpp", "qedx_runtime.cpp", "qedx_batch.cpp",
                "qedx_hosttools.cpp"]
# measurement tool kept out of the evaluation library (include/qedx_probe.h)
PROBE_SOURCES = ["qedx_probe.cpp"]
PROBE_LIB = os.path.join(PKG, "libqedx_probe.so")
DEVICE_HEADERS = ["qedx_device.h", "qedx_rambo.h"]


def embed_headers() -> None:
    parts = []
    for h in DEVICE_HEADERS:
        txt = open(os.path.join(CSRC, h)).read().replace("#pragma once\n", "")
        parts.append(txt)
    body = "\n".join(parts)
    assert ")QEDXHDR\"" not in body
    out = 'R"QEDXHDR(' + body + ')QEDXHDR"\n'
    path = os.path.join(CSRC, "qedx_device_embed.inc")
    if not os.path.exists(path) or open(path).read() != out:
        with open(path, "w") as f:
            f.write(out)


def _compile_objects(sources, verbose):
    objs, cmds = [], []
    for s in sources:
        o = os.path.join(CSRC, "_build", s.replace(".cpp", ".o"))
        os.makedirs(os.path.dirname(o), exist_ok=True)
        objs.append(o)
        cmds.append(["g++", "-std=c++17", "-O2", "-fPIC", "-Wall", "-Wno-unused-function",
                     "-D__HIP_PLATFORM_AMD__", f"-I{ROCM}/include", "-c", os.path.join(CSRC, s), "-o", o]
                    + HOST_EXTRA_FLAGS)
    with cf.ThreadPoolExecutor(max_workers=len(cmds)) as ex:
        futs = [ex.submit(subprocess.run, c, capture_output=True, text=True) for c in cmds]
        for c, f in zip(cmds, futs):
            r = f.result()
            if r.returncode != 0:
                raise RuntimeError("compile failed: " + " ".join(c) + "\n" + r.stderr)
            if verbose and r.stderr:
                print(r.stderr, file=sys.stderr)
    return objs


def _link(out, objs, extra):
    tmp = out + ".tmp"
    link = ["g++", "-shared", "-o", tmp] + objs + extra + [f"-L{ROCM}/lib", "-lamdhip64",
                                                          f"-Wl,-rpath,{ROCM}/lib"] + HOST_EXTRA_FLAGS
    r = subprocess.run(link, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError("link failed: " + r.stderr)
    os.replace(tmp, out)


# extra host compile/link flags (e.g. a sanitizer build of the host library);
# the generated GPU code is compiled by the library itself, never with these
HOST_EXTRA_FLAGS = os.environ.get("QEDX_HOST_FLAGS", "").split()


# the library's one HIP-compiled unit: the per-device scratch array of the
# allocation-free entry point (a __device__ symbol needs the HIP compiler)
HIP_SOURCES = ["qedx_scratch.hip"]


def _compile_hip_objects(sources, verbose):
    objs = []
    for s in sources:
        o = os.path.join(CSRC, "_build", s.replace(".hip", ".o"))
        os.makedirs(os.path.dirname(o), exist_ok=True)
        cmd = [os.path.join(ROCM, "bin", "hipcc"), "-std=c++17", "-O2", "-fPIC", "--offload-arch=gfx950",
               "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops", "-c", os.path.join(CSRC, s), "-o", o]
        r = subprocess.run(cmd, capture_output=True, text=True)
        if r.returncode != 0:
            raise RuntimeError("compile failed: " + " ".join(cmd) + "\n" + r.stderr)
        if verbose and r.stderr:
            print(r.stderr, file=sys.stderr)
        objs.append(o)
    return objs


def build_library(verbose: bool = False) -> None:
    embed_headers()
    _link(LIB, _compile_objects(HOST_SOURCES, verbose) + _compile_hip_objects(HIP_SOURCES, verbose), [])
    # the probe library resolves the code-object cache and error reporting
    # from libqedx.so next to it
    _link(PROBE_LIB, _compile_objects(PROBE_SOURCES, verbose), [f"-L{PKG}", "-lqedx", "-Wl,-rpath,$ORIGIN"])


from paper_2511_19456_amd._lib import QedVariant  # noqa: E402  (ctypes layout of qed_variant)


# (n, mode, precision[, variant fields]) built ahead of time: SUM 0 / PER_POINT 1;
# FP64 0 / FP32C 1.  The variant fields are keyword arguments of QedVariant
# (lane_bits, order, rewrite, ...); absent = the library default shape.
DEFAULT_KERNELS = [
    (1, 0, 0), (2, 0, 0), (3, 0, 0), (4, 0, 0),
    (1, 1, 0), (2, 1, 0), (3, 1, 0), (4, 1, 0), (5, 1, 0), (6, 1, 0),
    (3, 0, 1), (1, 1, 1), (2, 1, 1), (3, 1, 1), (4, 1, 1), (5, 1, 1), (6, 1, 1),
    # distributive rewrite (bench legs and parity tests)
    (2, 0, 0, dict(rewrite=1)), (3, 0, 0, dict(rewrite=1)), (3, 0, 0, dict(rewrite=1, lane_bits=7)),
    (4, 0, 0, dict(rewrite=1)), (4, 1, 0, dict(rewrite=1)), (5, 1, 0, dict(rewrite=1)), (6, 1, 0, dict(rewrite=1)),
    (1, 1, 0, dict(rewrite=1)), (2, 1, 0, dict(rewrite=1)), (3, 1, 0, dict(rewrite=1)),
    (3, 0, 1, dict(rewrite=1)), (5, 1, 1, dict(rewrite=1)),
    # the join of the distributive n = 3 helicity sum on the FP64 matrix cores (experiment)
    (3, 0, 0, dict(rewrite=1, order=128)),
    # kernel shapes the parity tests exercise
    (3, 0, 0, dict(lane_bits=7)), (3, 0, 0, dict(lane_bits=5, order=4)), (3, 0, 0, dict(lane_bits=63, order=4)),
    (3, 1, 0, dict(order=4)), (3, 0, 0, dict(lane_bits=5, order=16)), (3, 0, 0, dict(lane_bits=5, loop_bits=2, order=32)),
    (3, 1, 0, dict(order=24)),
    # reduction experiment (Sec. III-D): n = 4, one configuration per point, unsplit graph after
    # k of the 280 single node reductions (seeded order 1)
    (4, 1, 0, dict(partial_steps=0, partial_seed=1)), (4, 1, 0, dict(partial_steps=70, partial_seed=1)),
    (4, 1, 0, dict(partial_steps=140, partial_seed=1)), (4, 1, 0, dict(partial_steps=210, partial_seed=1)),
    (4, 1, 0, dict(partial_steps=280, partial_seed=1)),
    # Table I orientation e- gamma^n_in -> e- gamma (crossed processes, eval kernel only)
    (1, 0, 0, dict(n_in=2)), (1, 0, 0, dict(n_in=3)), (1, 0, 0, dict(n_in=4)), (1, 0, 1, dict(n_in=3)),
    (1, 1, 0, dict(n_in=2)), (1, 1, 0, dict(n_in=3)), (1, 1, 0, dict(n_in=4)), (1, 1, 0, dict(n_in=5)),
    (1, 1, 0, dict(n_in=6)), (1, 1, 1, dict(n_in=3)), (1, 1, 1, dict(n_in=6)), (2, 0, 0, dict(n_in=2)),
    (1, 1, 0, dict(n_in=6, rewrite=1)),
    # FP32C per point without the FP64 pass (bench leg and tests)
    (3, 1, 1, dict(fixup=-1)), (5, 1, 1, dict(fixup=-1)),
    # one-photon current cache shapes the parity tests exercise
    (4, 1, 0, dict(order=8)), (4, 1, 0, dict(order=264)), (4, 1, 0, dict(order=520)), (5, 1, 0, dict(order=1288)),
    (6, 1, 0, dict(order=264)), (4, 1, 1, dict(order=520)), (6, 1, 1, dict(order=1288)),
]


def prebuild_kernels(kernels=DEFAULT_KERNELS, jobs: int = 8, verbose: bool = True) -> dict:
    lib = ctypes.CDLL(LIB)
    lib.qed_prebuild.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_void_p, ctypes.c_int,
                                 ctypes.POINTER(ctypes.c_double)]
    lib.qed_prebuild.restype = ctypes.c_int
    lib.qed_prebuild_crossed.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_void_p,
                                         ctypes.POINTER(ctypes.c_double)]
    lib.qed_prebuild_crossed.restype = ctypes.c_int
    lib.qed_last_error.restype = ctypes.c_char_p

    def one(k):
        n, mode, prec = k[:3]
        var = None
        n_in = 1
        if len(k) > 3:
            kw = dict(k[3])
            n_in = kw.pop("n_in", 1)
            if "partial_steps" in kw:
                kw["partial"] = 1
            var = QedVariant(**kw) if kw else None
        ms = ctypes.c_double(0.0)
        t = time.time()
        vp = ctypes.byref(var) if var is not None else None
        if n_in == 1:
            rc = lib.qed_prebuild(n, mode, prec, vp, 1, ctypes.byref(ms))
        else:
            rc = lib.qed_prebuild_crossed(n_in, n, mode, prec, vp, ctypes.byref(ms))
        err = lib.qed_last_error().decode() if rc else ""
        return k, rc, ms.value, time.time() - t, err

    out = {}
    with cf.ThreadPoolExecutor(max_workers=jobs) as ex:
        for k, rc, ms, wall, err in ex.map(one, kernels):
            out[str(k)] = (rc, ms)
            if verbose:
                extra = f" {k[3]}" if len(k) > 3 else ""
                print(f"[qedx build] kernel n={k[0]} mode={k[1]} prec={k[2]}{extra}: rc={rc} "
                      f"compile={ms / 1e3:.1f}s", flush=True)
            if rc:
                raise RuntimeError(f"kernel prebuild failed for {k}: {err}")
    return out


BATCH_MODULES = [((1, 2, 3, 4, 5, 6), 0, 0), ((1, 2, 3, 4, 5, 6), 1, 0), ((1, 2, 3, 4, 5, 6), 0, 1)]


def prebuild_batches(verbose: bool = True) -> None:
    lib = ctypes.CDLL(LIB)
    lib.qed_batch_prebuild.argtypes = [ctypes.POINTER(ctypes.c_int), ctypes.c_int, ctypes.c_int, ctypes.c_int,
                                       ctypes.POINTER(ctypes.c_double)]
    lib.qed_last_error.restype = ctypes.c_char_p

    def one(spec):
        ns, prec, rewrite = spec
        arr = (ctypes.c_int * len(ns))(*ns)
        ms = ctypes.c_double(0)
        rc = lib.qed_batch_prebuild(arr, len(ns), prec, rewrite, ctypes.byref(ms))
        return spec, rc, ms.value, lib.qed_last_error().decode() if rc else ""

    with cf.ThreadPoolExecutor(max_workers=len(BATCH_MODULES)) as ex:
        for spec, rc, ms, err in ex.map(one, BATCH_MODULES):
            if verbose:
                print(f"[qedx build] batch module {spec}: rc={rc} compile={ms / 1e3:.1f}s", flush=True)
            if rc:
                raise RuntimeError(f"batch prebuild failed for {spec}: {err}")


def prebuild_probe(verbose: bool = True) -> None:
    ctypes.CDLL(LIB, mode=ctypes.RTLD_GLOBAL)
    lib = ctypes.CDLL(PROBE_LIB)
    lib.qed_pipe_probe_prebuild.argtypes = [ctypes.POINTER(ctypes.c_double)]
    lib.qed_pipe_probe_prebuild.restype = ctypes.c_int
    lib.qed_last_error.restype = ctypes.c_char_p
    ms = ctypes.c_double(0.0)
    rc = lib.qed_pipe_probe_prebuild(ctypes.byref(ms))
    if rc:
        raise RuntimeError(f"probe prebuild failed: {lib.qed_last_error().decode()}")
    if verbose:
        print(f"[qedx build] FP64 pipe probe: compile={ms.value / 1e3:.1f}s", flush=True)


def main(argv=None) -> None:
    ap = argparse.ArgumentParser()
    ap.add_argument("--no-kernels", action="store_true")
    ap.add_argument("--jobs", type=int, default=8)
    a = ap.parse_args(argv)
    build_library()
    if not a.no_kernels:
        prebuild_kernels(jobs=a.jobs)
        prebuild_batches()
        prebuild_probe()


if __name__ == "__main__":
    main()
