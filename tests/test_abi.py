"""The C ABI: the libraries load without a GPU and export every function
declared in include/*.h; the generated kernel source is self-contained."""
import ctypes
import os
import re

import pytest

from paper_2511_19456_amd import _lib
from paper_2511_19456_amd import qedx as Q

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared(header):
    txt = open(os.path.join(ROOT, "include", header)).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    return sorted(set(re.findall(r"^\s*(?:const\s+)?\w+\s*\**\s*(qed_\w+)\s*\(", txt, flags=re.M)))


# header -> (library that exports it, the binding's signature table)
HEADERS = {"qedx.h": (_lib.LIB_PATH, _lib.SIGNATURES), "qedx_tools.h": (_lib.LIB_PATH, _lib.SIGNATURES),
           "qedx_probe.h": (_lib.PROBE_LIB_PATH, _lib.PROBE_SIGNATURES)}


def test_every_declared_symbol_is_exported():
    assert sorted(f for f in os.listdir(os.path.join(ROOT, "include")) if f.endswith(".h")) == sorted(HEADERS)
    _lib.lib()  # the probe library resolves its runtime from libqedx.so
    total = 0
    for header, (path, sigs) in HEADERS.items():
        L = ctypes.CDLL(path)
        names = _declared(header)
        total += len(names)
        for n in names:
            assert hasattr(L, n), (header, n)
        # and the binding declares every one of them
        assert set(names) <= set(sigs), (header, set(names) - set(sigs))
    assert total >= 20


def test_product_header_holds_no_tools():
    """The evaluation ABI (qedx.h) declares the entry points of the hot path
    and their build/inspection calls only; host tools and the probe live in
    their own headers."""
    prod = set(_declared("qedx.h"))
    assert not prod & set(_declared("qedx_tools.h"))
    assert not any(n.startswith("qed_pipe_probe") for n in prod)
    assert not any(n.startswith("qed_graph_") for n in prod)
    for n in ("qed_process_create", "qed_eval", "qed_rambo", "qed_eval_grad", "qed_batch_plan_create",
              "qed_batch_launch", "qed_process_info"):
        assert n in prod


def test_emitted_source_is_self_contained():
    src = Q.emit_source(2, "sum", "fp64")
    assert 'extern "C" __global__' in src and "qedx_eval_n" in src
    assert "#include \"" not in src  # device header is inlined
    src = Q.emit_source(5, "per_point", "fp32c")
    assert "comp_acc" in src and "qx::dot<float>" in src


def test_status_codes_for_bad_processes():
    L = _lib.lib()
    h = ctypes.c_void_p()
    assert L.qed_process_create(0, 0, 0, None, ctypes.byref(h)) == _lib.QED_ERR_UNSUPPORTED
    assert L.qed_process_create(7, 0, 0, None, ctypes.byref(h)) == _lib.QED_ERR_UNSUPPORTED
    assert L.qed_process_create(3, 5, 0, None, ctypes.byref(h)) == _lib.QED_ERR_INVALID_ARG
    assert L.qed_process_create(3, 0, 9, None, ctypes.byref(h)) == _lib.QED_ERR_INVALID_ARG
    assert L.qed_process_create(3, 0, 0, None, None) == _lib.QED_ERR_INVALID_ARG
    assert b"n must be" in L.qed_last_error() or len(L.qed_last_error()) > 0
    v = _lib.QedVariant(0, 0, 100, 0, 0, 0, 0)
    assert L.qed_process_create(3, 0, 0, ctypes.byref(v), ctypes.byref(h)) == _lib.QED_ERR_INVALID_ARG
    v = _lib.QedVariant(1, 0, 0, 0, 0, 0, 0)
    assert L.qed_process_create(3, 1, 0, ctypes.byref(v), ctypes.byref(h)) == _lib.QED_ERR_INVALID_ARG


def test_null_process_and_negative_sizes():
    L = _lib.lib()
    assert L.qed_eval(None, None, None, 0, None, None) == _lib.QED_ERR_INVALID_ARG
    assert L.qed_rambo(None, None, 10.0, 0, None, None) == _lib.QED_ERR_INVALID_ARG
    assert L.qed_eval_grad(None, None, 10.0, None, 0, None, None, None, 0, None) == _lib.QED_ERR_INVALID_ARG
    b = ctypes.c_int64()
    assert L.qed_eval_grad_workspace_size(None, 10, ctypes.byref(b)) == _lib.QED_ERR_INVALID_ARG


def test_compile_failure_is_reported(tmp_path, monkeypatch):
    """A broken compiler flag must surface as QED_ERR_COMPILE with hipcc's message."""
    import subprocess
    import sys
    code = (
        "import ctypes, sys; sys.path.insert(0, %r)\n"
        "from paper_2511_19456_amd import _lib\n"
        "L = _lib.lib(); ms = ctypes.c_double()\n"
        "rc = L.qed_prebuild(1, 1, 0, None, 0, ctypes.byref(ms))\n"
        "print(rc); print(L.qed_last_error().decode()[:200])\n" % ROOT)
    env = dict(os.environ, QEDX_CACHE_DIR=str(tmp_path), QEDX_EXTRA_FLAGS="--this-flag-does-not-exist")
    r = subprocess.run([sys.executable, "-c", code], env=env, capture_output=True, text=True, timeout=300)
    lines = r.stdout.strip().splitlines()
    assert lines[0] == str(_lib.QED_ERR_COMPILE), r.stdout + r.stderr
    assert "hipcc failed" in r.stdout


def test_corrupt_cache_entry_is_rebuilt(tmp_path):
    """A code object whose checksum does not match is recompiled, not loaded."""
    import subprocess
    import sys
    code = (
        "import ctypes, sys, glob; sys.path.insert(0, %r)\n"
        "from paper_2511_19456_amd import _lib\n"
        "L = _lib.lib(); ms = ctypes.c_double()\n"
        "assert L.qed_prebuild(1, 1, 0, None, 0, ctypes.byref(ms)) == 0\n"
        "f = [x for x in glob.glob(%r + '/*.hsaco') if 'aux' not in x][0]\n"
        "open(f, 'r+b').write(b'garbage!')\n"
        "ms2 = ctypes.c_double()\n"
        "assert L.qed_prebuild(1, 1, 0, None, 0, ctypes.byref(ms2)) == 0\n"
        "print(ms.value > 0, ms2.value > 0)\n" % (ROOT, str(tmp_path)))
    env = dict(os.environ, QEDX_CACHE_DIR=str(tmp_path))
    r = subprocess.run([sys.executable, "-c", code], env=env, capture_output=True, text=True, timeout=300)
    assert r.stdout.strip() == "True True", r.stdout + r.stderr


def test_status_codes_for_crossed_processes_and_the_pipe_probe():
    """Argument checks that run before any device call."""
    L = _lib.lib()
    ms = ctypes.c_double()
    h = ctypes.c_void_p()
    # n_in + n_out <= 7, both >= 1
    assert L.qed_prebuild_crossed(4, 4, 1, 0, None, ctypes.byref(ms)) == _lib.QED_ERR_UNSUPPORTED
    assert L.qed_prebuild_crossed(0, 2, 1, 0, None, ctypes.byref(ms)) == _lib.QED_ERR_UNSUPPORTED
    assert L.qed_process_create_crossed(2, 0, 0, 0, None, ctypes.byref(h)) == _lib.QED_ERR_UNSUPPORTED
    assert L.qed_process_create_crossed(2, 1, 0, 0, None, None) == _lib.QED_ERR_INVALID_ARG
    # a fix-up threshold below 1 is rejected
    v = Q.make_variant(fix_kappa=0.5)
    assert L.qed_prebuild(3, 1, 1, ctypes.byref(v), 0, ctypes.byref(ms)) == _lib.QED_ERR_INVALID_ARG
    # pipe probe: kind, sizes, iteration counts and buffers are checked first
    P = _lib.probe_lib()
    assert P.qed_pipe_probe(3, 1, 8, 0, 1.0, 0.0, None, None, None, None, None) == _lib.QED_ERR_INVALID_ARG
    assert P.qed_pipe_probe(0, 0, 8, 0, 1.0, 0.0, None, None, None, None, None) == _lib.QED_ERR_INVALID_ARG
    assert P.qed_pipe_probe(1, 1, 7, 0, 1.0, 0.0, None, None, None, None, None) == _lib.QED_ERR_INVALID_ARG
    assert P.qed_pipe_probe(0, 1, 8, 0, 1.0, 0.0, None, None, None, None, None) == _lib.QED_ERR_INVALID_ARG


def test_fp32c_per_point_source_has_the_fp64_pass():
    src = Q.emit_source(4, "per_point", "fp32c")
    assert "_fix(" in src and "_b64(" in src and "fix_kappa" in src and "__ballot" in src
    off = Q.emit_source(4, "per_point", "fp32c", Q.make_variant(fixup=-1))
    assert "_fix(" not in off and "fix_kappa" not in off
    assert "_fix(" not in Q.emit_source(4, "per_point", "fp64")


def test_default_kernel_shapes():
    """The measured default shapes (helicity coverage, schedule, join split,
    fix-up) that the bench and the documentation rely on."""
    def tag(n, mode, prec, **kw):
        src = Q.emit_source(n, mode, prec, Q.make_variant(**kw) if kw else None)
        return src.splitlines()[0].split("generated by qedx: ")[1]
    # 4 photons, FP64 sum: e-_out spin on lanes, one block per partition
    # (the two lanes share the e-_in side, order flag 2048, and its one-photon
    # currents are cached in LDS, 4096)
    assert tag(3, "sum", "fp64") == "nin1_nout3_p0_m0_e59_l4_o0_b256_s2_j1_r6148_w0"
    # FP32C and the distributive rewrite keep both spins on lanes, shared block
    assert "_l5_o0_" in tag(3, "sum", "fp32c") and "_r0_" in tag(3, "sum", "fp32c")
    assert "_l5_o0_" in tag(3, "sum", "fp64", rewrite=1)
    # an explicit coverage keeps the shared block unless an order is given
    assert "_l7_o0_" in tag(3, "sum", "fp64", lane_bits=7) and "_r0_" in tag(3, "sum", "fp64", lane_bits=7)
    # 5 photons, FP64 sum: e-_in spin and 3 photons in the graph, 2 looped
    assert tag(4, "sum", "fp64") == "nin1_nout4_p0_m0_e27_l4_o96_b256_s2_j1_r10244_w0"
    # per point: join split ceil(P/2) for 5 and 7 photons, slot loop with the
    # one-photon current cache (2 lanes and the e-_in side at 5 photons, 4
    # lanes and both sides at 6 and 7; FP64 and FP32C alike)
    assert tag(4, "per_point", "fp64") == "nin1_nout4_p0_m1_e0_l0_o0_b256_s3_j1_r1288_w2"
    assert tag(5, "per_point", "fp64") == "nin1_nout5_p0_m1_e0_l0_o0_b256_s3_j1_r520_w2"
    assert tag(6, "per_point", "fp64") == "nin1_nout6_p0_m1_e0_l0_o0_b256_s4_j1_r520_w0"
    assert tag(5, "per_point", "fp32c") == "nin1_nout5_p1_m1_e0_l0_o0_b256_s3_j1_r520_w0_f1"
    assert tag(4, "per_point", "fp32c") == "nin1_nout4_p1_m1_e0_l0_o0_b256_s3_j1_r1288_w2_f1"
    assert "_r8_" in tag(4, "per_point", "fp64", rewrite=0, order=8)
    # FP32C per point carries the FP64 pass
    assert tag(5, "per_point", "fp32c").endswith("_f1")
    assert not tag(5, "per_point", "fp32c", fixup=-1).endswith("_f1")
