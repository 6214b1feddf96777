"""ctypes declarations of the qedx C ABI (include/qedx.h).

Argument marshalling only: every step of the computation runs in the native
library and its generated HIP kernels.  Loading fails loudly when the library
has not been built.
"""
from __future__ import annotations

import ctypes
import os

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libqedx.so")
PROBE_LIB_PATH = os.path.join(_HERE, "libqedx_probe.so")

c_int, c_int64, c_uint32, c_uint64, c_double, c_void_p, c_char_p = (
    ctypes.c_int, ctypes.c_int64, ctypes.c_uint32, ctypes.c_uint64, ctypes.c_double, ctypes.c_void_p,
    ctypes.c_char_p)

QED_OK, QED_ERR_INVALID_ARG, QED_ERR_UNSUPPORTED, QED_ERR_HIP, QED_ERR_COMPILE, QED_ERR_OOM = range(6)
STATUS_NAMES = {0: "QED_OK", 1: "QED_ERR_INVALID_ARG", 2: "QED_ERR_UNSUPPORTED", 3: "QED_ERR_HIP",
                4: "QED_ERR_COMPILE", 5: "QED_ERR_OOM"}
HEL_SUM, HEL_PER_POINT = 0, 1
FP64, FP32C = 0, 1


class QedVariant(ctypes.Structure):
    _fields_ = [("lane_bits", c_uint32), ("loop_bits", c_uint32), ("block", ctypes.c_int32),
                ("split", ctypes.c_int32), ("min_waves", ctypes.c_int32), ("order", ctypes.c_int32),
                ("use_defaults", ctypes.c_int32), ("rewrite", ctypes.c_int32),
                ("partial", ctypes.c_int32), ("partial_steps", ctypes.c_int32), ("partial_seed", ctypes.c_uint32),
                ("fixup", ctypes.c_int32), ("fix_kappa", ctypes.c_float)]


class QedInfo(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int32), ("mode", ctypes.c_int32), ("precision", ctypes.c_int32),
                ("nodes_unreduced", c_int64), ("nodes_reduced", c_int64),
                ("n_V", c_int64), ("n_S1", c_int64), ("n_dot", c_int64), ("n_prop", c_int64),
                ("flops_per_point", c_double),
                ("lanes_per_point", ctypes.c_int32), ("block", ctypes.c_int32),
                ("vgpr", ctypes.c_int32), ("agpr", ctypes.c_int32), ("sgpr", ctypes.c_int32),
                ("scratch_bytes", ctypes.c_int32), ("lds_bytes", ctypes.c_int32),
                ("create_ms_build", c_double), ("create_ms_reduce", c_double), ("create_ms_emit", c_double),
                ("create_ms_compile", c_double), ("create_ms_load", c_double),
                ("cache_hit", ctypes.c_int32), ("kernel_tag", ctypes.c_char * 160),
                ("code_hash", ctypes.c_char * 24), ("kernel_name", ctypes.c_char * 48), ("n_in", ctypes.c_int32),
                ("fixup", ctypes.c_int32), ("fix_kappa", ctypes.c_double)]


class QedSegment(ctypes.Structure):
    _fields_ = [("proc", c_void_p), ("momenta", c_void_p), ("hel", c_void_p), ("N", c_int64), ("out", c_void_p)]


# exported symbol -> (restype, argtypes); the header declares every one
SIGNATURES = {
    "qed_process_create": (c_int, [c_int, c_int, c_int, ctypes.POINTER(QedVariant), ctypes.POINTER(c_void_p)]),
    "qed_process_create_crossed": (c_int, [c_int, c_int, c_int, c_int, ctypes.POINTER(QedVariant),
                                           ctypes.POINTER(c_void_p)]),
    "qed_process_destroy": (c_int, [c_void_p]),
    "qed_process_info": (c_int, [c_void_p, ctypes.POINTER(QedInfo)]),
    "qed_eval": (c_int, [c_void_p, c_void_p, c_void_p, c_int64, c_void_p, c_void_p]),
    "qed_rambo": (c_int, [c_void_p, c_void_p, c_double, c_int64, c_void_p, c_void_p]),
    "qed_eval_grad": (c_int, [c_void_p, c_void_p, c_double, c_void_p, c_int64, c_void_p, c_void_p, c_void_p,
                              c_int64, c_void_p]),
    "qed_eval_grad_workspace_size": (c_int, [c_void_p, c_int64, ctypes.POINTER(c_int64)]),
    "qed_eval_grad_noalloc": (c_int, [c_void_p, c_void_p, c_double, c_void_p, c_int64, c_void_p, c_void_p,
                                      c_void_p]),
    "qed_batch_plan_create": (c_int, [ctypes.POINTER(QedSegment), c_int, c_int, ctypes.POINTER(c_void_p)]),
    "qed_batch_launch": (c_int, [c_void_p, c_void_p]),
    "qed_batch_plan_destroy": (c_int, [c_void_p]),
    "qed_batch_info": (c_int, [c_void_p, ctypes.POINTER(c_int64), ctypes.POINTER(c_int), ctypes.POINTER(c_int)]),
    "qed_batch_prebuild": (c_int, [ctypes.POINTER(c_int), c_int, c_int, c_int, ctypes.POINTER(c_double)]),
    "qed_last_error": (c_char_p, []),
    "qed_cache_dir": (c_char_p, []),
    "qed_graph_counts": (c_int, [c_int, c_int, c_uint32, c_int, c_int, ctypes.POINTER(c_int64)]),
    "qed_graph_interpret": (c_int, [c_int, c_int, c_uint32, c_int, c_int, c_void_p, c_void_p, c_int64,
                                    c_void_p]),
    "qed_graph_reduction_check": (c_int, [c_int, c_int, c_uint32, c_int, c_uint64, c_char_p, c_char_p,
                                          c_int64, ctypes.POINTER(c_int64)]),
    "qed_emit_source": (c_int, [c_int, c_int, c_int, ctypes.POINTER(QedVariant), c_char_p, c_int64,
                                ctypes.POINTER(c_int64)]),
    "qed_prebuild": (c_int, [c_int, c_int, c_int, ctypes.POINTER(QedVariant), c_int,
                             ctypes.POINTER(c_double)]),
    "qed_prebuild_crossed": (c_int, [c_int, c_int, c_int, c_int, ctypes.POINTER(QedVariant),
                                     ctypes.POINTER(c_double)]),
    "qed_graph_grad_interpret": (c_int, [c_int, c_int, c_int, c_void_p, c_int64, c_void_p, c_void_p]),
    "qed_rambo_vjp_host": (c_int, [c_int, c_void_p, c_double, c_void_p, c_int64, c_void_p, c_void_p]),
    "qed_graph_partial": (c_int, [c_int, c_int, c_int64, ctypes.c_uint64, c_void_p, c_void_p, c_int64, c_void_p,
                                  ctypes.POINTER(c_int64)]),
    "qed_graph_metrics": (c_int, [c_int, c_int, c_uint32, c_int, c_int, c_int, ctypes.POINTER(c_double),
                                  ctypes.POINTER(c_double)]),
    "qed_graph_adjoint_metrics": (c_int, [c_int, c_uint32, c_int, c_int, ctypes.POINTER(c_double),
                                          ctypes.POINTER(c_double)]),
}

# the measurement library (include/qedx_probe.h)
PROBE_SIGNATURES = {
    "qed_pipe_probe": (c_int, [c_int, c_int64, c_int64, c_int64, c_double, c_double, c_void_p, c_void_p,
                               c_void_p, c_void_p, c_void_p]),
    "qed_pipe_probe_prebuild": (c_int, [ctypes.POINTER(c_double)]),
    "qed_recip_probe": (c_int, [c_void_p, c_int64, c_void_p, c_void_p, c_void_p]),
}

_lib = None
_probe = None


class QedError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"{STATUS_NAMES.get(status, status)}: {msg}")
        self.status = status


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"qedx native library not found at {LIB_PATH}; build it with "
                               "`python -c 'import __graft_entry__ as g; g.build()'`")
        L = ctypes.CDLL(LIB_PATH)
        for name, (res, args) in SIGNATURES.items():
            fn = getattr(L, name)
            fn.restype = res
            fn.argtypes = args
        _lib = L
    return _lib


def probe_lib():
    """libqedx_probe.so (FP64 pipe probe, reciprocal probe); it reports errors through libqedx.s
    qed_last_error."""
    global _probe
    if _probe is None:
        lib()
        if not os.path.exists(PROBE_LIB_PATH):
            raise RuntimeError(f"qedx probe library not found at {PROBE_LIB_PATH}; run build()")
        L = ctypes.CDLL(PROBE_LIB_PATH)
        for name, (res, args) in PROBE_SIGNATURES.items():
            fn = getattr(L, name)
            fn.restype = res
            fn.argtypes = args
        _probe = L
    return _probe


def check(status: int) -> None:
    if status != QED_OK:
        raise QedError(status, lib().qed_last_error().decode(errors="replace"))
