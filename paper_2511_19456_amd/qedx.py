"""Python binding of the qedx library (torch tensors in, torch tensors out).

PyTorch provides device memory and the current HIP stream; every step of the
matrix-element computation runs in the native library's generated kernels.
There is no CPU fallback: without a GPU or without the built library these
functions raise.
"""
from __future__ import annotations

import ctypes
from typing import Optional, Sequence

import torch

from . import _lib
from ._lib import QedInfo, QedSegment, QedVariant, check, lib

_MODES = {"sum": _lib.HEL_SUM, "per_point": _lib.HEL_PER_POINT}
_PRECS = {"fp64": _lib.FP64, "fp32c": _lib.FP32C}


def _stream() -> ctypes.c_void_p:
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


def _ptr(t: Optional[torch.Tensor]) -> ctypes.c_void_p:
    return ctypes.c_void_p(0 if t is None else t.data_ptr())


def _need_gpu() -> None:
    if not torch.cuda.is_available():
        raise RuntimeError("qedx kernels need a ROCm GPU (gfx950); none is visible")


def _dev_tensor(t: torch.Tensor, dtype: torch.dtype, rows: int, name: str) -> torch.Tensor:
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise TypeError(f"{name} must be a GPU tensor")
    if t.dtype != dtype:
        raise TypeError(f"{name} must be {dtype}")
    if t.dim() != 2 or t.shape[0] != rows:
        raise ValueError(f"{name} must have shape [{rows}, N], got {tuple(t.shape)}")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    return t


def make_variant(lane_bits: int = 0, loop_bits: int = 0, block: int = 0, split: int = 0,
                 min_waves: int = 0, order: int = 0, rewrite: int = 0,
                 partial_steps: Optional[int] = None, partial_seed: int = 0,
                 fixup: int = 0, fix_kappa: float = 0.0) -> QedVariant:
    """Kernel shape (fields of qed_variant); rewrite=1 adds the distributive
    rewrite after node reduction; partial_steps=k builds the paper's unsplit
    graph after only k single node reductions (seeded random order);
    fixup=-1 turns off the FP64 pass of FP32C per-point kernels, fix_kappa sets
    its cancellation threshold.  Zero fields take the library default."""
    part = partial_steps is not None
    return QedVariant(lane_bits, loop_bits, block, split, min_waves, order, 0, rewrite, int(part),
                      int(partial_steps or 0), int(partial_seed), int(fixup), float(fix_kappa))


class QedProcess:
    """e- gamma -> e- n gamma at tree level, one compiled kernel variant.

    mode: 'sum' (all 2^(n+3) spin/polarisation configurations) or 'per_point'
    (one configuration per point from a uint32 code).  precision: 'fp64' or
    'fp32c' (FP32 currents with compensated diagram sum, FP64 kinematics).
    n_in > 1 gives the crossed process e- gamma^n_in -> e- gamma^n (Table I
    uses n = 1): particle order [e-_in, gamma_in..., e-_out, gamma_out...],
    eval only (no RAMBO, no gradient, no batches).
    """

    def __init__(self, n: int, mode: str = "sum", precision: str = "fp64",
                 variant: Optional[QedVariant] = None, n_in: int = 1):
        _need_gpu()
        L = lib()
        self.n = int(n)
        self.n_in = int(n_in)
        self.mode = mode
        self.precision = precision
        self.n_particles = self.n + self.n_in + 2
        h = ctypes.c_void_p()
        vp = ctypes.byref(variant) if variant is not None else None
        torch.cuda.current_device()
        if self.n_in == 1:
            check(L.qed_process_create(self.n, _MODES[mode], _PRECS[precision], vp, ctypes.byref(h)))
        else:
            check(L.qed_process_create_crossed(self.n_in, self.n, _MODES[mode], _PRECS[precision], vp,
                                               ctypes.byref(h)))
        self._h = h

    def __del__(self):
        h = getattr(self, "_h", None)
        if h is not None and h.value:
            try:
                lib().qed_process_destroy(h)
            except Exception:
                pass
            self._h = None

    @property
    def handle(self) -> ctypes.c_void_p:
        return self._h

    def info(self) -> dict:
        inf = QedInfo()
        check(lib().qed_process_info(self._h, ctypes.byref(inf)))
        d = {k: getattr(inf, k) for k, _ in QedInfo._fields_}
        d["kernel_tag"] = inf.kernel_tag.decode()
        d["code_hash"] = inf.code_hash.decode()
        d["kernel_name"] = inf.kernel_name.decode()
        return d

    def eval(self, momenta: torch.Tensor, hel: Optional[torch.Tensor] = None,
             out: Optional[torch.Tensor] = None) -> torch.Tensor:
        """|M|^2 for SoA momenta [4(n+n_in+2), N] (float64, device) -> [N] float64."""
        _dev_tensor(momenta, torch.float64, 4 * self.n_particles, "momenta")
        N = momenta.shape[1]
        if hel is not None:
            if hel.dtype not in (torch.int32, torch.uint32) or not hel.is_cuda or hel.shape != (N,):
                raise ValueError("hel must be a device int32/uint32 tensor of shape [N]")
            hel = hel.contiguous()
        if out is None:
            out = torch.empty(N, dtype=torch.float64, device=momenta.device)
        elif out.shape != (N,) or out.dtype != torch.float64 or not out.is_cuda or not out.is_contiguous():
            raise ValueError("out must be a contiguous float64 device tensor of shape [N]")
        check(lib().qed_eval(self._h, _ptr(momenta), _ptr(hel), N, _ptr(out), _stream()))
        return out

    def rambo(self, uniforms: torch.Tensor, sqrt_s: float, out: Optional[torch.Tensor] = None) -> torch.Tensor:
        """RAMBO momenta [4(n+3), N] from uniforms [4(n+1), N] at sqrt(s)."""
        _dev_tensor(uniforms, torch.float64, 4 * (self.n + 1), "uniforms")
        N = uniforms.shape[1]
        if out is None:
            out = torch.empty(4 * self.n_particles, N, dtype=torch.float64, device=uniforms.device)
        check(lib().qed_rambo(self._h, _ptr(uniforms), float(sqrt_s), N, _ptr(out), _stream()))
        return out

    def grad_workspace_bytes(self, N: int) -> int:
        """Device workspace qed_eval_grad uses for N points in one chunk."""
        b = ctypes.c_int64()
        check(lib().qed_eval_grad_workspace_size(self._h, int(N), ctypes.byref(b)))
        return b.value

    def eval_grad(self, uniforms: torch.Tensor, sqrt_s: float, out: Optional[tuple] = None,
                  workspace: Optional[torch.Tensor] = None):
        """(log|M|^2 [N], d log|M|^2 / d uniforms [4(n+1), N]) through RAMBO.
        `out` = (val, grad) preallocated device tensors, or None.  `workspace`
        is a uint8 device tensor for the split gradient (n = 4); by default
        one chunk's worth is taken from torch's allocator on the current
        stream."""
        _dev_tensor(uniforms, torch.float64, 4 * (self.n + 1), "uniforms")
        N = uniforms.shape[1]
        if out is None:
            val = torch.empty(N, dtype=torch.float64, device=uniforms.device)
            grad = torch.empty(4 * (self.n + 1), N, dtype=torch.float64, device=uniforms.device)
        else:
            val, grad = out
            _dev_tensor(grad, torch.float64, 4 * (self.n + 1), "grad")
            if val.shape != (N,) or val.dtype != torch.float64 or not val.is_cuda or not val.is_contiguous() \
                    or grad.shape[1] != N:
                raise ValueError("out must be (float64 [N], float64 [4(n+1), N]) contiguous device tensors")
        if workspace is None:
            nb = self.grad_workspace_bytes(N)
            workspace = torch.empty(nb, dtype=torch.uint8, device=uniforms.device) if nb else None
        elif workspace.dtype != torch.uint8 or not workspace.is_cuda or not workspace.is_contiguous():
            raise ValueError("workspace must be a contiguous uint8 device tensor")
        nbytes = 0 if workspace is None else workspace.numel()
        check(lib().qed_eval_grad(self._h, _ptr(uniforms), float(sqrt_s), None, N, _ptr(val), _ptr(grad),
                                  _ptr(workspace), nbytes, _stream()))
        return val, grad

    def eval_grad_noalloc(self, uniforms: torch.Tensor, sqrt_s: float, out: tuple):
        """eval_grad through qed_eval_grad_noalloc: the library's fixed
        per-device scratch instead of a workspace; `out` = (val [N],
        grad [4(n+1), N]) preallocated float64 device tensors.  Calls that
        overlap on one GPU share the scratch and must be serialised."""
        _dev_tensor(uniforms, torch.float64, 4 * (self.n + 1), "uniforms")
        N = uniforms.shape[1]
        val, grad = out
        _dev_tensor(grad, torch.float64, 4 * (self.n + 1), "grad")
        if val.shape != (N,) or val.dtype != torch.float64 or not val.is_cuda or not val.is_contiguous() \
                or grad.shape[1] != N:
            raise ValueError("out must be (float64 [N], float64 [4(n+1), N]) contiguous device tensors")
        check(lib().qed_eval_grad_noalloc(self._h, _ptr(uniforms), float(sqrt_s), None, N, _ptr(val), _ptr(grad),
                                          _stream()))
        return val, grad


class QedLogM2(torch.autograd.Function):
    """log|M|^2 (helicity sum) of RAMBO points as a differentiable function of
    the uniforms.  The forward calls qed_eval_grad, which returns log|M|^2 and
    its gradient from one pass of the library's kernels; the gradient is kept
    for the backward, which only scales it by grad_output."""

    @staticmethod
    def forward(ctx, uniforms: torch.Tensor, proc: QedProcess, sqrt_s: float):
        val, g = proc.eval_grad(uniforms.contiguous(), sqrt_s)
        ctx.save_for_backward(g)
        return val

    @staticmethod
    def backward(ctx, grad_out: torch.Tensor):
        (g,) = ctx.saved_tensors
        return g * grad_out[None, :], None, None


class BatchPlan:
    """Mixed-process batch: one persistent launch over several segments."""

    def __init__(self, segments: Sequence[tuple], tile_points: int = 0):
        _need_gpu()
        arr = (QedSegment * len(segments))()
        self._keep = []
        for i, (proc, mom, hel, out) in enumerate(segments):
            N = mom.shape[1]
            _dev_tensor(mom, torch.float64, 4 * proc.n_particles, "momenta")
            arr[i] = QedSegment(proc.handle.value, mom.data_ptr(), 0 if hel is None else hel.data_ptr(), N,
                                out.data_ptr())
            self._keep.append((proc, mom, hel, out))
        h = ctypes.c_void_p()
        check(lib().qed_batch_plan_create(arr, len(segments), int(tile_points), ctypes.byref(h)))
        self._h = h

    def launch(self) -> None:
        check(lib().qed_batch_launch(self._h, _stream()))

    def info(self) -> dict:
        t, g, c = ctypes.c_int64(), ctypes.c_int(), ctypes.c_int()
        check(lib().qed_batch_info(self._h, ctypes.byref(t), ctypes.byref(g), ctypes.byref(c)))
        return {"tiles": t.value, "grid": g.value, "chunk": c.value}

    def __del__(self):
        h = getattr(self, "_h", None)
        if h is not None and h.value:
            try:
                lib().qed_batch_plan_destroy(h)
            except Exception:
                pass
            self._h = None


# ---------------------------------------------------------------------------
# host graph tools (no GPU)
# ---------------------------------------------------------------------------
COUNT_KEYS = ("total", "data", "compute", "U", "V", "S1", "S2", "Dot", "Sum", "HelSum")


def graph_counts(n: int, n_in: int = 1, enum_mask: int = 0, split: Optional[int] = None,
                 reduced: bool = False) -> dict:
    split = split if split is not None else (n + n_in) // 2
    c = (ctypes.c_int64 * 10)()
    check(lib().qed_graph_counts(n, n_in, enum_mask, split, int(reduced), c))
    return dict(zip(COUNT_KEYS, list(c)))


def graph_interpret(n: int, mom_points, hel=None, n_in: int = 1, enum_mask: int = 0,
                    split: Optional[int] = None, reduced: bool = True):
    import numpy as np
    split = split if split is not None else (n + n_in) // 2
    m = np.ascontiguousarray(np.asarray(mom_points, dtype=np.float64))
    N = m.shape[0]
    out = np.zeros(N, dtype=np.float64)
    h = None if hel is None else np.ascontiguousarray(np.asarray(hel, dtype=np.uint32))
    check(lib().qed_graph_interpret(n, n_in, enum_mask, split, int(reduced), m.ctypes.data,
                                    None if h is None else h.ctypes.data, N, out.ctypes.data))
    return out


def graph_metrics(n: int, n_in: int = 1, enum_mask: int = 0, split: Optional[int] = None,
                  reduced: bool = True, fp32: bool = False):
    split = split if split is not None else (n + n_in) // 2
    c, d = ctypes.c_double(), ctypes.c_double()
    check(lib().qed_graph_metrics(n, n_in, enum_mask, split, int(reduced), int(fp32), ctypes.byref(c),
                                  ctypes.byref(d)))
    return c.value, d.value


def graph_adjoint_metrics(n: int, enum_mask: int = 0, split: Optional[int] = None, reduced: bool = True):
    """(forward C(DAG), reverse-mode cost) in FLOPs per point for e- gamma -> e- n gamma."""
    split = split if split is not None else (n + 1) // 2
    c, a = ctypes.c_double(), ctypes.c_double()
    check(lib().qed_graph_adjoint_metrics(n, enum_mask, split, int(reduced), ctypes.byref(c), ctypes.byref(a)))
    return c.value, a.value


def reduction_check(n: int, seed: int, n_in: int = 1, enum_mask: int = 0, split: Optional[int] = None):
    split = split if split is not None else (n + n_in) // 2
    size = 1 << 22
    a = ctypes.create_string_buffer(size)
    b = ctypes.create_string_buffer(size)
    steps = ctypes.c_int64()
    check(lib().qed_graph_reduction_check(n, n_in, enum_mask, split, seed, a, b, size, ctypes.byref(steps)))
    return a.value.decode(), b.value.decode(), steps.value


def emit_source(n: int, mode: str = "sum", precision: str = "fp64",
                variant: Optional[QedVariant] = None) -> str:
    ln = ctypes.c_int64()
    vp = ctypes.byref(variant) if variant is not None else None
    check(lib().qed_emit_source(n, _MODES[mode], _PRECS[precision], vp, None, 0, ctypes.byref(ln)))
    buf = ctypes.create_string_buffer(ln.value + 1)
    check(lib().qed_emit_source(n, _MODES[mode], _PRECS[precision], vp, buf, ln.value + 1, ctypes.byref(ln)))
    return buf.value.decode()


def graph_partial(n: int, steps: int, seed: int, mom_points=None, hel=None, split: Optional[int] = None):
    """Counts (and, given points, interpreted |A|^2) of the unreduced graph after
    `steps` single node reductions in the seeded random order."""
    import numpy as np
    split = split if split is not None else (n + 1) // 2
    c = (ctypes.c_int64 * 10)()
    if mom_points is None:
        check(lib().qed_graph_partial(n, split, steps, seed, None, None, 0, None, c))
        return dict(zip(COUNT_KEYS, list(c))), None
    m = np.ascontiguousarray(np.asarray(mom_points, dtype=np.float64))
    N = m.shape[0]
    out = np.zeros(N, dtype=np.float64)
    h = None if hel is None else np.ascontiguousarray(np.asarray(hel, dtype=np.uint32))
    check(lib().qed_graph_partial(n, split, steps, seed, m.ctypes.data, None if h is None else h.ctypes.data, N,
                                  out.ctypes.data, c))
    return dict(zip(COUNT_KEYS, list(c))), out
