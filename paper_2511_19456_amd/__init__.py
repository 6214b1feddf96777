"""qedx: batched tree-level QED |M|^2 for e- gamma -> e- n gamma on MI355X.

The computation graph of all (n+1)! Feynman diagrams is generated, node-reduced
and compiled into straight-line gfx950 kernels by the native library
``libqedx.so`` (C ABI in include/qedx.h).  Importing this package does not load
the library; the first call that needs it does, and fails loudly if it has not
been built.
"""
import importlib

_API = ("QedProcess", "QedLogM2", "BatchPlan", "make_variant", "graph_counts", "graph_interpret",
        "graph_metrics", "reduction_check", "emit_source", "graph_partial")
__all__ = list(_API)


def __getattr__(name):
    if name in _API:
        return getattr(importlib.import_module(".qedx", __name__), name)
    raise AttributeError(name)
