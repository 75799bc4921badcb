"""MI355X (gfx950) hot path of patch-based AMR MHD.

The compute runs in ``libamrx.so`` (host bookkeeping in C++, kernels in HIP);
this package only loads it, allocates its device arenas with PyTorch and
marshals arguments.  Importing the binding raises if the library is missing:
there is no CPU fallback.
"""
from .binding import FP32, FP32_MIXED, FP64, PLAIN, BATCHED, GRAPH, PERSISTENT, CONCURRENT, LAYERED, AmrxError, Hierarchy, load_library

__all__ = ["FP32", "FP32_MIXED", "FP64", "PLAIN", "BATCHED", "GRAPH", "PERSISTENT", "CONCURRENT", "LAYERED", "AmrxError", "Hierarchy", "load_library"]
