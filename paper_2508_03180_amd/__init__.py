"""MI355X-native renderer of Duplex-GS (arXiv 2508.03180).

The per-frame hot path (cell rasterization, onesweep radix sort of per-cell
(tile, depth) keys, the hybrid weighted-sum compositor with cell-level early
termination) runs in hand-written HIP kernels behind the C ABI declared in
include/duplexgs.h; this package is the Python binding.
"""
from . import scenes  # noqa: F401  (input generators, no renderer arithmetic)

__all__ = ["scenes", "renderer", "_capi"]
