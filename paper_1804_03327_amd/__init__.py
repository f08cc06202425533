"""Direction-optimized BFS (push-pull) as Boolean masked matvec on AMD Instinct MI355X.

The compute path is libdobfs.so: hand-written HIP kernels for gfx950 behind the C ABI of
include/dobfs.h. `dobfs` is its thin ctypes binding; `helpers` adds torch conveniences
(output allocation, bit-vector packing) that do no BFS arithmetic.
"""
from . import dobfs  # noqa: F401
from .dobfs import DobfsError, Graph  # noqa: F401

__all__ = ["dobfs", "DobfsError", "Graph"]
