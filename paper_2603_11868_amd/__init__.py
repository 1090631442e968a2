"""MI355X (gfx950) WCSPH hot path: cell-linked-list neighbour search and the
SPH pair sweeps as HIP kernels behind the C ABI of include/sph.h.

``paper_2603_11868_amd.sph`` is the ctypes binding (same names as the C ABI)
plus ``Simulation``, which allocates torch device buffers for a workload.
"""
from . import sph  # noqa: F401

__all__ = ["sph"]
