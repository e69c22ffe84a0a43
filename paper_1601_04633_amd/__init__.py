"""Double-MRT thermal lattice Boltzmann time step (Li, Yang & Zhang,
arXiv:1601.04633) for AMD MI355X (gfx950).

The compute path is ``libdmrt.so`` (hand-written HIP kernels behind a C ABI,
declared in ``include/dmrt.h``).  ``paper_1601_04633_amd.dmrt`` is the thin
ctypes binding with the same names; importing this package does not load the
library, so the seeded input module can be used without a GPU.
"""
__all__ = ["dmrt", "inputs"]
