"""Strict label propagation (GVE-LPA, arXiv 2312.08140) on AMD MI355X.

The label-scan sweep runs in hand-written HIP kernels for gfx950 behind the C
ABI declared in ``include/gvelpa.h``; ``paper_2312_08140_amd.abi`` is its thin
ctypes binding.  ``graphgen`` builds seeded synthetic inputs.
"""
__all__ = ["graphgen", "abi"]
