"""MI355X (gfx950) preconditioned steepest descent solver for periodic
regularised p-Laplacian problems (Feng, Salgado, Wang & Wise, arXiv:1607.01475).

The solver runs in the HIP library ``libpsd.so`` (C ABI in ``include/psd.h``);
``paper_1607_01475_amd.psd`` is the thin Python binding.
"""
__all__ = ["psd"]
