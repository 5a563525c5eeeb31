"""MI355X-native SP2 / SP2ACC density-matrix expansion (arXiv:1909.12533).

The hot path lives in ``libsp2dm.so`` (HIP kernels for gfx950 behind the C ABI
of ``include/sp2dm.h``); ``sp2`` is its Python binding and ``autograd`` wraps
the hand-written adjoint as a ``torch.autograd.Function``.
"""
__all__ = ["sp2", "build"]
