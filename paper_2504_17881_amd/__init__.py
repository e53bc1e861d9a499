"""Pauli-rotation state-vector engine for AMD MI355X (gfx950).

The product is ``lib/libprx.so`` (C ABI declared in ``include/prx.h``): HIP
kernels that apply sequences of Pauli rotations exp(i phi P) to a 2^n complex
state in HBM, the host planner that segments a schedule into HBM passes, the
product-formula schedule builders, and FP64 overlap reductions.
``paper_2504_17881_amd.prx`` is its ctypes binding with the same names.
"""
__all__ = ["prx"]
