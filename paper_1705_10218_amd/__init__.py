"""MI355X-native local block-sparse matrix multiply (arXiv:1705.10218, Section 2).

C = alpha * op(A) * op(B) + beta * C over block-CSR matrices of small dense
FP64 blocks, with on-the-fly and post-multiply norm filtering.  The work runs
in hand-written HIP kernels for gfx950 behind the C ABI declared in
``include/bsmm.h``; ``paper_1705_10218_amd.bsmm`` is the thin ctypes binding.
Importing this package loads nothing; the binding loads ``libbsmm.so`` on
first use and raises if it is missing.
"""
__all__ = ["bsmm", "inputs"]
