"""MI355X-native exact QAOA-for-QUBO statevector engine.

The compute path is a C-ABI shared library of hand-written HIP kernels for
gfx950 (``libqaoa_qubo.so``, declared in ``include/qaoa_qubo.h``).  Importing
this package loads nothing; ``paper_2606_26297_amd.native`` loads the library
and fails loudly when it is missing.
"""
__all__ = ["workloads", "native", "qaoa"]
