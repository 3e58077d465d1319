"""MI355X-native exact-exchange (EXX) pair kernel (arXiv:2011.07209).

The compute path is the C-ABI library ``libexx.so`` (hand-written HIP for
gfx950) declared in ``include/exx.h``; ``paper_2011_07209_amd.exx`` is a thin
ctypes binding with the same names.  ``synth`` generates seeded inputs.
Importing the package loads nothing; the binding loads the library on first use
and raises if it is missing.
"""
__all__ = ["synth", "exx"]
