"""MI355X (gfx950) library for the data-parallel hot path of the monolithic
FE^2 scheme (arXiv:2312.12771).

The compute path is the C-ABI shared library ``libfe2.so`` (include/fe2.h)
built from csrc/ by ``build.py``; ``paper_2312_12771_amd.fe2`` is its thin
ctypes binding.  Importing ``fe2`` raises ImportError when the library has
not been built.
"""
__all__ = ["fe2", "build"]
