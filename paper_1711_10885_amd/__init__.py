"""Matrix-free weighted SIPG discontinuous Galerkin operator on MI355X.

The compute path lives in the HIP library ``libdgmf.so`` (``csrc/``) behind the
C ABI of ``include/dg.h``; ``binding`` marshals arguments to it with ctypes.
Importing this package loads nothing: ``binding.load()`` opens the library and
raises if it has not been built.
"""
