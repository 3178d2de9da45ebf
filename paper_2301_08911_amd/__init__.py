"""MI355X-native periodic homogenization solver (arXiv 2301.08911 hot path).

The compute path is the gfx950 HIP library ``libhmg.so`` behind the C ABI of
``include/hmg.h``; :mod:`paper_2301_08911_amd.hmg` is its thin ctypes binding.
Importing the package loads nothing; the library is loaded (and must exist)
the first time a :class:`~paper_2301_08911_amd.hmg.Context` is created.
"""

__all__ = ["hmg", "inputs", "build"]
