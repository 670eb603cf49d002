"""Exact vertex-priority butterfly counting (BFC-VP) on one MI355X GPU.

The counting path is the HIP library ``libbfc.so`` (C ABI in ``include/bfc.h``);
``paper_1812_00283_amd.bfc`` is its ctypes binding.  Importing this package
loads nothing; ``bfc.load()`` raises if the library has not been built.
"""
__all__ = ["bfc"]
