"""MI355X-native Newton step of the stabilised P1-P1 hyperelastic solid.

The compute path is the HIP library ``libhfsi.so`` (C ABI in include/hfsi.h)
built from ``csrc/`` by ``build.py``; ``hfsi`` is its ctypes binding.
"""
__all__ = ["hfsi", "build"]
