"""Kinetic compressive sensing (direct parametric PET) on MI355X: HIP library + Python binding.

``kcs`` holds the thin binding of the C ABI in include/kcs.h; ``inputs`` generates seeded
synthetic studies.  The arithmetic of the method runs only in libkcs.so.
"""
