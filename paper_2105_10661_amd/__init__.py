"""MI355X-native hierarchical-inverse EMT network solver (gfx950 HIP kernels behind a C ABI).

Submodules are imported explicitly: ``cases`` (seeded inputs, no GPU) and
``hinv`` (the ctypes binding of libhinv.so, which needs the built library).
"""
