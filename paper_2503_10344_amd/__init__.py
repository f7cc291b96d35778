"""PDLP for LP relaxations on AMD Instinct MI355X (gfx950).

The solver lives in libpdlp.so (HIP kernels behind the C-ABI of include/pdlp.h); `pdlp` is its thin
Python binding and `generators` builds the seeded synthetic workloads. Importing the package does
not load the library; `pdlp.load()` does, and fails loudly if it has not been built.
"""
__all__ = ["pdlp", "generators", "build"]
