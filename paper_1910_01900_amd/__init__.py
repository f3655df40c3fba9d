"""MI355X (gfx950) matrix-free SIPG operator and hybrid multigrid solver.

The compute path is the HIP library libhmg.so (C ABI in include/hmg.h);
`paper_1910_01900_amd.hmg` is its thin ctypes binding, `inputs` holds the
seeded synthetic input generators, `build` compiles the library.
"""
__all__ = ["hmg", "inputs", "build"]
