"""MI355X-native Fourier-Galerkin projected-CG solver for corrosion-driven
fracture in fractal porous media (after Pundir, Kammer, Angst, arXiv 2305.13081).

``fgcg``   thin ctypes binding of the C ABI in include/fgcg.h (libfgcg.so)
``inputs`` seeded synthetic microstructures
``build``  hipcc build of the in-tree library
"""
