"""MI355X-native Pi_MatMul: the ciphertext x plaintext linear-layer protocol of
Liu & Liu, arXiv 2305.18396 (Algorithm 1), as HIP kernels for gfx950 behind a
C-ABI library (``libpimm.so``) with a thin ctypes binding (``pimm``).

Submodules are imported on demand so that the seeded input generators
(``workloads``) stay usable on machines without the built library.
"""
__all__ = ["pimm", "workloads"]
