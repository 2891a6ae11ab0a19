"""MI355X-native SquareSort (arXiv 2407.14801): HIP kernels behind a C ABI.

The compute path is ``libsquaresort.so`` (hand-written HIP for gfx950);
``binding`` is a thin ctypes layer over it.  Nothing here falls back to the
CPU: if the library is missing, importing ``binding`` raises.
"""
__all__ = ["binding", "datagen"]
