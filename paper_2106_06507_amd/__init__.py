"""MI355X (gfx950) n-gluon tree amplitudes with the Berends-Giele recursion.

The computation lives in libbg.so (HIP kernels behind the C ABI of
include/bg.h); ``api`` marshals torch tensors into it.  Nothing here falls back
to a CPU implementation.
"""
__all__ = ["api", "build", "workmodel"]
