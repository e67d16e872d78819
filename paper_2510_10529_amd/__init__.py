"""MI355X (gfx950) inverse-DFT hot path: spectral-FE Kohn-Sham operator, Chebyshev-filtered
subspace iteration, batched projected MINRES adjoint, density-loss gradient.

The compute path is libinvdft.so (HIP, built in-tree by ``build.py``); ``api`` is a thin
ctypes binding over its C ABI (include/invdft.h) and ``inverse`` holds the autograd
Function and the L-BFGS driver. Importing this package does not load the library;
the first call does, and fails loudly if it was not built.
"""
__all__ = ["api", "inverse"]
