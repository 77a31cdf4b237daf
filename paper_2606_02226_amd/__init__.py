"""MI355X-native chaos game of composable function systems (CFS).

The hot path (random streams, selection, maps, composed transforms, splats,
adjoint, batched scheduling) runs in the HIP kernels of ``libcfs.so``, whose
C ABI is ``include/cfs.h``.  ``api`` marshals torch tensors into that ABI;
``autograd`` wraps the differentiable splat.  Importing this package loads
nothing; the library is loaded on first use and must have been built in-tree.
"""
__all__ = ["api"]
