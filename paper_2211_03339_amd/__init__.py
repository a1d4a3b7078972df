"""MI355X-native mixed-precision preconditioned Jacobi eigensolver (Zhang & Bai,
arXiv 2211.03339): FP32 eigensolve -> FP64 modified Gram-Schmidt -> FP64
Q^T A Q -> FP64 round-robin parallel Jacobi sweeps, plus the one-sided Jacobi
SVD, a batched path and a learned warm start.  The compute runs in the HIP
library ``libjacobi.so`` (C-ABI in ``include/jacobi.h``); ``jacobi`` is its
thin Python binding."""
