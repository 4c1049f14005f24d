// Dense FP64 linear algebra on the device for the SCF step.
#pragma once

#include "mess_internal.hpp"

namespace mess {

// C[M x N] = alpha * op(A) * op(B) + beta * C, row-major; op(A) is M x K
// (A stored K x M when ta), op(B) is K x N (B stored N x K when tb).
int gemm(hipStream_t s, bool ta, bool tb, int M, int N, int K, double alpha, const double *A, int lda,
         const double *B, int ldb, double beta, double *C, int ldc);

// Batched square products on packed block-diagonal matrices: for each
// block m (n_m x n_m at offset off[m], device arrays), C_m = alpha op(A_m)
// op(B_m) + beta C_m.  nmax >= every n_m sizes the grid.
int gemm_blocks(hipStream_t s, bool ta, bool tb, int nmol, int nmax, const int64_t *off, const int *nb,
                double alpha, const double *A, const double *B, double beta, double *C);

// Eigen-decomposition of a symmetric n x n matrix A (device, row-major,
// destroyed): eigenvalues w[n] ascending, eigenvectors as the columns of
// V[n x n] (row-major), by cyclic Jacobi rotations in one workgroup.
int jacobi_eigh(hipStream_t s, int n, double *A, double *w, double *V, double *work);

// out = a*X + b*Y (elementwise, n values).
int axpby(hipStream_t s, int64_t n, double a, const double *X, double b, const double *Y, double *out);

}  // namespace mess
