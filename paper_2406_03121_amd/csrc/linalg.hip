// Dense FP64 linear algebra for the SCF step: a tiled GEMM, a one-workgroup
// cyclic Jacobi eigensolver (used once per geometry for the overlap matrix)
// and elementwise helpers.
#include <cmath>

#include "linalg.hpp"

namespace mess {

// ------------------------------------------------------------------ GEMM
//
// One wave per 16 x 16 output tile on the FP64 matrix cores
// (v_mfma_f64_16x16x4), operands read straight from global memory in the
// instruction's lane layout (these products are small and cached: N <=
// ~1000), K unrolled by 16 so that the loads of four steps are in flight
// together; batched block-diagonal products (gemm_blocks) run the same tile
// code over every molecule's blocks.

typedef double lg_double4 __attribute__((ext_vector_type(4)));

// One 16 x 16 tile (rows row0.., columns col0..) of C = alpha op(A) op(B) +
// beta C by one 64-lane wave.  Lane l supplies A(row0 + l % 16, k + l / 16)
// and B(k + l / 16, col0 + l % 16) for each step of 4 in k, and holds
// C(row0 + l / 16 + 4 q, col0 + l % 16) in element q of the accumulator
// (the FP64 instruction's lane layout).
template <bool TA, bool TB>
__device__ __forceinline__ void gemm_tile_mfma(int M, int N, int K, double alpha, const double *__restrict__ A,
                                               int lda, const double *__restrict__ B, int ldb, double beta,
                                               double *__restrict__ C, int ldc, int row0, int col0) {
    const int l = threadIdx.x;
    const int ar = row0 + l % 16, bc = col0 + l % 16, kq = l / 16;
    const bool aon = ar < M, bon = bc < N;
    auto ldA = [&](int k) -> double {
        return (aon && k < K) ? (TA ? A[(int64_t)k * lda + ar] : A[(int64_t)ar * lda + k]) : 0.0;
    };
    auto ldB = [&](int k) -> double {
        return (bon && k < K) ? (TB ? B[(int64_t)bc * ldb + k] : B[(int64_t)k * ldb + bc]) : 0.0;
    };
    // four independent accumulation chains (steps 4 st + 16 i), summed at
    // the end, so consecutive matrix instructions do not wait on each other
    lg_double4 acc[4];
#pragma unroll
    for (int st = 0; st < 4; ++st) acc[st] = {0.0, 0.0, 0.0, 0.0};
    int k0 = 0;
    for (; k0 + 16 <= K; k0 += 16) {
        double a[4], b[4];
#pragma unroll
        for (int st = 0; st < 4; ++st) {
            a[st] = ldA(k0 + 4 * st + kq);
            b[st] = ldB(k0 + 4 * st + kq);
        }
#pragma unroll
        for (int st = 0; st < 4; ++st) acc[st] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[st], b[st], acc[st], 0, 0, 0);
    }
    for (; k0 < K; k0 += 4) acc[0] = __builtin_amdgcn_mfma_f64_16x16x4f64(ldA(k0 + kq), ldB(k0 + kq), acc[0], 0, 0, 0);
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        const int r = row0 + l / 16 + 4 * q, c = col0 + l % 16;
        if (r < M && c < N) {
            double v = alpha * ((acc[0][q] + acc[1][q]) + (acc[2][q] + acc[3][q]));
            if (beta != 0.0) v += beta * C[(int64_t)r * ldc + c];
            C[(int64_t)r * ldc + c] = v;
        }
    }
}

template <bool TA, bool TB>
__global__ void __launch_bounds__(64) k_gemm_mfma(int M, int N, int K, double alpha, const double *__restrict__ A,
                                                  int lda, const double *__restrict__ B, int ldb, double beta,
                                                  double *__restrict__ C, int ldc) {
    gemm_tile_mfma<TA, TB>(M, N, K, alpha, A, lda, B, ldb, beta, C, ldc, blockIdx.y * 16, blockIdx.x * 16);
}

// Batched square products over a packed block-diagonal layout: block m is
// n_m x n_m at offset off[m] in A, B and C; blockIdx.z strides over blocks.
// Each block's product is computed exactly as gemm() computes it (the same
// tile code, so a molecule of a batch gets the same bits as alone).
template <bool TA, bool TB>
__global__ void __launch_bounds__(64) k_gemm_blocks(int nmol, const int64_t *__restrict__ off,
                                                    const int *__restrict__ nb, double alpha,
                                                    const double *__restrict__ A, const double *__restrict__ B,
                                                    double beta, double *__restrict__ C) {
    for (int m = blockIdx.z; m < nmol; m += gridDim.z) {
        const int n = nb[m];
        const int row0 = blockIdx.y * 16, col0 = blockIdx.x * 16;
        if (row0 >= n || col0 >= n) continue;  // uniform over the wave
        const int64_t o = off[m];
        gemm_tile_mfma<TA, TB>(n, n, n, alpha, A + o, n, B + o, n, beta, C + o, n, row0, col0);
    }
}

int gemm(hipStream_t s, bool ta, bool tb, int M, int N, int K, double alpha, const double *A, int lda,
         const double *B, int ldb, double beta, double *C, int ldc) {
    if (M <= 0 || N <= 0) return MESS_OK;
    const dim3 grid((N + 15) / 16, (M + 15) / 16), blk(64);
    if (!ta && !tb)
        hipLaunchKernelGGL((k_gemm_mfma<false, false>), grid, blk, 0, s, M, N, K, alpha, A, lda, B, ldb, beta, C, ldc);
    else if (ta && !tb)
        hipLaunchKernelGGL((k_gemm_mfma<true, false>), grid, blk, 0, s, M, N, K, alpha, A, lda, B, ldb, beta, C, ldc);
    else if (!ta && tb)
        hipLaunchKernelGGL((k_gemm_mfma<false, true>), grid, blk, 0, s, M, N, K, alpha, A, lda, B, ldb, beta, C, ldc);
    else
        hipLaunchKernelGGL((k_gemm_mfma<true, true>), grid, blk, 0, s, M, N, K, alpha, A, lda, B, ldb, beta, C, ldc);
    MESS_LAUNCH_CHECK();
    return MESS_OK;
}

int gemm_blocks(hipStream_t s, bool ta, bool tb, int nmol, int nmax, const int64_t *off, const int *nb,
                double alpha, const double *A, const double *B, double beta, double *C) {
    if (nmol <= 0 || nmax <= 0) return MESS_OK;
    dim3 grid((nmax + 15) / 16, (nmax + 15) / 16, (unsigned)(nmol < 65535 ? nmol : 65535)), blk(64);
    if (!ta && !tb)
        hipLaunchKernelGGL((k_gemm_blocks<false, false>), grid, blk, 0, s, nmol, off, nb, alpha, A, B, beta, C);
    else if (ta && !tb)
        hipLaunchKernelGGL((k_gemm_blocks<true, false>), grid, blk, 0, s, nmol, off, nb, alpha, A, B, beta, C);
    else if (!ta && tb)
        hipLaunchKernelGGL((k_gemm_blocks<false, true>), grid, blk, 0, s, nmol, off, nb, alpha, A, B, beta, C);
    else
        hipLaunchKernelGGL((k_gemm_blocks<true, true>), grid, blk, 0, s, nmol, off, nb, alpha, A, B, beta, C);
    MESS_LAUNCH_CHECK();
    return MESS_OK;
}

__global__ void k_axpby(int64_t n, double a, const double *__restrict__ X, double b, const double *__restrict__ Y,
                        double *__restrict__ out) {
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        out[i] = a * X[i] + (Y ? b * Y[i] : 0.0);
}

int axpby(hipStream_t s, int64_t n, double a, const double *X, double b, const double *Y, double *out) {
    int64_t g = (n + 255) / 256;
    if (g > 4096) g = 4096;
    if (g < 1) g = 1;
    hipLaunchKernelGGL(k_axpby, dim3((unsigned)g), dim3(256), 0, s, n, a, X, b, Y, out);
    MESS_LAUNCH_CHECK();
    return MESS_OK;
}

// ------------------------------------------------------------- Jacobi
//
// Two-sided cyclic Jacobi with the round-robin ("circle") ordering: in each
// of the m-1 rounds of a sweep (m = n rounded up to even) the indices are
// split into m/2 disjoint pairs (p, q); each pair's rotation
//   tau = (a_qq - a_pp) / (2 a_pq), t = sign(tau) / (|tau| + sqrt(1 + tau^2)),
//   c = 1/sqrt(1 + t^2), s = t c
// annihilates a_pq; rows then columns of A, and the columns of V, are
// rotated for all pairs at once.  Sweeps stop when every off-diagonal
// element is below 1e-14 sqrt(|a_pp a_qq|) (or after 20 sweeps).

__global__ void __launch_bounds__(1024) k_jacobi(int n, double *__restrict__ A, double *__restrict__ V,
                                                 double *__restrict__ w) {
    __shared__ double cs[512], sn[512];
    __shared__ int pp[512], qq[512];
    __shared__ double red[1024];
    __shared__ int done;
    const int tid = threadIdx.x;
    const int m = n + (n & 1);
    const int npairs = m / 2;
    for (int idx = tid; idx < n * n; idx += 1024) V[idx] = (idx / n == idx % n) ? 1.0 : 0.0;
    __syncthreads();
    for (int sweep = 0; sweep < 20; ++sweep) {
        // convergence test: every |a_pq| <= 1e-14 sqrt(|a_pp a_qq|)
        double worst = 0.0;
        for (int idx = tid; idx < n * n; idx += 1024) {
            const int i = idx / n, j = idx % n;
            if (i == j) continue;
            const double d = sqrt(fabs(A[(int64_t)i * n + i] * A[(int64_t)j * n + j]));
            const double a = fabs(A[idx]);
            const double ratio = d > 0.0 ? a / d : (a > 0.0 ? 1.0 : 0.0);
            worst = fmax(worst, ratio);
        }
        red[tid] = worst;
        __syncthreads();
        for (int st = 512; st > 0; st >>= 1) {
            if (tid < st) red[tid] = fmax(red[tid], red[tid + st]);
            __syncthreads();
        }
        if (tid == 0) done = red[0] <= 1e-14 ? 1 : 0;
        __syncthreads();
        if (done) break;
        for (int r = 0; r < m - 1; ++r) {
            if (tid < npairs) {
                int p, q;
                if (tid == 0) {
                    p = r;
                    q = m - 1;
                } else {
                    p = (r + tid) % (m - 1);
                    q = (r - tid + (m - 1)) % (m - 1);
                }
                if (p > q) { const int t = p; p = q; q = t; }
                double c = 1.0, s = 0.0;
                if (q < n) {
                    const double apq = A[(int64_t)p * n + q];
                    if (apq != 0.0) {
                        const double app = A[(int64_t)p * n + p], aqq = A[(int64_t)q * n + q];
                        const double tau = (aqq - app) / (2.0 * apq);
                        const double t = (tau >= 0.0 ? 1.0 : -1.0) / (fabs(tau) + sqrt(1.0 + tau * tau));
                        c = 1.0 / sqrt(1.0 + t * t);
                        s = t * c;
                    }
                }
                pp[tid] = p; qq[tid] = q; cs[tid] = c; sn[tid] = s;
            }
            __syncthreads();
            // rows: A <- J^T A
            for (int it = tid; it < npairs * n; it += 1024) {
                const int k = it / n, j = it % n;
                const int p = pp[k], q = qq[k];
                if (q >= n) continue;
                const double c = cs[k], s = sn[k];
                const double ap = A[(int64_t)p * n + j], aq = A[(int64_t)q * n + j];
                A[(int64_t)p * n + j] = c * ap - s * aq;
                A[(int64_t)q * n + j] = s * ap + c * aq;
            }
            __syncthreads();
            // columns: A <- A J, V <- V J
            for (int it = tid; it < 2 * npairs * n; it += 1024) {
                const int which = it / (npairs * n);
                const int rem = it % (npairs * n);
                const int k = rem / n, i = rem % n;
                const int p = pp[k], q = qq[k];
                if (q >= n) continue;
                const double c = cs[k], s = sn[k];
                double *X = which ? V : A;
                const double xp = X[(int64_t)i * n + p], xq = X[(int64_t)i * n + q];
                X[(int64_t)i * n + p] = c * xp - s * xq;
                X[(int64_t)i * n + q] = s * xp + c * xq;
            }
            __syncthreads();
        }
    }
    for (int i = tid; i < n; i += 1024) w[i] = A[(int64_t)i * n + i];
}

// Sort eigenpairs ascending: rank of each eigenvalue (ties by index), then
// gather the columns of V into Vs.
__global__ void __launch_bounds__(1024) k_sort_eig(int n, const double *__restrict__ w, const double *__restrict__ V,
                                                   double *__restrict__ ws, double *__restrict__ Vs) {
    for (int i = threadIdx.x; i < n; i += 1024) {
        const double wi = w[i];
        int r = 0;
        for (int j = 0; j < n; ++j) r += (w[j] < wi) || (w[j] == wi && j < i);
        ws[r] = wi;
        for (int row = 0; row < n; ++row) Vs[(int64_t)row * n + r] = V[(int64_t)row * n + i];
    }
}

int jacobi_eigh(hipStream_t s, int n, double *A, double *w, double *V, double *work) {
    if (n > 1024) {
        set_error("eigensolver: n = %d exceeds the 1024 supported", n);
        return MESS_E_UNSUPPORTED;
    }
    // work: n*n (unsorted vectors) + n (unsorted values)
    double *Vu = work, *wu = work + (int64_t)n * n;
    hipLaunchKernelGGL(k_jacobi, dim3(1), dim3(1024), 0, s, n, A, Vu, wu);
    MESS_LAUNCH_CHECK();
    hipLaunchKernelGGL(k_sort_eig, dim3(1), dim3(1024), 0, s, n, wu, Vu, w, V);
    MESS_LAUNCH_CHECK();
    return MESS_OK;
}

}  // namespace mess
