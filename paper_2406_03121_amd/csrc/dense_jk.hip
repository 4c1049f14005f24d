// J and K of many densities from a dense ERI tensor (section 3: the Coulomb
// and exchange matrices are contractions of the repulsion integrals with the
// density), as matrix products over the composite indices r = (i, j),
// c = (k, l) of the N^2 x N^2 views of the tensor:
//   J[d][r] = sum_c (ij|kl) D_d[c],     K[d][r] = sum_c (ik|jl) D_d[c],
// so that with many densities the contraction is a dense product whose
// arithmetic intensity grows with the density count.  Two forms of the same
// tiling: 256-thread blocks own 64 rows x 64 densities (each tensor element
// staged once serves 64 densities); per step of 16 columns the block stages
// the 64 x 16 tensor panel and the 16 x 64 density panel in LDS (coalesced
// loads: the tensor rows are contiguous in l), then
//   - MFMA: each wave issues 4 x 4 v_mfma 16x16x4 products (FP64 or FP32
//     operands, accumulation in the operand precision) on its 16 rows and
//     the four 16-density column tiles;
//   - VALU: each lane accumulates 16 densities of one row with FMAs.
// The column range is split over blockIdx.z when the row and density tiles
// alone leave the chip's 256 CUs underfilled (a 105-function tensor has
// 173 row tiles); split parts add into the zeroed output with FP64/FP32
// atomics.  The two forms are compared by rocprof on the same inputs.
#include <algorithm>

#include "mess_internal.hpp"

namespace mess {

constexpr int kDjRows = 64, kDjDens = 64, kDjK = 32;

typedef double dj_double4 __attribute__((ext_vector_type(4)));
typedef float dj_float4 __attribute__((ext_vector_type(4)));

template <typename Real> struct DjVec;
template <> struct DjVec<double> { using type = dj_double4; };
template <> struct DjVec<float> { using type = dj_float4; };

template <typename Real>
__device__ __forceinline__ typename DjVec<Real>::type dj_mfma(Real a, Real b, typename DjVec<Real>::type c) {
    if constexpr (sizeof(Real) == 8)
        return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
    else
        return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
}

// KMODE 0: A(r, c) = eri[r M + c] (J); 1: A((i,j), (k,l)) = eri[((i N + k) N + j) N + l] (K)
template <typename Real, int KMODE, bool MFMA>
__global__ void __launch_bounds__(256) k_dense_jk(int N, int nd, int64_t chunk, const Real *__restrict__ eri,
                                                  const Real *__restrict__ D, Real *__restrict__ out) {
    __shared__ Real As[kDjRows][kDjK + 1];
    __shared__ Real Bs[kDjK][kDjDens + 1];
    const int64_t M = (int64_t)N * N;
    const int64_t r0 = (int64_t)blockIdx.x * kDjRows;
    const int d0 = blockIdx.y * kDjDens;
    const int t = threadIdx.x, w = t / 64, l = t % 64;
    typename DjVec<Real>::type acc[4];
#pragma unroll
    for (int ct = 0; ct < 4; ++ct) acc[ct] = {0, 0, 0, 0};
    Real vacc[16];
#pragma unroll
    for (int j = 0; j < 16; ++j) vacc[j] = 0;
    const int64_t cb = (int64_t)blockIdx.z * chunk, ce = cb + chunk < M ? cb + chunk : M;
    const bool split = gridDim.z > 1;
    for (int64_t c0 = cb; c0 < ce; c0 += kDjK) {
        // tensor panel: 64 rows x 16 columns, four elements per thread
        for (int e = t; e < kDjRows * kDjK; e += 256) {
            const int rr = e / kDjK, cc = e % kDjK;
            const int64_t r = r0 + rr, c = c0 + cc;
            Real v = 0;
            if (r < M && c < ce) {
                if (KMODE == 0) {
                    v = eri[r * M + c];
                } else {
                    const int64_t i = r / N, j = r % N, k = c / N, ll = c % N;
                    v = eri[((i * N + k) * N + j) * N + ll];
                }
            }
            As[rr][cc] = v;
        }
        // density panel: 16 columns x 64 densities, four elements per thread
        for (int e = t; e < kDjK * kDjDens; e += 256) {
            const int cc = e % kDjK, dd = e / kDjK;
            const int64_t c = c0 + cc;
            Bs[cc][dd] = (c < ce && d0 + dd < nd) ? D[(int64_t)(d0 + dd) * M + c] : Real(0);
        }
        __syncthreads();
        if constexpr (MFMA) {
            // A operand: row l % 16 of this wave's rows, column 4 s + l / 16;
            // B operand: row 4 s + l / 16, density 16 ct + l % 16
#pragma unroll
            for (int s = 0; s < kDjK / 4; ++s) {
                const Real a = As[16 * w + l % 16][4 * s + l / 16];
#pragma unroll
                for (int ct = 0; ct < 4; ++ct) acc[ct] = dj_mfma<Real>(a, Bs[4 * s + l / 16][16 * ct + l % 16], acc[ct]);
            }
        } else {
#pragma unroll
            for (int kk = 0; kk < kDjK; ++kk) {
                const Real a = As[16 * w + l % 16][kk];
#pragma unroll
                for (int j = 0; j < 16; ++j) vacc[j] = fma(a, Bs[kk][16 * (l / 16) + j], vacc[j]);
            }
        }
        __syncthreads();
    }
    if constexpr (MFMA) {
        // result element q of lane l: density 16 ct + l % 16 and, of the
        // wave's 16 rows, row 4 (l / 16) + q for the FP32 product but
        // row l / 16 + 4 q for the FP64 one (measured lane layouts)
#pragma unroll
        for (int ct = 0; ct < 4; ++ct)
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                const int rw = sizeof(Real) == 8 ? l / 16 + 4 * q : 4 * (l / 16) + q;
                const int64_t r = r0 + 16 * w + rw;
                const int d = d0 + 16 * ct + l % 16;
                if (r < M && d < nd) {
                    if (split) unsafeAtomicAdd(&out[(int64_t)d * M + r], acc[ct][q]);
                    else out[(int64_t)d * M + r] = acc[ct][q];
                }
            }
    } else {
#pragma unroll
        for (int j = 0; j < 16; ++j) {
            const int64_t r = r0 + 16 * w + l % 16;
            const int d = d0 + 16 * (l / 16) + j;
            if (r < M && d < nd) {
                if (split) unsafeAtomicAdd(&out[(int64_t)d * M + r], vacc[j]);
                else out[(int64_t)d * M + r] = vacc[j];
            }
        }
    }
}

template <typename Real>
__global__ void k_dj_zero(int64_t n, Real *__restrict__ p) {
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        p[i] = Real(0);
}

template <typename Real, bool MFMA>
static void launch_dense(int N, int nd, const Real *eri, const Real *D, Real *J, Real *K, hipStream_t s) {
    const int64_t M = (int64_t)N * N;
    const unsigned gx = (unsigned)((M + kDjRows - 1) / kDjRows), gy = (unsigned)((nd + kDjDens - 1) / kDjDens);
    // split the columns until about 2048 blocks (8 per CU), in chunks of at
    // least 64 staging steps
    int64_t nz = 2048 / std::max<int64_t>(1, (int64_t)gx * gy);
    nz = std::max<int64_t>(1, std::min<int64_t>(nz, M / (64 * kDjK)));
    const int64_t chunk = ((M + nz - 1) / nz + kDjK - 1) / kDjK * kDjK;
    nz = (M + chunk - 1) / chunk;
    const dim3 grid(gx, gy, (unsigned)nz);
    const int64_t nout = (int64_t)nd * M;
    const unsigned zb = (unsigned)std::min<int64_t>((nout + 255) / 256, 65536);
    if (J) {
        if (nz > 1) hipLaunchKernelGGL(k_dj_zero<Real>, dim3(zb), dim3(256), 0, s, nout, J);
        hipLaunchKernelGGL((k_dense_jk<Real, 0, MFMA>), grid, dim3(256), 0, s, N, nd, chunk, eri, D, J);
    }
    if (K) {
        if (nz > 1) hipLaunchKernelGGL(k_dj_zero<Real>, dim3(zb), dim3(256), 0, s, nout, K);
        hipLaunchKernelGGL((k_dense_jk<Real, 1, MFMA>), grid, dim3(256), 0, s, N, nd, chunk, eri, D, K);
    }
}

}  // namespace mess

using namespace mess;

extern "C" int mess_jk_dense(const void *eri, int32_t n, int32_t ndens, const void *D, void *J, void *K,
                             int32_t prec, int32_t form, mess_stream stream) {
    if (!eri || !D || n < 1 || ndens < 1) {
        set_error("mess_jk_dense: need eri, D, n >= 1 and ndens >= 1");
        return MESS_E_ARG;
    }
    if ((prec != MESS_FP64 && prec != MESS_FP32) || (form != MESS_DENSE_VALU && form != MESS_DENSE_MFMA)) {
        set_error("mess_jk_dense: prec must be MESS_FP64 or MESS_FP32, form MESS_DENSE_VALU or MESS_DENSE_MFMA");
        return MESS_E_ARG;
    }
    if ((int64_t)n * n > ((int64_t)1 << 31) / 2 || ndens > 65535 * kDjDens) {
        set_error("mess_jk_dense: n or ndens out of range");
        return MESS_E_ARG;
    }
    if (!J && !K) return MESS_OK;
    hipStream_t s = static_cast<hipStream_t>(stream);
    const bool mf = form == MESS_DENSE_MFMA;
    if (prec == MESS_FP64) {
        auto *e = static_cast<const double *>(eri);
        auto *d = static_cast<const double *>(D);
        if (mf) launch_dense<double, true>(n, ndens, e, d, static_cast<double *>(J), static_cast<double *>(K), s);
        else launch_dense<double, false>(n, ndens, e, d, static_cast<double *>(J), static_cast<double *>(K), s);
    } else {
        auto *e = static_cast<const float *>(eri);
        auto *d = static_cast<const float *>(D);
        if (mf) launch_dense<float, true>(n, ndens, e, d, static_cast<float *>(J), static_cast<float *>(K), s);
        else launch_dense<float, false>(n, ndens, e, d, static_cast<float *>(J), static_cast<float *>(K), s);
    }
    MESS_LAUNCH_CHECK();
    return MESS_OK;
}
