// Boys function F_m(T) = int_0^1 u^{2m} exp(-T u^2) du (paper section 3: the
// closed-form electron repulsion integrals reduce to it), evaluated by the
// device routines that the integral kernels call, so that they can be checked
// on their own:
//   form 0: F_0..F_m together, as the recursion kernels take them: Taylor
//           sum of F_m about the nearest grid point T_k = k/16 (T < 60),
//           downward recurrence F_j = (2T F_{j+1} + exp(-T)) / (2j+1), and
//           the large-T form (2j-1)!!/(2T)^j sqrt(pi/T)/2 for T >= 60;
//   form 1: each F_j on its own (Taylor sum of order j, no recurrence), as
//           the table-driven kernel takes them.
// FP64, or the FP32 forms of the mixed-precision kernels (T rounded to FP32,
// results widened to FP64 on output).
#include "coop.hpp"

namespace mess {

template <int M, typename Real>
__global__ void __launch_bounds__(256) k_boys_rec(int64_t n, const double *__restrict__ T, BoysTabs bt,
                                                  double *__restrict__ F) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    if (!(T[i] >= 0.0)) {  // negative or NaN: no table row, NaN out
        for (int j = 0; j <= M; ++j) F[i * (M + 1) + j] = __builtin_nan("");
        return;
    }
    Real f[M + 1];
    boys_eval<M, Real>((Real)T[i], bt, f);
    static_for<0, M + 1>([&](auto J) { F[i * (M + 1) + J] = (double)f[J]; });
}

template <typename Real>
__global__ void __launch_bounds__(256) k_boys_direct(int64_t n, int m, const double *__restrict__ T, BoysTabs bt,
                                                     double *__restrict__ F) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    if (!(T[i] >= 0.0)) {
        for (int j = 0; j <= m; ++j) F[i * (m + 1) + j] = __builtin_nan("");
        return;
    }
    const Real t = (Real)T[i];
    for (int j = 0; j <= m; ++j) F[i * (m + 1) + j] = (double)coop_boys_r<Real>(j, t, bt);
}

template <typename Real, int M>
static void launch_rec(int64_t n, const double *T, const BoysTabs &bt, double *F, hipStream_t s) {
    hipLaunchKernelGGL((k_boys_rec<M, Real>), dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, n, T, bt, F);
}

template <typename Real>
static void launch_rec_m(int m, int64_t n, const double *T, const BoysTabs &bt, double *F, hipStream_t s) {
    switch (m) {
    case 0: launch_rec<Real, 0>(n, T, bt, F, s); break;
    case 1: launch_rec<Real, 1>(n, T, bt, F, s); break;
    case 2: launch_rec<Real, 2>(n, T, bt, F, s); break;
    case 3: launch_rec<Real, 3>(n, T, bt, F, s); break;
    case 4: launch_rec<Real, 4>(n, T, bt, F, s); break;
    case 5: launch_rec<Real, 5>(n, T, bt, F, s); break;
    case 6: launch_rec<Real, 6>(n, T, bt, F, s); break;
    case 7: launch_rec<Real, 7>(n, T, bt, F, s); break;
    default: launch_rec<Real, 8>(n, T, bt, F, s); break;
    }
}

}  // namespace mess

using namespace mess;

extern "C" int mess_boys(const mess_basis *B, int32_t prec, int32_t form, int32_t m, const double *T, int64_t n,
                         double *F, mess_stream stream) {
    if (!B || (n > 0 && (!T || !F))) {
        set_error("mess_boys: basis, T or F is NULL");
        return MESS_E_ARG;
    }
    if (m < 0 || m > 8 || (form != 0 && form != 1) || (prec != MESS_FP64 && prec != MESS_FP32) || n < 0 ||
        n > ((int64_t)1 << 31) * 256) {
        set_error("mess_boys: need 0 <= m <= 8, form 0 or 1, prec FP64 or FP32, 0 <= n (got m=%d form=%d)", m,
                  form);
        return MESS_E_ARG;
    }
    if (n == 0) return MESS_OK;
    hipStream_t s = static_cast<hipStream_t>(stream);
    const BoysTabs bt{B->d_boys, B->d_boys_exp, B->d_boys_f, B->d_boys_exp_f, B->d_boys_t};
    const dim3 grid((unsigned)((n + 255) / 256));
    if (form == 0) {
        if (prec == MESS_FP64) launch_rec_m<double>(m, n, T, bt, F, s);
        else launch_rec_m<float>(m, n, T, bt, F, s);
    } else if (prec == MESS_FP64) {
        hipLaunchKernelGGL(k_boys_direct<double>, grid, dim3(256), 0, s, n, (int)m, T, bt, F);
    } else {
        hipLaunchKernelGGL(k_boys_direct<float>, grid, dim3(256), 0, s, n, (int)m, T, bt, F);
    }
    MESS_LAUNCH_CHECK();
    return MESS_OK;
}
