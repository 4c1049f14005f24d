// mess_eri and mess_jk: class-by-class launches over the unique
// shell-quartet work lists, then the symmetrisation J = Gj + Gj^T,
// K = Gk + Gk^T of the half-matrices the digestion accumulates.
#include "class_ops.hpp"
#include "mess_internal.hpp"

#include <algorithm>
#include <mutex>

namespace mess {

int get_work_lists(mess_basis *B, double tau, hipStream_t s, WorkLists **out);
int fill_class_launch(const mess_basis *B, const ClassList &cl, hipStream_t s, ClassLaunch &L);
int jk_stored(mess_basis *B, const double *D, double *Gj, double *Gk, int prec, double tau, hipStream_t s);
int jk_det(mess_basis *B, const double *D, double *Gj, double *Gk, int prec, double tau, hipStream_t s);
int eri_blocks(mess_basis *B, int prec, double tau, void *out, size_t out_bytes, hipStream_t s);

__global__ void k_fill_zero(double *__restrict__ p, int64_t n) {
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        p[i] = 0.0;
}

// out = G + G^T for every diagonal block of a packed block-diagonal matrix
// (block m: n_m x n_m at offset moff[m]); blockIdx.z strides over blocks.
__global__ void k_symmetrise(const double *__restrict__ G, int nmol, const int64_t *__restrict__ moff,
                             const int *__restrict__ nb, double *__restrict__ out) {
    const int i = blockIdx.y * blockDim.y + threadIdx.y;
    const int j = blockIdx.x * blockDim.x + threadIdx.x;
    for (int m = blockIdx.z; m < nmol; m += gridDim.z) {
        const int n = nb[m];
        if (i < n && j < n) {
            const int64_t o = moff[m];
            out[o + (int64_t)i * n + j] = G[o + (int64_t)i * n + j] + G[o + (int64_t)j * n + i];
        }
    }
}

int zero_async(double *p, int64_t n, hipStream_t s) {
    if (n <= 0) return MESS_OK;
    int64_t g = (n + 255) / 256;
    if (g > 65536) g = 65536;
    hipLaunchKernelGGL(k_fill_zero, dim3((unsigned)g), dim3(256), 0, s, p, n);
    MESS_LAUNCH_CHECK();
    return MESS_OK;
}

int symmetrise_async(const mess_basis *B, const double *G, double *out, hipStream_t s) {
    const int N = B->nbf_max;
    dim3 blk(32, 8), grd((N + 31) / 32, (N + 7) / 8, (unsigned)std::min(B->n_mol, 65535));
    hipLaunchKernelGGL(k_symmetrise, grd, blk, 0, s, G, B->n_mol, B->d_mol_moff, B->d_mol_nbf, out);
    MESS_LAUNCH_CHECK();
    return MESS_OK;
}

// Gj, Gk (device, packed block-diagonal, may be NULL) <- half-matrices of J and K.
int jk_direct_half(mess_basis *B, const double *D, double *Gj, double *Gk, int prec, double tau,
                   hipStream_t s) {
    WorkLists *W = nullptr;
    MESS_TRY(get_work_lists(B, tau, s, &W));
    if (Gj) MESS_TRY(zero_async(Gj, B->packed, s));
    if (Gk) MESS_TRY(zero_async(Gk, B->packed, s));
    const bool prof = prof_on();
    for (const ClassList &cl : W->classes) {
        if (cl.total == 0) continue;
        ClassLaunch L;
        fill_class_launch(B, cl, s, L);
        // arithmetic of this class: a build asked for in FP32 runs a class in
        // FP64 where the FP32 form table says its FP64 kernel is faster
        const int cp = (prec == MESS_FP32 && class_form(cl.cb, cl.ck, MESS_FP32) == kFormFp64) ? MESS_FP64 : prec;
        if (prof) {
            double fp = 0.0, fq = 0.0;
            class_flops(cl.cb, cl.ck, &fp, &fq, cp);
            // FP32 launches are recorded under class index + 64
            prof_record(s, class_index(cl.cb, cl.ck) + (cp == MESS_FP32 ? 64 : 0), true, cl.total,
                        cl.prim_quartets,
                        fp * (double)cl.prim_quartets + fq * (double)cl.total);
        }
        MESS_TRY(dispatch_class(cl.cb, cl.ck, [&](auto CB, auto CK) {
            return ClassOps<decltype(CB)::value, decltype(CK)::value>::jk(L, D, Gj, Gk, cp);
        }));
        if (prof) prof_record(s, 0, false, 0, 0, 0.0);
    }
    return MESS_OK;
}

int jk_full(mess_basis *B, const double *D, double *J, double *K, int mode, int prec, double tau,
            hipStream_t s) {
    double *Gj = J ? static_cast<double *>(B->scratch_jk) : nullptr;
    double *Gk = K ? static_cast<double *>(B->scratch_jk) + B->packed : nullptr;
    if (mode == MESS_JK_DIRECT)
        MESS_TRY(jk_direct_half(B, D, Gj, Gk, prec, tau, s));
    else if (mode == MESS_JK_DETERMINISTIC)
        MESS_TRY(jk_det(B, D, Gj, Gk, prec, tau, s));
    else
        MESS_TRY(jk_stored(B, D, Gj, Gk, prec, tau, s));
    if (J) MESS_TRY(symmetrise_async(B, Gj, J, s));
    if (K) MESS_TRY(symmetrise_async(B, Gk, K, s));
    return MESS_OK;
}

// Fixed device workspace of the allocation-free J/K entry point: the two
// half matrices Gj, Gk of at most kNoAllocMaxPacked doubles each (8 MB in
// all per device, held until the process ends).  Host code never passes the
// array's name to a kernel: it uses the per-device address below.
constexpr int64_t kNoAllocMaxPacked = int64_t(1) << 19;
static __device__ __align__(256) double scratch[2 * kNoAllocMaxPacked];

constexpr int kMaxDevices = 64;
static std::mutex g_scratch_mutex;
static double *g_scratch_ptr[kMaxDevices] = {};

// Device address of `scratch` on the current device, looked up once per
// device (each device holds its own copy of the array).
static int scratch_address(double **out) {
    int dev = 0;
    MESS_HIP(hipGetDevice(&dev));
    if (dev < 0 || dev >= kMaxDevices) {
        set_error("mess_jk_noalloc: device index %d beyond %d", dev, kMaxDevices);
        return MESS_E_DEVICE;
    }
    std::lock_guard<std::mutex> lk(g_scratch_mutex);
    if (!g_scratch_ptr[dev]) {
        void *p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p) {
            set_error("mess_jk_noalloc: hipGetSymbolAddress(scratch) failed: %s", hipGetErrorString(e));
            return MESS_E_DEVICE;
        }
        g_scratch_ptr[dev] = static_cast<double *>(p);
    }
    *out = g_scratch_ptr[dev];
    return MESS_OK;
}

}  // namespace mess

using namespace mess;

extern "C" {

int mess_eri(const mess_basis *basis, int32_t layout, int32_t prec, double schwarz_tol, void *out,
             size_t out_bytes, mess_stream stream) {
    if (!basis || !out) {
        set_error("mess_eri: NULL basis or output");
        return MESS_E_ARG;
    }
    if (prec != MESS_FP64 && prec != MESS_FP32) {
        set_error("mess_eri: unknown precision %d", prec);
        return MESS_E_UNSUPPORTED;
    }
    if (layout != MESS_ERI_DENSE && layout != MESS_ERI_BLOCKS) {
        set_error("mess_eri: unknown layout %d", layout);
        return MESS_E_UNSUPPORTED;
    }
    auto *B = const_cast<mess_basis *>(basis);
    if (layout == MESS_ERI_BLOCKS)
        return eri_blocks(B, prec, schwarz_tol, out, out_bytes, static_cast<hipStream_t>(stream));
    if (B->n_mol != 1) {
        set_error("mess_eri: the dense tensor is built for a single molecule, not a batch of %d", B->n_mol);
        return MESS_E_UNSUPPORTED;
    }
    const int64_t N = B->nbf;
    const size_t need = sizeof(double) * (size_t)(N * N * N * N);
    if (out_bytes < need) {
        set_error("mess_eri: output holds %zu bytes, %zu needed", out_bytes, need);
        return MESS_E_SIZE;
    }
    hipStream_t s = static_cast<hipStream_t>(stream);
    WorkLists *W = nullptr;
    MESS_TRY(get_work_lists(B, schwarz_tol, s, &W));
    MESS_TRY(zero_async(static_cast<double *>(out), N * N * N * N, s));
    for (const ClassList &cl : W->classes) {
        if (cl.total == 0) continue;
        ClassLaunch L;
        fill_class_launch(B, cl, s, L);
        MESS_TRY(dispatch_class(cl.cb, cl.ck, [&](auto CB, auto CK) {
            return ClassOps<decltype(CB)::value, decltype(CK)::value>::dense(L, static_cast<double *>(out), prec);
        }));
    }
    return MESS_OK;
}

int mess_jk(const mess_basis *basis, const double *D, double *J, double *K, int32_t mode, int32_t prec,
            double schwarz_tol, mess_stream stream) {
    if (!basis || !D) {
        set_error("mess_jk: NULL basis or density");
        return MESS_E_ARG;
    }
    if (mode != MESS_JK_DIRECT && mode != MESS_JK_STORED && mode != MESS_JK_DETERMINISTIC) {
        set_error("mess_jk: unknown mode %d", mode);
        return MESS_E_UNSUPPORTED;
    }
    if (prec != MESS_FP64 && prec != MESS_FP32) {
        set_error("mess_jk: unknown precision %d", prec);
        return MESS_E_UNSUPPORTED;
    }
    if (!J && !K) return MESS_OK;
    return jk_full(const_cast<mess_basis *>(basis), D, J, K, mode, prec, schwarz_tol,
                   static_cast<hipStream_t>(stream));
}

int mess_jk_noalloc(const mess_basis *basis, const double *D, double *J, double *K, int32_t prec,
                    double schwarz_tol, mess_stream stream) {
    if (!basis || !D) {
        set_error("mess_jk_noalloc: NULL basis or density");
        return MESS_E_ARG;
    }
    if (prec != MESS_FP64 && prec != MESS_FP32) {
        set_error("mess_jk_noalloc: unknown precision %d", prec);
        return MESS_E_UNSUPPORTED;
    }
    auto *B = const_cast<mess_basis *>(basis);
    if (B->packed > kNoAllocMaxPacked) {
        set_error("mess_jk_noalloc: %lld matrix elements exceed the fixed workspace of %lld per matrix",
                  (long long)B->packed, (long long)kNoAllocMaxPacked);
        return MESS_E_SIZE;
    }
    if (prof_on()) {
        set_error("mess_jk_noalloc: class profiling is on (it records events); turn it off first");
        return MESS_E_ARG;
    }
    const double tau = schwarz_tol > 0.0 ? schwarz_tol : 0.0;
    auto it = B->lists.find(tau);
    bool ready = it != B->lists.end();
    if (ready)
        for (const ClassList &cl : it->second->classes)
            if (cl.total > 0 && !coop_program_cached(cl.cb, cl.ck)) ready = false;
    if (!ready) {
        set_error("mess_jk_noalloc: the work lists for schwarz_tol %g are not built yet; call mess_jk once "
                  "with this basis, precision and tolerance first", schwarz_tol);
        return MESS_E_ARG;
    }
    if (!J && !K) return MESS_OK;
    double *ws = nullptr;
    MESS_TRY(scratch_address(&ws));
    hipStream_t s = static_cast<hipStream_t>(stream);
    double *Gj = J ? ws : nullptr;
    double *Gk = K ? ws + kNoAllocMaxPacked : nullptr;
    MESS_TRY(jk_direct_half(B, D, Gj, Gk, prec, tau, s));
    if (J) MESS_TRY(symmetrise_async(B, Gj, J, s));
    if (K) MESS_TRY(symmetrise_async(B, Gk, K, s));
    return MESS_OK;
}

}  // extern "C"
