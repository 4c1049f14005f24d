// mess_jk(MESS_JK_STORED): the unique, Schwarz-screened shell-quartet blocks
// are computed once per (basis, precision, threshold) into device memory,
// one structure-of-arrays region per angular class (element k of quartet t
// at base[k * nq + t]; quartet-major, base[t * NOUT + k], for the classes
// stored_aos_class names), and every later call streams them into J/K.
// The same blocks are what mess_eri(MESS_ERI_BLOCKS) exports (always
// structure-of-arrays), and what the deterministic J/K mode digests with
// exact fixed-point accumulation.
#include <algorithm>

#include "class_ops.hpp"
#include "eri_kernels.hpp"
#include "mess_internal.hpp"

namespace mess {

int get_work_lists(mess_basis *B, double tau, hipStream_t s, WorkLists **out);
int fill_class_launch(const mess_basis *B, const ClassList &cl, hipStream_t s, ClassLaunch &L);

struct StoredEri {
    int prec = MESS_FP64;
    double tau = 0.0;
    std::vector<void *> base;      // per class (index into WorkLists::classes)
    std::vector<int64_t> bytes;
    int64_t total_bytes = 0;
};

void free_stored(mess_basis *B) {
    for (auto &kv : B->stored) {
        for (void *p : kv.second->base)
            if (p) hipFree(p);
        delete kv.second;
    }
    B->stored.clear();
}

static int nout_of(int cb, int ck) {
    return ncart(pair_class_la(cb)) * ncart(pair_class_lb(cb)) * ncart(pair_class_la(ck)) *
           ncart(pair_class_lb(ck));
}

static int get_stored(mess_basis *B, int prec, double tau, hipStream_t s, WorkLists **Wout, StoredEri **out) {
    if (!(tau > 0.0)) tau = 0.0;
    WorkLists *W = nullptr;
    MESS_TRY(get_work_lists(B, tau, s, &W));
    *Wout = W;
    auto key = std::make_pair(prec, tau);
    auto it = B->stored.find(key);
    if (it != B->stored.end()) {
        *out = it->second;
        return MESS_OK;
    }
    auto *E = new StoredEri();
    E->prec = prec;
    E->tau = tau;
    const size_t rsz = prec == MESS_FP32 ? sizeof(float) : sizeof(double);
    int rc = MESS_OK;
    for (const ClassList &cl : W->classes) {
        void *p = nullptr;
        const int64_t nbytes = (int64_t)rsz * nout_of(cl.cb, cl.ck) * cl.total;
        if (cl.total > 0 && hipMalloc(&p, nbytes) != hipSuccess) {
            set_error("mess_jk(STORED): cannot allocate %lld bytes for class (%d,%d)", (long long)nbytes, cl.cb,
                      cl.ck);
            rc = MESS_E_NOMEM;
            break;
        }
        E->base.push_back(p);
        E->bytes.push_back(cl.total > 0 ? nbytes : 0);
        E->total_bytes += cl.total > 0 ? nbytes : 0;
        if (cl.total == 0) continue;
        ClassLaunch L;
        fill_class_launch(B, cl, s, L);
        rc = dispatch_class(cl.cb, cl.ck, [&](auto CB, auto CK) {
            return ClassOps<decltype(CB)::value, decltype(CK)::value>::store(L, p, prec);
        });
        if (rc != MESS_OK) break;
        if (stored_aos_class(cl.cb, cl.ck)) {
            // kept quartet-major: copy, then release the structure-of-arrays region
            void *a = nullptr;
            if (hipMalloc(&a, nbytes) != hipSuccess) {
                set_error("mess_jk(STORED): cannot allocate %lld bytes for class (%d,%d)", (long long)nbytes, cl.cb,
                          cl.ck);
                rc = MESS_E_NOMEM;
                break;
            }
            rc = to_aos(p, a, nout_of(cl.cb, cl.ck), cl.total, prec, s);
            if (rc == MESS_OK && hipStreamSynchronize(s) != hipSuccess) {
                set_error("mess_jk(STORED): block transpose failed");
                rc = MESS_E_DEVICE;
            }
            hipFree(rc == MESS_OK ? p : a);
            if (rc != MESS_OK) break;
            E->base.back() = a;
        }
    }
    if (rc != MESS_OK) {
        for (void *p : E->base)
            if (p) hipFree(p);
        delete E;
        return rc;
    }
    B->stored[key] = E;
    *out = E;
    return MESS_OK;
}

int zero_async(double *p, int64_t n, hipStream_t s);

int jk_stored(mess_basis *B, const double *D, double *Gj, double *Gk, int prec, double tau, hipStream_t s) {
    WorkLists *W = nullptr;
    StoredEri *E = nullptr;
    MESS_TRY(get_stored(B, prec, tau, s, &W, &E));
    if (Gj) MESS_TRY(zero_async(Gj, B->packed, s));
    if (Gk) MESS_TRY(zero_async(Gk, B->packed, s));
    const bool prof = prof_on();
    for (size_t c = 0; c < W->classes.size(); ++c) {
        const ClassList &cl = W->classes[c];
        if (cl.total == 0) continue;
        ClassLaunch L;
        fill_class_launch(B, cl, s, L);
        // recorded under class index + 32, with the bytes streamed in the
        // operation-count field
        if (prof) prof_record(s, 32 + class_index(cl.cb, cl.ck), true, cl.total, cl.prim_quartets, (double)E->bytes[c]);
        MESS_TRY(dispatch_class(cl.cb, cl.ck, [&](auto CB, auto CK) {
            return ClassOps<decltype(CB)::value, decltype(CK)::value>::jk_stored(L, E->base[c], prec, D, Gj, Gk);
        }));
        if (prof) prof_record(s, 0, false, 0, 0, 0.0);
    }
    return MESS_OK;
}

// ------------------------------------------------------------ ERI blocks

// Element count of every class's block region for (basis, tau), in class
// order (cls = cb (cb + 1) / 2 + ck), and the total.
static int block_layout(mess_basis *B, double tau, hipStream_t s, WorkLists **Wout, std::vector<int64_t> &elems) {
    WorkLists *W = nullptr;
    MESS_TRY(get_work_lists(B, tau, s, &W));
    elems.assign(kNumClasses, 0);
    for (const ClassList &cl : W->classes) elems[class_index(cl.cb, cl.ck)] = (int64_t)nout_of(cl.cb, cl.ck) * cl.total;
    *Wout = W;
    return MESS_OK;
}

int eri_blocks(mess_basis *B, int prec, double tau, void *out, size_t out_bytes, hipStream_t s) {
    if (!(tau > 0.0)) tau = 0.0;
    WorkLists *W = nullptr;
    std::vector<int64_t> elems;
    MESS_TRY(block_layout(B, tau, s, &W, elems));
    const size_t rsz = prec == MESS_FP32 ? sizeof(float) : sizeof(double);
    int64_t total = 0;
    for (int64_t e : elems) total += e;
    if (out_bytes < rsz * (size_t)total) {
        set_error("mess_eri(BLOCKS): output holds %zu bytes, %zu needed", out_bytes, rsz * (size_t)total);
        return MESS_E_SIZE;
    }
    int64_t off = 0;
    for (const ClassList &cl : W->classes) {
        const int cls = class_index(cl.cb, cl.ck);
        if (cl.total > 0) {
            ClassLaunch L;
            fill_class_launch(B, cl, s, L);
            void *p = static_cast<char *>(out) + rsz * off;
            MESS_TRY(dispatch_class(cl.cb, cl.ck, [&](auto CB, auto CK) {
                return ClassOps<decltype(CB)::value, decltype(CK)::value>::store(L, p, prec);
            }));
        }
        off += elems[cls];
    }
    return MESS_OK;
}

// ------------------------------------------------- deterministic J/K
//
// Exact, order-independent accumulation: every contribution v (an FP64
// partial sum computed by one lane in a fixed order) is added as the
// 128-bit two's-complement integer X = round_toward_zero(|v| 2^80) (sign
// applied) to an accumulator of two 64-bit words with integer atomics; the
// carry out of the low word is detected from the value the low atomic
// returns.  Integer addition is associative, so the sum, and its one
// rounding back to FP64, do not depend on the order in which the GPU
// retires the atomics.  Resolution 2^-80, range |value| < 2^46 (larger or
// non-finite contributions set an error flag).

constexpr double kFixScale = 1208925819614629174706176.0;  // 2^80
constexpr double kFixHiScale = 65536.0;                    // 2^16: high word units of 2^-16

__device__ __forceinline__ void fix_add(unsigned long long *__restrict__ acc, double v, int *__restrict__ flag) {
    if (v == 0.0) return;
    const double a = fabs(v);
    if (!(a < 70368744177664.0)) {  // 2^46, also catches NaN
        atomicOr(flag, 1);
        return;
    }
    const double sh = a * kFixHiScale;
    const double fh = floor(sh);
    unsigned long long hi = (unsigned long long)fh;
    unsigned long long lo = (unsigned long long)((sh - fh) * 18446744073709551616.0);  // (frac) 2^64 < 2^64
    if (v < 0.0) {
        lo = ~lo + 1ull;
        hi = ~hi + (lo == 0ull ? 1ull : 0ull);
    }
    const unsigned long long old = atomicAdd(&acc[0], lo);
    const unsigned long long dh = hi + ((old + lo < old) ? 1ull : 0ull);
    if (dh) atomicAdd(&acc[1], dh);
}

__device__ __forceinline__ double fix_value(unsigned long long lo, unsigned long long hi) {
    const bool neg = (long long)hi < 0;
    if (neg) {
        lo = ~lo + 1ull;
        hi = ~hi + (lo == 0ull ? 1ull : 0ull);
    }
    const double r = (double)hi * (1.0 / kFixHiScale) + (double)lo * (1.0 / kFixScale);
    return neg ? -r : r;
}

__global__ void k_fix_zero(unsigned long long *__restrict__ p, int64_t n) {
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        p[i] = 0ull;
}

__global__ void k_fix_finish(const unsigned long long *__restrict__ acc, int64_t n, double *__restrict__ G) {
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        G[i] = fix_value(acc[2 * i], acc[2 * i + 1]);
}

// One wave per stored quartet; lane t computes target element t of the six
// families (Gj[a,b], Gj[c,d], Gk[a,c], Gk[b,c], Gk[a,d], Gk[b,d]) as a sum in
// a fixed order, then adds it exactly.
template <typename Real>
__global__ void __launch_bounds__(64) k_jk_det(const PairInfo *__restrict__ pairs, int bra_off, int ket_off,
                                               int nbra, int same_class, const int64_t *__restrict__ rowstart,
                                               const int2 *__restrict__ rowmap, int64_t total, int NA, int NB,
                                               int NC, int ND, const Real *__restrict__ base, int64_t es, int64_t qs,
                                               const double *__restrict__ D, unsigned long long *__restrict__ Aj,
                                               unsigned long long *__restrict__ Ak, int *__restrict__ flag) {
    const int lane = threadIdx.x;
    for (int64_t q = blockIdx.x; q < total; q += gridDim.x) {
        const int2 ij = quartet_pairs(rowstart, rowmap, nbra, q);
        const PairInfo bra = pairs[bra_off + ij.x];
        const PairInfo ket = pairs[ket_off + ij.y];
        double fac = 1.0;
        if (bra.sa == bra.sb) fac *= 0.5;
        if (ket.sa == ket.sb) fac *= 0.5;
        if (same_class && ij.x == ij.y) fac *= 0.5;
        const int N = bra.mN;
        const double *Dm = D + bra.moff;
        auto O = [&](int a, int b, int c, int d) {
            return (double)base[(int64_t)(((a * NB + b) * NC + c) * ND + d) * es + q * qs];
        };
        auto Dv = [&](int r, int c) { return Dm[(int64_t)r * N + c]; };
        const int a0 = bra.bfa, b0 = bra.bfb, c0 = ket.bfa, d0 = ket.bfb;
        const int t_ab = Aj ? NA * NB : 0, t_cd = Aj ? NC * ND : 0;
        const int t_ac = Ak ? NA * NC : 0, t_bc = Ak ? NB * NC : 0, t_ad = Ak ? NA * ND : 0, t_bd = Ak ? NB * ND : 0;
        const int ntgt = t_ab + t_cd + t_ac + t_bc + t_ad + t_bd;
        for (int t = lane; t < ntgt; t += 64) {
            int r = t;
            double sum = 0.0;
            int64_t dst;
            unsigned long long *acc;
            if (r < t_ab) {
                const int a = r / NB, b = r % NB;
                for (int c = 0; c < NC; ++c)
                    for (int d = 0; d < ND; ++d) sum += O(a, b, c, d) * Dv(c0 + c, d0 + d);
                sum *= 2.0 * fac;
                dst = (int64_t)(a0 + a) * N + b0 + b;
                acc = Aj;
            } else if ((r -= t_ab) < t_cd) {
                const int c = r / ND, d = r % ND;
                for (int a = 0; a < NA; ++a)
                    for (int b = 0; b < NB; ++b) sum += O(a, b, c, d) * Dv(a0 + a, b0 + b);
                sum *= 2.0 * fac;
                dst = (int64_t)(c0 + c) * N + d0 + d;
                acc = Aj;
            } else if ((r -= t_cd) < t_ac) {
                const int a = r / NC, c = r % NC;
                for (int b = 0; b < NB; ++b)
                    for (int d = 0; d < ND; ++d) sum += O(a, b, c, d) * Dv(b0 + b, d0 + d);
                sum *= fac;
                dst = (int64_t)(a0 + a) * N + c0 + c;
                acc = Ak;
            } else if ((r -= t_ac) < t_bc) {
                const int b = r / NC, c = r % NC;
                for (int a = 0; a < NA; ++a)
                    for (int d = 0; d < ND; ++d) sum += O(a, b, c, d) * Dv(a0 + a, d0 + d);
                sum *= fac;
                dst = (int64_t)(b0 + b) * N + c0 + c;
                acc = Ak;
            } else if ((r -= t_bc) < t_ad) {
                const int a = r / ND, d = r % ND;
                for (int b = 0; b < NB; ++b)
                    for (int c = 0; c < NC; ++c) sum += O(a, b, c, d) * Dv(b0 + b, c0 + c);
                sum *= fac;
                dst = (int64_t)(a0 + a) * N + d0 + d;
                acc = Ak;
            } else {
                r -= t_ad;
                const int b = r / ND, d = r % ND;
                for (int a = 0; a < NA; ++a)
                    for (int c = 0; c < NC; ++c) sum += O(a, b, c, d) * Dv(a0 + a, c0 + c);
                sum *= fac;
                dst = (int64_t)(b0 + b) * N + d0 + d;
                acc = Ak;
            }
            fix_add(acc + 2 * (bra.moff + dst), sum, flag);
        }
    }
}

// Gj, Gk (either may be NULL) <- half matrices of J and K from the stored
// blocks of (prec, tau), accumulated exactly: bitwise the same result on
// every run.  Synchronises the stream (reads the range flag).
int jk_det(mess_basis *B, const double *D, double *Gj, double *Gk, int prec, double tau, hipStream_t s) {
    WorkLists *W = nullptr;
    StoredEri *E = nullptr;
    MESS_TRY(get_stored(B, prec, tau, s, &W, &E));
    if (!B->det_acc) {
        // 2 accumulators (J, K) x packed elements x 2 words, then the flag
        MESS_HIP(hipMalloc(&B->det_acc, sizeof(unsigned long long) * (4 * (size_t)B->packed + 1)));
    }
    auto *Aj = static_cast<unsigned long long *>(B->det_acc);
    auto *Ak = Aj + 2 * B->packed;
    int *flag = reinterpret_cast<int *>(Aj + 4 * B->packed);
    const int64_t nz = 4 * B->packed + 1;
    hipLaunchKernelGGL(k_fix_zero, dim3((unsigned)std::min<int64_t>((nz + 255) / 256, 65536)), dim3(256), 0, s, Aj,
                       nz);
    MESS_LAUNCH_CHECK();
    for (size_t c = 0; c < W->classes.size(); ++c) {
        const ClassList &cl = W->classes[c];
        if (cl.total == 0) continue;
        const int NA = ncart(pair_class_la(cl.cb)), NB = ncart(pair_class_lb(cl.cb)),
                  NC = ncart(pair_class_la(cl.ck)), ND = ncart(pair_class_lb(cl.ck));
        const unsigned g = (unsigned)std::min<int64_t>(cl.total, 1 << 20);
        // element stride and quartet stride of the class's stored layout
        const bool aos = stored_aos_class(cl.cb, cl.ck);
        const int64_t es = aos ? 1 : cl.total, qs = aos ? (int64_t)NA * NB * NC * ND : 1;
        const PairInfo *pairs = B->d_pairs;
        const int boff = B->pair_class_off[cl.cb], koff = B->pair_class_off[cl.ck];
        if (prec == MESS_FP32)
            hipLaunchKernelGGL(k_jk_det<float>, dim3(g), dim3(64), 0, s, pairs, boff, koff, cl.nrow, cl.cb == cl.ck,
                               cl.d_rowstart, cl.d_rowmap, cl.total, NA, NB, NC, ND,
                               static_cast<const float *>(E->base[c]), es, qs, D, Gj ? Aj : nullptr, Gk ? Ak : nullptr,
                               flag);
        else
            hipLaunchKernelGGL(k_jk_det<double>, dim3(g), dim3(64), 0, s, pairs, boff, koff, cl.nrow, cl.cb == cl.ck,
                               cl.d_rowstart, cl.d_rowmap, cl.total, NA, NB, NC, ND,
                               static_cast<const double *>(E->base[c]), es, qs, D, Gj ? Aj : nullptr,
                               Gk ? Ak : nullptr, flag);
        MESS_LAUNCH_CHECK();
    }
    const unsigned gf = (unsigned)std::min<int64_t>((B->packed + 255) / 256, 65536);
    if (Gj) hipLaunchKernelGGL(k_fix_finish, dim3(gf), dim3(256), 0, s, Aj, B->packed, Gj);
    if (Gk) hipLaunchKernelGGL(k_fix_finish, dim3(gf), dim3(256), 0, s, Ak, B->packed, Gk);
    MESS_LAUNCH_CHECK();
    int hflag = 0;
    MESS_HIP(hipMemcpyAsync(&hflag, flag, sizeof(int), hipMemcpyDeviceToHost, s));
    MESS_HIP(hipStreamSynchronize(s));
    if (hflag) {
        set_error("deterministic J/K: a contribution is not finite or exceeds 2^46 in magnitude");
        return MESS_E_NUMERIC;
    }
    return MESS_OK;
}

}  // namespace mess

using namespace mess;

extern "C" int mess_eri_quartets(const mess_basis *basis, double schwarz_tol, int64_t *counts, int32_t *shells) {
    if (!basis) {
        set_error("mess_eri_quartets: NULL basis");
        return MESS_E_ARG;
    }
    auto *B = const_cast<mess_basis *>(basis);
    const double tau = schwarz_tol > 0.0 ? schwarz_tol : 0.0;
    WorkLists *W = nullptr;
    MESS_TRY(get_work_lists(B, tau, nullptr, &W));
    int64_t pos = 0;
    for (const ClassList &cl : W->classes) {
        const int cls = class_index(cl.cb, cl.ck);
        if (counts) counts[cls] = cl.total;
        if (!shells) continue;
        const int boff = B->pair_class_off[cl.cb], koff = B->pair_class_off[cl.ck];
        for (int r = 0; r < cl.nrow; ++r) {
            const PairInfo &bra = B->pairs_host[boff + cl.h_rowmap[r].x];
            for (int64_t t = cl.h_rowstart[r]; t < cl.h_rowstart[r + 1]; ++t) {
                const PairInfo &ket = B->pairs_host[koff + cl.h_rowmap[r].y + (int)(t - cl.h_rowstart[r])];
                int32_t *o = shells + 4 * (pos + t);
                o[0] = bra.sa; o[1] = bra.sb; o[2] = ket.sa; o[3] = ket.sb;
            }
        }
        pos += cl.total;
    }
    return MESS_OK;
}
