// Shared pieces of the wave-per-quartet kernels (table-driven k_coop in
// coop.hip, primitive-lane k_plane in plane.hip): the argument block of the
// step tables, the per-mode output (horizontal recursion, dense store,
// Schwarz factor or J/K digestion) of one quartet.
#pragma once

#include <algorithm>

#include "class_ops.hpp"
#include "eri_kernels.hpp"
#include "mess_internal.hpp"

namespace mess {

// Coefficient slots of the vertical-recursion steps (per primitive quartet):
enum : int {
    kC0 = 0,                 // 0
    kPA = 1, kWP = 4,        // PA_xyz, WP_xyz (bra)
    kQC = 7, kWQ = 10,       // QC_xyz, WQ_xyz (ket)
    kO2P = 13, kO2PR = 14,   // 1/(2p), rho/(2p^2)
    kO2Q = 15, kO2QR = 16,   // 1/(2q), rho/(2q^2)
    kO2PQ = 17,              // 1/(2(p+q))
    kNCoef = 18
};
// Horizontal-recursion coefficients: 0 -> 0, 1 -> 1, 2..4 -> AB, 5..7 -> CD.
enum : int { kH0 = 0, kH1 = 1, kHAB = 2, kHCD = 5, kNHCoef = 8 };

struct CoopArgs {
    const int4 *vops;
    const int *vlev;
    const unsigned short *accsrc;
    const int4 *hops;
    const int *hlev;
    const unsigned short *outslot;
    const double *outscale;
    int nV, nH, nacc, nout, nvlev, nhlev, L;
    int nvbra;  // VRR levels [0, nvbra) are bra steps, the rest ket steps
    int NA, NB, NC, ND;
};

enum { kModeSchwarz = 0, kModeDense = 1, kModeJK = 2, kModeStore64 = 3, kModeStore32 = 4 };

__device__ __forceinline__ double coop_boys(int m, double T, const double *__restrict__ tab) {
    // F_m(T), m <= 8, directly (no recurrence): Taylor about the nearest grid
    // point for T < 60, the large-T form (2m-1)!!/(2T)^m sqrt(pi/T)/2 above.
    if (T < kBoysTmax) {
        const int k = __double2int_rn(T * kBoysInvStep);
        const double md = static_cast<double>(k) * (1.0 / kBoysInvStep) - T;
        const double *row = tab + k * kBoysN + m;
        double f = row[7];
        f = row[6] + md * (1.0 / 7.0) * f;
        f = row[5] + md * (1.0 / 6.0) * f;
        f = row[4] + md * (1.0 / 5.0) * f;
        f = row[3] + md * (1.0 / 4.0) * f;
        f = row[2] + md * (1.0 / 3.0) * f;
        f = row[1] + md * (1.0 / 2.0) * f;
        return row[0] + md * f;
    }
    const double rT = 1.0 / T;
    double f = 0.5 * sqrt(M_PI * rT);
    for (int n = 0; n < m; ++n) f *= (2 * n + 1) * 0.5 * rT;
    return f;
}

// F_m(T) in the kernel's arithmetic: FP64 form of coop_boys, or FP32 Taylor for
// 1e-3 <= T <= 30 with the FP64 form rounded to FP32 outside.
template <typename Real>
__device__ __forceinline__ Real coop_boys_r(int m, Real T, const BoysTabs &bt) {
    if constexpr (sizeof(Real) == 8) {
        return coop_boys(m, T, bt.tab);
    } else {
        if (T < 1e-3f || T > 30.0f) return (float)coop_boys(m, (double)T, bt.tab);
        const int k = __float2int_rn(T * (float)kBoysInvStep);
        const float md = (float)k * (float)(1.0 / kBoysInvStep) - T;
        const float *row = bt.tabf + k * kBoysN + m;
        float f = row[5];
        f = row[4] + md * (1.0f / 5.0f) * f;
        f = row[3] + md * (1.0f / 4.0f) * f;
        f = row[2] + md * (1.0f / 3.0f) * f;
        f = row[1] + md * (1.0f / 2.0f) * f;
        return row[0] + md * f;
    }
}

__device__ __forceinline__ double run_op(const int4 op, const double *__restrict__ V, const double *__restrict__ c) {
    const int s1 = op.x >> 16, s2 = op.y & 0xffff, s3 = op.y >> 16, s4 = op.z & 0xffff, s5 = op.z >> 16;
    const int w = op.w;
    const int a1 = w & 31, a2 = (w >> 5) & 31, a3 = (w >> 10) & 31, a4 = (w >> 15) & 31, a5 = (w >> 20) & 31;
    const double k3 = (double)((w >> 25) & 7), k5 = (double)((w >> 28) & 7);
    double v = c[a1] * V[s1] + c[a2] * V[s2];
    if (k3 != 0.0) v += k3 * (c[a3] * V[s3] - c[a4] * V[s4]);
    if (k5 != 0.0) v += k5 * c[a5] * V[s5];
    return v;
}

// J/K digestion of one quartet's block by a wave: lanes over the elements of
// the six target families Gj[a,b], Gj[c,d], Gk[a,c], Gk[b,c], Gk[a,d],
// Gk[b,d] (each a sum over the block weighted by density elements).
template <int NT = 64, typename OF>
__device__ __forceinline__ void wave_digest(const int lane, const int NA, const int NB, const int NC, const int ND,
                                            const double fac, const int a0, const int b0, const int c0, const int d0,
                                            OF &&O, const double *__restrict__ D, const int N,
                                            double *__restrict__ Gj, double *__restrict__ Gk) {
    auto Dv = [&](int r, int cidx) { return D[(int64_t)r * N + cidx]; };
    const int nab = NA * NB, ncd = NC * ND;
    const int t_ab = Gj ? nab : 0, t_cd = Gj ? ncd : 0;
    const int t_ac = Gk ? NA * NC : 0, t_bc = Gk ? NB * NC : 0, t_ad = Gk ? NA * ND : 0, t_bd = Gk ? NB * ND : 0;
    const int ntgt = t_ab + t_cd + t_ac + t_bc + t_ad + t_bd;
    for (int t = lane; t < ntgt; t += NT) {
        int r = t;
        double s = 0.0;
        if (r < t_ab) {
            const int a = r / NB, b = r % NB;
            for (int cc = 0; cc < NC; ++cc)
                for (int d = 0; d < ND; ++d) s += O(a, b, cc, d) * Dv(c0 + cc, d0 + d);
            unsafeAtomicAdd(&Gj[(int64_t)(a0 + a) * N + b0 + b], 2.0 * fac * s);
            continue;
        }
        r -= t_ab;
        if (r < t_cd) {
            const int cc = r / ND, d = r % ND;
            for (int a = 0; a < NA; ++a)
                for (int b = 0; b < NB; ++b) s += O(a, b, cc, d) * Dv(a0 + a, b0 + b);
            unsafeAtomicAdd(&Gj[(int64_t)(c0 + cc) * N + d0 + d], 2.0 * fac * s);
            continue;
        }
        r -= t_cd;
        if (r < t_ac) {
            const int a = r / NC, cc = r % NC;
            for (int b = 0; b < NB; ++b)
                for (int d = 0; d < ND; ++d) s += O(a, b, cc, d) * Dv(b0 + b, d0 + d);
            unsafeAtomicAdd(&Gk[(int64_t)(a0 + a) * N + c0 + cc], fac * s);
            continue;
        }
        r -= t_ac;
        if (r < t_bc) {
            const int b = r / NC, cc = r % NC;
            for (int a = 0; a < NA; ++a)
                for (int d = 0; d < ND; ++d) s += O(a, b, cc, d) * Dv(a0 + a, d0 + d);
            unsafeAtomicAdd(&Gk[(int64_t)(b0 + b) * N + c0 + cc], fac * s);
            continue;
        }
        r -= t_bc;
        if (r < t_ad) {
            const int a = r / ND, d = r % ND;
            for (int b = 0; b < NB; ++b)
                for (int cc = 0; cc < NC; ++cc) s += O(a, b, cc, d) * Dv(b0 + b, c0 + cc);
            unsafeAtomicAdd(&Gk[(int64_t)(a0 + a) * N + d0 + d], fac * s);
            continue;
        }
        r -= t_ad;
        {
            const int b = r / ND, d = r % ND;
            for (int a = 0; a < NA; ++a)
                for (int cc = 0; cc < NC; ++cc) s += O(a, b, cc, d) * Dv(a0 + a, c0 + cc);
            unsafeAtomicAdd(&Gk[(int64_t)(b0 + b) * N + d0 + d], fac * s);
        }
    }
}

// Horizontal recursion of the accumulated [e0|f0] (in H[0, nacc)) and the
// per-mode output of one quartet, shared by the wave.
// NT: threads of the block sharing the quartet (lane = thread index).
template <int MODE, int NT = 64>
__device__ __forceinline__ void coop_finish(const CoopArgs &A, double *__restrict__ H, double *__restrict__ hc,
                                            const int lane, const PairInfo &bra, const PairInfo &ket, const int i,
                                            const int j, const int bra_off, const int same_class,
                                            const double *__restrict__ D, const int N, double *__restrict__ out0,
                                            double *__restrict__ out1, const int64_t q = 0, const int64_t total = 0) {
        if (lane == 0) {
            hc[kH0] = 0.0; hc[kH1] = 1.0;
            hc[kHAB + 0] = bra.ABx; hc[kHAB + 1] = bra.ABy; hc[kHAB + 2] = bra.ABz;
            hc[kHCD + 0] = ket.ABx; hc[kHCD + 1] = ket.ABy; hc[kHCD + 2] = ket.ABz;
        }
        __syncthreads();
        for (int lv = 0; lv < A.nhlev; ++lv) {
            const int b0 = A.hlev[lv], b1 = A.hlev[lv + 1];
            for (int o = b0 + lane; o < b1; o += NT) {
                const int4 op = A.hops[o];
                H[op.x & 0xffff] = run_op(op, H, hc);
            }
            __syncthreads();
        }
        // output element o = ((a*NB + b)*NC + c)*ND + d is H[outslot[o]] * outscale[o]
        const int NB = A.NB, NC = A.NC, ND = A.ND, NA = A.NA;
        auto O = [&](int a, int b, int cc, int d) {
            const int o = ((a * NB + b) * NC + cc) * ND + d;
            return H[A.outslot[o]] * A.outscale[o];
        };
        if (MODE == kModeSchwarz) {
            if (lane == 0) {
                double m = 0.0;
                for (int a = 0; a < NA; ++a)
                    for (int b = 0; b < NB; ++b) m = fmax(m, fabs(O(a, b, a, b)));
                out0[bra_off + i] = sqrt(m);
            }
        } else if (MODE == kModeStore64 || MODE == kModeStore32) {
            for (int o = lane; o < A.nout; o += NT) {
                const double v = H[A.outslot[o]] * A.outscale[o];
                if (MODE == kModeStore64) out0[(int64_t)o * total + q] = v;
                else reinterpret_cast<float *>(out0)[(int64_t)o * total + q] = (float)v;
            }
        } else if (MODE == kModeDense) {
            const int64_t NN = N;
            for (int o = lane; o < A.nout; o += NT) {
                const int d = o % ND, cc = (o / ND) % NC, b = (o / (ND * NC)) % NB, a = o / (ND * NC * NB);
                const double v = H[A.outslot[o]] * A.outscale[o];
                const int64_t ia = bra.bfa + a, ib = bra.bfb + b, ic = ket.bfa + cc, id = ket.bfb + d;
                out0[((ia * NN + ib) * NN + ic) * NN + id] = v;
                out0[((ib * NN + ia) * NN + ic) * NN + id] = v;
                out0[((ia * NN + ib) * NN + id) * NN + ic] = v;
                out0[((ib * NN + ia) * NN + id) * NN + ic] = v;
                out0[((ic * NN + id) * NN + ia) * NN + ib] = v;
                out0[((id * NN + ic) * NN + ia) * NN + ib] = v;
                out0[((ic * NN + id) * NN + ib) * NN + ia] = v;
                out0[((id * NN + ic) * NN + ib) * NN + ia] = v;
            }
        } else {
            double fac = 1.0;
            if (bra.sa == bra.sb) fac *= 0.5;
            if (ket.sa == ket.sb) fac *= 0.5;
            if (same_class && i == j) fac *= 0.5;
            wave_digest<NT>(lane, NA, NB, NC, ND, fac, bra.bfa, bra.bfb, ket.bfa, ket.bfb, O, D + bra.moff, bra.mN,
                            out0 ? out0 + bra.moff : nullptr, out1 ? out1 + bra.moff : nullptr);
        }
}


// Wave-per-primitive-quartet launch of one class in one precision
// (wave.hip, compiled once per class and precision).  With lds_out != NULL
// only reports the dynamic LDS bytes the launch needs.
template <int CB, int CK, typename Real>
struct WaveOps {
    static void launch(int mode, const CoopArgs &A, const ClassLaunch &L, int64_t total, unsigned g,
                       const double *D, double *out0, double *out1, size_t *lds_out);
};

// Primitive-lane launch of one class in one precision (plane.hip, compiled
// once per class and precision).
template <int CB, int CK, typename Real>
struct PlaneOps {
    static void launch(int mode, const CoopArgs &A, const ClassLaunch &L, int64_t total, unsigned g, size_t lds,
                       const double *D, double *out0, double *out1);
};

}  // namespace mess
