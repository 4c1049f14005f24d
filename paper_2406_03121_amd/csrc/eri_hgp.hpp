// Device code for contracted electron-repulsion integrals over one shell
// quartet (ab|cd), l <= 2, by Obara-Saika vertical recursion on primitive
// quartets followed by Head-Gordon-Pople horizontal recursion on the
// contracted intermediates.  Every loop is unrolled at compile time for the
// angular class (LA, LB, LC, LD), so every intermediate has a fixed register
// slot and no index is computed at run time.
//
// The integrals are the closed-form Gaussian integrals of section 3 of the
// paper (the four-centre Coulomb integrals that the Fock matrix needs).
#pragma once

#include "mess_internal.hpp"

namespace mess {

// ------------------------------------------------------------------ Boys
//
// F_n(T) = int_0^1 t^{2n} exp(-T t^2) dt.
// T < 60: the highest order needed, F_L, from an 8-term Taylor expansion
// about the nearest grid point T_k = k/16 (|T - T_k| <= 1/32, truncation
// below 3e-17 relative) using dF_n/dT = -F_{n+1}; exp(-T) the same way from
// exp(-T_k); then the downward recurrence F_n = (2T F_{n+1} + e^{-T})/(2n+1),
// which is stable.  T >= 60: F_0 = sqrt(pi/T)/2 (erf(sqrt T) = 1 and
// e^{-T} < 1e-26 relative to every F_n, n <= 8, there) and the upward
// recurrence F_{n+1} = (2n+1) F_n / (2T).

// 1/sqrt(x), x > 0: the hardware estimate refined by Newton steps
// y <- y (3 - x y^2) / 2, each of which squares the relative error (two in
// FP64 reach rounding level, one in FP32).
__device__ __forceinline__ double rsqrt_nr(double x) {
    double y = __builtin_amdgcn_rsq(x);
    const double hx = 0.5 * x;
    y = y * fma(-hx * y, y, 1.5);
    y = y * fma(-hx * y, y, 1.5);
    return y;
}
__device__ __forceinline__ float rsqrt_nr(float x) {
    const float y = __builtin_amdgcn_rsqf(x);
    return y * fmaf(-0.5f * x * y, y, 1.5f);
}

template <int L>
__device__ __forceinline__ void boys_f64(double T, const double *__restrict__ tab,
                                         const double *__restrict__ etab, double (&F)[L + 1]) {
    if (T < kBoysTmax) {
        const int k = __double2int_rn(T * kBoysInvStep);
        const double md = static_cast<double>(k) * (1.0 / kBoysInvStep) - T;  // -(T - T_k), exact
        const double *row = tab + k * kBoysN + L;
        double f = row[7];
        f = row[6] + md * (1.0 / 7.0) * f;
        f = row[5] + md * (1.0 / 6.0) * f;
        f = row[4] + md * (1.0 / 5.0) * f;
        f = row[3] + md * (1.0 / 4.0) * f;
        f = row[2] + md * (1.0 / 3.0) * f;
        f = row[1] + md * (1.0 / 2.0) * f;
        f = row[0] + md * f;
        F[L] = f;
        if constexpr (L > 0) {
            double e = 1.0 + md * (1.0 / 7.0);
            e = 1.0 + md * (1.0 / 6.0) * e;
            e = 1.0 + md * (1.0 / 5.0) * e;
            e = 1.0 + md * (1.0 / 4.0) * e;
            e = 1.0 + md * (1.0 / 3.0) * e;
            e = 1.0 + md * (1.0 / 2.0) * e;
            e = 1.0 + md * e;
            e *= etab[k];
            const double t2 = 2.0 * T;
            static_for<0, L>([&](auto I) {
                constexpr int m = L - 1 - decltype(I)::value;
                F[m] = (t2 * F[m + 1] + e) * (1.0 / (2 * m + 1));
            });
        }
    } else {
        const double sT = rsqrt_nr(T), rT = sT * sT;
        F[0] = 0.88622692545275801365 * sT;  // sqrt(pi) / 2
        static_for<0, L>([&](auto I) {
            constexpr int m = decltype(I)::value;
            F[m + 1] = F[m] * ((2 * m + 1) * 0.5) * rT;
        });
    }
}

// FP32 Boys function (mixed-precision path): FP32 Taylor expansion about the
// grid point (6 terms, |T - T_k| <= 1/32, truncation 1.3e-12 relative) and
// FP32 downward recurrence for 1e-3 <= T <= 30; the FP64 evaluation above,
// rounded to FP32, for T < 1e-3 and T > 30.
struct BoysTabs {
    const double *tab, *etab;
    const float *tabf, *etabf;
    const double *tabt;  // F_{L+i}(T_k) / i! per order L (FP64 Taylor with no per-term scaling)
};

// FP64 F_0..F_L as boys_f64, the Taylor sums in Horner form on the
// prescaled table (F_{L+i}(T_k)/i!) and the constants 1/i! for exp(-T):
// seven FMAs each.
template <int L>
__device__ __forceinline__ void boys_f64t(double T, const double *__restrict__ tabt, const double *__restrict__ etab,
                                          double (&F)[L + 1]) {
    if (T < kBoysTmax) {
        const int k = __double2int_rn(T * kBoysInvStep);
        const double md = static_cast<double>(k) * (1.0 / kBoysInvStep) - T;  // -(T - T_k), exact
        const double *row = tabt + ((size_t)L * kBoysRows + k) * 8;
        double f = row[7];
        f = row[6] + md * f;
        f = row[5] + md * f;
        f = row[4] + md * f;
        f = row[3] + md * f;
        f = row[2] + md * f;
        f = row[1] + md * f;
        f = row[0] + md * f;
        F[L] = f;
        if constexpr (L > 0) {
            double e = 1.0 / 5040.0;
            e = 1.0 / 720.0 + md * e;
            e = 1.0 / 120.0 + md * e;
            e = 1.0 / 24.0 + md * e;
            e = 1.0 / 6.0 + md * e;
            e = 0.5 + md * e;
            e = 1.0 + md * e;
            e = 1.0 + md * e;
            e *= etab[k];
            const double t2 = 2.0 * T;
            static_for<0, L>([&](auto I) {
                constexpr int m = L - 1 - decltype(I)::value;
                F[m] = (t2 * F[m + 1] + e) * (1.0 / (2 * m + 1));
            });
        }
    } else {
        const double sT = rsqrt_nr(T), rT = sT * sT;
        F[0] = 0.88622692545275801365 * sT;  // sqrt(pi) / 2
        static_for<0, L>([&](auto I) {
            constexpr int m = decltype(I)::value;
            F[m + 1] = F[m] * ((2 * m + 1) * 0.5) * rT;
        });
    }
}

template <int L>
__device__ __forceinline__ void boys_f32(float T, const BoysTabs &bt, float (&F)[L + 1]) {
    if (T < 1e-3f || T > 30.0f) {
        double Fd[L + 1];
        boys_f64<L>((double)T, bt.tab, bt.etab, Fd);
        static_for<0, L + 1>([&](auto M) { F[M] = (float)Fd[M]; });
        return;
    }
    const int k = __float2int_rn(T * (float)kBoysInvStep);
    const float md = (float)k * (float)(1.0 / kBoysInvStep) - T;
    const float *row = bt.tabf + k * kBoysN + L;
    float f = row[5];
    f = row[4] + md * (1.0f / 5.0f) * f;
    f = row[3] + md * (1.0f / 4.0f) * f;
    f = row[2] + md * (1.0f / 3.0f) * f;
    f = row[1] + md * (1.0f / 2.0f) * f;
    f = row[0] + md * f;
    F[L] = f;
    if constexpr (L > 0) {
        float e = 1.0f + md * (1.0f / 5.0f);
        e = 1.0f + md * (1.0f / 4.0f) * e;
        e = 1.0f + md * (1.0f / 3.0f) * e;
        e = 1.0f + md * (1.0f / 2.0f) * e;
        e = 1.0f + md * e;
        e *= bt.etabf[k];
        const float t2 = 2.0f * T;
        static_for<0, L>([&](auto I) {
            constexpr int m = L - 1 - decltype(I)::value;
            F[m] = (t2 * F[m + 1] + e) * (1.0f / (2 * m + 1));
        });
    }
}

template <int L, typename Real>
__device__ __forceinline__ void boys_eval(Real T, const BoysTabs &bt, Real (&F)[L + 1]) {
    if constexpr (sizeof(Real) == 8)
        boys_f64t<L>(T, bt.tabt, bt.etab, F);
    else
        boys_f32<L>(T, bt, F);
}

template <typename Real> struct PrimPairOf;
template <> struct PrimPairOf<double> { using type = PrimPair; };
template <> struct PrimPairOf<float> { using type = PrimPairF; };
template <typename Real> using PrimPairT = typename PrimPairOf<Real>::type;

// ------------------------------------------------------------ class dims

template <int LA_, int LB_, int LC_, int LD_>
struct ClassDims {
    static constexpr int LA = LA_, LB = LB_, LC = LC_, LD = LD_;
    static constexpr int LAB = LA + LB, LCD = LC + LD, L = LAB + LCD;
    static constexpr int NE = cart_off(LAB + 1), NF = cart_off(LCD + 1);
    static constexpr int E0 = cart_off(LA), F0 = cart_off(LC);
    static constexpr int NEA = NE - E0, NFA = NF - F0;
    static constexpr int NA = ncart(LA), NB = ncart(LB), NC = ncart(LC), ND = ncart(LD);
    static constexpr int NAB = NA * NB, NCD = NC * ND;
    static constexpr int NOUT = NAB * NCD;
};

__host__ __device__ constexpr int cmax(int a, int b) { return a > b ? a : b; }

// Orientation of the vertical recursion.  (ab|cd) = (cd|ab), so the
// recursion may build the contracted [e0|f0] with the ket pair on the e side
// instead.  The e-side intermediates [e0|00]^(m) stay live through the whole
// ket recursion, so putting the pair of lower total momentum there shrinks
// the live set of one primitive quartet (e.g. (dd|ds): 262 -> 154 values,
// (dd|dp): 437 -> 343) with about the same number of steps.  Chosen per
// class from a count of live values and steps of both orders; classes with
// a ds bra on an s or p ket, and the small ones, keep the bra side.  Used by
// the primitive-lane kernels, whose registers hold one primitive quartet's
// recursion.
__host__ __device__ constexpr bool swap_vrr(int LA, int LB, int LC, int LD) {
    return (LA + LB) > (LC + LD) && (LA + LB + LC + LD) >= 3 && !(LA == 2 && LB == 0);
}

template <class Dm>
struct VrrOrient {
    static constexpr bool swap = swap_vrr(Dm::LA, Dm::LB, Dm::LC, Dm::LD);
};

// ---------------------------------------------------- primitive quartet
//
// [e0|f0] for la <= |e| <= la+lb, lc <= |f| <= lc+ld of one primitive
// quartet (Obara-Saika vertical recursion; the bra direction i is the first
// non-zero one of e + 1_i, the ket direction j the last non-zero one of
// f + 1_j):
//   bra VRR: [e+1_i|0]^(m) = PA_i [e]^(m) + WP_i [e]^(m+1)
//                           + e_i/(2p) ([e-1_i]^(m) - rho/p [e-1_i]^(m+1))
//   ket VRR: [e|f+1_j]^(m) = QC_j [e|f]^(m) + WQ_j [e|f]^(m+1)
//                           + f_j/(2q) ([e|f-1_j]^(m) - rho/q [e|f-1_j]^(m+1))
//                           + e_j/(2(p+q)) [e-1_j|f]^(m+1)
//   base:    [0|0]^(m) = 2 pi^{5/2} / (p q sqrt(p+q)) K_ab K_cd F_m(rho |PQ|^2)

// Depth-first order of the ket components |f| <= LCD:
// each f != 0 is built from its parent f - 1_j along its LAST non-zero
// direction j, and the components are visited in pre-order of that tree
// (px, dxx, dxy, dxz, py, dyy, dyz, pz, dzz for LCD = 2), so the
// intermediates of one branch die before the next branch starts.
__host__ __device__ constexpr int last_dir(const Cart c) { return c.z > 0 ? 2 : (c.y > 0 ? 1 : 0); }

template <int LCD>
struct KetDfs {
    static constexpr int NF = cart_off(LCD + 1);
    int seq[NF];   // visiting order
    int rank[NF];  // position of f among the output components (|f| >= LC) in that order
};

template <int LC, int LCD>
__host__ __device__ constexpr KetDfs<LCD> make_ket_dfs() {
    KetDfs<LCD> r{};
    int stack[KetDfs<LCD>::NF + 3] = {};
    int sp = 0, n = 0, nout = 0;
    stack[sp++] = 0;
    while (sp > 0) {
        const int f = stack[--sp];
        r.seq[n++] = f;
        const Cart c = cart_of(f);
        if (c.l() >= LC) r.rank[f] = nout++;
        if (c.l() < LCD)
            for (int j = 2; j >= last_dir(c); --j) stack[sp++] = c.plus(j).idx();
    }
    return r;
}

template <int LC, int LCD>
inline constexpr KetDfs<LCD> kKetDfs = make_ket_dfs<LC, LCD>();

// Second-level subtrees of the depth-first ket tree: f with |f| >= 2 is
// built from the |f| = 2 component holding its first two directions in the
// order x, y, z; groups xx xy xz yy yz zz = bits 0..5.  A |f| = 1 component
// (p_x, p_y, p_z) is the parent of the groups below it: bits 0-2, 3-4, 5.
__host__ __device__ constexpr int ket_dir_n(const Cart c, int k) {
    // k-th direction (0-based) of f listed as x...x y...y z...z
    return k < c.x ? 0 : (k < c.x + c.y ? 1 : 2);
}
__host__ __device__ constexpr int ket_group_mask(const Cart c) {
    if (c.l() == 0) return 63;
    const int d1 = ket_dir_n(c, 0);
    if (c.l() == 1) return d1 == 0 ? 7 : (d1 == 1 ? 24 : 32);
    const int d2 = ket_dir_n(c, 1);
    constexpr int base[3] = {0, 3, 5};
    return 1 << (base[d1] + d2 - d1);
}

// One primitive quartet: the recursions above with the ket components in
// the depth-first order; every output [e0|f0] (la <= |e| <= la+lb,
// lc <= |f| <= lc+ld) is handed to out(integral_constant<x>, value) as soon
// as it is final, in the order rank(f) * NEA + (e - E0), where
// x = (f - F0) * NEA + (e - E0).  AC = A - C (bra and ket anchor centres);
// P - Q = AC + PA - QC is exact zero when all four shells share one atom.
// SUB (a mask of the second-level groups above) restricts the ket recursion
// to some subtrees of the depth-first tree: a class may be evaluated in
// passes over disjoint group sets, each repeating the base and e-side
// recursion (and the |f| = 1 parents it needs), so that one pass's
// intermediates are dead before the next starts (fewer live values for the
// largest classes).  A component is emitted by the pass holding the lowest
// group below it, so with passes in increasing group order the outputs keep
// their depth-first order.  With PRE, the base values [00|00]^(m) come
// from pre[64 m] (written by prim_base for the same primitive quartet, so
// that passes share one Boys evaluation) instead of being evaluated here.
//
// prim_base: the base values [00|00]^(m) = 2 pi^{5/2} K_P K_Q /
// (p q sqrt(p+q)) F_m(T), m = 0..L, of one primitive quartet.
template <int L, typename Real>
__device__ __forceinline__ void prim_base(const PrimPairT<Real> &P, const PrimPairT<Real> &Q, const Real (&AC)[3],
                                          const BoysTabs &bt, Real (&V0)[L + 1]) {
    const Real p = P.p, q = Q.p;
    const Real spq = rsqrt_nr(p + q);
    const Real rho = p * q * (spq * spq);
    const Real PQx = AC[0] + (P.PAx - Q.PAx), PQy = AC[1] + (P.PAy - Q.PAy), PQz = AC[2] + (P.PAz - Q.PAz);
    const Real T = rho * (PQx * PQx + PQy * PQy + PQz * PQz);
    const Real pref = P.Kr * Q.Kr * spq;  // 2 pi^{5/2} K_P K_Q / (p q sqrt(p+q))
    Real F[L + 1];
    boys_eval<L, Real>(T, bt, F);
    static_for<0, L + 1>([&](auto M) { V0[decltype(M)::value] = pref * F[decltype(M)::value]; });
}

template <class Dm, typename Real, int SUB = 63, bool PRE = false, class Out>
__device__ __forceinline__ void prim_quartet(const PrimPairT<Real> &P, const PrimPairT<Real> &Q,
                                                 const Real (&AC)[3], const BoysTabs &bt, Out &&out,
                                                 const Real *pre = nullptr) {
    constexpr int L = Dm::L, NE = Dm::NE, NF = Dm::NF, LA = Dm::LA, LC = Dm::LC, LCD = Dm::LCD;
    const Real p = P.p, q = Q.p;
    const Real pq = p + q;
    const Real spq = rsqrt_nr(pq);
    const Real rpq = spq * spq;
    const Real PQx = AC[0] + (P.PAx - Q.PAx), PQy = AC[1] + (P.PAy - Q.PAy), PQz = AC[2] + (P.PAz - Q.PAz);

    Real V[NF][NE][L + 1];
    if constexpr (PRE) {
        // volatile: each pass reads its own copy, so the compiler does not
        // merge the passes' recursions into one long-lived set of values
        const volatile Real *pv = pre;
        static_for<0, L + 1>([&](auto M) { V[0][0][decltype(M)::value] = pv[64 * decltype(M)::value]; });
    } else {
        Real V0[L + 1];
        prim_base<L, Real>(P, Q, AC, bt, V0);
        static_for<0, L + 1>([&](auto M) { V[0][0][decltype(M)::value] = V0[decltype(M)::value]; });
    }

    if constexpr (Dm::LAB > 0) {
        const Real PA[3] = {P.PAx, P.PAy, P.PAz};
        const Real WP[3] = {-q * rpq * PQx, -q * rpq * PQy, -q * rpq * PQz};
        const Real oo2p = Real(0.5) * P.rp, rho_p = q * rpq;
        static_for<1, NE>([&](auto EI) {
            constexpr int e = decltype(EI)::value;
            constexpr Cart c = cart_of(e);
            constexpr int i = c.dir();
            constexpr int ei = c.get(i);
            constexpr int e1 = c.minus(i).idx();
            static_for<0, L - c.l() + 1>([&](auto MI) {
                constexpr int m = decltype(MI)::value;
                Real v = PA[i] * V[0][e1][m] + WP[i] * V[0][e1][m + 1];
                if constexpr (ei >= 2) {
                    constexpr int e2 = c.minus(i, 2).idx();
                    v += Real(ei - 1) * oo2p * (V[0][e2][m] - rho_p * V[0][e2][m + 1]);
                }
                V[0][e][m] = v;
            });
        });
    }
    auto emit_f = [&](auto FI) {
        constexpr int f = decltype(FI)::value;
        constexpr int gm = ket_group_mask(cart_of(f));
        constexpr bool mine = (SUB & (gm & -gm)) != 0;  // lowest group below f
        if constexpr (cart_of(f).l() >= LC && mine) {
            static_for<Dm::E0, NE>([&](auto EI) {
                constexpr int e = decltype(EI)::value;
                out(std::integral_constant<int, (f - Dm::F0) * Dm::NEA + (e - Dm::E0)>{}, V[f][e][0]);
            });
        }
    };
    if constexpr (LCD == 0) {
        emit_f(std::integral_constant<int, 0>{});
    } else {
        const Real QC[3] = {Q.PAx, Q.PAy, Q.PAz};
        const Real WQ[3] = {p * rpq * PQx, p * rpq * PQy, p * rpq * PQz};
        const Real oo2q = Real(0.5) * Q.rp, rho_q = p * rpq, oo2pq = Real(0.5) * rpq;
        static_for<0, NF>([&](auto SI) {
            constexpr int f = kKetDfs<LC, LCD>.seq[decltype(SI)::value];
            if constexpr (f > 0 && (SUB & ket_group_mask(cart_of(f))) != 0) {
                constexpr Cart cf = cart_of(f);
                constexpr int nf = cf.l();
                constexpr int j = last_dir(cf);
                constexpr int fj = cf.get(j);
                constexpr int f1 = cf.minus(j).idx();
                constexpr int emin = cart_off(cmax(0, LA - (LCD - nf)));
                static_for<emin, NE>([&](auto EI) {
                    constexpr int e = decltype(EI)::value;
                    constexpr Cart ce = cart_of(e);
                    constexpr int ej = ce.get(j);
                    static_for<0, L - ce.l() - nf + 1>([&](auto MI) {
                        constexpr int m = decltype(MI)::value;
                        Real v = QC[j] * V[f1][e][m] + WQ[j] * V[f1][e][m + 1];
                        if constexpr (fj >= 2) {
                            constexpr int f2 = cf.minus(j, 2).idx();
                            v += Real(fj - 1) * oo2q * (V[f2][e][m] - rho_q * V[f2][e][m + 1]);
                        }
                        if constexpr (ej >= 1) {
                            constexpr int e1 = ce.minus(j).idx();
                            v += Real(ej) * oo2pq * V[f1][e1][m + 1];
                        }
                        V[f][e][m] = v;
                    });
                });
            }
            emit_f(std::integral_constant<int, f>{});
        });
    }
}

// --------------------------------------------------------------- HRR
//
// (a, b+1_i| = (a+1_i, b| + AB_i (a, b|, applied to contracted integrals.
// X[e - off(la)] for la <= |e| <= la+lb  ->  Y[a][b], |a| = la, |b| = lb.

template <int LA, int LB, typename Real>
__device__ __forceinline__ void hrr_1(const Real (&X)[cart_off(LA + LB + 1) - cart_off(LA)],
                                      const Real AB[3], Real (&Y)[ncart(LA) * ncart(LB)]) {
    constexpr int LAB = LA + LB;
    constexpr int E0 = cart_off(LA), NE = cart_off(LAB + 1);
    if constexpr (LB == 0) {
        static_for<0, ncart(LA)>([&](auto I) { Y[decltype(I)::value] = X[decltype(I)::value]; });
    } else {
        Real T[cart_off(LB + 1)][NE];
        static_for<E0, NE>([&](auto EI) {
            constexpr int e = decltype(EI)::value;
            T[0][e] = X[e - E0];
        });
        static_for<1, cart_off(LB + 1)>([&](auto BI) {
            constexpr int b = decltype(BI)::value;
            constexpr Cart cb = cart_of(b);
            constexpr int k = cb.l();
            constexpr int i = cb.dir();
            constexpr int b1 = cb.minus(i).idx();
            static_for<E0, cart_off(LAB - k + 1)>([&](auto AI) {
                constexpr int a = decltype(AI)::value;
                constexpr int a1 = cart_of(a).plus(i).idx();
                T[b][a] = T[b1][a1] + AB[i] * T[b1][a];
            });
        });
        static_for<0, ncart(LA)>([&](auto AI) {
            static_for<0, ncart(LB)>([&](auto BI) {
                constexpr int a = decltype(AI)::value, b = decltype(BI)::value;
                Y[a * ncart(LB) + b] = T[cart_off(LB) + b][E0 + a];
            });
        });
    }
}

template <int L>
__device__ constexpr double comp_scale(int local) {
    return cart_is_mixed_d(cart_of(cart_off(L) + local)) ? kSqrt3 : 1.0;
}

// ------------------------------------------------- contracted quartet
//
// out[((a*NB + b)*NC + c)*ND + d] = (ab|cd) for normalised Cartesian
// components a, b, c, d of the bra pair's shells (sa, sb) and the ket
// pair's shells (sc, sd).

template <class Dm, typename Real>
__device__ __forceinline__ void eri_quartet(const PairInfo &bra, const PairInfo &ket,
                                            const PrimPairT<Real> *__restrict__ pp, const BoysTabs &bt,
                                            Real (&out)[Dm::NOUT]) {
    // acc[f - F0][e - E0] = contracted [e0|f0], e on the bra side.  The
    // per-lane kernels keep the bra on the e side in every class: their
    // registers go mostly to the contracted intermediates, and the swapped
    // order has more steps where it has fewer live values (measured slower
    // for (dd|ps), (dp|ps)).
    Real acc[Dm::NFA][Dm::NEA];
    static_for<0, Dm::NFA>([&](auto F) {
        static_for<0, Dm::NEA>([&](auto E) { acc[decltype(F)::value][decltype(E)::value] = Real(0); });
    });
    const Real AC[3] = {Real(bra.Ax - ket.Ax), Real(bra.Ay - ket.Ay), Real(bra.Az - ket.Az)};
    // Lanes of a wave take consecutive quartets of one bra row: the ket's
    // primitive pairs (different for every lane) are read once each, the
    // bra's (the same for the wave) in the inner loop.  When every active
    // lane has the same bra pair (the usual case), its primitive pairs are
    // read once for the wave through the scalar cache.
    auto add = [&](auto X, Real v) {
        constexpr int x = decltype(X)::value;
        acc[x / Dm::NEA][x % Dm::NEA] += v;
    };
    const int pbu = __builtin_amdgcn_readfirstlane(bra.pp0);
    if (__all(bra.pp0 == pbu)) {
        const int nbu = __builtin_amdgcn_readfirstlane(bra.npp);
        const PrimPairT<Real> *__restrict__ pb = pp + pbu;
        for (int ik = 0; ik < ket.npp; ++ik) {
            const PrimPairT<Real> Q = pp[ket.pp0 + ik];
            for (int ib = 0; ib < nbu; ++ib) prim_quartet<Dm, Real>(pb[ib], Q, AC, bt, add);
        }
    } else {
        for (int ik = 0; ik < ket.npp; ++ik) {
            const PrimPairT<Real> Q = pp[ket.pp0 + ik];
            for (int ib = 0; ib < bra.npp; ++ib) prim_quartet<Dm, Real>(pp[bra.pp0 + ib], Q, AC, bt, add);
        }
    }
    // bra HRR for every ket index f
    const Real AB[3] = {Real(bra.ABx), Real(bra.ABy), Real(bra.ABz)};
    const Real CD[3] = {Real(ket.ABx), Real(ket.ABy), Real(ket.ABz)};
    Real Y[Dm::NFA][Dm::NAB];
    static_for<0, Dm::NFA>([&](auto F) {
        constexpr int f = decltype(F)::value;
        hrr_1<Dm::LA, Dm::LB, Real>(acc[f], AB, Y[f]);
    });
    // ket HRR for every bra (a, b)
    static_for<0, Dm::NAB>([&](auto AB_) {
        constexpr int ab = decltype(AB_)::value;
        Real Xk[Dm::NFA];
        static_for<0, Dm::NFA>([&](auto F) { Xk[decltype(F)::value] = Y[decltype(F)::value][ab]; });
        Real Yk[Dm::NCD];
        hrr_1<Dm::LC, Dm::LD, Real>(Xk, CD, Yk);
        constexpr int a = ab / Dm::NB, b = ab % Dm::NB;
        constexpr double sab = comp_scale<Dm::LA>(a) * comp_scale<Dm::LB>(b);
        static_for<0, Dm::NCD>([&](auto CD_) {
            constexpr int cd = decltype(CD_)::value;
            constexpr int c = cd / Dm::ND, d = cd % Dm::ND;
            constexpr double s = sab * comp_scale<Dm::LC>(c) * comp_scale<Dm::LD>(d);
            if constexpr (s == 1.0)
                out[ab * Dm::NCD + cd] = Yk[cd];
            else
                out[ab * Dm::NCD + cd] = Yk[cd] * Real(s);
        });
    });
}

template <class Dm>
__device__ __forceinline__ void eri_quartet_f64(const PairInfo &bra, const PairInfo &ket,
                                                const PrimPair *__restrict__ pp, const BoysTabs &bt,
                                                double (&out)[Dm::NOUT]) {
    eri_quartet<Dm, double>(bra, ket, pp, bt, out);
}

}  // namespace mess
