// Shell-quartet kernels: Schwarz factors, dense ERI store, direct J/K.
// One lane per shell quartet; quartets of one angular class per launch.
#pragma once

#include "eri_hgp.hpp"

namespace mess {

template <int CB, int CK>
using ClassOf = ClassDims<pair_class_la(CB), pair_class_lb(CB), pair_class_la(CK), pair_class_lb(CK)>;

// Row of thread t in a ragged work list: largest i with rowstart[i] <= t.
__device__ __forceinline__ int find_row(const int64_t *__restrict__ rowstart, int nbra, int64_t t) {
    int lo = 0, hi = nbra;
    while (hi - lo > 1) {
        const int mid = (lo + hi) >> 1;
        if (rowstart[mid] <= t) lo = mid; else hi = mid;
    }
    return lo;
}

// (bra, ket) pair indices, relative to their classes, of quartet t.
__device__ __forceinline__ int2 quartet_pairs(const int64_t *__restrict__ rowstart, const int2 *__restrict__ rowmap,
                                              int nrow, int64_t t) {
    const int r = find_row(rowstart, nrow, t);
    const int2 m = rowmap[r];
    return make_int2(m.x, m.y + static_cast<int>(t - rowstart[r]));
}

// Q = sqrt(max_{a in sa, b in sb} |(ab|ab)|) for every pair of one class.
template <class Dm>
__global__ void __launch_bounds__(64) k_schwarz(const PairInfo *__restrict__ pairs, int off, int n,
                                                const PrimPair *__restrict__ pp, BoysTabs bt,
                                                double *__restrict__ Q) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const PairInfo pr = pairs[off + i];
    double out[Dm::NOUT];
    eri_quartet_f64<Dm>(pr, pr, pp, bt, out);
    double m = 0.0;
    static_for<0, Dm::NAB>([&](auto I) {
        constexpr int ab = decltype(I)::value;
        m = fmax(m, fabs(out[ab * Dm::NCD + ab]));
    });
    Q[off + i] = sqrt(m);
}

// Dense N^4 store: every unique quartet writes its block to all eight
// index permutations.
template <class Dm, typename Real>
__global__ void __launch_bounds__(128) k_eri_dense(const PairInfo *__restrict__ pairs, int bra_off,
                                                   int ket_off, int nbra,
                                                   const int64_t *__restrict__ rowstart, const int2 *__restrict__ rowmap,
                                                   const PrimPairT<Real> *__restrict__ pp, BoysTabs bt,
                                                   int64_t N, double *__restrict__ eri) {
    const int64_t total = rowstart[nbra];
    for (int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; t < total;
         t += (int64_t)gridDim.x * blockDim.x) {
        const int2 ij = quartet_pairs(rowstart, rowmap, nbra, t);
        const int i = ij.x, j = ij.y;
        const PairInfo bra = pairs[bra_off + i];
        const PairInfo ket = pairs[ket_off + j];
        Real out[Dm::NOUT];
        eri_quartet<Dm, Real>(bra, ket, pp, bt, out);
        static_for<0, Dm::NOUT>([&](auto I) {
            constexpr int k = decltype(I)::value;
            constexpr int a = k / (Dm::NB * Dm::NCD), b = (k / Dm::NCD) % Dm::NB;
            constexpr int c = (k / Dm::ND) % Dm::NC, d = k % Dm::ND;
            const int64_t ia = bra.bfa + a, ib = bra.bfb + b, ic = ket.bfa + c, id = ket.bfb + d;
            const double v = (double)out[k];
            eri[((ia * N + ib) * N + ic) * N + id] = v;
            eri[((ib * N + ia) * N + ic) * N + id] = v;
            eri[((ia * N + ib) * N + id) * N + ic] = v;
            eri[((ib * N + ia) * N + id) * N + ic] = v;
            eri[((ic * N + id) * N + ia) * N + ib] = v;
            eri[((id * N + ic) * N + ia) * N + ib] = v;
            eri[((ic * N + id) * N + ib) * N + ia] = v;
            eri[((id * N + ic) * N + ib) * N + ia] = v;
        });
    }
}

// Stored layout of one class: element k of quartet t at base[k * nq + t]
// (structure of arrays, so that consecutive lanes touch consecutive words).
template <class Dm, typename Real>
__global__ void __launch_bounds__(128) k_eri_store(const PairInfo *__restrict__ pairs, int bra_off, int ket_off,
                                                   int nbra, const int64_t *__restrict__ rowstart, const int2 *__restrict__ rowmap,
                                                   const PrimPairT<Real> *__restrict__ pp, BoysTabs bt,
                                                   Real *__restrict__ base) {
    const int64_t total = rowstart[nbra];
    for (int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; t < total;
         t += (int64_t)gridDim.x * blockDim.x) {
        const int2 ij = quartet_pairs(rowstart, rowmap, nbra, t);
        const int i = ij.x, j = ij.y;
        const PairInfo bra = pairs[bra_off + i];
        const PairInfo ket = pairs[ket_off + j];
        Real out[Dm::NOUT];
        eri_quartet<Dm, Real>(bra, ket, pp, bt, out);
        static_for<0, Dm::NOUT>([&](auto I) { base[(int64_t)decltype(I)::value * total + t] = out[I]; });
    }
}

// Digest one unique quartet block into the half-matrices Gj, Gk
// (J = Gj + Gj^T, K = Gk + Gk^T).  With v' = v / ((1+d_ab)(1+d_cd)(1+d_ab,cd)):
//   Gj[a,b] += 2 v' D[c,d]      Gj[c,d] += 2 v' D[a,b]
//   Gk[a,c] += v' D[b,d]        Gk[b,c] += v' D[a,d]
//   Gk[a,d] += v' D[b,c]        Gk[b,d] += v' D[a,c]
// which is the sum of the eight permutation updates of (ab|cd).
// The partial sums run in the integrals' arithmetic (Real) and are added to
// the FP64 half-matrices.
template <class Dm, typename Real>
__device__ __forceinline__ void digest_jk(const Real (&out)[Dm::NOUT], double fac, int a0, int b0,
                                          int c0, int d0, const double *__restrict__ D, int N,
                                          double *__restrict__ Gj, double *__restrict__ Gk) {
    constexpr int NA = Dm::NA, NB = Dm::NB, NC = Dm::NC, ND = Dm::ND;
    auto O = [&](int a, int b, int c, int d) -> Real { return out[((a * NB + b) * NC + c) * ND + d]; };
    auto Dv = [&](int r, int c) -> Real { return Real(D[(int64_t)r * N + c]); };
    if (Gj) {
        Real Dcd[NC][ND], Dab[NA][NB];
        static_for<0, NC>([&](auto C) { static_for<0, ND>([&](auto Dd) {
            Dcd[C][Dd] = Dv(c0 + C, d0 + Dd); }); });
        static_for<0, NA>([&](auto A) { static_for<0, NB>([&](auto B) {
            Dab[A][B] = Dv(a0 + A, b0 + B); }); });
        static_for<0, NA>([&](auto A) { static_for<0, NB>([&](auto B) {
            Real s = Real(0);
            static_for<0, NC>([&](auto C) { static_for<0, ND>([&](auto Dd) {
                s += O(A, B, C, Dd) * Dcd[C][Dd]; }); });
            unsafeAtomicAdd(&Gj[(int64_t)(a0 + A) * N + b0 + B], 2.0 * fac * (double)s);
        }); });
        static_for<0, NC>([&](auto C) { static_for<0, ND>([&](auto Dd) {
            Real s = Real(0);
            static_for<0, NA>([&](auto A) { static_for<0, NB>([&](auto B) {
                s += O(A, B, C, Dd) * Dab[A][B]; }); });
            unsafeAtomicAdd(&Gj[(int64_t)(c0 + C) * N + d0 + Dd], 2.0 * fac * (double)s);
        }); });
    }
    if (Gk) {
        Real Dbd[NB][ND], Dad[NA][ND], Dbc[NB][NC], Dac[NA][NC];
        static_for<0, NB>([&](auto B) { static_for<0, ND>([&](auto Dd) { Dbd[B][Dd] = Dv(b0 + B, d0 + Dd); }); });
        static_for<0, NA>([&](auto A) { static_for<0, ND>([&](auto Dd) { Dad[A][Dd] = Dv(a0 + A, d0 + Dd); }); });
        static_for<0, NB>([&](auto B) { static_for<0, NC>([&](auto C) { Dbc[B][C] = Dv(b0 + B, c0 + C); }); });
        static_for<0, NA>([&](auto A) { static_for<0, NC>([&](auto C) { Dac[A][C] = Dv(a0 + A, c0 + C); }); });
        static_for<0, NA>([&](auto A) { static_for<0, NC>([&](auto C) {
            Real s = Real(0);
            static_for<0, NB>([&](auto B) { static_for<0, ND>([&](auto Dd) { s += O(A, B, C, Dd) * Dbd[B][Dd]; }); });
            unsafeAtomicAdd(&Gk[(int64_t)(a0 + A) * N + c0 + C], fac * (double)s);
        }); });
        static_for<0, NB>([&](auto B) { static_for<0, NC>([&](auto C) {
            Real s = Real(0);
            static_for<0, NA>([&](auto A) { static_for<0, ND>([&](auto Dd) { s += O(A, B, C, Dd) * Dad[A][Dd]; }); });
            unsafeAtomicAdd(&Gk[(int64_t)(b0 + B) * N + c0 + C], fac * (double)s);
        }); });
        static_for<0, NA>([&](auto A) { static_for<0, ND>([&](auto Dd) {
            Real s = Real(0);
            static_for<0, NB>([&](auto B) { static_for<0, NC>([&](auto C) { s += O(A, B, C, Dd) * Dbc[B][C]; }); });
            unsafeAtomicAdd(&Gk[(int64_t)(a0 + A) * N + d0 + Dd], fac * (double)s);
        }); });
        static_for<0, NB>([&](auto B) { static_for<0, ND>([&](auto Dd) {
            Real s = Real(0);
            static_for<0, NA>([&](auto A) { static_for<0, NC>([&](auto C) { s += O(A, B, C, Dd) * Dac[A][C]; }); });
            unsafeAtomicAdd(&Gk[(int64_t)(b0 + B) * N + d0 + Dd], fac * (double)s);
        }); });
    }
}

template <class Dm, typename Real>
__global__ void __launch_bounds__(128) k_jk_direct(const PairInfo *__restrict__ pairs, int bra_off,
                                                   int ket_off, int nbra, int same_class,
                                                   const int64_t *__restrict__ rowstart, const int2 *__restrict__ rowmap,
                                                   const PrimPairT<Real> *__restrict__ pp, BoysTabs bt,
                                                   const double *__restrict__ D, int N,
                                                   double *__restrict__ Gj, double *__restrict__ Gk) {
    const int64_t total = rowstart[nbra];
    for (int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; t < total;
         t += (int64_t)gridDim.x * blockDim.x) {
        const int2 ij = quartet_pairs(rowstart, rowmap, nbra, t);
        const int i = ij.x, j = ij.y;
        const PairInfo bra = pairs[bra_off + i];
        const PairInfo ket = pairs[ket_off + j];
        Real out[Dm::NOUT];
        eri_quartet<Dm, Real>(bra, ket, pp, bt, out);
        double fac = 1.0;
        if (bra.sa == bra.sb) fac *= 0.5;
        if (ket.sa == ket.sb) fac *= 0.5;
        if (same_class && i == j) fac *= 0.5;
        digest_jk<Dm, Real>(out, fac, bra.bfa, bra.bfb, ket.bfa, ket.bfb, D + bra.moff, bra.mN,
                            Gj ? Gj + bra.moff : nullptr, Gk ? Gk + bra.moff : nullptr);
    }
}

// J/K from stored blocks: one lane per quartet streams its NOUT values.
template <class Dm, typename Real>
__global__ void __launch_bounds__(128) k_jk_stored(const PairInfo *__restrict__ pairs, int bra_off, int ket_off,
                                                   int nbra, int same_class, const int64_t *__restrict__ rowstart, const int2 *__restrict__ rowmap,
                                                   const Real *__restrict__ base, const double *__restrict__ D,
                                                   int N, double *__restrict__ Gj, double *__restrict__ Gk) {
    const int64_t total = rowstart[nbra];
    for (int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; t < total;
         t += (int64_t)gridDim.x * blockDim.x) {
        const int2 ij = quartet_pairs(rowstart, rowmap, nbra, t);
        const int i = ij.x, j = ij.y;
        const PairInfo bra = pairs[bra_off + i];
        const PairInfo ket = pairs[ket_off + j];
        Real out[Dm::NOUT];
        static_for<0, Dm::NOUT>([&](auto I) { out[I] = base[(int64_t)decltype(I)::value * total + t]; });
        double fac = 1.0;
        if (bra.sa == bra.sb) fac *= 0.5;
        if (ket.sa == ket.sb) fac *= 0.5;
        if (same_class && i == j) fac *= 0.5;
        digest_jk<Dm, Real>(out, fac, bra.bfa, bra.bfb, ket.bfa, ket.bfb, D + bra.moff, bra.mN,
                            Gj ? Gj + bra.moff : nullptr, Gk ? Gk + bra.moff : nullptr);
    }
}

// J/K by bra segments: one 256-thread block per segment of one bra's
// quartets (at most kSegLen sharing the bra pair (ab)).  Every
// exchange family and J[a,b] index rows of the bra pair's functions, so they
// are accumulated in LDS (K rows of a and b, NA + NB rows of the molecule's
// N columns) and in registers (J[a,b], reduced over the wave), and flushed
// to the half-matrices once per segment; only J[c,d] goes to global memory
// per quartet.  This cuts the FP64 global atomics, which bound the
// streaming digestion and much of the direct one for the low classes, by a
// factor of up to six.  DIRECT: each quartet's block is computed by the
// recursion instead of read from the store (base unused).
template <class Dm, typename Real, bool DIRECT = false>
__global__ void __launch_bounds__(256) k_jk_rows(const PairInfo *__restrict__ pairs, int bra_off, int ket_off,
                                                        int same_class, const int64_t *__restrict__ rowstart,
                                                        const int2 *__restrict__ rowmap, const int4 *__restrict__ segs,
                                                        int nseg, const Real *__restrict__ base, int64_t total,
                                                        const double *__restrict__ Dall, double *__restrict__ Gjall,
                                                        double *__restrict__ Gkall,
                                                        const PrimPairT<Real> *__restrict__ pp = nullptr,
                                                        BoysTabs bt = BoysTabs{}) {
    constexpr int NA = Dm::NA, NB = Dm::NB, NC = Dm::NC, ND = Dm::ND;
    extern __shared__ double lds[];
    for (int sidx = blockIdx.x; sidx < nseg; sidx += gridDim.x) {
        const int4 sg = segs[sidx];
        const int i = rowmap[sg.x].x;
        const PairInfo bra = pairs[bra_off + i];
        const int N = bra.mN, a0 = bra.bfa, b0 = bra.bfb;
        const double *D = Dall + bra.moff;
        double *Gj = Gjall ? Gjall + bra.moff : nullptr;
        double *Gk = Gkall ? Gkall + bra.moff : nullptr;
        double *Ka = lds, *Kb = lds + NA * N, *Jab = lds + (NA + NB) * N;
        const int nl = (NA + NB) * N + NA * NB;
        for (int e = threadIdx.x; e < nl; e += 256) lds[e] = 0.0;
        __syncthreads();
        auto Dv = [&](int r, int c) -> Real { return Real(D[(int64_t)r * N + c]); };
        Real Dab[NA][NB];
        static_for<0, NA>([&](auto A) { static_for<0, NB>([&](auto B) { Dab[A][B] = Dv(a0 + A, b0 + B); }); });
        Real jab[NA][NB];
        static_for<0, NA>([&](auto A) { static_for<0, NB>([&](auto B) { jab[A][B] = Real(0); }); });
        int r = sg.x;  // row of this thread's quartet q (rows of one bra, in order)
        for (int64_t q = sg.y + threadIdx.x; q < sg.z; q += 256) {
            while (r + 1 < sg.w && rowstart[r + 1] <= q) ++r;
            const int j = rowmap[r].y + (int)(q - rowstart[r]);
            const PairInfo ket = pairs[ket_off + j];
            const int c0 = ket.bfa, d0 = ket.bfb;
            Real out[Dm::NOUT];
            if constexpr (DIRECT)
                eri_quartet<Dm, Real>(bra, ket, pp, bt, out);
            else
                static_for<0, Dm::NOUT>([&](auto I) { out[I] = base[(int64_t)decltype(I)::value * total + q]; });
            double fac = 1.0;
            if (bra.sa == bra.sb) fac *= 0.5;
            if (ket.sa == ket.sb) fac *= 0.5;
            if (same_class && i == j) fac *= 0.5;
            auto O = [&](int a, int b, int c, int d) -> Real { return out[((a * NB + b) * NC + c) * ND + d]; };
            if (Gj) {
                Real Dcd[NC][ND];
                static_for<0, NC>([&](auto C) { static_for<0, ND>([&](auto Dd) { Dcd[C][Dd] = Dv(c0 + C, d0 + Dd); }); });
                static_for<0, NA>([&](auto A) { static_for<0, NB>([&](auto B) {
                    Real s = Real(0);
                    static_for<0, NC>([&](auto C) { static_for<0, ND>([&](auto Dd) { s += O(A, B, C, Dd) * Dcd[C][Dd]; }); });
                    jab[A][B] += Real(fac) * s;
                }); });
                static_for<0, NC>([&](auto C) { static_for<0, ND>([&](auto Dd) {
                    Real s = Real(0);
                    static_for<0, NA>([&](auto A) { static_for<0, NB>([&](auto B) { s += O(A, B, C, Dd) * Dab[A][B]; }); });
                    unsafeAtomicAdd(&Gj[(int64_t)(c0 + C) * N + d0 + Dd], 2.0 * fac * (double)s);
                }); });
            }
            if (Gk) {
                Real Dbd[NB][ND], Dad[NA][ND], Dbc[NB][NC], Dac[NA][NC];
                static_for<0, NB>([&](auto B) { static_for<0, ND>([&](auto Dd) { Dbd[B][Dd] = Dv(b0 + B, d0 + Dd); }); });
                static_for<0, NA>([&](auto A) { static_for<0, ND>([&](auto Dd) { Dad[A][Dd] = Dv(a0 + A, d0 + Dd); }); });
                static_for<0, NB>([&](auto B) { static_for<0, NC>([&](auto C) { Dbc[B][C] = Dv(b0 + B, c0 + C); }); });
                static_for<0, NA>([&](auto A) { static_for<0, NC>([&](auto C) { Dac[A][C] = Dv(a0 + A, c0 + C); }); });
                static_for<0, NA>([&](auto A) { static_for<0, NC>([&](auto C) {
                    Real s = Real(0);
                    static_for<0, NB>([&](auto B) { static_for<0, ND>([&](auto Dd) { s += O(A, B, C, Dd) * Dbd[B][Dd]; }); });
                    __hip_atomic_fetch_add(&Ka[A * N + c0 + C], fac * (double)s, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
                }); });
                static_for<0, NB>([&](auto B) { static_for<0, NC>([&](auto C) {
                    Real s = Real(0);
                    static_for<0, NA>([&](auto A) { static_for<0, ND>([&](auto Dd) { s += O(A, B, C, Dd) * Dad[A][Dd]; }); });
                    __hip_atomic_fetch_add(&Kb[B * N + c0 + C], fac * (double)s, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
                }); });
                static_for<0, NA>([&](auto A) { static_for<0, ND>([&](auto Dd) {
                    Real s = Real(0);
                    static_for<0, NB>([&](auto B) { static_for<0, NC>([&](auto C) { s += O(A, B, C, Dd) * Dbc[B][C]; }); });
                    __hip_atomic_fetch_add(&Ka[A * N + d0 + Dd], fac * (double)s, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
                }); });
                static_for<0, NB>([&](auto B) { static_for<0, ND>([&](auto Dd) {
                    Real s = Real(0);
                    static_for<0, NA>([&](auto A) { static_for<0, NC>([&](auto C) { s += O(A, B, C, Dd) * Dac[A][C]; }); });
                    __hip_atomic_fetch_add(&Kb[B * N + d0 + Dd], fac * (double)s, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
                }); });
            }
        }
        if (Gj) {
            // J[a,b]: sum over the wave, then the waves' sums in LDS
            static_for<0, NA>([&](auto A) { static_for<0, NB>([&](auto B) {
                double v = (double)jab[A][B];
                for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
                if ((threadIdx.x & 63) == 0)
                    __hip_atomic_fetch_add(&Jab[A * NB + B], v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
            }); });
        }
        __syncthreads();
        if (Gk)
            for (int e = threadIdx.x; e < (NA + NB) * N; e += 256) {
                const double v = lds[e];
                if (v == 0.0) continue;
                const int row = e < NA * N ? a0 + e / N : b0 + (e - NA * N) / N;
                unsafeAtomicAdd(&Gk[(int64_t)row * N + e % N], v);
            }
        if (Gj)
            for (int e = threadIdx.x; e < NA * NB; e += 256)
                unsafeAtomicAdd(&Gj[(int64_t)(a0 + e / NB) * N + b0 + e % NB], 2.0 * Jab[e]);
        __syncthreads();  // LDS reused by the next segment
    }
}

// J/K from stored blocks by groups of G consecutive bras of one molecule
// (sorted neighbours: similar primitive counts and Schwarz factors, so their
// ket prefixes nearly coincide).  A group's quartets are laid out as tiles,
// one per ket bucket, each a G x (longest row) rectangle whose rows are the
// bras' work-list rows; one 256-thread block takes a group, a thread a ket
// of a tile, and the thread loops over the G bras.  Every sum that indexes
// a ket alone (J[c,d]) is then reduced over the G bras in registers before
// its one global atomic; sums of a bra (J[a,b]) stay in registers for the
// whole group, the exchange rows of the G bras' functions in LDS (flushed
// once per group).  The ket's pair record and density block are read once
// per G quartets.  Store reads stay coalesced: consecutive threads take
// consecutive kets of one row.
template <class Dm, typename Real, int G>
__global__ void __launch_bounds__(256) k_jk_group(const PairInfo *__restrict__ pairs, int bra_off, int ket_off,
                                                  int same_class, const int64_t *__restrict__ rowstart,
                                                  const int4 *__restrict__ groups, int ngroups,
                                                  const int4 *__restrict__ tiles, const int *__restrict__ grows,
                                                  const Real *__restrict__ base, int64_t total,
                                                  const double *__restrict__ Dall, double *__restrict__ Gjall,
                                                  double *__restrict__ Gkall) {
    constexpr int NA = Dm::NA, NB = Dm::NB, NC = Dm::NC, ND = Dm::ND, NR = NA + NB;
    extern __shared__ double lds[];
    for (int gi = blockIdx.x; gi < ngroups; gi += gridDim.x) {
        const int4 gr = groups[gi];
        const int ng = gr.w;
        const PairInfo first = pairs[bra_off + gr.z];
        const int N = first.mN;
        const double *D = Dall + first.moff;
        double *Gj = Gjall ? Gjall + first.moff : nullptr;
        double *Gk = Gkall ? Gkall + first.moff : nullptr;
        // LDS: exchange rows of bra g (its a functions, then its b
        // functions) at (g NR + row) N, J[a,b] of the bras after them, then
        // the function index of every row slot
        double *Jab = lds + G * NR * N;
        int *rowfn = reinterpret_cast<int *>(Jab + G * NA * NB);
        for (int e = threadIdx.x; e < G * NR * N + G * NA * NB; e += 256) lds[e] = 0.0;
        int a0[G], b0[G], bi[G];
        Real fb[G], Dab[G][NA][NB], jab[G][NA][NB];
        static_for<0, G>([&](auto Gi) {
            constexpr int g = decltype(Gi)::value;
            const bool on = g < ng;
            const PairInfo p = pairs[bra_off + gr.z + (on ? g : 0)];
            a0[g] = p.bfa;
            b0[g] = p.bfb;
            bi[g] = on ? gr.z + g : -1;
            fb[g] = on ? (p.sa == p.sb ? Real(0.5) : Real(1)) : Real(0);
            static_for<0, NA>([&](auto A) { static_for<0, NB>([&](auto B) {
                Dab[g][A][B] = Real(D[(int64_t)(a0[g] + A) * N + b0[g] + B]);
                jab[g][A][B] = Real(0);
            }); });
            if ((int)threadIdx.x < NR) rowfn[g * NR + threadIdx.x] = threadIdx.x < NA ? a0[g] + threadIdx.x : b0[g] + threadIdx.x - NA;
        });
        __syncthreads();
        const int4 lt = tiles[gr.y - 1];
        const int nk = lt.w + lt.z;
        int t = gr.x;
        int4 tl = tiles[t];
        int64_t rs[G];
        int cnt[G];
        auto load_tile = [&]() {
            static_for<0, G>([&](auto Gi) {
                constexpr int g = decltype(Gi)::value;
                const int r = grows[tl.x + g];
                rs[g] = r >= 0 ? rowstart[r] : 0;
                cnt[g] = r >= 0 ? (int)(rowstart[r + 1] - rs[g]) : 0;
            });
        };
        load_tile();
        for (int idx = threadIdx.x; idx < nk; idx += 256) {
            if (t + 1 < gr.y && tiles[t + 1].w <= idx) {
                do ++t; while (t + 1 < gr.y && tiles[t + 1].w <= idx);
                tl = tiles[t];
                load_tile();
            }
            const int k = idx - tl.w;
            const int j = tl.y + k;
            const PairInfo ket = pairs[ket_off + j];
            const int c0 = ket.bfa, d0 = ket.bfb;
            const Real fk = ket.sa == ket.sb ? Real(0.5) : Real(1);
            Real Dcd[NC][ND], jcd[NC][ND];
            static_for<0, NC>([&](auto C) { static_for<0, ND>([&](auto Dd) {
                Dcd[C][Dd] = Real(D[(int64_t)(c0 + C) * N + d0 + Dd]);
                jcd[C][Dd] = Real(0);
            }); });
            static_for<0, G>([&](auto Gi) {
                constexpr int g = decltype(Gi)::value;
                if (k < cnt[g]) {
                    const int64_t q = rs[g] + k;
                    Real out[Dm::NOUT];
                    static_for<0, Dm::NOUT>([&](auto I) { out[I] = base[(int64_t)decltype(I)::value * total + q]; });
                    Real fac = fb[g] * fk;
                    if (same_class && bi[g] == j) fac *= Real(0.5);
                    auto O = [&](int a, int b, int c, int d) -> Real { return out[((a * NB + b) * NC + c) * ND + d]; };
                    if (Gj) {
                        static_for<0, NA>([&](auto A) { static_for<0, NB>([&](auto B) {
                            Real s = Real(0);
                            static_for<0, NC>([&](auto C) { static_for<0, ND>([&](auto Dd) { s += O(A, B, C, Dd) * Dcd[C][Dd]; }); });
                            jab[g][A][B] += fac * s;
                        }); });
                        static_for<0, NC>([&](auto C) { static_for<0, ND>([&](auto Dd) {
                            Real s = Real(0);
                            static_for<0, NA>([&](auto A) { static_for<0, NB>([&](auto B) { s += O(A, B, C, Dd) * Dab[g][A][B]; }); });
                            jcd[C][Dd] += fac * s;
                        }); });
                    }
                    if (Gk) {
                        auto Dv = [&](int r, int c) -> Real { return Real(D[(int64_t)r * N + c]); };
                        double *Ka = lds + g * NR * N, *Kb = Ka + NA * N;
                        Real Dbd[NB][ND], Dad[NA][ND], Dbc[NB][NC], Dac[NA][NC];
                        static_for<0, NB>([&](auto B) { static_for<0, ND>([&](auto Dd) { Dbd[B][Dd] = Dv(b0[g] + B, d0 + Dd); }); });
                        static_for<0, NA>([&](auto A) { static_for<0, ND>([&](auto Dd) { Dad[A][Dd] = Dv(a0[g] + A, d0 + Dd); }); });
                        static_for<0, NB>([&](auto B) { static_for<0, NC>([&](auto C) { Dbc[B][C] = Dv(b0[g] + B, c0 + C); }); });
                        static_for<0, NA>([&](auto A) { static_for<0, NC>([&](auto C) { Dac[A][C] = Dv(a0[g] + A, c0 + C); }); });
                        static_for<0, NA>([&](auto A) { static_for<0, NC>([&](auto C) {
                            Real s = Real(0);
                            static_for<0, NB>([&](auto B) { static_for<0, ND>([&](auto Dd) { s += O(A, B, C, Dd) * Dbd[B][Dd]; }); });
                            __hip_atomic_fetch_add(&Ka[A * N + c0 + C], (double)(fac * s), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
                        }); });
                        static_for<0, NB>([&](auto B) { static_for<0, NC>([&](auto C) {
                            Real s = Real(0);
                            static_for<0, NA>([&](auto A) { static_for<0, ND>([&](auto Dd) { s += O(A, B, C, Dd) * Dad[A][Dd]; }); });
                            __hip_atomic_fetch_add(&Kb[B * N + c0 + C], (double)(fac * s), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
                        }); });
                        static_for<0, NA>([&](auto A) { static_for<0, ND>([&](auto Dd) {
                            Real s = Real(0);
                            static_for<0, NB>([&](auto B) { static_for<0, NC>([&](auto C) { s += O(A, B, C, Dd) * Dbc[B][C]; }); });
                            __hip_atomic_fetch_add(&Ka[A * N + d0 + Dd], (double)(fac * s), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
                        }); });
                        static_for<0, NB>([&](auto B) { static_for<0, ND>([&](auto Dd) {
                            Real s = Real(0);
                            static_for<0, NA>([&](auto A) { static_for<0, NC>([&](auto C) { s += O(A, B, C, Dd) * Dac[A][C]; }); });
                            __hip_atomic_fetch_add(&Kb[B * N + d0 + Dd], (double)(fac * s), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
                        }); });
                    }
                }
            });
            if (Gj)
                static_for<0, NC>([&](auto C) { static_for<0, ND>([&](auto Dd) {
                    if (jcd[C][Dd] != Real(0)) unsafeAtomicAdd(&Gj[(int64_t)(c0 + C) * N + d0 + Dd], 2.0 * (double)jcd[C][Dd]);
                }); });
        }
        if (Gj)
            static_for<0, G>([&](auto Gi) {
                constexpr int g = decltype(Gi)::value;
                static_for<0, NA>([&](auto A) { static_for<0, NB>([&](auto B) {
                    double v = (double)jab[g][A][B];
                    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
                    if ((threadIdx.x & 63) == 0)
                        __hip_atomic_fetch_add(&Jab[(g * NA + A) * NB + B], v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
                }); });
            });
        __syncthreads();
        if (Gk)
            for (int e = threadIdx.x; e < ng * NR * N; e += 256) {
                const double v = lds[e];
                if (v != 0.0) unsafeAtomicAdd(&Gk[(int64_t)rowfn[e / N] * N + e % N], v);
            }
        if (Gj)
            for (int e = threadIdx.x; e < ng * NA * NB; e += 256) {
                const int g = e / (NA * NB), ab = e % (NA * NB);
                unsafeAtomicAdd(&Gj[(int64_t)rowfn[g * NR + ab / NB] * N + rowfn[g * NR + NA + ab % NB]], 2.0 * Jab[e]);
            }
        __syncthreads();  // LDS reused by the next group
    }
}

// J/K from stored blocks for classes whose block is too large to hold in
// registers: the same bra-row segments (K rows of the bra functions in
// LDS, J[a,b] in registers, one flush per segment), with the block of each
// quartet streamed element by element in (a, b, c, d) order; the density
// rows of the bra functions are staged in LDS next to the K rows.  Per
// element six FMAs; K partial sums are flushed to LDS per (a, b) and per a,
// J[c,d] to global memory per quartet.
template <class Dm, typename Real>
__global__ void __launch_bounds__(256) k_jk_stored_stream(const PairInfo *__restrict__ pairs, int bra_off, int ket_off,
                                                          int same_class, const int64_t *__restrict__ rowstart,
                                                          const int2 *__restrict__ rowmap, const int4 *__restrict__ segs,
                                                          int nseg, const Real *__restrict__ base, int64_t total,
                                                          const double *__restrict__ Dall, double *__restrict__ Gjall,
                                                          double *__restrict__ Gkall) {
    constexpr int NA = Dm::NA, NB = Dm::NB, NC = Dm::NC, ND = Dm::ND;
    extern __shared__ double lds[];
    auto lds_add = [](double *p, double v) {
        __hip_atomic_fetch_add(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
    };
    for (int sidx = blockIdx.x; sidx < nseg; sidx += gridDim.x) {
        const int4 sg = segs[sidx];
        const int i = rowmap[sg.x].x;
        const PairInfo bra = pairs[bra_off + i];
        const int N = bra.mN, a0 = bra.bfa, b0 = bra.bfb;
        const double *D = Dall + bra.moff;
        double *Gj = Gjall ? Gjall + bra.moff : nullptr;
        double *Gk = Gkall ? Gkall + bra.moff : nullptr;
        double *Ka = lds, *Kb = lds + NA * N, *Da = lds + (NA + NB) * N, *Db = Da + NA * N;
        double *Jab = Db + NB * N;
        // K rows zeroed, density rows (same layout) copied, J[a,b] zeroed
        for (int e = threadIdx.x; e < (NA + NB) * N; e += 256) {
            const int row = e < NA * N ? a0 + e / N : b0 + (e - NA * N) / N;
            lds[e] = 0.0;
            Da[e] = D[(int64_t)row * N + e % N];
        }
        if (threadIdx.x < NA * NB) Jab[threadIdx.x] = 0.0;
        __syncthreads();
        Real jab[NA][NB];
        static_for<0, NA>([&](auto A) { static_for<0, NB>([&](auto B) { jab[A][B] = Real(0); }); });
        int r = sg.x;
        for (int64_t q = sg.y + threadIdx.x; q < sg.z; q += 256) {
            while (r + 1 < sg.w && rowstart[r + 1] <= q) ++r;
            const int j = rowmap[r].y + (int)(q - rowstart[r]);
            const PairInfo ket = pairs[ket_off + j];
            const int c0 = ket.bfa, d0 = ket.bfb;
            double fac = 1.0;
            if (bra.sa == bra.sb) fac *= 0.5;
            if (ket.sa == ket.sb) fac *= 0.5;
            if (same_class && i == j) fac *= 0.5;
            Real Dcd[NC][ND], jcd[NC][ND];
            static_for<0, NC>([&](auto C) {
                static_for<0, ND>([&](auto Dd) {
                    Dcd[C][Dd] = Real(D[(int64_t)(c0 + C) * N + d0 + Dd]);
                    jcd[C][Dd] = Real(0);
                });
            });
            static_for<0, NA>([&](auto A) {
                Real kac[NC], kad[ND];
                static_for<0, NC>([&](auto C) { kac[C] = Real(0); });
                static_for<0, ND>([&](auto Dd) { kad[Dd] = Real(0); });
                static_for<0, NB>([&](auto B) {
                    const Real dab = Real(Da[A * N + b0 + B]);
                    Real dad[ND], dbd[ND], kbd[ND], kbc[NC];
                    static_for<0, ND>([&](auto Dd) {
                        dad[Dd] = Real(Da[A * N + d0 + Dd]);
                        dbd[Dd] = Real(Db[B * N + d0 + Dd]);
                        kbd[Dd] = Real(0);
                    });
                    Real s = Real(0);
                    static_for<0, NC>([&](auto C) {
                        const Real dac = Real(Da[A * N + c0 + C]), dbc = Real(Db[B * N + c0 + C]);
                        kbc[C] = Real(0);
                        static_for<0, ND>([&](auto Dd) {
                            constexpr int e = ((decltype(A)::value * NB + decltype(B)::value) * NC + decltype(C)::value) * ND +
                                              decltype(Dd)::value;
                            const Real o = base[(int64_t)e * total + q];
                            s += o * Dcd[C][Dd];
                            jcd[C][Dd] += o * dab;
                            kac[C] += o * dbd[Dd];
                            kbc[C] += o * dad[Dd];
                            kad[Dd] += o * dbc;
                            kbd[Dd] += o * dac;
                        });
                    });
                    jab[A][B] += Real(fac) * s;
                    if (Gk) {
                        static_for<0, NC>([&](auto C) { lds_add(&Kb[B * N + c0 + C], fac * (double)kbc[C]); });
                        static_for<0, ND>([&](auto Dd) { lds_add(&Kb[B * N + d0 + Dd], fac * (double)kbd[Dd]); });
                    }
                });
                if (Gk) {
                    static_for<0, NC>([&](auto C) { lds_add(&Ka[A * N + c0 + C], fac * (double)kac[C]); });
                    static_for<0, ND>([&](auto Dd) { lds_add(&Ka[A * N + d0 + Dd], fac * (double)kad[Dd]); });
                }
            });
            if (Gj)
                static_for<0, NC>([&](auto C) {
                    static_for<0, ND>([&](auto Dd) {
                        unsafeAtomicAdd(&Gj[(int64_t)(c0 + C) * N + d0 + Dd], 2.0 * fac * (double)jcd[C][Dd]);
                    });
                });
        }
        if (Gj) {
            static_for<0, NA>([&](auto A) { static_for<0, NB>([&](auto B) {
                double v = (double)jab[A][B];
                for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
                if ((threadIdx.x & 63) == 0) lds_add(&Jab[A * NB + B], v);
            }); });
        }
        __syncthreads();
        if (Gk)
            for (int e = threadIdx.x; e < (NA + NB) * N; e += 256) {
                const double v = lds[e];
                if (v == 0.0) continue;
                const int row = e < NA * N ? a0 + e / N : b0 + (e - NA * N) / N;
                unsafeAtomicAdd(&Gk[(int64_t)row * N + e % N], v);
            }
        if (Gj)
            for (int e = threadIdx.x; e < NA * NB; e += 256)
                unsafeAtomicAdd(&Gj[(int64_t)(a0 + e / NB) * N + b0 + e % NB], 2.0 * Jab[e]);
        __syncthreads();  // LDS reused by the next segment
    }
}

}  // namespace mess
