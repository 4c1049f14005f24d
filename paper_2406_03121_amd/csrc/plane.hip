// Primitive-lane kernel of one high angular class in one precision.  This
// file is compiled once per (class, precision) with -DMESS_PCB=<bra pair
// class> -DMESS_PCK=<ket pair class> -DMESS_PREAL=<double|float>.
#include "coop.hpp"

#ifndef MESS_PCB
#error "compile with -DMESS_PCB, -DMESS_PCK, -DMESS_PREAL"
#endif

namespace mess {

// --------------------------------------------------- primitive lanes
//
// Alternative mapping for classes whose unrolled recursion fits in one
// lane's registers but whose contracted intermediates do not: one wave per
// shell quartet, lane k evaluating primitive quartet k (then k + 64, ...)
// with the fully unrolled recursion; after each round of 64 the wave sums
// the intermediates with a butterfly reduce-scatter (six exchange steps,
// each lane keeping half of what it holds), so lane l ends with the sums of
// intermediates [l*NPER, (l+1)*NPER).  The horizontal recursion and output
// then run table-driven as in k_coop.

template <int NP, int C, int O, typename Real>
__device__ __forceinline__ void rs_step(Real (&v)[NP], const int lane) {
    const bool up = (lane & O) != 0;
    static_for<0, C / 2>([&](auto I) {
        constexpr int k = decltype(I)::value;
        const Real lo = v[k], hi = v[k + C / 2];
        const Real send = up ? lo : hi;
        const Real keep = up ? hi : lo;
        v[k] = keep + __shfl_xor(send, O, 64);
    });
}

template <class Dm, int MODE, typename Real>
__global__ void __launch_bounds__(64) k_plane(CoopArgs A, const PairInfo *__restrict__ pairs, int bra_off,
                                              int ket_off, int nbra, int same_class,
                                              const int64_t *__restrict__ rowstart, const int2 *__restrict__ rowmap, int64_t total,
                                              const PrimPairT<Real> *__restrict__ pp, BoysTabs bt,
                                              const double *__restrict__ D, int N,
                                              double *__restrict__ out0, double *__restrict__ out1) {
    constexpr int NACC = Dm::NFA * Dm::NEA;
    constexpr int NP = ((NACC + 63) / 64) * 64, NPER = NP / 64;
    extern __shared__ double lds[];
    double *H = lds;
    double *hc = lds + A.nH;
    const int lane = threadIdx.x;
    for (int64_t q = blockIdx.x; q < total; q += gridDim.x) {
        int i, j;
        if (MODE == kModeSchwarz) {
            i = j = (int)q;
        } else {
            const int2 ij = quartet_pairs(rowstart, rowmap, nbra, q);
            i = ij.x;
            j = ij.y;
        }
        const PairInfo bra = pairs[bra_off + i];
        const PairInfo ket = pairs[(MODE == kModeSchwarz ? bra_off : ket_off) + j];
        const Real AC[3] = {Real(bra.Ax - ket.Ax), Real(bra.Ay - ket.Ay), Real(bra.Az - ket.Az)};
        Real part[NPER];
        static_for<0, NPER>([&](auto I) { part[I] = Real(0); });
        const int nprim = bra.npp * ket.npp;
        for (int k0 = 0; k0 < nprim; k0 += 64) {
            const int k = k0 + lane;
            Real a[Dm::NFA][Dm::NEA];
            static_for<0, Dm::NFA>([&](auto F) {
                static_for<0, Dm::NEA>([&](auto E) { a[decltype(F)::value][decltype(E)::value] = Real(0); });
            });
            if (k < nprim) {
                const PrimPairT<Real> P = pp[bra.pp0 + k / ket.npp];
                const PrimPairT<Real> Q = pp[ket.pp0 + k % ket.npp];
                prim_quartet<Dm, Real>(P, Q, AC, bt, a);
            }
            Real v[NP];
            static_for<0, NP>([&](auto I) {
                constexpr int x = decltype(I)::value;
                if constexpr (x < NACC) v[x] = a[x / Dm::NEA][x % Dm::NEA];
                else v[x] = Real(0);
            });
            rs_step<NP, NP, 32>(v, lane);
            rs_step<NP, NP / 2, 16>(v, lane);
            rs_step<NP, NP / 4, 8>(v, lane);
            rs_step<NP, NP / 8, 4>(v, lane);
            rs_step<NP, NP / 16, 2>(v, lane);
            rs_step<NP, NP / 32, 1>(v, lane);
            static_for<0, NPER>([&](auto I) { part[I] += v[I]; });
        }
        static_for<0, NPER>([&](auto I) {
            const int idx = lane * NPER + decltype(I)::value;
            if (idx < NACC) H[idx] = (double)part[I];
        });
        __syncthreads();
        coop_finish<MODE>(A, H, hc, lane, bra, ket, i, j, bra_off, same_class, D, N, out0, out1, q, total);
        __syncthreads();
    }
}


template <>
void PlaneOps<MESS_PCB, MESS_PCK, MESS_PREAL>::launch(int mode, const CoopArgs &A, const ClassLaunch &L,
                                                      int64_t total, unsigned g, size_t lds, const double *D,
                                                      double *out0, double *out1) {
    using Dm = ClassOf<MESS_PCB, MESS_PCK>;
    using R = MESS_PREAL;
    const BoysTabs bt{L.tab, L.etab, L.tabf, L.etabf};
    const PrimPairT<R> *pp;
    pp = reinterpret_cast<const PrimPairT<R> *>(sizeof(R) == 8 ? (const void *)L.pp : (const void *)L.ppf);
    switch (mode) {
        case kModeSchwarz:
            hipLaunchKernelGGL((k_plane<Dm, kModeSchwarz, R>), dim3(g), dim3(64), lds, L.stream, A, L.pairs, L.bra_off,
                               L.ket_off, L.nbra, L.same_class, L.rowstart, L.rowmap, total, pp, bt, D, L.N, out0, out1);
            break;
        case kModeDense:
            hipLaunchKernelGGL((k_plane<Dm, kModeDense, R>), dim3(g), dim3(64), lds, L.stream, A, L.pairs, L.bra_off,
                               L.ket_off, L.nbra, L.same_class, L.rowstart, L.rowmap, total, pp, bt, D, L.N, out0, out1);
            break;
        case kModeStore64:
            hipLaunchKernelGGL((k_plane<Dm, kModeStore64, R>), dim3(g), dim3(64), lds, L.stream, A, L.pairs, L.bra_off,
                               L.ket_off, L.nbra, L.same_class, L.rowstart, L.rowmap, total, pp, bt, D, L.N, out0, out1);
            break;
        case kModeStore32:
            hipLaunchKernelGGL((k_plane<Dm, kModeStore32, R>), dim3(g), dim3(64), lds, L.stream, A, L.pairs, L.bra_off,
                               L.ket_off, L.nbra, L.same_class, L.rowstart, L.rowmap, total, pp, bt, D, L.N, out0, out1);
            break;
        default:
            hipLaunchKernelGGL((k_plane<Dm, kModeJK, R>), dim3(g), dim3(64), lds, L.stream, A, L.pairs, L.bra_off,
                               L.ket_off, L.nbra, L.same_class, L.rowstart, L.rowmap, total, pp, bt, D, L.N, out0, out1);
    }
}

}  // namespace mess
