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
// the intermediates with butterfly reduce-scatters over blocks of 64 (six
// exchange steps, each lane keeping half of what it holds), so lane l ends
// with the sums of intermediates 64 b + l.  The horizontal recursion and output
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

// Position of intermediate x = (f - F0) NEA + (e - E0) in the order
// prim_quartet hands them out, and its inverse (tables evaluated once per
// class at compile time).  Blocks of 64 are cut in that order, so a block is
// complete (and reduced) after 64 consecutive outputs and at most one block
// is pending at a time.
template <class Dm, int NACC>
struct PlaneBlocks {
    int pos[NACC];
    int xof[NACC];
};
template <class Dm, int NACC>
__host__ __device__ constexpr PlaneBlocks<Dm, NACC> make_plane_blocks() {
    PlaneBlocks<Dm, NACC> r{};
    const KetDfs<Dm::LCD> kd = make_ket_dfs<Dm::LC, Dm::LCD>();
    for (int x = 0; x < NACC; ++x) {
        r.pos[x] = kd.rank[Dm::F0 + x / Dm::NEA] * Dm::NEA + x % Dm::NEA;
        r.xof[r.pos[x]] = x;
    }
    return r;
}
template <class Dm, int NACC>
inline constexpr PlaneBlocks<Dm, NACC> kPlaneBlocks = make_plane_blocks<Dm, NACC>();
template <class Dm, int NACC>
__constant__ PlaneBlocks<Dm, NACC> kPlaneBlocksDev = make_plane_blocks<Dm, NACC>();

template <class Dm>
inline constexpr int kPlaneBlockSize = 32;
// recursion passes per primitive quartet over ket subtrees: 2: x | y z;
// 3: x | y | z; 6: one pass per second-level component (xx, xy, xz, yy,
// yz, zz), the fewest live values for the most repeated work
#ifndef MESS_PLANE_PASSES
#define MESS_PLANE_PASSES 1
#endif
template <class Dm>
inline constexpr int kPlanePasses = MESS_PLANE_PASSES;

// with several passes, the base values [00|00]^(m) are evaluated once per
// primitive quartet and read by every pass from LDS (MESS_PLANE_SHARE=0:
// every pass evaluates them itself)
#ifndef MESS_PLANE_SHARE
#define MESS_PLANE_SHARE 1
#endif

// MESS_PLANE_WAVES=n asks for n waves per SIMD (register budget 512 / n)
#if defined(MESS_PLANE_WAVES)
#define MESS_PLANE_OCC __attribute__((amdgpu_waves_per_eu(MESS_PLANE_WAVES, MESS_PLANE_WAVES)))
#else
#define MESS_PLANE_OCC
#endif

template <class Dm, int MODE, typename Real>
__global__ void __launch_bounds__(64) MESS_PLANE_OCC k_plane(CoopArgs A, const PairInfo *__restrict__ pairs, int bra_off,
                                              int ket_off, int nbra, int same_class,
                                              const int64_t *__restrict__ rowstart, const int2 *__restrict__ rowmap, int64_t total,
                                              const PrimPairT<Real> *__restrict__ pp, BoysTabs bt,
                                              const double *__restrict__ D, int N,
                                              double *__restrict__ out0, double *__restrict__ out1) {
    constexpr int NACC = Dm::NFA * Dm::NEA;
    // reduction block: 64 outputs, or 32 where the recursion itself nearly
    // fills the registers (at most one block of outputs is pending)
    constexpr int BS = kPlaneBlockSize<Dm>;
    constexpr int NP = ((NACC + BS - 1) / BS) * BS, NPER = NP / BS;
    // the recursion may run with the ket pair on the e side (fewer live
    // values); intermediates are then numbered in that orientation and put
    // back in the class's own order when stored to LDS
    constexpr bool SW = VrrOrient<Dm>::swap;
    using Dr = std::conditional_t<SW, ClassDims<Dm::LC, Dm::LD, Dm::LA, Dm::LB>, Dm>;
    extern __shared__ double lds[];
    double *H = lds;
    double *hc = lds + A.nH;
    const int lane = threadIdx.x;
    // base values [00|00]^(m) of this lane's primitive quartet, element m at
    // bfl[64 m], shared by the recursion passes (one Boys evaluation)
    Real *bfl = reinterpret_cast<Real *>(lds + A.nH + kNHCoef) + lane;
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
        // anchor difference of the recursion's e-side and f-side pairs
        const Real sg = SW ? Real(-1) : Real(1);
        const Real AC[3] = {sg * Real(bra.Ax - ket.Ax), sg * Real(bra.Ay - ket.Ay), sg * Real(bra.Az - ket.Az)};
        Real part[NPER];
        static_for<0, NPER>([&](auto I) { part[I] = Real(0); });
        const int nprim = bra.npp * ket.npp;
        for (int k0 = 0; k0 < nprim; k0 += 64) {
            const int k = k0 + lane;
            // lanes past the end evaluate primitive quartet 0 with zero
            // weight, so the recursion and the reductions stay one
            // straight-line block
            const int kk = k < nprim ? k : 0;
            PrimPairT<Real> P = pp[bra.pp0 + kk / ket.npp];
            const PrimPairT<Real> Q = pp[ket.pp0 + kk % ket.npp];
            if (k >= nprim) P.Kr = Real(0);
            // intermediates in blocks of 64; each block is reduce-scattered
            // over the wave (lane l keeps entry 64 b + l) as soon as its last
            // entry is final, so finished outputs do not stay live through
            // the rest of the recursion
            Real vb[NPER][BS];
            static_for<NACC, NP>([&](auto X) {
                constexpr int x = decltype(X)::value;
                vb[x / BS][x % BS] = Real(0);
            });
            auto emit = [&](auto X, Real val) {
                constexpr int ps = kPlaneBlocks<Dr, NACC>.pos[decltype(X)::value];
                constexpr int b = ps / BS;
                vb[b][ps % BS] = val;
                if constexpr (ps % BS == BS - 1 || ps == NACC - 1) {
                    if constexpr (BS == 64) rs_step<64, 64, 32>(vb[b], lane);
                    rs_step<BS, 32, 16>(vb[b], lane);
                    rs_step<BS, 16, 8>(vb[b], lane);
                    rs_step<BS, 8, 4>(vb[b], lane);
                    rs_step<BS, 4, 2>(vb[b], lane);
                    rs_step<BS, 2, 1>(vb[b], lane);
                    // blocks of 32: lanes l and l ^ 32 hold halves of entry l % 32
                    if constexpr (BS == 32) vb[b][0] += __shfl_xor(vb[b][0], 32, 64);
                    part[b] += vb[b][0];
                }
            };
            // classes whose recursion outgrows the registers run it in
            // passes over disjoint subtrees of the ket tree (outputs stay in
            // order, so the reduction blocks are unchanged)
            constexpr bool PRE = MESS_PLANE_SHARE && kPlanePasses<Dm> > 1;
            if constexpr (PRE) {
                Real V0[Dr::L + 1];
                if constexpr (SW)
                    prim_base<Dr::L, Real>(Q, P, AC, bt, V0);
                else
                    prim_base<Dr::L, Real>(P, Q, AC, bt, V0);
                static_for<0, Dr::L + 1>([&](auto M) { bfl[64 * decltype(M)::value] = V0[decltype(M)::value]; });
            }
            auto run = [&](auto SUBC) {
                constexpr int SUB = decltype(SUBC)::value;
                if constexpr (SW)
                    prim_quartet<Dr, Real, SUB, PRE>(Q, P, AC, bt, emit, bfl);
                else
                    prim_quartet<Dr, Real, SUB, PRE>(P, Q, AC, bt, emit, bfl);
            };
            // passes over second-level ket groups (xx xy xz | yy yz | zz)
            if constexpr (kPlanePasses<Dm> == 2) {
                run(std::integral_constant<int, 7>{});
                run(std::integral_constant<int, 56>{});
            } else if constexpr (kPlanePasses<Dm> == 3) {
                run(std::integral_constant<int, 7>{});
                run(std::integral_constant<int, 24>{});
                run(std::integral_constant<int, 32>{});
            } else if constexpr (kPlanePasses<Dm> == 6) {
                run(std::integral_constant<int, 1>{});
                run(std::integral_constant<int, 2>{});
                run(std::integral_constant<int, 4>{});
                run(std::integral_constant<int, 8>{});
                run(std::integral_constant<int, 16>{});
                run(std::integral_constant<int, 32>{});
            } else {
                run(std::integral_constant<int, 63>{});
            }
        }
        static_for<0, NPER>([&](auto I) {
            const int ps = BS * decltype(I)::value + lane;
            if (lane < BS && ps < NACC) {
                const int x = kPlaneBlocksDev<Dr, NACC>.xof[ps];
                // swapped: x = (e - E0) NFA + (f - F0) holds [e0|f0]
                const int h = SW ? (x % Dm::NFA) * Dm::NEA + x / Dm::NFA : x;
                H[h] = (double)part[I];
            }
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
    const BoysTabs bt{L.tab, L.etab, L.tabf, L.etabf, L.tabt};
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
