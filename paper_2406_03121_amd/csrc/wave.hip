// Wave-per-primitive-quartet kernel of one high angular class in one
// precision (compiled once per class and precision with -DMESS_WCB,
// -DMESS_WCK, -DMESS_WREAL).
//
// A 256-thread block takes one shell quartet; each of its four waves runs
// the Obara-Saika vertical recursion of every fourth primitive quartet.
// Inside a wave the lanes share the recursion of one primitive quartet:
// lane slot p owns the intermediate pair (e, m) for the whole kernel, so a
// step of component f reads the parent's (e, m), (e, m+1) and
// (e - 1_j, m+1) and the grandparent's (e, m), (e, m+1) at offsets that are
// fixed per lane, and writes its own (e, m).  Each recursion level has one
// dense [e][m] block of LDS per wave; the ket components are visited depth
// first, so a level's block always holds the current ancestor at that level.
// The pairs are numbered so that the ones a ket level uses are a prefix
// (numbered by the deepest level that uses them), and the lanes owning an
// output pair [e0|f0]^(0) accumulate it over the wave's primitive quartets
// in registers: no reduction across lanes until the quartet is done.  The
// four waves' sums then meet in LDS, and the horizontal recursion and output
// run table-driven as in k_coop.
#include "coop.hpp"

#ifndef MESS_WCB
#error "compile with -DMESS_WCB, -DMESS_WCK, -DMESS_WREAL"
#endif

namespace mess {

template <class Dr>
struct WaveMap {
    static constexpr int L = Dr::L, LP = L + 1, NE = Dr::NE, LA = Dr::LA, LAB = Dr::LAB, LCD = Dr::LCD;
    static constexpr int NPAIR = NE * LP;
    static constexpr int NSLOT = ((NPAIR + 63) / 64) * 64;
    int pe[NSLOT], pm[NSLOT];  // pair of slot p (e = -1: unused)
    int cnt[LCD + 1];          // slots used by ket level nf: [0, cnt[nf])
    int nout;                  // output pairs (|e| >= LA, m = 0): slots [0, nout)
};

// Lowest |e| a ket level nf needs (outputs need |e| >= LA at level LCD).
__host__ __device__ constexpr int wave_emin(int LA, int LCD, int nf) { return cmax(0, LA - (LCD - nf)); }

template <class Dr>
__host__ __device__ constexpr WaveMap<Dr> make_wave_map() {
    using W = WaveMap<Dr>;
    WaveMap<Dr> r{};
    for (int p = 0; p < W::NSLOT; ++p) {
        r.pe[p] = -1;
        r.pm[p] = 0;
    }
    // deepest ket level using (e, m): levels are nested, so sorting by it
    // makes every level's pairs a prefix
    int depth[W::NPAIR] = {};
    for (int e = 0; e < W::NE; ++e)
        for (int m = 0; m < W::LP; ++m) {
            const int le = cart_of(e).l();
            int d = 0;
            for (int nf = 1; nf <= W::LCD; ++nf)
                if (le >= wave_emin(W::LA, W::LCD, nf) && m <= W::L - le - nf) d = nf;
            depth[e * W::LP + m] = d;
        }
    int n = 0;
    // output pairs first
    for (int e = cart_off(W::LA); e < W::NE; ++e) {
        r.pe[n] = e;
        r.pm[n] = 0;
        ++n;
    }
    r.nout = n;
    for (int d = W::LCD; d >= 1; --d)
        for (int e = 0; e < W::NE; ++e)
            for (int m = 0; m < W::LP; ++m) {
                if (depth[e * W::LP + m] != d) continue;
                if (m == 0 && e >= cart_off(W::LA)) continue;  // already placed
                r.pe[n] = e;
                r.pm[n] = m;
                ++n;
            }
    for (int nf = 0; nf <= W::LCD; ++nf) {
        int c = 0;
        for (int p = 0; p < n; ++p)
            if (depth[r.pe[p] * W::LP + r.pm[p]] >= (nf == 0 ? 1 : nf)) ++c;
        r.cnt[nf] = c;
    }
    return r;
}

// Checks, at compile time, that every slot a ket level uses is valid there
// and that the prefixes hold.
template <class Dr>
__host__ __device__ constexpr bool wave_map_ok() {
    using W = WaveMap<Dr>;
    const WaveMap<Dr> r = make_wave_map<Dr>();
    for (int nf = 1; nf <= W::LCD; ++nf) {
        if (r.cnt[nf] > r.cnt[nf - 1] && nf > 1) return false;
        for (int p = 0; p < r.cnt[nf]; ++p) {
            if (r.pe[p] < 0 || r.pe[p] >= W::NE) return false;
            const int le = cart_of(r.pe[p]).l();
            if (le < wave_emin(W::LA, W::LCD, nf) || r.pm[p] > W::L - le - nf) return false;
        }
    }
    // every pair a level needs is in its prefix
    for (int nf = 1; nf <= W::LCD; ++nf) {
        int need = 0;
        for (int e = 0; e < W::NE; ++e) {
            const int le = cart_of(e).l();
            if (le >= wave_emin(W::LA, W::LCD, nf))
                for (int m = 0; m <= W::L - le - nf; ++m) ++need;
        }
        if (need != r.cnt[nf]) return false;
    }
    return r.nout == W::NE - cart_off(W::LA) && r.nout <= 64;
}

template <class Dr>
__constant__ WaveMap<Dr> kWaveMapDev = make_wave_map<Dr>();
template <class Dr>
inline constexpr WaveMap<Dr> kWaveMap = make_wave_map<Dr>();

// Per-component tables of the e side (index < NE): first non-zero
// direction i, its exponent, and the indices of e - 1_i, e - 2_i.
template <int NE>
struct ECart {
    int dir[NE], ei[NE], e1[NE], e2[NE];
    int m1[3][NE];  // e - 1_j for j = x, y, z (or e itself when e_j = 0)
    int ej[3][NE];
};
template <int NE>
__host__ __device__ constexpr ECart<NE> make_ecart() {
    ECart<NE> t{};
    for (int e = 0; e < NE; ++e) {
        const Cart c = cart_of(e);
        const int i = c.l() > 0 ? c.dir() : 0;
        t.dir[e] = i;
        t.ei[e] = c.get(i);
        t.e1[e] = c.l() > 0 ? c.minus(i).idx() : 0;
        t.e2[e] = c.get(i) >= 2 ? c.minus(i, 2).idx() : 0;
        for (int j = 0; j < 3; ++j) {
            t.ej[j][e] = c.get(j);
            t.m1[j][e] = c.get(j) > 0 ? c.minus(j).idx() : e;
        }
    }
    return t;
}
template <int NE>
__constant__ ECart<NE> kECartDev = make_ecart<NE>();

// Orders LDS traffic of one wave between recursion steps (the lanes read
// what other lanes of the same wave wrote).  The LDS performs the
// operations of one wave in issue order, so wavefront-scope fences (which
// only stop the compiler from moving memory operations across them) are
// enough: no wait for outstanding LDS operations is needed.
__device__ __forceinline__ void wave_step_sync() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// The bra stays on the e side here: the f side's components are the
// recursion steps of a wave, so the pair of larger momentum there means
// more steps with less work each (measured slower for (dd|ds), (dd|dp)).
template <class Dm>
struct WaveOrient {
    static constexpr bool swap = false;
    using Dr = Dm;
};

template <class Dm, typename Real>
struct WaveLds {
    using Dr = typename WaveOrient<Dm>::Dr;
    static constexpr int LP = Dr::L + 1;
    static constexpr int BLOCK = Dr::NE * LP;                  // one level
    static constexpr int PER_WAVE = (Dr::LCD + 1) * BLOCK;     // Real elements per wave
    static constexpr int VRR_DOUBLES = (4 * PER_WAVE * (int)sizeof(Real) + 7) / 8;
};

template <class Dm, int MODE, typename Real>
__global__ void __launch_bounds__(256) k_wave(CoopArgs A, int region, const PairInfo *__restrict__ pairs,
                                              int bra_off, int ket_off, int nbra, int same_class,
                                              const int64_t *__restrict__ rowstart, const int2 *__restrict__ rowmap,
                                              int64_t total, const PrimPairT<Real> *__restrict__ pp, BoysTabs bt,
                                              const double *__restrict__ D, int N, double *__restrict__ out0,
                                              double *__restrict__ out1) {
    using WO = WaveOrient<Dm>;
    using Dr = typename WO::Dr;
    constexpr bool SW = WO::swap;
    using WM = WaveMap<Dr>;
    constexpr int L = Dr::L, LP = L + 1, NE = Dr::NE, LAB = Dr::LAB, LCD = Dr::LCD, LC = Dr::LC;
    constexpr int NSUB = (kWaveMap<Dr>.cnt[1] + 63) / 64;  // lane slots the ket levels use
    constexpr int NFO = Dr::NFA;                             // output components on the f side
    static_assert(wave_map_ok<Dr>(), "wave pair map");
    using Lds = WaveLds<Dm, Real>;

    extern __shared__ double lds[];
    const int tid = threadIdx.x;
    const int wave = tid >> 6, lane = tid & 63;
    Real *R = reinterpret_cast<Real *>(lds) + wave * Lds::PER_WAVE;
    double *H = lds;                 // after the primitive loop: accumulators and HRR slots
    double *hc = lds + region;       // HRR coefficients

    // this lane's pairs for the ket levels: own offset, (e - 1_j, m + 1)
    // offsets, e_j
    int own[NSUB], e1o[NSUB][3];
    Real ejr[NSUB][3];
    static_for<0, NSUB>([&](auto S) {
        constexpr int s = decltype(S)::value;
        const int p = 64 * s + lane;
        const int e = kWaveMapDev<Dr>.pe[p], m = kWaveMapDev<Dr>.pm[p];
        const int ee = e < 0 ? 0 : e;
        own[s] = ee * LP + m;
        for (int j = 0; j < 3; ++j) {
            const int ej = kECartDev<NE>.ej[j][ee];
            e1o[s][j] = ej > 0 ? kECartDev<NE>.m1[j][ee] * LP + m + 1 : own[s];
            ejr[s][j] = Real(ej);
        }
    });
    const bool out_lane = lane < kWaveMap<Dr>.nout;

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
        // the recursion's e-side and f-side pairs
        const PairInfo &pe = SW ? ket : bra;
        const PairInfo &pf = SW ? bra : ket;
        const Real ACx = Real(pe.Ax - pf.Ax), ACy = Real(pe.Ay - pf.Ay), ACz = Real(pe.Az - pf.Az);
        Real acc[NFO];
        static_for<0, NFO>([&](auto F) { acc[decltype(F)::value] = Real(0); });
        const int npe = pe.npp, npf = pf.npp;
        const int npq = npe * npf;
        for (int k = wave; k < npq; k += 4) {
            const PrimPairT<Real> P = pp[pe.pp0 + k / npf];
            const PrimPairT<Real> Q = pp[pf.pp0 + k % npf];
            const Real p = P.p, qq = Q.p, pq = p + qq, spq = rsqrt_nr(pq), rpq = spq * spq;
            const Real PQx = ACx + (P.PAx - Q.PAx), PQy = ACy + (P.PAy - Q.PAy), PQz = ACz + (P.PAz - Q.PAz);
            const Real T = p * qq * rpq * (PQx * PQx + PQy * PQy + PQz * PQz);
            const Real PA[3] = {P.PAx, P.PAy, P.PAz};
            const Real WP[3] = {-qq * rpq * PQx, -qq * rpq * PQy, -qq * rpq * PQz};
            const Real QC[3] = {Q.PAx, Q.PAy, Q.PAz};
            const Real WQ[3] = {p * rpq * PQx, p * rpq * PQy, p * rpq * PQz};
            const Real o2p = Real(0.5) * P.rp, o2pr = o2p * (qq * rpq);
            const Real o2q = Real(0.5) * Q.rp, o2qr = o2q * (p * rpq);
            const Real o2pq = Real(0.5) * rpq;
            // [0|0]^(m) = 2 pi^{5/2} K_P K_Q / (p q sqrt(p+q)) F_m(T)
            if (lane <= L) R[lane] = P.Kr * Q.Kr * spq * coop_boys_r<Real>(lane, T, bt);
            wave_step_sync();
            // e-side recursion, level by level: [e+1_i|0]^(m)
            static_for<1, LAB + 1>([&](auto NI) {
                constexpr int n = decltype(NI)::value;
                constexpr int MW = L + 1 - n;                 // m = 0 .. L - n
                constexpr int ITEMS = ncart(n) * MW;
                static_for<0, (ITEMS + 63) / 64>([&](auto SI) {
                    const int it = 64 * decltype(SI)::value + lane;
                    if (it < ITEMS) {
                        const int e = cart_off(n) + it / MW, m = it % MW;
                        const int d = kECartDev<NE>.dir[e];
                        const int e1 = kECartDev<NE>.e1[e] * LP + m;
                        const Real pa = d == 0 ? PA[0] : (d == 1 ? PA[1] : PA[2]);
                        const Real wp = d == 0 ? WP[0] : (d == 1 ? WP[1] : WP[2]);
                        Real v = pa * R[e1] + wp * R[e1 + 1];
                        const int ei = kECartDev<NE>.ei[e];
                        if (ei >= 2) {
                            const int e2 = kECartDev<NE>.e2[e] * LP + m;
                            v += Real(ei - 1) * (o2p * R[e2] - o2pr * R[e2 + 1]);
                        }
                        R[e * LP + m] = v;
                    }
                });
                wave_step_sync();
            });
            // f-side recursion, depth first: level nf's block holds the
            // current ancestor at that level
            static_for<0, Dr::NF>([&](auto SI) {
                constexpr int f = kKetDfs<LC, LCD>.seq[decltype(SI)::value];
                if constexpr (f > 0) {
                    constexpr Cart cf = cart_of(f);
                    constexpr int nf = cf.l();
                    constexpr int jd = last_dir(cf);
                    constexpr int fj = cf.get(jd);
                    constexpr int cnt = kWaveMap<Dr>.cnt[nf];
                    Real *R1 = R + (nf - 1) * Lds::BLOCK;
                    Real *R0 = R + nf * Lds::BLOCK;
                    static_for<0, (cnt + 63) / 64>([&](auto S) {
                        constexpr int s = decltype(S)::value;
                        if (64 * s + lane < cnt) {
                            const int o = own[s];
                            Real v = QC[jd] * R1[o] + WQ[jd] * R1[o + 1] + ejr[s][jd] * o2pq * R1[e1o[s][jd]];
                            if constexpr (fj >= 2) {
                                const Real *R2 = R + (nf - 2) * Lds::BLOCK;
                                v += Real(fj - 1) * (o2q * R2[o] - o2qr * R2[o + 1]);
                            }
                            R0[o] = v;
                            if constexpr (s == 0 && nf >= LC) {
                                if (out_lane) acc[f - Dr::F0] += v;
                            }
                        }
                    });
                    wave_step_sync();
                }
            });
        }
        // the four waves' sums into H[(f - F0) NEA + (e - E0)] in the class's
        // own orientation: each wave writes its own copy (after H), then the
        // copies are added in wave order, so the result does not depend on
        // timing (the deterministic J/K mode relies on reproducible blocks)
        __syncthreads();
        double *Hw = H + A.nacc;
        if (out_lane) {
            const int e = kWaveMapDev<Dr>.pe[lane];
            static_for<0, NFO>([&](auto F) {
                constexpr int fo = decltype(F)::value;
                const int x = SW ? (e - Dr::E0) * Dm::NEA + fo : fo * Dm::NEA + (e - Dr::E0);
                Hw[wave * A.nacc + x] = (double)acc[fo];
            });
        }
        __syncthreads();
        for (int s = tid; s < A.nacc; s += 256)
            H[s] = ((Hw[s] + Hw[A.nacc + s]) + Hw[2 * A.nacc + s]) + Hw[3 * A.nacc + s];
        __syncthreads();
        coop_finish<MODE, 256>(A, H, hc, tid, bra, ket, i, j, bra_off, same_class, D, N, out0, out1, q, total);
        __syncthreads();
    }
}

template <>
void WaveOps<MESS_WCB, MESS_WCK, MESS_WREAL>::launch(int mode, const CoopArgs &A, const ClassLaunch &L,
                                                     int64_t total, unsigned g, const double *D, double *out0,
                                                     double *out1, size_t *lds_out) {
    using Dm = ClassOf<MESS_WCB, MESS_WCK>;
    using R = MESS_WREAL;
    using Lds = WaveLds<Dm, R>;
    // VRR blocks during the primitive loop; then the accumulators, the four
    // waves' copies of them, and the HRR slots
    const int region = std::max(std::max(Lds::VRR_DOUBLES, A.nH), 5 * A.nacc);
    const size_t lds = sizeof(double) * ((size_t)region + kNHCoef);
    if (lds_out) {
        *lds_out = lds;
        return;
    }
    const BoysTabs bt{L.tab, L.etab, L.tabf, L.etabf, L.tabt};
    const PrimPairT<R> *pp =
        reinterpret_cast<const PrimPairT<R> *>(sizeof(R) == 8 ? (const void *)L.pp : (const void *)L.ppf);
#define MESS_WAVE_GO(MODE)                                                                                       \
    hipLaunchKernelGGL((k_wave<Dm, MODE, R>), dim3(g), dim3(256), lds, L.stream, A, region, L.pairs, L.bra_off,  \
                       L.ket_off, L.nbra, L.same_class, L.rowstart, L.rowmap, total, pp, bt, D, L.N, out0, out1)
    switch (mode) {
        case kModeSchwarz: MESS_WAVE_GO(kModeSchwarz); break;
        case kModeDense: MESS_WAVE_GO(kModeDense); break;
        case kModeStore64: MESS_WAVE_GO(kModeStore64); break;
        case kModeStore32: MESS_WAVE_GO(kModeStore32); break;
        default: MESS_WAVE_GO(kModeJK);
    }
#undef MESS_WAVE_GO
}

}  // namespace mess
