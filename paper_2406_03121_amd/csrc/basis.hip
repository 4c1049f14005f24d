// Basis creation (normalisation, device tables), shell pairs, Schwarz
// factors and unique shell-quartet work lists.
#include <array>
#include <atomic>
#include <cmath>
#include <cstdarg>
#include <cstring>
#include <thread>

#include "class_ops.hpp"
#include "mess_internal.hpp"

namespace mess {

// ------------------------------------------------------------- errors

static thread_local char g_err[512] = "";

void set_error(const char *fmt, ...) {
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(g_err, sizeof(g_err), fmt, ap);
    va_end(ap);
}

// --------------------------------------------------------------- Boys
//
// Table of F_n(T_k), T_k = k/16, n < 16, built on the host in extended
// precision: F_15 from its power series
//   F_n(T) = e^{-T} sum_i (2T)^i / ((2n+1)(2n+3)...(2n+2i+1))
// (all terms positive), lower orders by the stable downward recurrence
//   F_n = (2T F_{n+1} + e^{-T}) / (2n+1).

static void build_boys_table(std::vector<double> &tab, std::vector<double> &etab, std::vector<double> &tabt) {
    tab.assign((size_t)kBoysRows * kBoysN, 0.0);
    etab.assign(kBoysRows, 0.0);
    tabt.assign((size_t)kBoysTL * kBoysRows * 8, 0.0);
    for (int k = 0; k < kBoysRows; ++k) {
        const long double T = (long double)k / (long double)kBoysInvStep;
        const long double eT = expl(-T);
        const int n = kBoysN - 1;
        long double term = 1.0L / (2 * n + 1), sum = term;
        for (int i = 1; i < 4000; ++i) {
            term *= 2.0L * T / (long double)(2 * n + 2 * i + 1);
            sum += term;
            if (term < 1e-22L * sum) break;
        }
        long double F[kBoysN];
        F[n] = eT * sum;
        for (int m = n - 1; m >= 0; --m) F[m] = (2.0L * T * F[m + 1] + eT) / (long double)(2 * m + 1);
        for (int m = 0; m < kBoysN; ++m) tab[(size_t)k * kBoysN + m] = (double)F[m];
        etab[k] = (double)eT;
        for (int L = 0; L < kBoysTL; ++L) {
            long double fact = 1.0L;
            for (int i = 0; i < 8; ++i) {
                if (i > 0) fact *= (long double)i;
                tabt[((size_t)L * kBoysRows + k) * 8 + i] = (double)(F[L + i] / fact);
            }
        }
    }
}

// ------------------------------------------------ normalisation (host)
//
// Contracted shell of angular momentum l: phi = N_c sum_p c_p N(a_p; l,0,0) g_p
// with N(a; l,0,0) = (2a/pi)^{3/4} (4a)^{l/2} / sqrt((2l-1)!!) and
// N_c^{-2} = sum_pq c_p c_q (2 sqrt(a_p a_q)/(a_p+a_q))^{l+3/2}.
// The remaining per-component factor sqrt((2l-1)!!/((2lx-1)!!(2ly-1)!!(2lz-1)!!))
// is applied to integrals at output time.

static double dfact_odd(int n) {
    double r = 1.0;
    for (int k = n; k > 1; k -= 2) r *= k;
    return r;
}

static void normalise(const int l, const int np, const double *a, const double *c, double *out) {
    double s = 0.0;
    for (int p = 0; p < np; ++p)
        for (int q = 0; q < np; ++q)
            s += c[p] * c[q] * pow(2.0 * sqrt(a[p] * a[q]) / (a[p] + a[q]), l + 1.5);
    const double nc = 1.0 / sqrt(s);
    for (int p = 0; p < np; ++p)
        out[p] = nc * c[p] * pow(2.0 * a[p] / M_PI, 0.75) * pow(4.0 * a[p], 0.5 * l) /
                 sqrt(dfact_odd(2 * l - 1));
}

// Primitive-pair screening.  For a primitive of exponent a and angular
// momentum l, every normalised Cartesian component obeys
//   |x^lx y^ly z^lz| e^{-a r^2} <= r^l e^{-a r^2} <= m e^{-(1-t) a r^2},
//   m = (l / (2 t a e))^{l/2}  (t = 0 and m = 1 for l = 0, t = 1/10 otherwise),
// times |c~| and the largest component scale (sqrt 3 for the mixed d).  The
// product of two such bounds is a single Gaussian of exponent p' = a' + b'
// with prefactor exp(-a'b'/p' |AB|^2); the Coulomb integral of two such
// non-negative Gaussians is at most 2 pi^{5/2} / (p' q' sqrt(p' + q')) (F_0 <= 1),
// and sqrt(p' + q') >= sqrt 2 (p' q')^{1/4}, so every primitive-quartet
// contribution |(uv|wx)| <= U_uv U_wx with
//   U_uv = w_u w_v exp(-a'b'/p' |AB|^2) 2^{1/4} pi^{5/4} p'^{-5/4}.
// A primitive pair with U_uv max(U) below eps is dropped, eps chosen so that
// all dropped quartets of one contracted integral together stay below
// 1e-14 (each pair keeps at least its largest term).
struct PrimScreen {
    std::vector<int> pp0, npp;
    std::vector<ushort2> uv;
    int64_t full = 0;  // unscreened primitive pairs
};

static PrimScreen screen_prim_pairs(const std::vector<int2> &pairs_ab, const double *xyz, const std::vector<int> &sh_atom,
                                    const std::vector<int> &sh_l, const std::vector<int> &sh_np,
                                    const std::vector<int> &sh_prim0, const double *alpha,
                                    const std::vector<double> &ct) {
    const double kE = 2.718281828459045, kPi = 3.141592653589793;
    const int nprim = (int)ct.size();
    std::vector<double> w(nprim), ap(nprim);
    for (size_t s = 0; s < sh_l.size(); ++s) {
        const int l = sh_l[s];
        const double t = l == 0 ? 0.0 : 0.1, smax = l == 2 ? std::sqrt(3.0) : 1.0;
        for (int u = sh_prim0[s]; u < sh_prim0[s] + sh_np[s]; ++u) {
            const double m = l == 0 ? 1.0 : std::pow(l / (2.0 * t * alpha[u] * kE), 0.5 * l);
            w[u] = std::fabs(ct[u]) * smax * m;
            ap[u] = (1.0 - t) * alpha[u];
        }
    }
    const double c0 = std::pow(2.0, 0.25) * std::pow(kPi, 1.25);
    // p^{-5/4} = 1 / (p p^{1/4}) from two square roots (the bound's
    // rounding is immaterial next to its slack)
    auto bound = [&](const double *A, const double *B, int pu, int pv) {
        const double r2 = (A[0] - B[0]) * (A[0] - B[0]) + (A[1] - B[1]) * (A[1] - B[1]) + (A[2] - B[2]) * (A[2] - B[2]);
        const double p = ap[pu] + ap[pv];
        return w[pu] * w[pv] * std::exp(-ap[pu] * ap[pv] / p * r2) * c0 / (p * std::sqrt(std::sqrt(p)));
    };
    // every primitive pair's bound once, then the cut against the largest
    std::vector<double> bnd;
    std::vector<int> boff(pairs_ab.size() + 1, 0);
    for (size_t i = 0; i < pairs_ab.size(); ++i) boff[i + 1] = boff[i] + sh_np[pairs_ab[i].x] * sh_np[pairs_ab[i].y];
    bnd.resize(boff.back());
    int nppmax = 1;
    for (const int2 &q : pairs_ab) nppmax = std::max(nppmax, sh_np[q.x] * sh_np[q.y]);
    // the bounds on host threads (contiguous ranges of pairs), then their maximum
    const int nt = (int)std::max(1u, std::min(16u, std::thread::hardware_concurrency()));
    std::vector<double> tmax(nt, 0.0);
    {
        std::vector<std::thread> pool;
        const size_t np = pairs_ab.size(), chunk = (np + nt - 1) / nt;
        for (int t = 0; t < nt; ++t)
            pool.emplace_back([&, t]() {
                double m = 0.0;
                for (size_t i = t * chunk; i < std::min(np, (t + 1) * chunk); ++i) {
                    const int2 q = pairs_ab[i];
                    const double *A = xyz + 3 * sh_atom[q.x], *B = xyz + 3 * sh_atom[q.y];
                    double *b = bnd.data() + boff[i];
                    for (int u = 0; u < sh_np[q.x]; ++u)
                        for (int v = 0; v < sh_np[q.y]; ++v) {
                            const double x = bound(A, B, sh_prim0[q.x] + u, sh_prim0[q.y] + v);
                            b[u * sh_np[q.y] + v] = x;
                            m = std::max(m, x);
                        }
                }
                tmax[t] = m;
            });
        for (auto &th : pool) th.join();
    }
    double umax = 0.0;
    for (double m : tmax) umax = std::max(umax, m);
    const double eps = 1e-14 / (2.0 * (double)nppmax * (double)nppmax);
    PrimScreen S;
    S.pp0.reserve(pairs_ab.size());
    S.npp.reserve(pairs_ab.size());
    for (size_t i = 0; i < pairs_ab.size(); ++i) {
        const int2 q = pairs_ab[i];
        const double *bq = bnd.data() + boff[i];
        const int k0 = (int)S.uv.size();
        S.pp0.push_back(k0);
        double best = -1.0;
        int bu = 0, bv = 0;
        for (int u = 0; u < sh_np[q.x]; ++u)
            for (int v = 0; v < sh_np[q.y]; ++v) {
                const double b = bq[u * sh_np[q.y] + v];
                if (b * umax >= eps) S.uv.push_back(make_ushort2((unsigned short)u, (unsigned short)v));
                if (b > best) {
                    best = b;
                    bu = u;
                    bv = v;
                }
            }
        if ((int)S.uv.size() == k0) S.uv.push_back(make_ushort2((unsigned short)bu, (unsigned short)bv));
        S.npp.push_back((int)S.uv.size() - k0);
        S.full += (int64_t)sh_np[q.x] * sh_np[q.y];
    }
    return S;
}

// ------------------------------------------------------ device kernels

struct ShellDev {
    double x, y, z;
    int prim0, nprim;
    int bf0, moff, mN;  // first function within its molecule; packed block of the molecule
};

__global__ void k_build_pairs(int n, const int2 *__restrict__ ab, const int *__restrict__ pp0,
                              const int *__restrict__ npp, const ushort2 *__restrict__ uv,
                              const ShellDev *__restrict__ sh, const double *__restrict__ alpha,
                              const double *__restrict__ ct, PairInfo *__restrict__ pairs,
                              PrimPair *__restrict__ pp) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const int sa = ab[i].x, sb = ab[i].y;
    const ShellDev A = sh[sa], B = sh[sb];
    PairInfo pi;
    pi.Ax = A.x; pi.Ay = A.y; pi.Az = A.z;
    pi.ABx = A.x - B.x; pi.ABy = A.y - B.y; pi.ABz = A.z - B.z;
    pi.pp0 = pp0[i];
    pi.npp = npp[i];
    pi.sa = sa; pi.sb = sb;
    pi.bfa = A.bf0; pi.bfb = B.bf0;
    pi.moff = A.moff; pi.mN = A.mN;
    pairs[i] = pi;
    const double ab2 = pi.ABx * pi.ABx + pi.ABy * pi.ABy + pi.ABz * pi.ABz;
    for (int k = pi.pp0; k < pi.pp0 + pi.npp; ++k) {
        const int u = uv[k].x, v = uv[k].y;
        const double a = alpha[A.prim0 + u], ca = ct[A.prim0 + u];
        const double b = alpha[B.prim0 + v], cb = ct[B.prim0 + v];
        const double p = a + b, rp = 1.0 / p;
        PrimPair q;
        q.PAx = -b * rp * pi.ABx;
        q.PAy = -b * rp * pi.ABy;
        q.PAz = -b * rp * pi.ABz;
        q.p = p;
        q.K = ca * cb * exp(-a * b * rp * ab2);
        q.rp = rp;
        // the primitive-quartet prefactor 2 pi^{5/2} K_P K_Q / (p q sqrt(p+q))
        // is then Kr_P Kr_Q (p+q)^{-1/2}
        q.Kr = 5.9149671727956129 * q.K * rp;
        q.pad1 = 0.0;
        pp[k] = q;
    }
}

// Rank of each pair within its (class, molecule) segment by descending
// primitive-pair count, then descending Q (ties by index), then
// perm[off + seg_lo + rank] = local index.  The pairs of a block of 256 lie
// in consecutive segments, so their union [seg_lo of the first, seg_hi of
// the last) is cut into chunks of kRankChunk (blockIdx.y), staged through
// LDS in tiles of 256; each thread counts the entries of its own segment
// that precede it and adds its count to cnt[i].
constexpr int kRankChunk = 1024;

__global__ void __launch_bounds__(256) k_rank_count(const double *__restrict__ Q, const PairInfo *__restrict__ pairs,
                                                    int off, int n, const int *__restrict__ seg_lo,
                                                    const int *__restrict__ seg_hi, int *__restrict__ cnt) {
    __shared__ double qs[256];
    __shared__ int ns[256];
    const int first = blockIdx.x * 256, last = min(n - 1, first + 255);
    const int i = first + threadIdx.x;
    const bool on = i < n;
    const int blo = seg_lo[off + first], bhi = seg_hi[off + last];
    const int c0 = blo + blockIdx.y * kRankChunk, c1 = min(bhi, c0 + kRankChunk);
    if (c0 >= c1) return;  // uniform over the block
    double qi = 0.0;
    int ni = 0, lo = 0, hi = 0;
    if (on) {
        qi = Q[off + i];
        ni = pairs[off + i].npp;
        lo = seg_lo[off + i];
        hi = seg_hi[off + i];
    }
    int rank = 0;
    for (int j0 = c0; j0 < c1; j0 += 256) {
        const int j = j0 + threadIdx.x;
        if (j < c1) {
            qs[threadIdx.x] = Q[off + j];
            ns[threadIdx.x] = pairs[off + j].npp;
        }
        __syncthreads();
        const int jb = max(lo, j0), je = min(hi, min(c1, j0 + 256));
        for (int jj = jb; jj < je; ++jj) {
            const double qj = qs[jj - j0];
            const int nj = ns[jj - j0];
            rank += (nj > ni) || (nj == ni && ((qj > qi) || (qj == qi && jj < i)));
        }
        __syncthreads();
    }
    if (on && rank) atomicAdd(&cnt[off + i], rank);
}

__global__ void k_rank_scatter(int off, int n, const int *__restrict__ seg_lo, const int *__restrict__ cnt,
                               int *__restrict__ perm) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) perm[off + seg_lo[off + i] + cnt[off + i]] = i;
}

__global__ void k_pp_to_f32(int64_t n, const PrimPair *__restrict__ pp, PrimPairF *__restrict__ ppf) {
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
        const PrimPair h = pp[i];
        ppf[i] = PrimPairF{(float)h.PAx, (float)h.PAy, (float)h.PAz, (float)h.p, (float)h.K, (float)h.rp, (float)h.Kr, 0.0f};
    }
}

__global__ void k_gather_pairs(int off, int n, const int *__restrict__ perm,
                               const PairInfo *__restrict__ src, const double *__restrict__ Qsrc,
                               PairInfo *__restrict__ dst, double *__restrict__ Qdst) {
    const int r = blockIdx.x * blockDim.x + threadIdx.x;
    if (r >= n) return;
    const int i = perm[off + r];
    dst[off + r] = src[off + i];
    Qdst[off + r] = Qsrc[off + i];
}

// ------------------------------------------------------- host helpers

static int make_class_launch(const mess_basis *B, ClassLaunch &L, hipStream_t s) {
    L.pairs = B->d_pairs;
    L.pp = B->d_pp;
    L.ppf = B->d_ppf;
    L.tab = B->d_boys;
    L.etab = B->d_boys_exp;
    L.tabt = B->d_boys_t;
    L.tabf = B->d_boys_f;
    L.etabf = B->d_boys_exp_f;
    L.N = B->nbf;
    L.stream = s;
    L.rowstart = nullptr;
    L.rowmap = nullptr;
    L.total = 0;
    L.bra_off = L.ket_off = L.nbra = L.same_class = 0;
    return MESS_OK;
}

int fill_class_launch(const mess_basis *B, const ClassList &cl, hipStream_t s, ClassLaunch &L) {
    make_class_launch(B, L, s);
    L.bra_off = B->pair_class_off[cl.cb];
    L.ket_off = B->pair_class_off[cl.ck];
    L.nbra = cl.nrow;
    L.same_class = cl.cb == cl.ck;
    L.rowstart = cl.d_rowstart;
    L.rowmap = cl.d_rowmap;
    L.segs = cl.d_segs;
    L.nseg = cl.d_segs ? cl.nseg : 0;
    L.groups = cl.d_groups;
    L.tiles = cl.d_tiles;
    L.grows = cl.d_grows;
    L.ngroups = cl.d_groups ? cl.ngroups : 0;
    L.nmax = B->nbf_max;
    L.total = cl.total;
    return MESS_OK;
}

int get_work_lists(mess_basis *B, double tau, hipStream_t s, WorkLists **out) {
    (void)s;
    if (!(tau > 0.0)) tau = 0.0;
    auto it = B->lists.find(tau);
    if (it != B->lists.end()) {
        *out = it->second;
        return MESS_OK;
    }
    auto *W = new WorkLists();
    W->tau = tau;
    // per class: host lists waiting for the single device copy
    struct Staged {
        std::vector<int4> segs, groups, tiles;
        std::vector<int> grows;
    };
    const std::vector<PairInfo> &P = B->pairs_host;
    const std::vector<double> &Q = B->pairQ_host;
    int rc = MESS_OK;
    // the 21 classes are independent: built on host threads, kept in class order
    std::vector<ClassList> built(kNumClasses);
    std::vector<Staged> staged(kNumClasses);
    auto build_class = [&](int cb, int ck) {
            ClassList &cl = built[class_index(cb, ck)];
            cl.cb = cb;
            cl.ck = ck;
            cl.nbra = B->pair_class_off[cb + 1] - B->pair_class_off[cb];
            const int boff = B->pair_class_off[cb], koff = B->pair_class_off[ck];
            const bool same = cb == ck;
            cl.h_rowstart.assign(1, 0);
            const int G = kGroupBras[cb];
            std::vector<int4> groups, tiles;
            std::vector<int> grows;
            for (int m = 0; m < B->n_mol; ++m) {
                // buckets of equal primitive count in the molecule's ket segment
                std::vector<int2> bk;
                const int k0 = B->seg_off[ck][m], k1 = k0 + B->seg_cnt[ck][m];
                for (int k = k0; k < k1;) {
                    int e = k + 1;
                    while (e < k1 && P[koff + e].npp == P[koff + k].npp) ++e;
                    bk.push_back(make_int2(k, e));
                    k = e;
                }
                const int i0 = B->seg_off[cb][m], i1 = i0 + B->seg_cnt[cb][m];
                const int mr0 = (int)cl.h_rowmap.size();
                for (int i = i0; i < i1; ++i) {
                    const double qi = Q[boff + i];
                    const int64_t nbp = P[boff + i].npp;
                    for (const int2 &b : bk) {
                        int cnt = b.y - b.x;
                        if (tau > 0.0) {
                            int lo = 0, hi = cnt;  // first ket with qi Q_j < tau
                            while (lo < hi) {
                                const int mid = (lo + hi) >> 1;
                                if (qi * Q[koff + b.x + mid] >= tau) lo = mid + 1; else hi = mid;
                            }
                            cnt = lo;
                        }
                        if (same) cnt = std::min(cnt, std::max(0, i - b.x + 1));
                        if (cnt <= 0) continue;
                        cl.h_rowmap.push_back(make_int2(i, b.x));
                        cl.h_rowstart.push_back(cl.h_rowstart.back() + cnt);
                        cl.prim_quartets += nbp * cnt * P[koff + b.x].npp;
                    }
                }
                if (G > 1) {
                    // rows of bra i: [first[i - i0], last[i - i0]) in bucket order
                    const int mr1 = (int)cl.h_rowmap.size();
                    std::vector<int> first(i1 - i0, -1), last(i1 - i0, -1);
                    for (int r = mr0; r < mr1; ++r) {
                        const int k = cl.h_rowmap[r].x - i0;
                        if (first[k] < 0) first[k] = r;
                        last[k] = r + 1;
                    }
                    for (int g0 = i0; g0 < i1; g0 += G) {
                        const int ng = std::min(G, i1 - g0), t0 = (int)tiles.size();
                        int ptr[8], kofs = 0;
                        for (int g = 0; g < ng; ++g) ptr[g] = first[g0 + g - i0];
                        for (const int2 &b : bk) {
                            const int rb = (int)grows.size();
                            int64_t maxc = 0;
                            for (int g = 0; g < G; ++g) {
                                int r = -1;
                                if (g < ng && ptr[g] >= 0 && ptr[g] < last[g0 + g - i0] &&
                                    cl.h_rowmap[ptr[g]].y == b.x) {
                                    r = ptr[g]++;
                                    maxc = std::max(maxc, cl.h_rowstart[r + 1] - cl.h_rowstart[r]);
                                }
                                grows.push_back(r);
                            }
                            if (maxc == 0) {
                                grows.resize(rb);
                                continue;
                            }
                            tiles.push_back(make_int4(rb, b.x, (int)maxc, kofs));
                            kofs += (int)maxc;
                        }
                        if ((int)tiles.size() > t0) groups.push_back(make_int4(t0, (int)tiles.size(), g0, ng));
                    }
                }
            }
            cl.nrow = (int)cl.h_rowmap.size();
            cl.total = cl.h_rowstart.back();
            std::vector<int4> segs;
            if (cl.total < ((int64_t)1 << 31))
                for (int r0 = 0; r0 < cl.nrow;) {
                    int r1 = r0 + 1;
                    while (r1 < cl.nrow && cl.h_rowmap[r1].x == cl.h_rowmap[r0].x) ++r1;
                    int rq = r0;  // row holding quartet q
                    for (int64_t q = cl.h_rowstart[r0]; q < cl.h_rowstart[r1]; q += kSegLen) {
                        const int64_t e = std::min(q + kSegLen, cl.h_rowstart[r1]);
                        while (cl.h_rowstart[rq + 1] <= q) ++rq;
                        segs.push_back(make_int4(rq, (int)q, (int)e, r1));
                    }
                    r0 = r1;
                }
            cl.nseg = (int)segs.size();
            if (cl.total >= ((int64_t)1 << 31)) groups.clear();
            cl.ngroups = (int)groups.size();
            staged[class_index(cb, ck)] = Staged{std::move(segs), std::move(groups), std::move(tiles), std::move(grows)};
    };
    {
        std::vector<std::thread> pool;
        std::atomic<int> next{0};
        const int nt = (int)std::min<unsigned>(kNumClasses, std::max(1u, std::thread::hardware_concurrency()));
        for (int t = 0; t < nt; ++t)
            pool.emplace_back([&]() {
                for (int c = next++; c < kNumClasses; c = next++) {
                    int cb = 0;
                    while ((cb + 1) * (cb + 2) / 2 <= c) ++cb;
                    build_class(cb, c - cb * (cb + 1) / 2);
                }
            });
        for (auto &th : pool) th.join();
    }
    // class order: cb ascending, ck ascending within (the fixed order of W->classes)
    for (int cb = 0; cb < kNumPairClasses; ++cb)
        for (int ck = 0; ck <= cb; ++ck) W->classes.push_back(std::move(built[class_index(cb, ck)]));
    {
        std::vector<Staged> ordered;
        for (int cb = 0; cb < kNumPairClasses; ++cb)
            for (int ck = 0; ck <= cb; ++ck) ordered.push_back(std::move(staged[class_index(cb, ck)]));
        staged.swap(ordered);
    }
    // every class's lists in one device buffer (one allocation, one copy)
    size_t bytes = 0;
    auto take = [&](size_t n) {
        const size_t o = bytes;
        bytes += (n + 255) / 256 * 256;
        return o;
    };
    std::vector<std::array<size_t, 6>> offs(W->classes.size());
    for (size_t c = 0; c < W->classes.size(); ++c) {
        const ClassList &cl = W->classes[c];
        const Staged &st = staged[c];
        if (cl.nrow > 0) {
            offs[c][0] = take(sizeof(int64_t) * (cl.nrow + 1));
            offs[c][1] = take(sizeof(int2) * cl.nrow);
        }
        if (cl.nseg > 0) offs[c][2] = take(sizeof(int4) * cl.nseg);
        if (cl.ngroups > 0) {
            offs[c][3] = take(sizeof(int4) * st.groups.size());
            offs[c][4] = take(sizeof(int4) * st.tiles.size());
            offs[c][5] = take(sizeof(int) * st.grows.size());
        }
    }
    if (bytes > 0) {
        std::vector<char> host(bytes);
        for (size_t c = 0; c < W->classes.size(); ++c) {
            const ClassList &cl = W->classes[c];
            const Staged &st = staged[c];
            if (cl.nrow > 0) {
                std::memcpy(host.data() + offs[c][0], cl.h_rowstart.data(), sizeof(int64_t) * (cl.nrow + 1));
                std::memcpy(host.data() + offs[c][1], cl.h_rowmap.data(), sizeof(int2) * cl.nrow);
            }
            if (cl.nseg > 0) std::memcpy(host.data() + offs[c][2], st.segs.data(), sizeof(int4) * cl.nseg);
            if (cl.ngroups > 0) {
                std::memcpy(host.data() + offs[c][3], st.groups.data(), sizeof(int4) * st.groups.size());
                std::memcpy(host.data() + offs[c][4], st.tiles.data(), sizeof(int4) * st.tiles.size());
                std::memcpy(host.data() + offs[c][5], st.grows.data(), sizeof(int) * st.grows.size());
            }
        }
        if (hipMalloc(&W->dbuf, bytes) != hipSuccess) {
            W->dbuf = nullptr;
            set_error("hipMalloc(work list, %zu bytes) failed", bytes);
            rc = MESS_E_NOMEM;
        } else if (hipMemcpy(W->dbuf, host.data(), bytes, hipMemcpyHostToDevice) != hipSuccess) {
            set_error("work list copy to the device failed");
            rc = MESS_E_DEVICE;
        }
    }
    if (rc == MESS_OK) {
        char *base = static_cast<char *>(W->dbuf);
        for (size_t c = 0; c < W->classes.size(); ++c) {
            ClassList &cl = W->classes[c];
            if (cl.nrow > 0) {
                cl.d_rowstart = reinterpret_cast<int64_t *>(base + offs[c][0]);
                cl.d_rowmap = reinterpret_cast<int2 *>(base + offs[c][1]);
            }
            if (cl.nseg > 0) cl.d_segs = reinterpret_cast<int4 *>(base + offs[c][2]);
            if (cl.ngroups > 0) {
                cl.d_groups = reinterpret_cast<int4 *>(base + offs[c][3]);
                cl.d_tiles = reinterpret_cast<int4 *>(base + offs[c][4]);
                cl.d_grows = reinterpret_cast<int *>(base + offs[c][5]);
            }
        }
    }
    if (rc != MESS_OK) {
        hipFree(W->dbuf);
        delete W;
        return rc;
    }
    B->lists[tau] = W;
    *out = W;
    return MESS_OK;
}

static void free_basis(mess_basis *B) {
    if (!B) return;
    for (auto &kv : B->lists) {
        hipFree(kv.second->dbuf);
        delete kv.second;
    }
    void free_stored(mess_basis *);
    free_stored(B);
    void free_xc(mess_basis *);
    free_xc(B);
    void free_guess_tables(mess_basis *);
    free_guess_tables(B);
    hipFree(B->d_xyz);
    hipFree(B->d_Zd);
    hipFree(B->d_boys);
    hipFree(B->d_boys_exp);
    hipFree(B->d_boys_t);
    hipFree(B->d_boys_f);
    hipFree(B->d_boys_exp_f);
    hipFree(B->d_pairs);
    hipFree(B->d_pairQ);
    hipFree(B->d_pp);
    hipFree(B->d_ppf);
    hipFree(B->scratch_jk);
    hipFree(B->det_acc);
    hipFree(B->d_mol_moff);
    hipFree(B->d_mol_nbf);
    delete B;
}

// Molecules are given back to back: molecule m owns atoms
// [atom0_m, atom0_m + natom_m) and shells [sh0_m, sh0_m + nsh_m), with
// shell_atom holding global atom indices.
static int create_impl(int n_mol, const int32_t *mol_natom, const int32_t *mol_nsh, const int32_t *charges,
                       int32_t n_atoms, const int32_t *Z, const double *xyz, int32_t n_shells,
                       const int32_t *shell_atom, const int32_t *shell_l, const int32_t *shell_nprim,
                       const double *exps, const double *coefs, mess_basis *B) {
    if (n_mol <= 0 || n_atoms <= 0 || n_shells <= 0 || !Z || !xyz || !shell_atom || !shell_l || !shell_nprim ||
        !exps || !coefs) {
        set_error("mess_basis_create: NULL array or non-positive count");
        return MESS_E_ARG;
    }
    B->n_mol = n_mol;
    B->nat = n_atoms;
    B->nsh = n_shells;
    B->Z.assign(Z, Z + n_atoms);
    B->xyz.assign(xyz, xyz + 3 * n_atoms);
    std::vector<int> atom_mol(n_atoms), shell_mol(n_shells);
    {
        int a0 = 0, s0 = 0;
        for (int m = 0; m < n_mol; ++m) {
            if (mol_natom[m] <= 0 || mol_nsh[m] <= 0) {
                set_error("mess_basis_create: molecule %d has no atoms or no shells", m);
                return MESS_E_ARG;
            }
            B->mol_atom0.push_back(a0);
            B->mol_natom.push_back(mol_natom[m]);
            B->mol_sh0.push_back(s0);
            B->mol_nsh.push_back(mol_nsh[m]);
            for (int a = a0; a < a0 + mol_natom[m] && a < n_atoms; ++a) atom_mol[a] = m;
            for (int q = s0; q < s0 + mol_nsh[m] && q < n_shells; ++q) shell_mol[q] = m;
            a0 += mol_natom[m];
            s0 += mol_nsh[m];
        }
        if (a0 != n_atoms || s0 != n_shells) {
            set_error("mess_basis_create: per-molecule atom/shell counts do not add up");
            return MESS_E_ARG;
        }
    }
    for (int a = 0; a < n_atoms; ++a) {
        if (Z[a] < 0 || Z[a] > 118) {
            set_error("mess_basis_create: atomic number %d out of range", Z[a]);
            return MESS_E_ARG;
        }
        for (int x = 0; x < 3; ++x)
            if (!std::isfinite(xyz[3 * a + x])) {
                set_error("mess_basis_create: non-finite coordinate of atom %d", a);
                return MESS_E_ARG;
            }
    }
    int nprim = 0, nbf = 0;
    B->sh_atom.resize(n_shells);
    B->sh_l.resize(n_shells);
    B->sh_np.resize(n_shells);
    B->sh_prim0.resize(n_shells);
    B->sh_bf0.resize(n_shells);
    for (int s = 0; s < n_shells; ++s) {
        const int m = shell_mol[s];
        if (shell_atom[s] < B->mol_atom0[m] || shell_atom[s] >= B->mol_atom0[m] + B->mol_natom[m]) {
            set_error("mess_basis_create: shell %d on atom %d out of range", s, shell_atom[s]);
            return MESS_E_ARG;
        }
        if (shell_l[s] < 0 || shell_l[s] > 2) {
            set_error("mess_basis_create: shell %d has l=%d; only s, p, d (l <= 2) are built", s,
                      shell_l[s]);
            return shell_l[s] < 0 ? MESS_E_ARG : MESS_E_UNSUPPORTED;
        }
        if (shell_nprim[s] < 1 || shell_nprim[s] > 16) {
            set_error("mess_basis_create: shell %d has %d primitives (1..16 allowed)", s, shell_nprim[s]);
            return MESS_E_ARG;
        }
        B->sh_atom[s] = shell_atom[s];
        B->sh_l[s] = shell_l[s];
        B->sh_np[s] = shell_nprim[s];
        B->sh_prim0[s] = nprim;
        B->sh_bf0[s] = nbf;
        nprim += shell_nprim[s];
        nbf += ncart(shell_l[s]);
    }
    B->nbf = nbf;
    // per molecule: functions, packed block, electrons, nuclear repulsion
    B->mol_moff.assign(1, 0);
    B->packed = 0;
    int tot_e = 0;
    double tot_en = 0.0;
    for (int m = 0; m < n_mol; ++m) {
        const int s0 = B->mol_sh0[m], s1 = s0 + B->mol_nsh[m];
        const int bf0 = B->sh_bf0[s0];
        const int bf1 = s1 < n_shells ? B->sh_bf0[s1] : nbf;
        B->mol_bf0.push_back(bf0);
        B->mol_nbf.push_back(bf1 - bf0);
        B->packed += (int64_t)(bf1 - bf0) * (bf1 - bf0);
        B->mol_moff.push_back(B->packed);
        int zsum = 0;
        double en = 0.0;
        const int a0 = B->mol_atom0[m], a1 = a0 + B->mol_natom[m];
        for (int a = a0; a < a1; ++a) {
            zsum += Z[a];
            for (int b = a0; b < a; ++b) {
                const double dx = xyz[3 * a] - xyz[3 * b], dy = xyz[3 * a + 1] - xyz[3 * b + 1],
                             dz = xyz[3 * a + 2] - xyz[3 * b + 2];
                const double r = sqrt(dx * dx + dy * dy + dz * dz);
                if (r == 0.0 && Z[a] * Z[b] != 0) {
                    set_error("mess_basis_create: atoms %d and %d coincide", a, b);
                    return MESS_E_ARG;
                }
                if (r > 0.0) en += (double)Z[a] * Z[b] / r;
            }
        }
        const int ne = zsum - (charges ? charges[m] : 0);
        if (ne < 0) {
            set_error("mess_basis_create: negative electron count in molecule %d", m);
            return MESS_E_ARG;
        }
        B->mol_nelec.push_back(ne);
        B->mol_nocc.push_back(ne / 2);
        B->mol_enuc.push_back(en);
        tot_e += ne;
        tot_en += en;
    }
    B->nelec = tot_e;
    B->nocc = tot_e / 2;
    B->enuc = tot_en;
    B->alpha.assign(exps, exps + nprim);
    B->ctilde.assign(nprim, 0.0);
    for (int p = 0; p < nprim; ++p)
        if (!(exps[p] > 0.0) || !std::isfinite(exps[p]) || !std::isfinite(coefs[p])) {
            set_error("mess_basis_create: primitive %d has exponent %g, coefficient %g", p, exps[p], coefs[p]);
            return MESS_E_ARG;
        }
    for (int s = 0; s < n_shells; ++s)
        normalise(B->sh_l[s], B->sh_np[s], exps + B->sh_prim0[s], coefs + B->sh_prim0[s],
                  B->ctilde.data() + B->sh_prim0[s]);
    for (int p = 0; p < nprim; ++p)
        if (!std::isfinite(B->ctilde[p])) {
            set_error("mess_basis_create: contraction of shell with primitive %d cannot be normalised", p);
            return MESS_E_ARG;
        }
    MESS_HIP(hipGetDevice(&B->device));

    // Boys tables
    std::vector<double> tab, etab;
    std::vector<double> tabt;
    build_boys_table(tab, etab, tabt);
    std::vector<float> tabf(tab.begin(), tab.end()), etabf(etab.begin(), etab.end());
    MESS_HIP(hipMalloc(&B->d_boys, sizeof(double) * tab.size()));
    MESS_HIP(hipMalloc(&B->d_boys_exp, sizeof(double) * etab.size()));
    MESS_HIP(hipMalloc(&B->d_boys_t, sizeof(double) * tabt.size()));
    MESS_HIP(hipMemcpy(B->d_boys_t, tabt.data(), sizeof(double) * tabt.size(), hipMemcpyHostToDevice));
    MESS_HIP(hipMalloc(&B->d_boys_f, sizeof(float) * tabf.size()));
    MESS_HIP(hipMalloc(&B->d_boys_exp_f, sizeof(float) * etabf.size()));
    MESS_HIP(hipMemcpy(B->d_boys, tab.data(), sizeof(double) * tab.size(), hipMemcpyHostToDevice));
    MESS_HIP(hipMemcpy(B->d_boys_exp, etab.data(), sizeof(double) * etab.size(), hipMemcpyHostToDevice));
    MESS_HIP(hipMemcpy(B->d_boys_f, tabf.data(), sizeof(float) * tabf.size(), hipMemcpyHostToDevice));
    MESS_HIP(hipMemcpy(B->d_boys_exp_f, etabf.data(), sizeof(float) * etabf.size(), hipMemcpyHostToDevice));

    // atoms
    std::vector<double> Zd(Z, Z + n_atoms);
    B->nbf_max = 0;
    for (int m = 0; m < n_mol; ++m) B->nbf_max = std::max(B->nbf_max, B->mol_nbf[m]);
    MESS_HIP(hipMalloc(&B->d_mol_moff, sizeof(int64_t) * (n_mol + 1)));
    MESS_HIP(hipMalloc(&B->d_mol_nbf, sizeof(int) * n_mol));
    MESS_HIP(hipMemcpy(B->d_mol_moff, B->mol_moff.data(), sizeof(int64_t) * (n_mol + 1), hipMemcpyHostToDevice));
    MESS_HIP(hipMemcpy(B->d_mol_nbf, B->mol_nbf.data(), sizeof(int) * n_mol, hipMemcpyHostToDevice));
    MESS_HIP(hipMalloc(&B->d_xyz, sizeof(double) * 3 * n_atoms));
    MESS_HIP(hipMalloc(&B->d_Zd, sizeof(double) * n_atoms));
    MESS_HIP(hipMemcpy(B->d_xyz, xyz, sizeof(double) * 3 * n_atoms, hipMemcpyHostToDevice));
    MESS_HIP(hipMemcpy(B->d_Zd, Zd.data(), sizeof(double) * n_atoms, hipMemcpyHostToDevice));

    // shell pairs (a, b) of one molecule with l_a > l_b, or l_a == l_b and
    // a >= b, grouped by class, then by molecule
    std::vector<int2> pairs_ab;
    std::vector<int> seg_lo, seg_hi;  // per pair: its (class, molecule) segment, relative to the class
    for (int c = 0; c < kNumPairClasses; ++c) {
        B->pair_class_off[c] = (int)pairs_ab.size();
        B->seg_off[c].assign(n_mol, 0);
        B->seg_cnt[c].assign(n_mol, 0);
        for (int m = 0; m < n_mol; ++m) {
            const int lo = (int)pairs_ab.size() - B->pair_class_off[c];
            const int s0 = B->mol_sh0[m], s1 = s0 + B->mol_nsh[m];
            for (int a = s0; a < s1; ++a)
                for (int b = s0; b < s1; ++b) {
                    const int la = B->sh_l[a], lb = B->sh_l[b];
                    if (!(la > lb || (la == lb && a >= b)) || pair_class_of(la, lb) != c) continue;
                    pairs_ab.push_back(make_int2(a, b));
                }
            const int hi = (int)pairs_ab.size() - B->pair_class_off[c];
            B->seg_off[c][m] = lo;
            B->seg_cnt[c][m] = hi - lo;
            for (int k = lo; k < hi; ++k) {
                seg_lo.push_back(lo);
                seg_hi.push_back(hi);
            }
        }
    }
    B->pair_class_off[kNumPairClasses] = (int)pairs_ab.size();
    B->npair = (int)pairs_ab.size();
    const PrimScreen screen =
        screen_prim_pairs(pairs_ab, xyz, B->sh_atom, B->sh_l, B->sh_np, B->sh_prim0, exps, B->ctilde);
    const int npp = (int)screen.uv.size();
    B->npp = npp;
    B->npp_full = screen.full;
    std::vector<ShellDev> shd(n_shells);
    for (int s = 0; s < n_shells; ++s) {
        const int a = B->sh_atom[s], m = shell_mol[s];
        shd[s] = ShellDev{xyz[3 * a], xyz[3 * a + 1], xyz[3 * a + 2], B->sh_prim0[s], B->sh_np[s],
                          B->sh_bf0[s] - B->mol_bf0[m], (int)B->mol_moff[m], B->mol_nbf[m]};
    }

    int2 *d_ab = nullptr;
    int *d_pp0 = nullptr, *d_npp = nullptr, *d_perm = nullptr, *d_cnt = nullptr, *d_seglo = nullptr, *d_seghi = nullptr;
    ushort2 *d_uv = nullptr;
    ShellDev *d_sh = nullptr;
    double *d_alpha = nullptr, *d_ct = nullptr, *d_Qraw = nullptr;
    PairInfo *d_pairs_raw = nullptr;
    int rc = MESS_OK;
    auto cleanup = [&]() {
        hipFree(d_ab); hipFree(d_pp0); hipFree(d_npp); hipFree(d_uv); hipFree(d_seglo); hipFree(d_seghi); hipFree(d_perm); hipFree(d_cnt); hipFree(d_sh);
        hipFree(d_alpha); hipFree(d_ct); hipFree(d_Qraw); hipFree(d_pairs_raw);
    };
#define MESS_HIPC(call)                                                                         \
    do {                                                                                        \
        hipError_t _e = (call);                                                                 \
        if (_e != hipSuccess) {                                                                 \
            set_error("%s failed: %s", #call, hipGetErrorString(_e));                           \
            cleanup();                                                                          \
            return _e == hipErrorOutOfMemory ? MESS_E_NOMEM : MESS_E_DEVICE;                    \
        }                                                                                       \
    } while (0)
    const int np_ = B->npair;
    MESS_HIPC(hipMalloc(&d_ab, sizeof(int2) * np_));
    MESS_HIPC(hipMalloc(&d_pp0, sizeof(int) * np_));
    MESS_HIPC(hipMalloc(&d_npp, sizeof(int) * np_));
    MESS_HIPC(hipMalloc(&d_uv, sizeof(ushort2) * npp));
    MESS_HIPC(hipMalloc(&d_seglo, sizeof(int) * np_));
    MESS_HIPC(hipMalloc(&d_seghi, sizeof(int) * np_));
    MESS_HIPC(hipMalloc(&d_perm, sizeof(int) * np_));
    MESS_HIPC(hipMalloc(&d_cnt, sizeof(int) * np_));
    MESS_HIPC(hipMemset(d_cnt, 0, sizeof(int) * np_));
    MESS_HIPC(hipMalloc(&d_sh, sizeof(ShellDev) * n_shells));
    MESS_HIPC(hipMalloc(&d_alpha, sizeof(double) * nprim));
    MESS_HIPC(hipMalloc(&d_ct, sizeof(double) * nprim));
    MESS_HIPC(hipMalloc(&d_Qraw, sizeof(double) * np_));
    MESS_HIPC(hipMalloc(&d_pairs_raw, sizeof(PairInfo) * np_));
    MESS_HIPC(hipMalloc(&B->d_pairs, sizeof(PairInfo) * np_));
    MESS_HIPC(hipMalloc(&B->d_pairQ, sizeof(double) * np_));
    MESS_HIPC(hipMalloc(&B->d_pp, sizeof(PrimPair) * npp));
    MESS_HIPC(hipMemcpy(d_ab, pairs_ab.data(), sizeof(int2) * np_, hipMemcpyHostToDevice));
    MESS_HIPC(hipMemcpy(d_pp0, screen.pp0.data(), sizeof(int) * np_, hipMemcpyHostToDevice));
    MESS_HIPC(hipMemcpy(d_npp, screen.npp.data(), sizeof(int) * np_, hipMemcpyHostToDevice));
    MESS_HIPC(hipMemcpy(d_uv, screen.uv.data(), sizeof(ushort2) * npp, hipMemcpyHostToDevice));
    MESS_HIPC(hipMemcpy(d_seglo, seg_lo.data(), sizeof(int) * np_, hipMemcpyHostToDevice));
    MESS_HIPC(hipMemcpy(d_seghi, seg_hi.data(), sizeof(int) * np_, hipMemcpyHostToDevice));
    MESS_HIPC(hipMemcpy(d_sh, shd.data(), sizeof(ShellDev) * n_shells, hipMemcpyHostToDevice));
    MESS_HIPC(hipMemcpy(d_alpha, exps, sizeof(double) * nprim, hipMemcpyHostToDevice));
    MESS_HIPC(hipMemcpy(d_ct, B->ctilde.data(), sizeof(double) * nprim, hipMemcpyHostToDevice));
    hipStream_t s = nullptr;
    hipLaunchKernelGGL(k_build_pairs, dim3((np_ + 127) / 128), dim3(128), 0, s, np_, d_ab, d_pp0, d_npp, d_uv, d_sh, d_alpha,
                       d_ct, d_pairs_raw, B->d_pp);
    MESS_HIPC(hipGetLastError());

    // Schwarz factors per pair (diagonal quartets), then sort each class by Q
    ClassLaunch L;
    make_class_launch(B, L, s);
    L.pairs = d_pairs_raw;
    for (int c = 0; c < kNumPairClasses && rc == MESS_OK; ++c) {
        const int off = B->pair_class_off[c], n = B->pair_class_off[c + 1] - off;
        if (n == 0) continue;
        rc = dispatch_class(c, c, [&](auto CB, auto CK) {
            return ClassOps<decltype(CB)::value, decltype(CK)::value>::schwarz(L, off, n, d_Qraw);
        });
    }
    if (rc != MESS_OK) {
        cleanup();
        return rc;
    }
    for (int c = 0; c < kNumPairClasses; ++c) {
        const int off = B->pair_class_off[c], n = B->pair_class_off[c + 1] - off;
        if (n == 0) continue;
        // chunks along y: the longest block span of this class, in kRankChunk
        int span = 0;
        for (int f = 0; f < n; f += 256)
            span = std::max(span, seg_hi[off + std::min(n - 1, f + 255)] - seg_lo[off + f]);
        const dim3 grid((unsigned)((n + 255) / 256), (unsigned)((span + kRankChunk - 1) / kRankChunk));
        hipLaunchKernelGGL(k_rank_count, grid, dim3(256), 0, s, d_Qraw, d_pairs_raw, off, n, d_seglo, d_seghi, d_cnt);
        hipLaunchKernelGGL(k_rank_scatter, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, off, n, d_seglo, d_cnt,
                           d_perm);
        hipLaunchKernelGGL(k_gather_pairs, dim3((n + 255) / 256), dim3(256), 0, s, off, n, d_perm, d_pairs_raw,
                           d_Qraw, B->d_pairs, B->d_pairQ);
    }
    MESS_HIPC(hipGetLastError());
    B->pairQ_host.resize(np_);
    MESS_HIPC(hipMemcpy(B->pairQ_host.data(), B->d_pairQ, sizeof(double) * np_, hipMemcpyDeviceToHost));
    B->pairs_host.resize(np_);
    MESS_HIPC(hipMemcpy(B->pairs_host.data(), B->d_pairs, sizeof(PairInfo) * np_, hipMemcpyDeviceToHost));
    for (int i = 0; i < np_; ++i)
        if (!std::isfinite(B->pairQ_host[i])) {
            set_error("mess_basis_create: non-finite Schwarz factor (pair %d)", i);
            cleanup();
            return MESS_E_NUMERIC;
        }
    // FP32 copy of the primitive-pair table
    MESS_HIPC(hipMalloc(&B->d_ppf, sizeof(PrimPairF) * npp));
    hipLaunchKernelGGL(k_pp_to_f32, dim3((unsigned)std::min<int64_t>(((int64_t)npp + 255) / 256, 65536)), dim3(256), 0,
                       s, (int64_t)npp, B->d_pp, B->d_ppf);
    MESS_HIPC(hipGetLastError());
    MESS_HIPC(hipStreamSynchronize(s));
    MESS_HIPC(hipMalloc(&B->scratch_jk, sizeof(double) * 2 * (size_t)B->packed));
#undef MESS_HIPC
    cleanup();
    return MESS_OK;
}

}  // namespace mess

using namespace mess;

extern "C" {

const char *mess_last_error(void) { return g_err; }

int mess_basis_create(int32_t n_atoms, const int32_t *Z, const double *xyz_bohr, int32_t n_shells,
                      const int32_t *shell_atom, const int32_t *shell_l, const int32_t *shell_nprim,
                      const double *exps, const double *coefs, int32_t charge, mess_basis **out) {
    g_err[0] = 0;
    if (!out) {
        set_error("mess_basis_create: out is NULL");
        return MESS_E_ARG;
    }
    *out = nullptr;
    auto *B = new mess_basis();
    int rc = create_impl(1, &n_atoms, &n_shells, &charge, n_atoms, Z, xyz_bohr, n_shells, shell_atom, shell_l,
                         shell_nprim, exps, coefs, B);
    if (rc != MESS_OK) {
        free_basis(B);
        return rc;
    }
    *out = B;
    return MESS_OK;
}

int mess_batch_create(int32_t n_mol, const int32_t *mol_atoms, const int32_t *mol_shells, const int32_t *charges,
                      const int32_t *Z, const double *xyz_bohr, const int32_t *shell_atom, const int32_t *shell_l,
                      const int32_t *shell_nprim, const double *exps, const double *coefs, mess_basis **out) {
    g_err[0] = 0;
    if (!out || n_mol <= 0 || !mol_atoms || !mol_shells || !shell_atom) {
        set_error("mess_batch_create: NULL argument or no molecules");
        return MESS_E_ARG;
    }
    *out = nullptr;
    int64_t na = 0, ns = 0;
    for (int m = 0; m < n_mol; ++m) {
        na += mol_atoms[m];
        ns += mol_shells[m];
    }
    if (na <= 0 || ns <= 0 || na > (1 << 30) || ns > (1 << 30)) {
        set_error("mess_batch_create: atom/shell totals out of range");
        return MESS_E_ARG;
    }
    // shell_atom is molecule-local: convert to global atom indices
    std::vector<int32_t> sa(ns);
    {
        int64_t a0 = 0, s0 = 0;
        for (int m = 0; m < n_mol; ++m) {
            for (int k = 0; k < mol_shells[m]; ++k) {
                const int32_t la = shell_atom[s0 + k];
                sa[s0 + k] = (la >= 0 && la < mol_atoms[m]) ? (int32_t)(a0 + la) : -1;
            }
            a0 += mol_atoms[m];
            s0 += mol_shells[m];
        }
    }
    auto *B = new mess_basis();
    int rc = create_impl(n_mol, mol_atoms, mol_shells, charges, (int32_t)na, Z, xyz_bohr, (int32_t)ns, sa.data(),
                         shell_l, shell_nprim, exps, coefs, B);
    if (rc != MESS_OK) {
        free_basis(B);
        return rc;
    }
    *out = B;
    return MESS_OK;
}

int mess_batch_info(const mess_basis *B, int32_t *n_mol, int32_t *nbf, int64_t *moff, int32_t *n_occ,
                    double *e_nuc) {
    if (!B) {
        set_error("mess_batch_info: basis is NULL");
        return MESS_E_ARG;
    }
    if (n_mol) *n_mol = B->n_mol;
    for (int m = 0; m < B->n_mol; ++m) {
        if (nbf) nbf[m] = B->mol_nbf[m];
        if (moff) moff[m] = B->mol_moff[m];
        if (n_occ) n_occ[m] = B->mol_nocc[m];
        if (e_nuc) e_nuc[m] = B->mol_enuc[m];
    }
    if (moff) moff[B->n_mol] = B->packed;
    return MESS_OK;
}

void mess_basis_destroy(mess_basis *basis) { free_basis(basis); }

int mess_prim_pairs(const mess_basis *basis, int64_t *kept, int64_t *full) {
    if (!basis) {
        set_error("mess_prim_pairs: NULL basis");
        return MESS_E_ARG;
    }
    if (kept) *kept = basis->npp;
    if (full) *full = basis->npp_full;
    return MESS_OK;
}

int mess_work_stats(const mess_basis *basis, double schwarz_tol, int32_t cls, int64_t *quartets,
                    int64_t *prim_quartets, double *alg_flops_jk) {
    if (!basis || cls < 0 || cls > 20) {
        set_error("mess_work_stats: NULL basis or class index outside 0..20");
        return MESS_E_ARG;
    }
    WorkLists *W = nullptr;
    MESS_TRY(get_work_lists(const_cast<mess_basis *>(basis), schwarz_tol, nullptr, &W));
    for (const ClassList &cl : W->classes)
        if (class_index(cl.cb, cl.ck) == cls) {
            double fp = 0.0, fq = 0.0;
            class_flops(cl.cb, cl.ck, &fp, &fq);
            if (quartets) *quartets = cl.total;
            if (prim_quartets) *prim_quartets = cl.prim_quartets;
            if (alg_flops_jk) *alg_flops_jk = fp * (double)cl.prim_quartets + fq * (double)cl.total;
            return MESS_OK;
        }
    if (quartets) *quartets = 0;
    if (prim_quartets) *prim_quartets = 0;
    if (alg_flops_jk) *alg_flops_jk = 0.0;
    return MESS_OK;
}

int mess_basis_info(const mess_basis *B, int32_t *nbf, int32_t *n_occ, double *e_nuc) {
    if (!B) {
        set_error("mess_basis_info: basis is NULL");
        return MESS_E_ARG;
    }
    if (nbf) *nbf = B->nbf;
    if (n_occ) *n_occ = B->nocc;
    if (e_nuc) *e_nuc = B->enuc;
    return MESS_OK;
}

}  // extern "C"
