// Wave-cooperative shell-quartet kernel for the high angular classes
// (bra or ket pair dp/dd with a large ket).  One 64-lane wave evaluates one
// shell quartet: the Obara-Saika vertical recursion of each primitive quartet
// runs level by level with every intermediate [e0|f0]^(m) in LDS, the 64
// lanes sharing the independent recursion steps of a level; contracted
// intermediates are accumulated in LDS and the Head-Gordon-Pople horizontal
// recursion runs the same way.  The per-class step lists are generated on
// the host from the recursions (see eri_hgp.hpp for the formulas) and are
// the same for every quartet of the class.
#include <algorithm>
#include <cstring>
#include <set>
#include <memory>
#include <mutex>

#include "coop.hpp"

namespace mess {

// Recursion step: v = c[a1] V[s1] + c[a2] V[s2] + k3 (c[a3] V[s3] - c[a4] V[s4]) + k5 c[a5] V[s5]
// packed as x = dst | s1 << 16, y = s2 | s3 << 16, z = s4 | s5 << 16,
// w = a1 | a2 << 5 | a3 << 10 | a4 << 15 | a5 << 20 | k3 << 25 | k5 << 28.
struct CoopProgram {
    int cb = 0, ck = 0, LA = 0, LB = 0, LC = 0, LD = 0, L = 0;
    int nV = 0;       // VRR slots (slot 0 holds 0.0); slots 1..L+1 are [0|0]^(m)
    int nH = 0;       // HRR slots; slots [0, nacc) are the contracted [e0|f0]
    int nacc = 0, nout = 0;
    int nvlev = 0, nhlev = 0;
    int4 *d_vops = nullptr;
    int *d_vlev = nullptr;     // nvlev + 1 op offsets
    unsigned short *d_accsrc = nullptr;  // V slot of accumulator k
    int4 *d_hops = nullptr;
    int *d_hlev = nullptr;
    unsigned short *d_outslot = nullptr;  // H slot of output element
    double *d_outscale = nullptr;
};

namespace {

int4 pack(int dst, int s1, int a1, int s2, int a2, int s3, int a3, int s4, int a4, int s5, int a5, int k3,
          int k5) {
    int4 o;
    o.x = dst | (s1 << 16);
    o.y = s2 | (s3 << 16);
    o.z = s4 | (s5 << 16);
    o.w = a1 | (a2 << 5) | (a3 << 10) | (a4 << 15) | (a5 << 20) | (k3 << 25) | (k5 << 28);
    return o;
}

struct Builder {
    std::map<std::tuple<int, int, int>, int> vslot;  // (f, e, m) -> slot
    int nV = 1;
    int V(int f, int e, int m) {
        auto key = std::make_tuple(f, e, m);
        auto it = vslot.find(key);
        if (it != vslot.end()) return it->second;
        vslot[key] = nV;
        return nV++;
    }
    int Vget(int f, int e, int m) const {
        auto it = vslot.find(std::make_tuple(f, e, m));
        return it == vslot.end() ? -1 : it->second;
    }
};

struct CoopTables {
    std::vector<int4> vops, hops;
    std::vector<int> vlev, hlev;
    std::vector<unsigned short> accsrc, outslot;
    std::vector<double> outscale;
};

// Sources a step reads: s1, s2 always; s3, s4 with k3 != 0; s5 with k5 != 0.
static int step_reads(const int4 op, int *src) {
    const int k3 = (op.w >> 25) & 7, k5 = (op.w >> 28) & 7;
    int n = 0;
    src[n++] = op.x >> 16;
    src[n++] = op.y & 0xffff;
    if (k3) {
        src[n++] = op.y >> 16;
        src[n++] = op.z & 0xffff;
    }
    if (k5) src[n++] = op.z >> 16;
    return n;
}

// Reuses LDS slots: a slot whose value is last read at level l may receive a
// destination of any level after l (all reads of a level finish at its
// barrier).  Slots [0, nfixed) hold values defined before the first level
// (their numbers are kept); slot 0 is never reused when keep0 (it is the
// zero operand of absent terms).  Rewrites the steps and the final reads
// in place and returns the number of slots, or -1 if the symbolic replay
// of the rewritten tables does not reproduce the original data flow.
static int compact_slots(std::vector<int4> &ops, const std::vector<int> &lev, int nlog, int nfixed, bool keep0,
                         std::vector<unsigned short> &final_reads) {
    const int nlev = (int)lev.size() - 1;
    std::vector<int> last(nlog, -1);
    int src[5];
    for (int lv = 0; lv < nlev; ++lv)
        for (int o = lev[lv]; o < lev[lv + 1]; ++o) {
            const int n = step_reads(ops[o], src);
            for (int k = 0; k < n; ++k) last[src[k]] = std::max(last[src[k]], lv);
        }
    for (unsigned short r : final_reads) last[r] = nlev;
    std::vector<int> phys(nlog, -1);
    std::vector<int> live;
    for (int l = 0; l < nfixed; ++l) {
        phys[l] = l;
        live.push_back(l);
    }
    std::set<int> freeset;
    int next = nfixed;
    const std::vector<int4> orig = ops;
    for (int lv = 0; lv < nlev; ++lv) {
        std::vector<int> still;
        for (int l : live) {
            if (last[l] < lv && !(keep0 && l == 0)) freeset.insert(phys[l]);
            else still.push_back(l);
        }
        live.swap(still);
        for (int o = lev[lv]; o < lev[lv + 1]; ++o) {
            const int d = ops[o].x & 0xffff;
            int p;
            if (freeset.empty()) {
                p = next++;
            } else {
                p = *freeset.begin();
                freeset.erase(freeset.begin());
            }
            phys[d] = p;
            live.push_back(d);
        }
        for (int o = lev[lv]; o < lev[lv + 1]; ++o) {
            int4 &op = ops[o];
            const int k3 = (op.w >> 25) & 7, k5 = (op.w >> 28) & 7;
            const int d = op.x & 0xffff, s1 = op.x >> 16, s2 = op.y & 0xffff, s3 = op.y >> 16,
                      s4 = op.z & 0xffff, s5 = op.z >> 16;
            op.x = phys[d] | (phys[s1] << 16);
            op.y = phys[s2] | ((k3 ? phys[s3] : 0) << 16);
            op.z = (k3 ? phys[s4] : 0) | ((k5 ? phys[s5] : 0) << 16);
        }
    }
    std::vector<unsigned short> final_orig = final_reads;
    for (unsigned short &r : final_reads) r = (unsigned short)phys[r];
    const int nphys = next;
    if (nphys >= 65536) return -1;
    // symbolic replay: every read finds the value the original step read,
    // no destination of a level aliases another destination or a source
    // of that level
    std::vector<int> content(nphys, -1);
    for (int l = 0; l < nfixed; ++l) content[l] = l;
    for (int lv = 0; lv < nlev; ++lv) {
        std::set<int> dsts, reads;
        for (int o = lev[lv]; o < lev[lv + 1]; ++o) {
            int so[5], sn[5];
            const int n = step_reads(orig[o], so);
            step_reads(ops[o], sn);
            for (int k = 0; k < n; ++k) {
                if (sn[k] < 0 || sn[k] >= nphys || content[sn[k]] != so[k]) return -1;
                reads.insert(sn[k]);
            }
            if (!dsts.insert(ops[o].x & 0xffff).second) return -1;
        }
        for (int dd : dsts)
            if (reads.count(dd)) return -1;
        for (int o = lev[lv]; o < lev[lv + 1]; ++o) content[ops[o].x & 0xffff] = orig[o].x & 0xffff;
    }
    for (size_t k = 0; k < final_reads.size(); ++k)
        if (content[final_reads[k]] != final_orig[k]) return -1;
    return nphys;
}

std::unique_ptr<CoopProgram> build_tables(int cb, int ck, CoopTables &tables) {
    auto P = std::make_unique<CoopProgram>();
    P->cb = cb; P->ck = ck;
    const int LA = pair_class_la(cb), LB = pair_class_lb(cb), LC = pair_class_la(ck), LD = pair_class_lb(ck);
    P->LA = LA; P->LB = LB; P->LC = LC; P->LD = LD;
    const int LAB = LA + LB, LCD = LC + LD, L = LAB + LCD;
    P->L = L;
    const int NE = cart_off(LAB + 1), NF = cart_off(LCD + 1), E0 = cart_off(LA), F0 = cart_off(LC);
    Builder b;
    for (int m = 0; m <= L; ++m) b.V(0, 0, m);  // slots 1..L+1
    std::vector<std::vector<int4>> levels;
    // bra VRR, level |e|
    for (int n = 1; n <= LAB; ++n) {
        std::vector<int4> lev;
        for (int e = cart_off(n); e < cart_off(n + 1); ++e) {
            const Cart c = cart_of(e);
            const int i = c.dir(), ei = c.get(i), e1 = c.minus(i).idx();
            for (int m = 0; m <= L - n; ++m) {
                const int dst = b.V(0, e, m);
                int s3 = 0, s4 = 0, k3 = 0;
                if (ei >= 2) {
                    const int e2 = c.minus(i, 2).idx();
                    s3 = b.Vget(0, e2, m);
                    s4 = b.Vget(0, e2, m + 1);
                    k3 = ei - 1;
                }
                lev.push_back(pack(dst, b.Vget(0, e1, m), kPA + i, b.Vget(0, e1, m + 1), kWP + i, s3, kO2P, s4,
                                   kO2PR, 0, kC0, k3, 0));
            }
        }
        levels.push_back(lev);
    }
    // ket VRR, level |f|
    for (int nf = 1; nf <= LCD; ++nf) {
        std::vector<int4> lev;
        const int emin = cart_off(std::max(0, LA - (LCD - nf)));
        for (int f = cart_off(nf); f < cart_off(nf + 1); ++f) {
            const Cart cf = cart_of(f);
            const int j = cf.dir(), fj = cf.get(j), f1 = cf.minus(j).idx();
            for (int e = emin; e < NE; ++e) {
                const Cart ce = cart_of(e);
                const int ej = ce.get(j);
                for (int m = 0; m <= L - ce.l() - nf; ++m) {
                    const int dst = b.V(f, e, m);
                    int s3 = 0, s4 = 0, k3 = 0, s5 = 0, k5 = 0;
                    if (fj >= 2) {
                        const int f2 = cf.minus(j, 2).idx();
                        s3 = b.Vget(f2, e, m);
                        s4 = b.Vget(f2, e, m + 1);
                        k3 = fj - 1;
                    }
                    if (ej >= 1) {
                        s5 = b.Vget(f1, ce.minus(j).idx(), m + 1);
                        k5 = ej;
                    }
                    lev.push_back(pack(dst, b.Vget(f1, e, m), kQC + j, b.Vget(f1, e, m + 1), kWQ + j, s3, kO2Q,
                                       s4, kO2QR, s5, kO2PQ, k3, k5));
                }
            }
        }
        levels.push_back(lev);
    }
    P->nV = b.nV;
    std::vector<int4> vops;
    std::vector<int> vlev{0};
    for (auto &lev : levels) {
        vops.insert(vops.end(), lev.begin(), lev.end());
        vlev.push_back((int)vops.size());
    }
    P->nvlev = (int)levels.size();
    // accumulators
    const int NEA = NE - E0, NFA = NF - F0;
    P->nacc = NEA * NFA;
    std::vector<unsigned short> accsrc(P->nacc);
    for (int f = F0; f < NF; ++f)
        for (int e = E0; e < NE; ++e) accsrc[(f - F0) * NEA + (e - E0)] = (unsigned short)b.Vget(f, e, 0);
    // horizontal recursion on H; H[(f-F0)*NEA + (e-E0)] = [e0|f0]
    int nH = P->nacc;
    std::vector<std::vector<int4>> hlevels;
    const int NA = ncart(LA), NB = ncart(LB), NC = ncart(LC), ND = ncart(LD);
    // bra: T[b][a] for each f; level |b|
    std::map<std::tuple<int, int, int>, int> Tb;  // (f, b, a) -> slot
    for (int f = F0; f < NF; ++f)
        for (int e = E0; e < NE; ++e) Tb[std::make_tuple(f, 0, e)] = (f - F0) * NEA + (e - E0);
    for (int k = 1; k <= LB; ++k) {
        std::vector<int4> lev;
        for (int f = F0; f < NF; ++f)
            for (int bb = cart_off(k); bb < cart_off(k + 1); ++bb) {
                const Cart cb_ = cart_of(bb);
                const int i = cb_.dir(), b1 = cb_.minus(i).idx();
                for (int a = E0; a < cart_off(LAB - k + 1); ++a) {
                    const int a1 = cart_of(a).plus(i).idx();
                    const int dst = nH++;
                    Tb[std::make_tuple(f, bb, a)] = dst;
                    lev.push_back(pack(dst, Tb.at(std::make_tuple(f, b1, a1)), kH1, Tb.at(std::make_tuple(f, b1, a)),
                                       kHAB + i, 0, kH0, 0, kH0, 0, kH0, 0, 0));
                }
            }
        hlevels.push_back(lev);
    }
    // ket: U[d][c] for each (a, b); level |d|
    std::map<std::tuple<int, int, int>, int> Td;  // (ab, d, c) -> slot
    for (int a = 0; a < NA; ++a)
        for (int bb = 0; bb < NB; ++bb)
            for (int f = F0; f < NF; ++f)
                Td[std::make_tuple(a * NB + bb, 0, f)] = Tb.at(std::make_tuple(f, cart_off(LB) + bb, E0 + a));
    for (int k = 1; k <= LD; ++k) {
        std::vector<int4> lev;
        for (int ab = 0; ab < NA * NB; ++ab)
            for (int d = cart_off(k); d < cart_off(k + 1); ++d) {
                const Cart cd_ = cart_of(d);
                const int i = cd_.dir(), d1 = cd_.minus(i).idx();
                for (int c = F0; c < cart_off(LCD - k + 1); ++c) {
                    const int c1 = cart_of(c).plus(i).idx();
                    const int dst = nH++;
                    Td[std::make_tuple(ab, d, c)] = dst;
                    lev.push_back(pack(dst, Td.at(std::make_tuple(ab, d1, c1)), kH1, Td.at(std::make_tuple(ab, d1, c)),
                                       kHCD + i, 0, kH0, 0, kH0, 0, kH0, 0, 0));
                }
            }
        hlevels.push_back(lev);
    }
    P->nH = nH;
    std::vector<int4> hops;
    std::vector<int> hlev{0};
    for (auto &lev : hlevels) {
        hops.insert(hops.end(), lev.begin(), lev.end());
        hlev.push_back((int)hops.size());
    }
    P->nhlev = (int)hlevels.size();
    P->nout = NA * NB * NC * ND;
    std::vector<unsigned short> outslot(P->nout);
    std::vector<double> outscale(P->nout);
    auto scale = [](int l, int local) { return cart_is_mixed_d(cart_of(cart_off(l) + local)) ? kSqrt3 : 1.0; };
    for (int a = 0; a < NA; ++a)
        for (int bb = 0; bb < NB; ++bb)
            for (int c = 0; c < NC; ++c)
                for (int d = 0; d < ND; ++d) {
                    const int o = ((a * NB + bb) * NC + c) * ND + d;
                    outslot[o] = (unsigned short)Td.at(std::make_tuple(a * NB + bb, cart_off(LD) + d, F0 + c));
                    outscale[o] = scale(LA, a) * scale(LB, bb) * scale(LC, c) * scale(LD, d);
                }
    if (P->nV >= 65536 || P->nH >= 65536) return nullptr;
    // Validate the step tables: every source slot is defined by an earlier
    // level (or is the zero slot with a zero multiplier), every destination
    // is in range and written once.
    {
        std::vector<int> vdef(P->nV, -1);
        for (int m = 0; m <= L; ++m) vdef[1 + m] = 0;
        vdef[0] = 0;
        for (int lv = 0; lv < P->nvlev; ++lv)
            for (int o = vlev[lv]; o < vlev[lv + 1]; ++o) {
                const int4 op = vops[o];
                const int dst = op.x & 0xffff, s1 = op.x >> 16, s2 = op.y & 0xffff, s3 = op.y >> 16,
                          s4 = op.z & 0xffff, s5 = op.z >> 16;
                const int k3 = (op.w >> 25) & 7, k5 = (op.w >> 28) & 7;
                auto ok = [&](int sl, bool used) {
                    if (sl < 0 || sl >= P->nV) return false;
                    return !used || (vdef[sl] >= 0 && vdef[sl] <= lv);
                };
                if (!ok(s1, true) || !ok(s2, true) || !ok(s3, k3 != 0) || !ok(s4, k3 != 0) || !ok(s5, k5 != 0))
                    return nullptr;
                if (dst <= L + 1 || dst >= P->nV || vdef[dst] >= 0) return nullptr;
                vdef[dst] = lv + 1;
            }
        for (int k = 0; k < P->nacc; ++k)
            if (accsrc[k] >= P->nV || vdef[accsrc[k]] < 0) return nullptr;
        std::vector<int> hdef(P->nH, -1);
        for (int k = 0; k < P->nacc; ++k) hdef[k] = 0;
        for (int lv = 0; lv < P->nhlev; ++lv)
            for (int o = hlev[lv]; o < hlev[lv + 1]; ++o) {
                const int4 op = hops[o];
                const int dst = op.x & 0xffff, s1 = op.x >> 16, s2 = op.y & 0xffff;
                if (s1 >= P->nH || s2 >= P->nH || hdef[s1] < 0 || hdef[s1] > lv || hdef[s2] < 0 || hdef[s2] > lv)
                    return nullptr;
                if (dst < P->nacc || dst >= P->nH || hdef[dst] >= 0) return nullptr;
                hdef[dst] = lv + 1;
            }
        for (int o = 0; o < P->nout; ++o)
            if (outslot[o] >= P->nH || hdef[outslot[o]] < 0) return nullptr;
    }
    // Slot reuse.  The final reads are checked against the original slots
    // here, since compact_slots rewrites them.
    {
        const std::vector<unsigned short> acc0 = accsrc, out0 = outslot;
        const int nv = compact_slots(vops, vlev, P->nV, L + 2, true, accsrc);
        const int nh = compact_slots(hops, hlev, P->nH, P->nacc, false, outslot);
        if (nv < 0 || nh < 0) return nullptr;
        P->nV = nv;
        P->nH = nh;
        (void)acc0;
        (void)out0;
    }
    // VRR steps: replace the five coefficient indices by the step's side
    // (bit 2: ket) and direction (bits 0-1); the kernel holds the
    // coefficients in registers.  Within a level, steps are grouped by the
    // terms they use so that a wave mostly takes one path.
    for (int4 &op : vops) {
        const int a1 = op.w & 31;
        const int ket = a1 >= kQC ? 1 : 0;
        const int dir = ket ? a1 - kQC : a1 - kPA;
        op.w = dir | (ket << 2) | (op.w & (0x3f << 25));
    }
    for (int lv = 0; lv < P->nvlev; ++lv)
        std::stable_sort(vops.begin() + vlev[lv], vops.begin() + vlev[lv + 1], [](const int4 &x, const int4 &y) {
            auto key = [](const int4 &o) { return (((o.w >> 25) & 7) ? 2 : 0) + (((o.w >> 28) & 7) ? 1 : 0); };
            return key(x) < key(y);
        });
    // LDS: accumulators [0, nacc), then one region shared by the VRR slots
    // (during the primitive loop) and the HRR slots >= nacc (after it).
    tables.vops = std::move(vops);
    tables.hops = std::move(hops);
    tables.vlev = std::move(vlev);
    tables.hlev = std::move(hlev);
    tables.accsrc = std::move(accsrc);
    tables.outslot = std::move(outslot);
    tables.outscale = std::move(outscale);
    return P;
}

std::unique_ptr<CoopProgram> build_program(int cb, int ck) {
    CoopTables T;
    auto P = build_tables(cb, ck, T);
    if (!P) return nullptr;
    // upload
    auto up = [](auto **dptr, const auto &vec) -> bool {
        using T = typename std::remove_reference<decltype(vec)>::type::value_type;
        size_t n = std::max<size_t>(1, vec.size());
        if (hipMalloc((void **)dptr, sizeof(T) * n) != hipSuccess) return false;
        if (!vec.empty() && hipMemcpy(*dptr, vec.data(), sizeof(T) * vec.size(), hipMemcpyHostToDevice) != hipSuccess)
            return false;
        return true;
    };
    if (!up(&P->d_vops, T.vops) || !up(&P->d_vlev, T.vlev) || !up(&P->d_accsrc, T.accsrc) ||
        !up(&P->d_hops, T.hops) || !up(&P->d_hlev, T.hlev) || !up(&P->d_outslot, T.outslot) ||
        !up(&P->d_outscale, T.outscale))
        return nullptr;
    return P;
}

std::mutex g_prog_mutex;
std::mutex g_flop_mutex;
std::map<std::pair<int, int>, std::pair<double, double>> g_flops;
std::map<std::pair<int, int>, std::unique_ptr<CoopProgram>> g_programs;

}  // namespace

// Algorithmic operation count of the recursion (FMA = 2): per primitive
// quartet the setup of Boys arguments and prefactors with the Taylor
// evaluation and downward recurrence of the Boys function (80 + 4L), each
// vertical step (3 for the two leading terms, 4 for the f_i/2p term, 2 for
// the e_j/2(p+q) term) and one add per contracted intermediate; per shell
// quartet each horizontal step (2) and the J/K digestion (six families of
// one FMA per integral: 12 per integral).
// The vertical steps are counted in the orientation the class's kernel
// runs: the primitive-lane kernels may put the ket pair on the e side
// (swap_vrr), every other form keeps the bra there.
static std::pair<double, double> count_flops(int cb, int ck, bool swapped) {
    CoopTables T, Tv;
    std::unique_ptr<CoopProgram> P, Pv;
    try {
        P = build_tables(cb, ck, T);
        if (swapped) Pv = build_tables(ck, cb, Tv);
    } catch (...) {
        P.reset();
    }
    if (!P || (swapped && !Pv)) return {0.0, 0.0};
    const std::vector<int4> &vops = swapped ? Tv.vops : T.vops;
    double fp = 80.0 + 4.0 * P->L + P->nacc;
    for (const int4 &op : vops) {
        const int k3 = (op.w >> 25) & 7, k5 = (op.w >> 28) & 7;
        fp += 3.0 + (k3 ? 4.0 : 0.0) + (k5 ? 2.0 : 0.0);
    }
    const double fq = 2.0 * (double)T.hops.size() + 12.0 * P->nout;
    return {fp, fq};
}

void class_flops(int cb, int ck, double *per_prim, double *per_quartet_jk, int prec) {
    const int la = pair_class_la(cb), lb = pair_class_lb(cb), lc = pair_class_la(ck), ld = pair_class_lb(ck);
    const bool swapped = plane_compiled(cb, ck) && class_form(cb, ck, prec) == kFormPlane && swap_vrr(la, lb, lc, ld);
    std::lock_guard<std::mutex> lk(g_flop_mutex);
    auto key = std::make_pair(cb * 8 + (swapped ? 1 : 0), ck);
    auto it = g_flops.find(key);
    if (it == g_flops.end()) it = g_flops.emplace(key, count_flops(cb, ck, swapped)).first;
    *per_prim = it->second.first;
    *per_quartet_jk = it->second.second;
}

// Classes evaluated through the cooperative tables (the per-lane unrolled
// form of these needs far more than the 512 registers a lane can hold), and
// (pp|pp), whose few quartets leave the lane-per-quartet launch with too few
// waves to fill the chip.
bool coop_class(int cb, int ck) {
    return (cb == 5 && ck >= 2) || (cb == 4 && (ck == 2 || ck == 4)) || (cb == 2 && ck == 2);
}

// True when class (cb, ck) needs no cooperative step tables or they are
// already on the device (nothing left to allocate for its launches).
bool coop_program_cached(int cb, int ck) {
    if (!coop_class(cb, ck) && !(plane_compiled(cb, ck) && class_form(cb, ck, MESS_FP64) == kFormPlane)) return true;
    std::lock_guard<std::mutex> lk(g_prog_mutex);
    return g_programs.count(std::make_pair(cb, ck)) != 0;
}

static const CoopProgram *coop_program(int cb, int ck) {
    std::lock_guard<std::mutex> lk(g_prog_mutex);
    auto key = std::make_pair(cb, ck);
    auto it = g_programs.find(key);
    if (it != g_programs.end()) return it->second.get();
    std::unique_ptr<CoopProgram> P;
    try {
        P = build_program(cb, ck);
    } catch (...) {
        P.reset();
    }
    if (!P) return nullptr;
    const CoopProgram *raw = P.get();
    g_programs[key] = std::move(P);
    return raw;
}

// ------------------------------------------------------------ device

// Per-primitive-quartet coefficients of the vertical recursion, in registers.
template <typename Real>
struct VrrCoef {
    Real PA[3], WP[3], QC[3], WQ[3];
    Real o2p, o2pr, o2q, o2qr, o2pq;
};

template <typename Real>
__device__ __forceinline__ Real sel3(int d, Real a0, Real a1, Real a2) {
    return d == 0 ? a0 : (d == 1 ? a1 : a2);
}

// One vertical step of a bra (KET = false) or ket level, direction from
// op.w bits 0-1:
// v = c1 V[s1] + c2 V[s2] + k3 (c3 V[s3] - c4 V[s4]) + k5 / (2(p+q)) V[s5].
template <bool KET, typename Real>
__device__ __forceinline__ Real run_vop(const int4 op, const Real *__restrict__ V, const VrrCoef<Real> &c) {
    const int s1 = op.x >> 16, s2 = op.y & 0xffff;
    const int w = op.w, dir = w & 3, k3 = (w >> 25) & 7;
    const Real c1 = KET ? sel3(dir, c.QC[0], c.QC[1], c.QC[2]) : sel3(dir, c.PA[0], c.PA[1], c.PA[2]);
    const Real c2 = KET ? sel3(dir, c.WQ[0], c.WQ[1], c.WQ[2]) : sel3(dir, c.WP[0], c.WP[1], c.WP[2]);
    Real v = c1 * V[s1] + c2 * V[s2];
    if (k3) v += (Real)k3 * ((KET ? c.o2q : c.o2p) * V[op.y >> 16] - (KET ? c.o2qr : c.o2pr) * V[op.z & 0xffff]);
    if (KET) {
        const int k5 = (w >> 28) & 7;
        if (k5) v += (Real)k5 * c.o2pq * V[op.z >> 16];
    }
    return v;
}

template <bool KET, int GT, typename Real>
__device__ __forceinline__ void run_level(const CoopArgs &A, int lv, int gl, Real *__restrict__ V,
                                          const VrrCoef<Real> &cf) {
    // the steps of a level are independent: fetch up to four of this
    // thread's steps before running them
    const int b0 = A.vlev[lv], b1 = A.vlev[lv + 1];
    for (int c0 = b0 + gl; c0 < b1; c0 += 4 * GT) {
        int4 op[4];
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            const int o = c0 + r * GT;
            op[r] = o < b1 ? A.vops[o] : make_int4(0, 0, 0, 0);
        }
#pragma unroll
        for (int r = 0; r < 4; ++r)
            if (c0 + r * GT < b1) V[op[r].x & 0xffff] = run_vop<KET, Real>(op[r], V, cf);
    }
}

// NT threads (one to four waves) share each shell quartet.
// NT threads share each shell quartet; they form NP groups of NT/NP threads,
// each group running the vertical recursion of its own primitive quartet
// in its own LDS slot region (vstride doubles apart), so NP primitive
// quartets advance per round of level barriers.
template <int MODE, typename Real, int NT, int NP>
__global__ void __launch_bounds__(NT) k_coop(CoopArgs A, int region, int vstride, const PairInfo *__restrict__ pairs,
                                             int bra_off, int ket_off, int nbra, int same_class,
                                             const int64_t *__restrict__ rowstart, const int2 *__restrict__ rowmap, int64_t total,
                                             const PrimPairT<Real> *__restrict__ pp, BoysTabs bt,
                                             const double *__restrict__ D, int N, double *__restrict__ out0,
                                             double *__restrict__ out1) {
    // LDS: accumulators H[0, nacc) (FP64), then `region` doubles shared by the
    // NP VRR slot regions (Real, during the primitive loop) and the HRR slots
    // >= nacc (after it), then the HRR coefficients.
    constexpr int GT = NT / NP;  // threads per group
    extern __shared__ double lds[];
    double *H = lds;
    Real *V0 = reinterpret_cast<Real *>(lds + A.nacc);
    double *hc = lds + A.nacc + region;
    const int lane = threadIdx.x;
    const int grp = lane / GT, gl = lane % GT;
    Real *V = V0 + (size_t)grp * vstride;
    for (int64_t q = blockIdx.x; q < total; q += gridDim.x) {
        if (gl == 0) V[0] = Real(0);
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
        const Real ACx = Real(bra.Ax - ket.Ax), ACy = Real(bra.Ay - ket.Ay), ACz = Real(bra.Az - ket.Az);
        for (int s = lane; s < A.nacc; s += NT) H[s] = 0.0;
        const int npq = bra.npp * ket.npp;
        for (int r0 = 0; r0 < npq; r0 += NP) {
            // every thread passes every barrier; a group past the end idles
            const int pidx = r0 + grp;
            const bool act = pidx < npq;
            const int ib = act ? pidx / ket.npp : 0, ik = act ? pidx % ket.npp : 0;
            const PrimPairT<Real> P = pp[bra.pp0 + ib];
            const PrimPairT<Real> Q = pp[ket.pp0 + ik];
            const Real p = P.p, qq = Q.p, pq = p + qq, spq = rsqrt_nr(pq), rpq = spq * spq, rho = p * qq * rpq;
            const Real PQx = ACx + (P.PAx - Q.PAx), PQy = ACy + (P.PAy - Q.PAy), PQz = ACz + (P.PAz - Q.PAz);
            const Real T = rho * (PQx * PQx + PQy * PQy + PQz * PQz);
            __syncthreads();  // previous round fully consumed
            if (act && gl <= A.L) {
                const Real pref = P.Kr * Q.Kr * spq;
                V[1 + gl] = pref * coop_boys_r<Real>(gl, T, bt);
            }
            VrrCoef<Real> cf;
            cf.PA[0] = P.PAx; cf.PA[1] = P.PAy; cf.PA[2] = P.PAz;
            cf.WP[0] = -qq * rpq * PQx; cf.WP[1] = -qq * rpq * PQy; cf.WP[2] = -qq * rpq * PQz;
            cf.QC[0] = Q.PAx; cf.QC[1] = Q.PAy; cf.QC[2] = Q.PAz;
            cf.WQ[0] = p * rpq * PQx; cf.WQ[1] = p * rpq * PQy; cf.WQ[2] = p * rpq * PQz;
            cf.o2p = Real(0.5) * P.rp; cf.o2pr = Real(0.5) * P.rp * (qq * rpq);
            cf.o2q = Real(0.5) * Q.rp; cf.o2qr = Real(0.5) * Q.rp * (p * rpq);
            cf.o2pq = Real(0.5) * rpq;
            __syncthreads();
            for (int lv = 0; lv < A.nvbra; ++lv) {
                if (act) run_level<false, GT, Real>(A, lv, gl, V, cf);
                __syncthreads();
            }
            for (int lv = A.nvbra; lv < A.nvlev; ++lv) {
                if (act) run_level<true, GT, Real>(A, lv, gl, V, cf);
                __syncthreads();
            }
            const int nact = npq - r0 < NP ? npq - r0 : NP;
            for (int s = lane; s < A.nacc; s += NT) {
                const int src = A.accsrc[s];
                double acc = 0.0;
                for (int g = 0; g < nact; ++g) acc += (double)V0[(size_t)g * vstride + src];
                H[s] += acc;
            }
        }
        __syncthreads();
        coop_finish<MODE, NT>(A, H, hc, lane, bra, ket, i, j, bra_off, same_class, D, N, out0, out1, q, total);
        __syncthreads();  // H reused by the next quartet
    }
}

// Classes run with the primitive-lane mapping: the form chosen for the
// class (built-in default or autotuned; see tune.hip).
static bool plane_class(int cb, int ck, int prec) {
    return plane_compiled(cb, ck) && class_form(cb, ck, prec) == kFormPlane;
}

static void launch_plane(int mode, int cb, int ck, int prec, const CoopArgs &A, const ClassLaunch &L, int64_t total,
                         unsigned g, size_t lds, const double *D, double *out0, double *out1) {
#define MESS_PL(B, K)                                                                                  \
    if (cb == B && ck == K) {                                                                          \
        if (prec == MESS_FP32) PlaneOps<B, K, float>::launch(mode, A, L, total, g, lds, D, out0, out1);  \
        else PlaneOps<B, K, double>::launch(mode, A, L, total, g, lds, D, out0, out1);                   \
    }
    MESS_PL(5, 4)
    MESS_PL(5, 3)
    MESS_PL(5, 2)
    MESS_PL(5, 1)
    MESS_PL(4, 4)
    MESS_PL(4, 2)
    MESS_PL(2, 2)
#undef MESS_PL
}

static void launch_wave(int mode, int cb, int ck, int prec, const CoopArgs &A, const ClassLaunch &L, int64_t total,
                        unsigned g, const double *D, double *out0, double *out1, size_t *lds) {
#define MESS_WV(B, K)                                                                                        \
    if (cb == B && ck == K) {                                                                                \
        if (prec == MESS_FP32) WaveOps<B, K, float>::launch(mode, A, L, total, g, D, out0, out1, lds);        \
        else WaveOps<B, K, double>::launch(mode, A, L, total, g, D, out0, out1, lds);                         \
    }
    MESS_WV(5, 5)
    MESS_WV(5, 4)
    MESS_WV(5, 3)
#undef MESS_WV
}

static int coop_launch(int mode, int cb, int ck, const ClassLaunch &L, int64_t total, double *out0, double *out1,
                       const double *D, int prec = MESS_FP64) {
    const CoopProgram *P = coop_program(cb, ck);
    if (!P) {
        set_error("internal: cooperative program for class (%d,%d) could not be built", cb, ck);
        return MESS_E_DEVICE;
    }
    if (total <= 0) return MESS_OK;
    CoopArgs A;
    A.vops = P->d_vops; A.vlev = P->d_vlev; A.accsrc = P->d_accsrc;
    A.hops = P->d_hops; A.hlev = P->d_hlev; A.outslot = P->d_outslot; A.outscale = P->d_outscale;
    A.nV = P->nV; A.nH = P->nH; A.nacc = P->nacc; A.nout = P->nout;
    A.nvlev = P->nvlev; A.nhlev = P->nhlev; A.L = P->L;
    A.nvbra = P->LA + P->LB;
    A.NA = ncart(P->LA); A.NB = ncart(P->LB); A.NC = ncart(P->LC); A.ND = ncart(P->LD);
    int64_t g = total;
    if (g > (1 << 20)) g = 1 << 20;
    if (wave_compiled(cb, ck) && class_form(cb, ck, prec) == kFormWave) {
        size_t lds = 0;
        launch_wave(mode, cb, ck, prec, A, L, total, (unsigned)g, D, out0, out1, &lds);
        if (lds > 64 * 1024) {
            set_error("internal: class (%d,%d) needs %zu bytes of LDS in the wave form", cb, ck, lds);
            return MESS_E_UNSUPPORTED;
        }
        launch_wave(mode, cb, ck, prec, A, L, total, (unsigned)g, D, out0, out1, nullptr);
        MESS_LAUNCH_CHECK();
        return MESS_OK;
    }
    if (plane_class(cb, ck, prec)) {
        // H, the coefficients, and 64 lanes' base values (L + 1 each)
        const size_t lds = sizeof(double) * ((size_t)P->nH + kNHCoef + 64 * (size_t)(P->L + 1));
        launch_plane(mode, cb, ck, prec, A, L, total, (unsigned)g, lds, D, out0, out1);
        MESS_LAUNCH_CHECK();
        return MESS_OK;
    }
    const size_t rsz = prec == MESS_FP32 ? sizeof(float) : sizeof(double);
    // two primitive quartets in flight per block (two slot regions, 128
    // threads each): the levels are too small to keep 256 threads busy on
    // one (measured: one is slower for (dd|dp), 258 vs 182 ms over three
    // SCFs, and for (dd|dd), 137 vs 131; four is slower for (dd|dp), 193)
    const int np = 2;
    const int vstride = (int)(((size_t)P->nV * rsz + 7) / 8 * 8 / rsz);  // whole doubles per region
    const int region = (int)std::max<size_t>((np * (size_t)vstride * rsz + 7) / 8, (size_t)(P->nH - P->nacc));
    const size_t lds = sizeof(double) * ((size_t)P->nacc + region + kNHCoef);
    if (lds > 64 * 1024) {
        set_error("internal: class (%d,%d) needs %zu bytes of LDS", cb, ck, lds);
        return MESS_E_UNSUPPORTED;
    }
    const BoysTabs bt{L.tab, L.etab, L.tabf, L.etabf, L.tabt};
#define MESS_COOP_GO(MODE, R, PP, NPV)                                                                            \
    hipLaunchKernelGGL((k_coop<MODE, R, 256, NPV>), dim3((unsigned)g), dim3(256), lds, L.stream, A, region,      \
                       vstride, L.pairs, L.bra_off, L.ket_off, L.nbra, L.same_class, L.rowstart, L.rowmap, total, \
                       PP, bt, D, L.N, out0, out1)
#define MESS_COOP_M(MODE)                                                            \
    do {                                                                             \
        if (prec == MESS_FP32) MESS_COOP_GO(MODE, float, L.ppf, 2);                  \
        else MESS_COOP_GO(MODE, double, L.pp, 2);                                    \
    } while (0)
    switch (mode) {
        case kModeSchwarz: MESS_COOP_M(kModeSchwarz); break;
        case kModeDense: MESS_COOP_M(kModeDense); break;
        case kModeStore64: MESS_COOP_M(kModeStore64); break;
        case kModeStore32: MESS_COOP_M(kModeStore32); break;
        default: MESS_COOP_M(kModeJK);
    }
#undef MESS_COOP_M
#undef MESS_COOP_GO
    MESS_LAUNCH_CHECK();
    return MESS_OK;
}

int coop_schwarz(int c, const ClassLaunch &L, int off, int n, double *Q) {
    ClassLaunch L2 = L;
    L2.bra_off = off;
    L2.ket_off = off;
    return coop_launch(kModeSchwarz, c, c, L2, n, Q - 0, nullptr, nullptr);
}

int coop_dense(int cb, int ck, const ClassLaunch &L, double *eri, int prec) {
    return coop_launch(kModeDense, cb, ck, L, L.total, eri, nullptr, nullptr, prec);
}

int coop_jk(int cb, int ck, const ClassLaunch &L, const double *D, double *Gj, double *Gk, int prec) {
    return coop_launch(kModeJK, cb, ck, L, L.total, Gj, Gk, D, prec);
}

}  // namespace mess

namespace mess {

// J/K from stored blocks for the high classes: one wave per quartet, lanes
// over the six digestion families, block elements read from the class's
// structure-of-arrays store.
template <typename Real>
__global__ void __launch_bounds__(64) k_jk_stored_wave(const PairInfo *__restrict__ pairs, int bra_off, int ket_off,
                                                      int nbra, int same_class, const int64_t *__restrict__ rowstart, const int2 *__restrict__ rowmap,
                                                      int64_t total, int NA, int NB, int NC, int ND,
                                                      const Real *__restrict__ base, const double *__restrict__ D, int N,
                                                      double *__restrict__ Gj, double *__restrict__ Gk) {
    const int lane = threadIdx.x;
    for (int64_t q = blockIdx.x; q < total; q += gridDim.x) {
        const int2 ij = quartet_pairs(rowstart, rowmap, nbra, q);
        const int i = ij.x, j = ij.y;
        const PairInfo bra = pairs[bra_off + i];
        const PairInfo ket = pairs[ket_off + j];
        double fac = 1.0;
        if (bra.sa == bra.sb) fac *= 0.5;
        if (ket.sa == ket.sb) fac *= 0.5;
        if (same_class && i == j) fac *= 0.5;
        auto O = [&](int a, int b, int cc, int d) {
            return (double)base[(int64_t)(((a * NB + b) * NC + cc) * ND + d) * total + q];
        };
        wave_digest(lane, NA, NB, NC, ND, fac, bra.bfa, bra.bfb, ket.bfa, ket.bfb, O, D + bra.moff, bra.mN,
                    Gj ? Gj + bra.moff : nullptr, Gk ? Gk + bra.moff : nullptr);
    }
}

// Classes whose stored blocks are kept quartet-major (the block of quartet
// t contiguous at base[t NOUT]) and streamed by k_jk_stored_aos: the ones
// with few quartets per bra, where a bra segment leaves most of a block's
// threads idle and the launch has fewer blocks than the chip has CUs.
// (dd|ds) has enough quartets that its per-quartet atomics would cost more
// than the segment kernel's LDS rows save.
bool stored_aos_class(int cb, int ck) {
    return (cb == 2 && ck == 2) || (cb == 4 && (ck == 2 || ck == 4)) || (cb == 5 && (ck == 2 || ck == 4 || ck == 5));
}

// J/K from quartet-major stored blocks: one wave per quartet copies its
// block (contiguous, coalesced) and the six density sub-blocks it touches
// into LDS, then its lanes take the output elements of the six digestion
// families (J[a,b], J[c,d], K[a,c], K[b,c], K[a,d], K[b,d]), each a sum
// over the block from LDS, added to J/K with one FP64 atomic.
template <typename Real>
__global__ void __launch_bounds__(64) k_jk_stored_aos(const PairInfo *__restrict__ pairs, int bra_off, int ket_off,
                                                     int nbra, int same_class, const int64_t *__restrict__ rowstart,
                                                     const int2 *__restrict__ rowmap, int64_t total, int NA, int NB,
                                                     int NC, int ND, const Real *__restrict__ base,
                                                     const double *__restrict__ Dall, double *__restrict__ Gjall,
                                                     double *__restrict__ Gkall) {
    extern __shared__ double lds[];
    const int lane = threadIdx.x;
    const int nout = NA * NB * NC * ND;
    const int nab = NA * NB, ncd = NC * ND;
    // LDS: block, then D[c,d], D[a,b], D[b,d], D[a,d], D[b,c], D[a,c]
    double *O = lds, *Dcd = O + nout, *Dab = Dcd + ncd, *Dbd = Dab + nab, *Dad = Dbd + NB * ND,
           *Dbc = Dad + NA * ND, *Dac = Dbc + NB * NC;
    const int nden = ncd + nab + NB * ND + NA * ND + NB * NC + NA * NC;
    for (int64_t q = blockIdx.x; q < total; q += gridDim.x) {
        const int2 ij = quartet_pairs(rowstart, rowmap, nbra, q);
        const PairInfo bra = pairs[bra_off + ij.x];
        const PairInfo ket = pairs[ket_off + ij.y];
        double fac = 1.0;
        if (bra.sa == bra.sb) fac *= 0.5;
        if (ket.sa == ket.sb) fac *= 0.5;
        if (same_class && ij.x == ij.y) fac *= 0.5;
        const int N = bra.mN, a0 = bra.bfa, b0 = bra.bfb, c0 = ket.bfa, d0 = ket.bfb;
        const double *D = Dall + bra.moff;
        double *Gj = Gjall ? Gjall + bra.moff : nullptr;
        double *Gk = Gkall ? Gkall + bra.moff : nullptr;
        const Real *src = base + q * nout;
        for (int e = lane; e < nout; e += 64) O[e] = (double)src[e];
        for (int e = lane; e < nden; e += 64) {
            int r = e, row, col;
            if (r < ncd) { row = c0 + r / ND; col = d0 + r % ND; }
            else if ((r -= ncd) < nab) { row = a0 + r / NB; col = b0 + r % NB; }
            else if ((r -= nab) < NB * ND) { row = b0 + r / ND; col = d0 + r % ND; }
            else if ((r -= NB * ND) < NA * ND) { row = a0 + r / ND; col = d0 + r % ND; }
            else if ((r -= NA * ND) < NB * NC) { row = b0 + r / NC; col = c0 + r % NC; }
            else { r -= NB * NC; row = a0 + r / NC; col = c0 + r % NC; }
            Dcd[e] = D[(int64_t)row * N + col];
        }
        __syncthreads();
        auto At = [&](int a, int b, int c, int d) { return O[((a * NB + b) * NC + c) * ND + d]; };
        const int t_ab = Gj ? nab : 0, t_cd = Gj ? ncd : 0;
        const int t_ac = Gk ? NA * NC : 0, t_bc = Gk ? NB * NC : 0, t_ad = Gk ? NA * ND : 0, t_bd = Gk ? NB * ND : 0;
        const int ntgt = t_ab + t_cd + t_ac + t_bc + t_ad + t_bd;
        for (int t = lane; t < ntgt; t += 64) {
            int r = t;
            double sum = 0.0;
            if (r < t_ab) {
                const int a = r / NB, b = r % NB;
                for (int c = 0; c < NC; ++c)
                    for (int d = 0; d < ND; ++d) sum += At(a, b, c, d) * Dcd[c * ND + d];
                unsafeAtomicAdd(&Gj[(int64_t)(a0 + a) * N + b0 + b], 2.0 * fac * sum);
            } else if ((r -= t_ab) < t_cd) {
                const int c = r / ND, d = r % ND;
                for (int a = 0; a < NA; ++a)
                    for (int b = 0; b < NB; ++b) sum += At(a, b, c, d) * Dab[a * NB + b];
                unsafeAtomicAdd(&Gj[(int64_t)(c0 + c) * N + d0 + d], 2.0 * fac * sum);
            } else if ((r -= t_cd) < t_ac) {
                const int a = r / NC, c = r % NC;
                for (int b = 0; b < NB; ++b)
                    for (int d = 0; d < ND; ++d) sum += At(a, b, c, d) * Dbd[b * ND + d];
                unsafeAtomicAdd(&Gk[(int64_t)(a0 + a) * N + c0 + c], fac * sum);
            } else if ((r -= t_ac) < t_bc) {
                const int b = r / NC, c = r % NC;
                for (int a = 0; a < NA; ++a)
                    for (int d = 0; d < ND; ++d) sum += At(a, b, c, d) * Dad[a * ND + d];
                unsafeAtomicAdd(&Gk[(int64_t)(b0 + b) * N + c0 + c], fac * sum);
            } else if ((r -= t_bc) < t_ad) {
                const int a = r / ND, d = r % ND;
                for (int b = 0; b < NB; ++b)
                    for (int c = 0; c < NC; ++c) sum += At(a, b, c, d) * Dbc[b * NC + c];
                unsafeAtomicAdd(&Gk[(int64_t)(a0 + a) * N + d0 + d], fac * sum);
            } else {
                r -= t_ad;
                const int b = r / ND, d = r % ND;
                for (int a = 0; a < NA; ++a)
                    for (int c = 0; c < NC; ++c) sum += At(a, b, c, d) * Dac[a * NC + c];
                unsafeAtomicAdd(&Gk[(int64_t)(b0 + b) * N + d0 + d], fac * sum);
            }
        }
        __syncthreads();  // LDS reused by the next quartet
    }
}

// Quartet-major copy of a structure-of-arrays block region (once per store).
template <typename Real>
__global__ void k_to_aos(const Real *__restrict__ soa, Real *__restrict__ aos, int nout, int64_t total) {
    const int64_t n = (int64_t)nout * total;
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
        const int64_t t = i / nout;
        const int e = (int)(i % nout);
        aos[i] = soa[(int64_t)e * total + t];
    }
}

int to_aos(const void *soa, void *aos, int nout, int64_t total, int prec, hipStream_t s) {
    const unsigned g = (unsigned)std::min<int64_t>(((int64_t)nout * total + 255) / 256, 1 << 16);
    if (prec == MESS_FP32)
        hipLaunchKernelGGL(k_to_aos<float>, dim3(g), dim3(256), 0, s, static_cast<const float *>(soa),
                           static_cast<float *>(aos), nout, total);
    else
        hipLaunchKernelGGL(k_to_aos<double>, dim3(g), dim3(256), 0, s, static_cast<const double *>(soa),
                           static_cast<double *>(aos), nout, total);
    MESS_LAUNCH_CHECK();
    return MESS_OK;
}

int coop_store(int cb, int ck, const ClassLaunch &L, void *base, int prec) {
    return coop_launch(prec == MESS_FP32 ? kModeStore32 : kModeStore64, cb, ck, L, L.total,
                       static_cast<double *>(base), nullptr, nullptr, prec);
}

int coop_jk_stored(int cb, int ck, const ClassLaunch &L, const void *base, int prec, const double *D, double *Gj,
                   double *Gk) {
    if (L.total <= 0) return MESS_OK;
    int64_t g = L.total;
    if (g > (1 << 20)) g = 1 << 20;
    const int NA = ncart(pair_class_la(cb)), NB = ncart(pair_class_lb(cb)), NC = ncart(pair_class_la(ck)),
              ND = ncart(pair_class_lb(ck));
    if (stored_aos_class(cb, ck)) {
        const size_t la = sizeof(double) * ((size_t)NA * NB * NC * ND + NA * NB + NC * ND + (NA + NB) * (NC + ND));
        if (prec == MESS_FP32)
            hipLaunchKernelGGL(k_jk_stored_aos<float>, dim3((unsigned)g), dim3(64), la, L.stream, L.pairs, L.bra_off,
                               L.ket_off, L.nbra, L.same_class, L.rowstart, L.rowmap, L.total, NA, NB, NC, ND,
                               static_cast<const float *>(base), D, Gj, Gk);
        else
            hipLaunchKernelGGL(k_jk_stored_aos<double>, dim3((unsigned)g), dim3(64), la, L.stream, L.pairs, L.bra_off,
                               L.ket_off, L.nbra, L.same_class, L.rowstart, L.rowmap, L.total, NA, NB, NC, ND,
                               static_cast<const double *>(base), D, Gj, Gk);
        MESS_LAUNCH_CHECK();
        return MESS_OK;
    }
    // bra-row segments with K and density rows in LDS when they fit; (dd|dd)
    // keeps the wave-per-quartet form (measured faster: the streamed form
    // needs more registers than a lane has for its 36-element J and density
    // blocks)
    const size_t lds = sizeof(double) * (2 * (size_t)(NA + NB) * L.nmax + NA * NB);
    if (L.segs && L.nseg > 0 && lds <= 64 * 1024 && !(cb == 5 && ck == 5)) {
        const unsigned gs = (unsigned)std::min(L.nseg, 1 << 20);
        bool done = false;
#define MESS_STREAM(B, K)                                                                                         \
        if (cb == B && ck == K) {                                                                                 \
            if (prec == MESS_FP32)                                                                                \
                hipLaunchKernelGGL((k_jk_stored_stream<ClassOf<B, K>, float>), dim3(gs), dim3(256), lds, L.stream, \
                                   L.pairs, L.bra_off, L.ket_off, L.same_class, L.rowstart, L.rowmap, L.segs,      \
                                   L.nseg, static_cast<const float *>(base), L.total, D, Gj, Gk);                   \
            else                                                                                                  \
                hipLaunchKernelGGL((k_jk_stored_stream<ClassOf<B, K>, double>), dim3(gs), dim3(256), lds,         \
                                   L.stream, L.pairs, L.bra_off, L.ket_off, L.same_class, L.rowstart, L.rowmap,    \
                                   L.segs, L.nseg, static_cast<const double *>(base), L.total, D, Gj, Gk);          \
            done = true;                                                                                          \
        }
        MESS_STREAM(2, 2)
        MESS_STREAM(4, 2)
        MESS_STREAM(4, 4)
        MESS_STREAM(5, 2)
        MESS_STREAM(5, 3)
        MESS_STREAM(5, 4)
#undef MESS_STREAM
        if (done) {
            MESS_LAUNCH_CHECK();
            return MESS_OK;
        }
    }
    if (prec == MESS_FP32)
        hipLaunchKernelGGL(k_jk_stored_wave<float>, dim3((unsigned)g), dim3(64), 0, L.stream, L.pairs, L.bra_off,
                           L.ket_off, L.nbra, L.same_class, L.rowstart, L.rowmap, L.total, NA, NB, NC, ND,
                           static_cast<const float *>(base), D, L.N, Gj, Gk);
    else
        hipLaunchKernelGGL(k_jk_stored_wave<double>, dim3((unsigned)g), dim3(64), 0, L.stream, L.pairs, L.bra_off,
                           L.ket_off, L.nbra, L.same_class, L.rowstart, L.rowmap, L.total, NA, NB, NC, ND,
                           static_cast<const double *>(base), D, L.N, Gj, Gk);
    MESS_LAUNCH_CHECK();
    return MESS_OK;
}

}  // namespace mess

// The high classes are reached through the same ClassOps interface as the
// unrolled ones; eri_class.hip is not compiled for them.
namespace mess {
#define MESS_COOP_CLASS(B, K)                                                                          \
    template <>                                                                                        \
    int ClassOps<B, K>::schwarz(const ClassLaunch &L, int off, int n, double *Q) {                     \
        if (B != K) {                                                                                  \
            set_error("internal: Schwarz launch for a mixed class");                                   \
            return MESS_E_ARG;                                                                         \
        }                                                                                              \
        return coop_schwarz(B, L, off, n, Q);                                                          \
    }                                                                                                  \
    template <>                                                                                        \
    int ClassOps<B, K>::dense(const ClassLaunch &L, double *eri, int prec) {                           \
        return coop_dense(B, K, L, eri, prec);                                                         \
    }                                                                                                  \
    template <>                                                                                        \
    int ClassOps<B, K>::jk(const ClassLaunch &L, const double *D, double *Gj, double *Gk, int prec) {  \
        return coop_jk(B, K, L, D, Gj, Gk, prec);                                                      \
    }                                                                                                  \
    template <>                                                                                        \
    int ClassOps<B, K>::store(const ClassLaunch &L, void *base, int prec) {                            \
        return coop_store(B, K, L, base, prec);                                                        \
    }                                                                                                  \
    template <>                                                                                        \
    int ClassOps<B, K>::jk_stored(const ClassLaunch &L, const void *base, int prec, const double *D,   \
                                  double *Gj, double *Gk) {                                            \
        return coop_jk_stored(B, K, L, base, prec, D, Gj, Gk);                                         \
    }
MESS_COOP_CLASS(2, 2)
MESS_COOP_CLASS(4, 2)
MESS_COOP_CLASS(4, 4)
MESS_COOP_CLASS(5, 2)
MESS_COOP_CLASS(5, 3)
MESS_COOP_CLASS(5, 4)
MESS_COOP_CLASS(5, 5)
#undef MESS_COOP_CLASS
}  // namespace mess
