// One angular class of shell quartets.  This file is compiled once per
// class with -DMESS_CB=<bra pair class> -DMESS_CK=<ket pair class>, so the
// 21 fully unrolled class kernels build in parallel.
#include <algorithm>

#include "class_ops.hpp"
#include "eri_kernels.hpp"

#ifndef MESS_CB
#error "compile with -DMESS_CB=<0..5> -DMESS_CK=<0..MESS_CB>"
#endif

namespace mess {

namespace {
inline unsigned grid_for(int64_t total, int block) {
    int64_t g = (total + block - 1) / block;
    if (g < 1) g = 1;
    if (g > (1 << 20)) g = 1 << 20;
    return static_cast<unsigned>(g);
}
}  // namespace

template <>
int ClassOps<MESS_CB, MESS_CK>::schwarz(const ClassLaunch &L, int off, int n, double *Q) {
    if constexpr (MESS_CB != MESS_CK) {
        set_error("internal: Schwarz launch for a mixed class");
        return MESS_E_ARG;
    } else {
        using Dm = ClassOf<MESS_CB, MESS_CK>;
        if (n <= 0) return MESS_OK;
        hipLaunchKernelGGL(k_schwarz<Dm>, dim3((n + 63) / 64), dim3(64), 0, L.stream, L.pairs, off, n,
                           L.pp, BoysTabs{L.tab, L.etab, L.tabf, L.etabf, L.tabt}, Q);
        MESS_LAUNCH_CHECK();
        return MESS_OK;
    }
}

template <>
int ClassOps<MESS_CB, MESS_CK>::dense(const ClassLaunch &L, double *eri, int prec) {
    using Dm = ClassOf<MESS_CB, MESS_CK>;
    if (L.total <= 0) return MESS_OK;
    const BoysTabs bt{L.tab, L.etab, L.tabf, L.etabf, L.tabt};
    if (prec == MESS_FP32)
        hipLaunchKernelGGL((k_eri_dense<Dm, float>), dim3(grid_for(L.total, 128)), dim3(128), 0, L.stream,
                           L.pairs, L.bra_off, L.ket_off, L.nbra, L.rowstart, L.rowmap, L.ppf, bt, (int64_t)L.N, eri);
    else
        hipLaunchKernelGGL((k_eri_dense<Dm, double>), dim3(grid_for(L.total, 128)), dim3(128), 0, L.stream,
                           L.pairs, L.bra_off, L.ket_off, L.nbra, L.rowstart, L.rowmap, L.pp, bt, (int64_t)L.N, eri);
    MESS_LAUNCH_CHECK();
    return MESS_OK;
}

template <>
int ClassOps<MESS_CB, MESS_CK>::jk(const ClassLaunch &L, const double *D, double *Gj, double *Gk,
                                   int prec) {
    using Dm = ClassOf<MESS_CB, MESS_CK>;
    if (L.total <= 0) return MESS_OK;
    // the primitive-lane form, where it is built and the form table picks it
    if (plane_compiled(MESS_CB, MESS_CK) && class_form(MESS_CB, MESS_CK, prec) == kFormPlane)
        return coop_jk(MESS_CB, MESS_CK, L, D, Gj, Gk, prec);
    const BoysTabs bt{L.tab, L.etab, L.tabf, L.etabf, L.tabt};
    if constexpr (!(MESS_CB == 4 && MESS_CK == 3) && !(MESS_CB == 3 && MESS_CK == 2)) {
        // one 256-thread block per bra segment, K rows of the bra functions
        // in LDS and J[a,b] in registers (one flush per segment), so only
        // J[c,d] takes a global atomic per quartet (not built for (dp|ds)
        // and (ds|pp), which spill and run 1.3-2.8x slower this way); the
        // default form of the low classes unless the form table says lane
        const size_t lds = sizeof(double) * ((size_t)(Dm::NA + Dm::NB) * L.nmax + Dm::NA * Dm::NB);
        if (L.segs && L.nseg > 0 && lds <= 48 * 1024 && class_form(MESS_CB, MESS_CK, prec) == kFormRows) {
            const unsigned g = (unsigned)std::min(L.nseg, 1 << 20);
            if (prec == MESS_FP32)
                hipLaunchKernelGGL((k_jk_rows<Dm, float, true>), dim3(g), dim3(256), lds, L.stream, L.pairs,
                                   L.bra_off, L.ket_off, L.same_class, L.rowstart, L.rowmap, L.segs, L.nseg,
                                   (const float *)nullptr, L.total, D, Gj, Gk, L.ppf, bt);
            else
                hipLaunchKernelGGL((k_jk_rows<Dm, double, true>), dim3(g), dim3(256), lds, L.stream, L.pairs,
                                   L.bra_off, L.ket_off, L.same_class, L.rowstart, L.rowmap, L.segs, L.nseg,
                                   (const double *)nullptr, L.total, D, Gj, Gk, L.pp, bt);
            MESS_LAUNCH_CHECK();
            return MESS_OK;
        }
    }
    if (prec == MESS_FP32)
        hipLaunchKernelGGL((k_jk_direct<Dm, float>), dim3(grid_for(L.total, 128)), dim3(128), 0, L.stream,
                           L.pairs, L.bra_off, L.ket_off, L.nbra, L.same_class, L.rowstart, L.rowmap, L.ppf, bt, D, L.N, Gj,
                           Gk);
    else
        hipLaunchKernelGGL((k_jk_direct<Dm, double>), dim3(grid_for(L.total, 128)), dim3(128), 0, L.stream,
                           L.pairs, L.bra_off, L.ket_off, L.nbra, L.same_class, L.rowstart, L.rowmap, L.pp, bt, D, L.N, Gj,
                           Gk);
    MESS_LAUNCH_CHECK();
    return MESS_OK;
}

template <>
int ClassOps<MESS_CB, MESS_CK>::store(const ClassLaunch &L, void *base, int prec) {
    using Dm = ClassOf<MESS_CB, MESS_CK>;
    if (L.total <= 0) return MESS_OK;
    const BoysTabs bt{L.tab, L.etab, L.tabf, L.etabf, L.tabt};
    if (prec == MESS_FP32)
        hipLaunchKernelGGL((k_eri_store<Dm, float>), dim3(grid_for(L.total, 128)), dim3(128), 0, L.stream, L.pairs,
                           L.bra_off, L.ket_off, L.nbra, L.rowstart, L.rowmap, L.ppf, bt, static_cast<float *>(base));
    else
        hipLaunchKernelGGL((k_eri_store<Dm, double>), dim3(grid_for(L.total, 128)), dim3(128), 0, L.stream, L.pairs,
                           L.bra_off, L.ket_off, L.nbra, L.rowstart, L.rowmap, L.pp, bt, static_cast<double *>(base));
    MESS_LAUNCH_CHECK();
    return MESS_OK;
}

template <>
int ClassOps<MESS_CB, MESS_CK>::jk_stored(const ClassLaunch &L, const void *base, int prec, const double *D,
                                          double *Gj, double *Gk) {
    using Dm = ClassOf<MESS_CB, MESS_CK>;
    if (L.total <= 0) return MESS_OK;
    constexpr int G = kGroupBras[MESS_CB];
    if constexpr (G > 1) {
        // groups of G bras: J[c,d] reduced over the group before its atomic
        const size_t lg = sizeof(double) * ((size_t)G * (Dm::NA + Dm::NB) * L.nmax + G * Dm::NA * Dm::NB) +
                          sizeof(int) * G * (Dm::NA + Dm::NB);
        if (L.groups && L.ngroups > 0 && lg <= 48 * 1024) {
            const unsigned g = (unsigned)std::min(L.ngroups, 1 << 20);
            if (prec == MESS_FP32)
                hipLaunchKernelGGL((k_jk_group<Dm, float, G>), dim3(g), dim3(256), lg, L.stream, L.pairs, L.bra_off,
                                   L.ket_off, L.same_class, L.rowstart, L.groups, L.ngroups, L.tiles, L.grows,
                                   static_cast<const float *>(base), L.total, D, Gj, Gk);
            else
                hipLaunchKernelGGL((k_jk_group<Dm, double, G>), dim3(g), dim3(256), lg, L.stream, L.pairs, L.bra_off,
                                   L.ket_off, L.same_class, L.rowstart, L.groups, L.ngroups, L.tiles, L.grows,
                                   static_cast<const double *>(base), L.total, D, Gj, Gk);
            MESS_LAUNCH_CHECK();
            return MESS_OK;
        }
    }
    const size_t lds = sizeof(double) * ((size_t)(Dm::NA + Dm::NB) * L.nmax + Dm::NA * Dm::NB);
    if (L.segs && L.nseg > 0 && lds <= 48 * 1024) {
        const unsigned g = (unsigned)std::min(L.nseg, 1 << 20);
        if (prec == MESS_FP32)
            hipLaunchKernelGGL((k_jk_rows<Dm, float>), dim3(g), dim3(256), lds, L.stream, L.pairs, L.bra_off,
                               L.ket_off, L.same_class, L.rowstart, L.rowmap, L.segs, L.nseg,
                               static_cast<const float *>(base), L.total, D, Gj, Gk);
        else
            hipLaunchKernelGGL((k_jk_rows<Dm, double>), dim3(g), dim3(256), lds, L.stream, L.pairs, L.bra_off,
                               L.ket_off, L.same_class, L.rowstart, L.rowmap, L.segs, L.nseg,
                               static_cast<const double *>(base), L.total, D, Gj, Gk);
        MESS_LAUNCH_CHECK();
        return MESS_OK;
    }
    if (prec == MESS_FP32)
        hipLaunchKernelGGL((k_jk_stored<Dm, float>), dim3(grid_for(L.total, 128)), dim3(128), 0, L.stream, L.pairs,
                           L.bra_off, L.ket_off, L.nbra, L.same_class, L.rowstart, L.rowmap, static_cast<const float *>(base),
                           D, L.N, Gj, Gk);
    else
        hipLaunchKernelGGL((k_jk_stored<Dm, double>), dim3(grid_for(L.total, 128)), dim3(128), 0, L.stream, L.pairs,
                           L.bra_off, L.ket_off, L.nbra, L.same_class, L.rowstart, L.rowmap, static_cast<const double *>(base),
                           D, L.N, Gj, Gk);
    MESS_LAUNCH_CHECK();
    return MESS_OK;
}

}  // namespace mess
