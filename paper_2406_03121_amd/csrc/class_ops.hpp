// Per-angular-class launchers.  Each of the 21 unique classes (pair class
// of the bra >= pair class of the ket) is compiled in its own object file
// (eri_class.hip built once per class) and reached through ClassOps.
#pragma once

#include "mess_internal.hpp"

namespace mess {

struct ClassLaunch {
    const PairInfo *pairs;
    const PrimPair *pp;
    const PrimPairF *ppf;
    const double *tab, *etab;
    const float *tabf, *etabf;
    const double *tabt;  // per-order Taylor table (F_{L+i}(T_k) / i!)
    int bra_off, ket_off, nbra, same_class;  // nbra: rows of the work list
    const int64_t *rowstart;
    const int2 *rowmap;  // per row: {bra index, first ket index}
    int64_t total;
    int N;
    hipStream_t stream;
    // stored-block digestion by bra-row segments (NULL: one lane per quartet)
    const int4 *segs = nullptr;  // {first row, first quartet, end quartet, end row}
    int nseg = 0;
    int nmax = 0;                // largest molecule dimension (LDS rows)
    // grouped stored digestion (NULL: by segments)
    const int4 *groups = nullptr, *tiles = nullptr;
    const int *grows = nullptr;
    int ngroups = 0;
};

// Direct J/K of class (cb, ck) through its cooperative tables (primitive-
// lane, wave or table-driven kernel; coop.hip).
int coop_jk(int cb, int ck, const ClassLaunch &L, const double *D, double *Gj, double *Gk, int prec);

// Stored-block layout (coop.hip): true when class (cb, ck) keeps its blocks
// quartet-major for J/K streaming (element e of quartet t at t NOUT + e)
// instead of structure-of-arrays (e total + t); to_aos converts a region.
bool stored_aos_class(int cb, int ck);
int to_aos(const void *soa, void *aos, int nout, int64_t total, int prec, hipStream_t s);

template <int CB, int CK>
struct ClassOps {
    // Q[off + i] for the n pairs of class CB (requires CB == CK).
    static int schwarz(const ClassLaunch &L, int off, int n, double *Q);
    // Dense N^4 FP64 store of every quartet in the list.
    static int dense(const ClassLaunch &L, double *eri, int prec);
    // Gj, Gk half-matrices (either may be NULL) from density D.
    static int jk(const ClassLaunch &L, const double *D, double *Gj, double *Gk, int prec);
    // Unique blocks of every quartet into base (FP64 or FP32 by prec),
    // element k of quartet t at base[k * total + t].
    static int store(const ClassLaunch &L, void *base, int prec);
    // Gj, Gk from the stored blocks.
    static int jk_stored(const ClassLaunch &L, const void *base, int prec, const double *D, double *Gj, double *Gk);
};

// Calls f(integral_constant<CB>, integral_constant<CK>) for a runtime
// (cb, ck) with cb >= ck.
template <typename F>
int dispatch_class(int cb, int ck, F &&f) {
    using std::integral_constant;
#define MESS_CASE(B, K) \
    case (B) * 6 + (K): return f(integral_constant<int, B>{}, integral_constant<int, K>{});
    switch (cb * 6 + ck) {
        MESS_CASE(0, 0)
        MESS_CASE(1, 0) MESS_CASE(1, 1)
        MESS_CASE(2, 0) MESS_CASE(2, 1) MESS_CASE(2, 2)
        MESS_CASE(3, 0) MESS_CASE(3, 1) MESS_CASE(3, 2) MESS_CASE(3, 3)
        MESS_CASE(4, 0) MESS_CASE(4, 1) MESS_CASE(4, 2) MESS_CASE(4, 3) MESS_CASE(4, 4)
        MESS_CASE(5, 0) MESS_CASE(5, 1) MESS_CASE(5, 2) MESS_CASE(5, 3) MESS_CASE(5, 4) MESS_CASE(5, 5)
        default: break;
    }
#undef MESS_CASE
    set_error("internal: bad class (%d,%d)", cb, ck);
    return MESS_E_ARG;
}


}  // namespace mess
