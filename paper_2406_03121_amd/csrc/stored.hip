// mess_jk(MESS_JK_STORED): the unique, Schwarz-screened shell-quartet blocks
// are computed once per (basis, precision, threshold) into device memory,
// one structure-of-arrays region per angular class (element k of quartet t
// at base[k * nq + t]), and every later call streams them into J/K.
#include <algorithm>

#include "class_ops.hpp"
#include "mess_internal.hpp"

namespace mess {

int get_work_lists(mess_basis *B, double tau, hipStream_t s, WorkLists **out);
int fill_class_launch(const mess_basis *B, const ClassList &cl, hipStream_t s, ClassLaunch &L);

struct StoredEri {
    int prec = MESS_FP64;
    double tau = 0.0;
    std::vector<void *> base;      // per class (index into WorkLists::classes)
    std::vector<int64_t> bytes;
    std::vector<int4 *> segs;      // per class: bra-row segments of the quartet list
    std::vector<int> nseg;
    int64_t total_bytes = 0;
};

void free_stored(mess_basis *B) {
    for (auto &kv : B->stored) {
        for (void *p : kv.second->base)
            if (p) hipFree(p);
        for (int4 *p : kv.second->segs)
            if (p) hipFree(p);
        delete kv.second;
    }
    B->stored.clear();
}

// Quartets of every bra (its consecutive rows [r0, r1) of the work list),
// cut into pieces of at most kSegLen: {r0, first, end, r1}.
constexpr int64_t kSegLen = 2048;
static int build_segments(const ClassList &cl, int4 **out, int *n) {
    std::vector<int4> v;
    for (int r0 = 0; r0 < cl.nrow;) {
        int r1 = r0 + 1;
        while (r1 < cl.nrow && cl.h_rowmap[r1].x == cl.h_rowmap[r0].x) ++r1;
        for (int64_t q = cl.h_rowstart[r0]; q < cl.h_rowstart[r1]; q += kSegLen) {
            const int64_t e = std::min(q + kSegLen, cl.h_rowstart[r1]);
            int rq = r0;  // row holding quartet q
            while (cl.h_rowstart[rq + 1] <= q) ++rq;
            v.push_back(make_int4(rq, (int)q, (int)e, r1));
        }
        r0 = r1;
    }
    *n = (int)v.size();
    *out = nullptr;
    if (v.empty()) return MESS_OK;
    if (cl.total >= ((int64_t)1 << 31)) return MESS_OK;  // quartet index beyond int: lane-per-quartet digestion
    if (hipMalloc(out, sizeof(int4) * v.size()) != hipSuccess ||
        hipMemcpy(*out, v.data(), sizeof(int4) * v.size(), hipMemcpyHostToDevice) != hipSuccess) {
        hipFree(*out);
        *out = nullptr;
        set_error("mess_jk(STORED): cannot allocate the row segments");
        return MESS_E_NOMEM;
    }
    return MESS_OK;
}

static int nout_of(int cb, int ck) {
    return ncart(pair_class_la(cb)) * ncart(pair_class_lb(cb)) * ncart(pair_class_la(ck)) *
           ncart(pair_class_lb(ck));
}

static int get_stored(mess_basis *B, int prec, double tau, hipStream_t s, WorkLists **Wout, StoredEri **out) {
    if (!(tau > 0.0)) tau = 0.0;
    WorkLists *W = nullptr;
    MESS_TRY(get_work_lists(B, tau, s, &W));
    *Wout = W;
    auto key = std::make_pair(prec, tau);
    auto it = B->stored.find(key);
    if (it != B->stored.end()) {
        *out = it->second;
        return MESS_OK;
    }
    auto *E = new StoredEri();
    E->prec = prec;
    E->tau = tau;
    const size_t rsz = prec == MESS_FP32 ? sizeof(float) : sizeof(double);
    int rc = MESS_OK;
    for (const ClassList &cl : W->classes) {
        void *p = nullptr;
        const int64_t nbytes = (int64_t)rsz * nout_of(cl.cb, cl.ck) * cl.total;
        if (cl.total > 0 && hipMalloc(&p, nbytes) != hipSuccess) {
            set_error("mess_jk(STORED): cannot allocate %lld bytes for class (%d,%d)", (long long)nbytes, cl.cb,
                      cl.ck);
            rc = MESS_E_NOMEM;
            break;
        }
        E->base.push_back(p);
        E->bytes.push_back(cl.total > 0 ? nbytes : 0);
        E->total_bytes += cl.total > 0 ? nbytes : 0;
        {
            int4 *sg = nullptr;
            int ns = 0;
            if (cl.total > 0) rc = build_segments(cl, &sg, &ns);
            E->segs.push_back(sg);
            E->nseg.push_back(sg ? ns : 0);
            if (rc != MESS_OK) break;
        }
        if (cl.total == 0) continue;
        ClassLaunch L;
        fill_class_launch(B, cl, s, L);
        rc = dispatch_class(cl.cb, cl.ck, [&](auto CB, auto CK) {
            return ClassOps<decltype(CB)::value, decltype(CK)::value>::store(L, p, prec);
        });
        if (rc != MESS_OK) break;
    }
    if (rc != MESS_OK) {
        for (void *p : E->base)
            if (p) hipFree(p);
        for (int4 *p : E->segs)
            if (p) hipFree(p);
        delete E;
        return rc;
    }
    B->stored[key] = E;
    *out = E;
    return MESS_OK;
}

int zero_async(double *p, int64_t n, hipStream_t s);

int jk_stored(mess_basis *B, const double *D, double *Gj, double *Gk, int prec, double tau, hipStream_t s) {
    WorkLists *W = nullptr;
    StoredEri *E = nullptr;
    MESS_TRY(get_stored(B, prec, tau, s, &W, &E));
    if (Gj) MESS_TRY(zero_async(Gj, B->packed, s));
    if (Gk) MESS_TRY(zero_async(Gk, B->packed, s));
    const bool prof = prof_on();
    for (size_t c = 0; c < W->classes.size(); ++c) {
        const ClassList &cl = W->classes[c];
        if (cl.total == 0) continue;
        ClassLaunch L;
        fill_class_launch(B, cl, s, L);
        L.segs = E->segs[c];
        L.nseg = E->nseg[c];
        L.nmax = B->nbf_max;
        // recorded under class index + 32, with the bytes streamed in the
        // operation-count field
        if (prof) prof_record(s, 32 + class_index(cl.cb, cl.ck), true, cl.total, cl.prim_quartets, (double)E->bytes[c]);
        MESS_TRY(dispatch_class(cl.cb, cl.ck, [&](auto CB, auto CK) {
            return ClassOps<decltype(CB)::value, decltype(CK)::value>::jk_stored(L, E->base[c], prec, D, Gj, Gk);
        }));
        if (prof) prof_record(s, 0, false, 0, 0, 0.0);
    }
    return MESS_OK;
}

}  // namespace mess
