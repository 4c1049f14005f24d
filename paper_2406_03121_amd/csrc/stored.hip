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
    int64_t total_bytes = 0;
};

void free_stored(mess_basis *B) {
    for (auto &kv : B->stored) {
        for (void *p : kv.second->base)
            if (p) hipFree(p);
        delete kv.second;
    }
    B->stored.clear();
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
