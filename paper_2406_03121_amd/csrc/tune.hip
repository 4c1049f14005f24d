// Kernel form of each angular class, and the autotuner that chooses it.
//
// Every class can be mapped onto the hardware in more than one way:
//  - lane:  one lane per shell quartet, recursion unrolled in registers;
//  - rows:  one 256-thread block per segment of a bra's quartets, exchange
//           rows of the bra functions in LDS (low classes);
//  - plane: one wave per shell quartet, one lane per primitive quartet;
//  - coop:  one block per shell quartet, the recursion table-driven in LDS;
//  - wave:  one block per shell quartet, one wave per primitive quartet,
//           lanes over the recursion's intermediates (wave.hip);
//  - fp64:  (mixed precision only) the class's FP64 kernel serves builds
//           asked for in FP32, where it is the faster one.
// Which is fastest depends on the class (registers, primitive counts) and
// on the workload, so the choice is a run-time table.  The built-in
// defaults come from measurements on MI355X; mess_autotune times every
// valid form of every class on a basis's own work lists and keeps the
// fastest.
#include <algorithm>
#include <mutex>
#include <vector>

#include "class_ops.hpp"
#include "mess_internal.hpp"

namespace mess {

int get_work_lists(mess_basis *B, double tau, hipStream_t s, WorkLists **out);
int fill_class_launch(const mess_basis *B, const ClassList &cl, hipStream_t s, ClassLaunch &L);
int zero_async(double *p, int64_t n, hipStream_t s);

namespace {
std::mutex g_form_mutex;
int g_form[2][kNumClasses] = {};  // [precision][class]; kFormAuto: built-in default
}  // namespace

bool plane_compiled(int cb, int ck) {
    // (dd|ps) is the one lane-kernel class the primitive-lane form beats
    // (3.25 -> 2.75 ms per 60-atom build); (dp|ps), (dp|ds) and (ds|pp)
    // measured 1.4-2x slower in it
    return (cb == 5 && ck >= 1 && ck <= 4) || (cb == 4 && (ck == 2 || ck == 4)) || (cb == 2 && ck == 2);
}

bool wave_compiled(int cb, int ck) { return cb == 5 && ck >= 3; }

bool rows_compiled(int cb, int ck) {
    // classes whose unrolled kernels include the bra-segment form: all but
    // (dp|ds) and (ds|pp) (measured per 60-atom build: 5.12 vs 3.85 ms and
    // 2.31 vs 1.37 ms against one lane per quartet)
    return !coop_class(cb, ck) && !(cb == 4 && ck == 3) && !(cb == 3 && ck == 2);
}

bool form_valid(int cb, int ck, int form, int prec) {
    if (form == kFormAuto) return true;
    if (form == kFormFp64) return prec == MESS_FP32;
    if (coop_class(cb, ck))
        return form == kFormCoop || (form == kFormPlane && plane_compiled(cb, ck)) ||
               (form == kFormWave && wave_compiled(cb, ck));
    if (form == kFormLane) return true;
    if (form == kFormRows) return rows_compiled(cb, ck);
    if (form == kFormPlane) return plane_compiled(cb, ck);
    return false;
}

static int default_form(int cb, int ck, int prec) {
    // FP32 builds: the classes with an s pair or a ps/pp pair against a lower
    // one run as fast or faster in FP64 (measured on MI355X; the FP32 Boys
    // function falls back to FP64 outside 1e-3 <= T <= 30, and FP32 and FP64
    // FMAs issue at the same rate without packed math)
    if (prec == MESS_FP32) {
        const int c = class_index(cb, ck);
        if (c == 0 || c == 1 || c == 3 || c == 4 || c == 8 || c == 10 || c == 11 || c == 15) return kFormFp64;
    }
    if (coop_class(cb, ck)) return (cb == 5 && ck == 5) ? kFormWave : kFormPlane;
    if (cb == 5 && ck == 1 && prec == MESS_FP64) return kFormPlane;
    return rows_compiled(cb, ck) ? kFormRows : kFormLane;
}

int class_form(int cb, int ck, int prec) {
    std::lock_guard<std::mutex> lk(g_form_mutex);
    const int f = g_form[prec == MESS_FP32 ? 1 : 0][class_index(cb, ck)];
    return f == kFormAuto ? default_form(cb, ck, prec) : f;
}

static void set_form(int prec, int cls, int form) {
    std::lock_guard<std::mutex> lk(g_form_mutex);
    g_form[prec == MESS_FP32 ? 1 : 0][cls] = form;
}

}  // namespace mess

using namespace mess;

extern "C" {

int mess_kernel_form(int32_t prec, int32_t cls, int32_t form, int32_t *active) {
    if (prec != MESS_FP64 && prec != MESS_FP32) {
        set_error("mess_kernel_form: unknown precision %d", prec);
        return MESS_E_ARG;
    }
    if (cls < 0 || cls >= kNumClasses) {
        set_error("mess_kernel_form: class index %d outside 0..%d", cls, kNumClasses - 1);
        return MESS_E_ARG;
    }
    int cb = 0;
    while ((cb + 1) * (cb + 2) / 2 <= cls) ++cb;
    const int ck = cls - cb * (cb + 1) / 2;
    if (form >= 0) {
        if (!form_valid(cb, ck, form, prec)) {
            set_error("mess_kernel_form: form %d is not available for class %d", form, cls);
            return MESS_E_UNSUPPORTED;
        }
        set_form(prec, cls, form);
    }
    if (active) *active = class_form(cb, ck, prec);
    return MESS_OK;
}

int mess_autotune(const mess_basis *basis, int32_t prec, double schwarz_tol, const double *D, int32_t reps,
                  int32_t *forms, double *ms, mess_stream stream) {
    if (!basis || !D) {
        set_error("mess_autotune: NULL basis or density");
        return MESS_E_ARG;
    }
    if (prec != MESS_FP64 && prec != MESS_FP32) {
        set_error("mess_autotune: unknown precision %d", prec);
        return MESS_E_ARG;
    }
    if (reps < 1 || reps > 100) {
        set_error("mess_autotune: reps %d outside 1..100", reps);
        return MESS_E_ARG;
    }
    auto *B = const_cast<mess_basis *>(basis);
    hipStream_t s = static_cast<hipStream_t>(stream);
    WorkLists *W = nullptr;
    MESS_TRY(get_work_lists(B, schwarz_tol, s, &W));
    double *Gj = static_cast<double *>(B->scratch_jk);
    double *Gk = Gj + B->packed;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    MESS_HIP(hipEventCreate(&e0));
    if (hipEventCreate(&e1) != hipSuccess) {
        hipEventDestroy(e0);
        set_error("mess_autotune: hipEventCreate failed");
        return MESS_E_DEVICE;
    }
    int rc = MESS_OK;
    if (ms)
        for (int k = 0; k < kNumClasses * kNumForms; ++k) ms[k] = -1.0;
    for (const ClassList &cl : W->classes) {
        const int cls = class_index(cl.cb, cl.ck);
        int best = kFormAuto;
        double best_ms = 0.0;
        if (cl.total > 0) {
            for (int form = 1; form < kNumForms && rc == MESS_OK; ++form) {
                if (!form_valid(cl.cb, cl.ck, form, prec)) continue;
                set_form(prec, cls, form);
                ClassLaunch L;
                fill_class_launch(B, cl, s, L);
                double tmin = 1e300;
                for (int r = 0; r <= reps && rc == MESS_OK; ++r) {  // the first run is a warm-up
                    rc = zero_async(Gj, 2 * B->packed, s);
                    if (rc != MESS_OK) break;
                    if (hipEventRecord(e0, s) != hipSuccess) rc = MESS_E_DEVICE;
                    if (rc == MESS_OK)
                        rc = dispatch_class(cl.cb, cl.ck, [&](auto CB, auto CK) {
                            return ClassOps<decltype(CB)::value, decltype(CK)::value>::jk(
                                L, D, Gj, Gk, form == kFormFp64 ? MESS_FP64 : prec);
                        });
                    if (rc == MESS_OK && (hipEventRecord(e1, s) != hipSuccess || hipEventSynchronize(e1) != hipSuccess))
                        rc = MESS_E_DEVICE;
                    float t = 0.0f;
                    if (rc == MESS_OK && hipEventElapsedTime(&t, e0, e1) != hipSuccess) rc = MESS_E_DEVICE;
                    if (rc == MESS_OK && r > 0) tmin = std::min(tmin, (double)t);
                }
                if (rc != MESS_OK) break;
                if (ms) ms[cls * kNumForms + form] = tmin;
                if (best == kFormAuto || tmin < best_ms) {
                    best = form;
                    best_ms = tmin;
                }
            }
        }
        if (rc != MESS_OK) {
            set_form(prec, cls, kFormAuto);
            break;
        }
        set_form(prec, cls, best);
        if (forms) forms[cls] = best == kFormAuto ? class_form(cl.cb, cl.ck, prec) : best;
    }
    hipEventDestroy(e0);
    hipEventDestroy(e1);
    if (rc == MESS_E_DEVICE) set_error("mess_autotune: device error while timing class kernels");
    return rc;
}

}  // extern "C"
