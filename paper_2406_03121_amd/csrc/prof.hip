// Optional timing of the shell-quartet class launches: when enabled, a pair
// of HIP events is recorded on the launch stream around every class launch
// together with the work it covers; mess_prof_read sums them per class.
#include <mutex>
#include <vector>

#include "mess_internal.hpp"

namespace mess {

namespace {
struct Rec {
    hipEvent_t a = nullptr, b = nullptr;
    int cls = 0;
    int64_t quartets = 0, prims = 0;
    double flops = 0.0;
};
std::mutex g_mu;
bool g_on = false;
std::vector<Rec> g_recs;
Rec g_open;
bool g_have_open = false;

void clear_locked() {
    for (auto &r : g_recs) {
        if (r.a) hipEventDestroy(r.a);
        if (r.b) hipEventDestroy(r.b);
    }
    g_recs.clear();
    g_have_open = false;
}
}  // namespace

bool prof_on() { return g_on; }

void prof_record(hipStream_t s, int cls, bool begin, int64_t quartets, int64_t prims, double flops) {
    std::lock_guard<std::mutex> lk(g_mu);
    if (!g_on) return;
    if (begin) {
        g_open = Rec{};
        if (hipEventCreate(&g_open.a) != hipSuccess) return;
        hipEventRecord(g_open.a, s);
        g_open.cls = cls;
        g_open.quartets = quartets;
        g_open.prims = prims;
        g_open.flops = flops;
        g_have_open = true;
    } else if (g_have_open) {
        if (hipEventCreate(&g_open.b) != hipSuccess) return;
        hipEventRecord(g_open.b, s);
        g_recs.push_back(g_open);
        g_have_open = false;
    }
}

}  // namespace mess

using namespace mess;

extern "C" {

int mess_prof_enable(int32_t on) {
    std::lock_guard<std::mutex> lk(g_mu);
    clear_locked();
    g_on = on != 0;
    return MESS_OK;
}

int mess_prof_read(int32_t cls, int64_t *launches, double *ms, double *alg_flops, int64_t *quartets,
                   int64_t *prim_quartets) {
    std::lock_guard<std::mutex> lk(g_mu);
    int64_t n = 0, q = 0, p = 0;
    double t = 0.0, f = 0.0;
    for (auto &r : g_recs) {
        if (cls >= 0 && r.cls != cls) continue;
        float e = 0.0f;
        if (hipEventSynchronize(r.b) != hipSuccess || hipEventElapsedTime(&e, r.a, r.b) != hipSuccess) {
            set_error("mess_prof_read: event query failed");
            return MESS_E_DEVICE;
        }
        ++n;
        t += e;
        q += r.quartets;
        p += r.prims;
        f += r.flops;
    }
    if (launches) *launches = n;
    if (ms) *ms = t;
    if (alg_flops) *alg_flops = f;
    if (quartets) *quartets = q;
    if (prim_quartets) *prim_quartets = p;
    return MESS_OK;
}

}  // extern "C"
