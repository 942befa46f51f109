// Event-based kernel timing (diagnostics section of the C ABI).
#include <cstring>
#include <mutex>

#include "vie_internal.h"

namespace {
struct Rec {
    const char *name;
    hipEvent_t a, b;
};
std::mutex g_mu;
bool g_on = false;
std::vector<Rec> g_recs;
std::vector<std::pair<hipEvent_t, hipEvent_t>> g_pool;
}  // namespace

static thread_local int g_noalloc_depth = 0;
NoAllocScope::NoAllocScope() { ++g_noalloc_depth; }
NoAllocScope::~NoAllocScope() { --g_noalloc_depth; }
bool in_noalloc() { return g_noalloc_depth > 0; }

ProfScope::ProfScope(const char *name, hipStream_t stream) : s(stream) {
    if (tune_active() || in_noalloc()) return;
    std::lock_guard<std::mutex> lk(g_mu);
    if (!g_on) return;
    hipEvent_t a, b;
    if (!g_pool.empty()) {
        a = g_pool.back().first;
        b = g_pool.back().second;
        g_pool.pop_back();
    } else if (hipEventCreate(&a) != hipSuccess || hipEventCreate(&b) != hipSuccess) {
        return;
    }
    if (hipEventRecord(a, s) != hipSuccess) return;
    slot = (int)g_recs.size();
    g_recs.push_back({name, a, b});
}

ProfScope::~ProfScope() {
    std::lock_guard<std::mutex> lk(g_mu);
    if (slot >= 0 && slot < (int)g_recs.size()) (void)hipEventRecord(g_recs[slot].b, s);
}

static void recycle() {
    for (auto &r : g_recs) g_pool.push_back({r.a, r.b});
    g_recs.clear();
}

extern "C" vie_status vie_profile_begin(void) {
    std::lock_guard<std::mutex> lk(g_mu);
    VIE_HIP(hipDeviceSynchronize());
    recycle();
    g_on = true;
    return VIE_OK;
}

extern "C" vie_status vie_profile_kernel(const char *name, double *total_ms, int64_t *launches) {
    if (!name || !total_ms || !launches) {
        vie_set_error("vie_profile_kernel: NULL argument");
        return VIE_EARG;
    }
    std::lock_guard<std::mutex> lk(g_mu);
    double t = 0;
    int64_t n = 0;
    for (auto &r : g_recs) {
        if (std::strcmp(r.name, name) != 0) continue;
        VIE_HIP(hipEventSynchronize(r.b));
        float ms = 0;
        VIE_HIP(hipEventElapsedTime(&ms, r.a, r.b));
        t += ms;
        ++n;
    }
    *total_ms = t;
    *launches = n;
    return VIE_OK;
}

extern "C" vie_status vie_profile_end(void) {
    std::lock_guard<std::mutex> lk(g_mu);
    g_on = false;
    VIE_HIP(hipDeviceSynchronize());
    recycle();
    return VIE_OK;
}
