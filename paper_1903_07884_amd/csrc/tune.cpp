// Launch-parameter autotuner: a grid search over the candidates a kernel family offers,
// each timed with HIP events on the caller's stream, the winner cached per problem shape
// for the life of the process.  Off by default (vie_autotune).
#include <cstdio>
#include <cstring>
#include <map>
#include <mutex>

#include "vie_internal.h"

namespace {
struct Entry {
    std::vector<int> choice;
    double ms;
    int candidates;
};
std::mutex g_mu;
bool g_on = false;
std::map<std::string, Entry> g_cache;
thread_local int g_active = 0;  // > 0 while candidates run: ProfScope records nothing
}  // namespace

bool tune_enabled() {
    std::lock_guard<std::mutex> lk(g_mu);
    return g_on;
}

bool tune_active() { return g_active > 0; }

bool tune_lookup(const std::string &key, std::vector<int> *choice) {
    std::lock_guard<std::mutex> lk(g_mu);
    auto it = g_cache.find(key);
    if (it == g_cache.end()) return false;
    *choice = it->second.choice;
    return true;
}

void tune_store(const std::string &key, const std::vector<int> &choice, double ms, int candidates) {
    std::lock_guard<std::mutex> lk(g_mu);
    g_cache[key] = Entry{choice, ms, candidates};
}

vie_status tune_check_choice(const std::string &key, const std::vector<int> &choice,
                             const std::vector<std::vector<int>> &cands) {
    for (auto &c : cands)
        if (c == choice) return VIE_OK;
    vie_set_error("autotune entry '" + key + "' holds a choice that is not one of this shape's candidates");
    return VIE_EARG;
}

vie_status tune_time(hipStream_t s, int reps, const std::function<vie_status()> &run, double *ms) {
    ++g_active;
    struct Guard {
        ~Guard() { --g_active; }
    } guard;
    VIE_CHECK(run());  // warm-up (first-launch attributes, scratch growth)
    hipEvent_t a, b;
    VIE_HIP(hipEventCreate(&a));
    if (hipEventCreate(&b) != hipSuccess) {
        (void)hipEventDestroy(a);
        vie_set_error("hipEventCreate failed");
        return VIE_EDEVICE;
    }
    vie_status st = VIE_OK;
    if (hipEventRecord(a, s) != hipSuccess) st = VIE_EDEVICE;
    for (int i = 0; i < reps && st == VIE_OK; ++i) st = run();
    if (st == VIE_OK && (hipEventRecord(b, s) != hipSuccess || hipEventSynchronize(b) != hipSuccess))
        st = VIE_EDEVICE;
    float t = 0;
    if (st == VIE_OK && hipEventElapsedTime(&t, a, b) != hipSuccess) st = VIE_EDEVICE;
    (void)hipEventDestroy(a);
    (void)hipEventDestroy(b);
    if (st == VIE_EDEVICE) vie_set_error("event timing failed during autotuning");
    *ms = t / reps;
    return st;
}

extern "C" vie_status vie_autotune(int32_t enable) {
    std::lock_guard<std::mutex> lk(g_mu);
    g_on = enable != 0;
    return VIE_OK;
}

extern "C" vie_status vie_autotune_set(const char *key, const int32_t *choice, int32_t n) {
    if (!key || n < 0 || n > 16 || (n > 0 && !choice)) {
        vie_set_error("vie_autotune_set: needs a key and 0..16 values");
        return VIE_EARG;
    }
    std::lock_guard<std::mutex> lk(g_mu);
    if (n == 0)
        g_cache.erase(key);
    else
        g_cache[key] = Entry{std::vector<int>(choice, choice + n), 0.0, 0};
    return VIE_OK;
}

extern "C" vie_status vie_autotune_report(char *buf, int64_t size, int64_t *needed) {
    std::string out;
    {
        std::lock_guard<std::mutex> lk(g_mu);
        for (auto &kv : g_cache) {
            out += kv.first + " ->";
            for (int c : kv.second.choice) out += " " + std::to_string(c);
            char tail[96];
            snprintf(tail, sizeof tail, "  (%.4f ms, %d candidates)\n", kv.second.ms, kv.second.candidates);
            out += tail;
        }
    }
    if (needed) *needed = (int64_t)out.size() + 1;
    if (buf && size > 0) {
        size_t n = std::min<size_t>((size_t)size - 1, out.size());
        memcpy(buf, out.data(), n);
        buf[n] = 0;
    }
    return VIE_OK;
}
