// FFT plans: radix factorisation and device twiddle tables; the device buffer type and its
// cache of released blocks.
#include <atomic>
#include <cmath>
#include <map>
#include <mutex>
#include <vector>

#include "vie_internal.h"

static int smallest_prime_factor(int n) {
    for (int p = 2; p * p <= n; ++p)
        if (n % p == 0) return p;
    return n;
}

bool fft_supported_length(int L) {
    if (L < 1) return false;
    int n = L;
    while (n > 1) {
        int p = smallest_prime_factor(n);
        if (p > VIE_FFT_MAX_PRIME) return false;
        n /= p;
    }
    return true;
}

int fft_good_length(int minL) {
    if (minL <= 1) return 1;
    for (int L = minL;; ++L) {
        int n = L;
        for (int p : {2, 3, 5})
            while (n % p == 0) n /= p;
        if (n == 1) return L;
    }
}

static void factor(int L, FftPlan *plan) {
    int n = L;
    plan->nrad = 0;
    while (n % 4 == 0) {
        plan->rad[plan->nrad++] = 4;
        n /= 4;
    }
    while (n % 2 == 0) {
        plan->rad[plan->nrad++] = 2;
        n /= 2;
    }
    while (n > 1) {
        int p = smallest_prime_factor(n);
        plan->rad[plan->nrad++] = p;
        n /= p;
    }
}

vie_status FftCache::get(int L, FftPlan *plan) {
    if (!fft_supported_length(L)) {
        vie_set_error("FFT length " + std::to_string(L) + " has a prime factor above " +
                      std::to_string(VIE_FFT_MAX_PRIME));
        return VIE_EARG;
    }
    Entry *e = nullptr;
    for (Entry *x : entries)
        if (x->L == L) e = x;
    if (!e) {
        e = new Entry();
        e->L = L;
        entries.push_back(e);
        std::vector<c128> h64(L);
        std::vector<c64> h32(L);
        const long double twopi = 6.283185307179586476925286766559005768L;
        for (int q = 0; q < L; ++q) {
            // exp(-2 pi i q / L), using the exactly representable reduction q/L in [0, 1)
            long double a = twopi * (long double)q / (long double)L;
            double c = (double)cosl(a), s = (double)(-sinl(a));
            // exact values on the axes
            if (4LL * q == 0) { c = 1.0; s = 0.0; }
            if (4LL * q == (long long)L) { c = 0.0; s = -1.0; }
            if (2LL * q == (long long)L) { c = -1.0; s = 0.0; }
            if (4LL * q == 3LL * L) { c = 0.0; s = 1.0; }
            h64[q] = mk(c, s);
            h32[q] = mk((float)c, (float)s);
        }
        VIE_CHECK(e->t64.ensure(sizeof(c128) * L));
        VIE_CHECK(e->t32.ensure(sizeof(c64) * L));
        VIE_HIP(hipMemcpy(e->t64.p, h64.data(), sizeof(c128) * L, hipMemcpyHostToDevice));
        VIE_HIP(hipMemcpy(e->t32.p, h32.data(), sizeof(c64) * L, hipMemcpyHostToDevice));
    }
    plan->L = L;
    factor(L, plan);
    plan->tw64 = e->t64.as<const c128>();
    plan->tw32 = e->t32.as<const c64>();
    return VIE_OK;
}

FftCache::~FftCache() {
    for (Entry *e : entries) {
        e->t64.release();
        e->t32.release();
        delete e;
    }
}

// Device bytes held by the library's buffers, and their high-water mark.
static std::atomic<uint64_t> g_dev_cur{0}, g_dev_peak{0};

// Released buffers are kept for reuse instead of being returned to the driver: freeing and
// re-allocating tens of GB (the Krylov bases of a batched solve) costs seconds in the driver
// at times.  A request takes the smallest cached block of at least its size and at most twice
// it; when the driver is out of memory the cache is returned and the allocation retried.
// A block released inside a library call carries an event recorded on that call's stream (the
// stream its last work was queued on): whoever takes it next waits for that event only.
// Released outside a call (destroy, trim), the device is synchronised instead.
namespace {
struct Block {
    void *p;
    hipEvent_t ev;       // nullptr: idle already
    hipStream_t stream;  // the stream ev was recorded on
};
std::mutex g_pool_mu;
std::multimap<size_t, Block> g_pool;  // size -> block
size_t g_pool_bytes = 0;
std::vector<std::pair<hipEvent_t, hipStream_t>> g_events;  // idle events, last stream (under g_pool_mu)
thread_local hipStream_t t_stream = nullptr;
thread_local int t_stream_depth = 0;

void pool_trim_locked() {
    for (auto &kv : g_pool) {
        if (kv.second.ev) {
            (void)hipEventSynchronize(kv.second.ev);
            g_events.emplace_back(kv.second.ev, kv.second.stream);
        }
        (void)hipFree(kv.second.p);
    }
    g_pool.clear();
    g_pool_bytes = 0;
}
}  // namespace

void pool_stream_retired(hipStream_t s) {
    // an event must not outlive the stream it was last recorded on: wait for the blocks
    // released on s and drop their events (fresh ones are created on demand)
    std::lock_guard<std::mutex> lk(g_pool_mu);
    for (auto &kv : g_pool)
        if (kv.second.ev && kv.second.stream == s) {
            (void)hipEventSynchronize(kv.second.ev);
            (void)hipEventDestroy(kv.second.ev);
            kv.second.ev = nullptr;
        }
    for (size_t i = 0; i < g_events.size();)
        if (g_events[i].second == s) {
            (void)hipEventDestroy(g_events[i].first);
            g_events[i] = g_events.back();
            g_events.pop_back();
        } else {
            ++i;
        }
}

StreamScope::StreamScope(hipStream_t s) : prev(t_stream) {
    t_stream = s;
    ++t_stream_depth;
}

StreamScope::~StreamScope() {
    t_stream = prev;
    --t_stream_depth;
}

extern "C" vie_status vie_device_bytes(uint64_t *current, uint64_t *peak, int32_t reset_peak) {
    if (reset_peak) g_dev_peak.store(g_dev_cur.load());
    if (current) *current = g_dev_cur.load();
    if (peak) *peak = g_dev_peak.load();
    return VIE_OK;
}

uint64_t pool_cached_bytes() {
    std::lock_guard<std::mutex> lk(g_pool_mu);
    return g_pool_bytes;
}

// Cached blocks back to the driver, each after its own last work.  The blocks leave the cache
// under its lock and are freed after it is released, so other threads' allocations and releases
// go on meanwhile (hipFree itself may still wait for the device).
void pool_trim_cached() {
    std::vector<Block> gone;
    {
        std::lock_guard<std::mutex> lk(g_pool_mu);
        for (auto &kv : g_pool) gone.push_back(kv.second);
        g_pool.clear();
        g_pool_bytes = 0;
    }
    for (Block &b : gone) {
        if (b.ev) {
            (void)hipEventSynchronize(b.ev);
            std::lock_guard<std::mutex> lk(g_pool_mu);
            g_events.emplace_back(b.ev, b.stream);
        }
        (void)hipFree(b.p);
    }
}

extern "C" vie_status vie_trim(void) {
    std::lock_guard<std::mutex> lk(g_pool_mu);
    VIE_HIP(hipDeviceSynchronize());
    pool_trim_locked();
    return VIE_OK;
}

vie_status DevBuf::ensure(size_t nbytes) {
    if (nbytes <= bytes && p) return VIE_OK;
    release();
    if (nbytes == 0) return VIE_OK;
    {
        hipEvent_t ev = nullptr;
        hipStream_t evs = nullptr;
        {
            std::lock_guard<std::mutex> lk(g_pool_mu);
            auto it = g_pool.lower_bound(nbytes);
            if (it != g_pool.end() && it->first <= 2 * nbytes) {
                p = it->second.p;
                ev = it->second.ev;
                evs = it->second.stream;
                bytes = it->first;
                g_pool_bytes -= it->first;
                g_pool.erase(it);
            }
        }
        if (ev) {  // the previous user's work on this block is done before it is handed out
            (void)hipEventSynchronize(ev);
            std::lock_guard<std::mutex> lk(g_pool_mu);
            g_events.emplace_back(ev, evs);
        }
    }
    if (!p) {
        hipError_t e = hipMalloc(&p, nbytes);
        if (e == hipErrorOutOfMemory) {
            std::lock_guard<std::mutex> lk(g_pool_mu);
            pool_trim_locked();
            e = hipMalloc(&p, nbytes);
        }
        if (e != hipSuccess) {
            p = nullptr;
            bytes = 0;
            vie_set_error("hipMalloc of " + std::to_string(nbytes) + " bytes failed: " + hipGetErrorString(e));
            return e == hipErrorOutOfMemory ? VIE_EOOM : VIE_EDEVICE;
        }
        bytes = nbytes;
    }
    const uint64_t cur = g_dev_cur.fetch_add(bytes) + bytes;
    uint64_t pk = g_dev_peak.load();
    while (cur > pk && !g_dev_peak.compare_exchange_weak(pk, cur)) {
    }
    return VIE_OK;
}

void DevBuf::release() {
    if (p) {
        hipEvent_t ev = nullptr;
        if (t_stream_depth > 0) {
            {
                std::lock_guard<std::mutex> lk(g_pool_mu);
                if (!g_events.empty()) {
                    ev = g_events.back().first;
                    g_events.pop_back();
                }
            }
            if (!ev && hipEventCreateWithFlags(&ev, hipEventDisableTiming) != hipSuccess) ev = nullptr;
            if (ev && hipEventRecord(ev, t_stream) != hipSuccess) {
                (void)hipEventDestroy(ev);
                ev = nullptr;
            }
        }
        if (!ev) (void)hipDeviceSynchronize();  // no call stream known: wait for everything
        std::lock_guard<std::mutex> lk(g_pool_mu);
        g_pool.emplace(bytes, Block{p, ev, t_stream});
        g_pool_bytes += bytes;
        g_dev_cur.fetch_sub(bytes);
    }
    p = nullptr;
    bytes = 0;
}
