// Request scheduler for many solves on one GPU (the serving part of the C ABI).
//
// Submitted requests wait in a FIFO queue.  A worker thread (one HIP stream each) takes the
// first queued request that can be admitted: its operator and preconditioner are found in the
// resident cache (shared with any solves running on them: the handles are read-only and each
// stream has its own scratch), or the bytes to build them fit the budget after evicting idle
// cache entries (least recently used first); the solve's own bytes must fit as well.  An entry
// is built once: requests for it wait while another worker builds it.  Later queued
// requests with the same device, preconditioner options and solver settings join it in one
// multi-RHS solve.  A request that has been passed over by later ones several times blocks
// further overtaking until it is admitted.
// Continuous batching: the solve's right-hand sides are slots.  At every restart-cycle
// boundary of the batched GMRES, a request whose columns have all ended is completed at once
// (its columns copied to the caller's host buffer, its waiter woken) and its slots are freed;
// a queued request for the same device and settings whose right-hand sides fit the free
// slots joins the running solve there, without a new admission (its memory is the slots').
// After the solve the operator and preconditioner return to the cache.
#include <algorithm>
#include <chrono>
#include <condition_variable>
#include <cstdio>
#include <cstring>
#include <deque>
#include <list>
#include <map>
#include <mutex>
#include <thread>
#include <vector>

#include "vie_internal.h"

// buffer cache of fft_host.cpp: bytes of the released blocks kept for reuse, and returning them
uint64_t pool_cached_bytes();
void pool_trim_cached();

namespace {
using Clock = std::chrono::steady_clock;

#define SERVE_MAX_OVERTAKE 8

uint64_t fnv1a(const void *p, size_t n, uint64_t h = 1469598103934665603ULL) {
    const unsigned char *c = static_cast<const unsigned char *>(p);
    for (size_t i = 0; i < n; ++i) {
        h ^= c[i];
        h *= 1099511628211ULL;
    }
    return h;
}

struct Req {
    int64_t id = 0;
    int32_t grid[3] = {0, 0, 0};
    double delta = 0, kb = 0;
    std::vector<double> chi, e;
    int nrhs = 0;
    int precond = 0;
    vie_pc_opts pco{};
    std::vector<int32_t> boxes, box_levels, box_homog;
    vie_solve_opts so{};
    double *x_out = nullptr;
    vie_solve_stats *st_out = nullptr;
    std::string key;        // device + preconditioner options: the cache key
    std::string batch_key;  // key + solver settings: requests that may share one solve
    Clock::time_point t_submit, t_start, t_end;
    vie_status status = VIE_OK;
    bool done = false;
    int cache_hit = 0, merged = 1, overtaken = 0, joined = 0;
    int cols_left = 0;      // columns of a running solve not yet ended
    bool finished = false;  // all columns ended and copied out
    std::string err;  // message of a failed build or solve
};

struct Entry {
    std::string key;
    vie_op op = nullptr;
    vie_pc pc = nullptr;
    uint64_t bytes = 0;  // resident bytes accounted for this entry
    int users = 0;       // solves running on it
    bool ready = false;  // built (until then the admitting worker is building it)
    uint64_t last = 0;
};

// One admitted solve: the requests merged into it and its accounting.
struct Batch {
    std::vector<Req *> reqs;  // requests of the solve not yet completed (a waiter may free the others)
    std::string key, batch_key;
    int n_total = 0;          // requests that took part, joiners included
    Entry *entry = nullptr;   // cache entry it runs on
    bool build = false;       // this solve builds the entry
    bool trim = false;        // return the released blocks cached for reuse before running
    int R = 0;
    uint64_t build_bytes = 0, run = 0;  // bytes committed for the build (while it runs) and the run
};

double ms_between(Clock::time_point a, Clock::time_point b) {
    return std::chrono::duration<double, std::milli>(b - a).count();
}
}  // namespace

struct vie_server_s {
    int workers_n = 4, max_rhs = 64;
    uint64_t budget = 0;
    int device = 0;
    std::mutex mu;
    std::condition_variable cv_work, cv_done;
    std::deque<Req *> queue;
    std::map<int64_t, Req *> reqs;
    std::list<Entry *> cache;
    uint64_t committed = 0, peak = 0, tick = 0;
    int64_t next_id = 1;
    bool stop = false;
    int running = 0;
    std::vector<std::thread> threads;
    int64_t n_submitted = 0, n_completed = 0, n_solves = 0, n_hits = 0, n_evicted = 0, n_shared = 0, n_trims = 0;
};

namespace {
void commit(vie_server srv, uint64_t b) {
    srv->committed += b;
    srv->peak = std::max(srv->peak, srv->committed);
}

void destroy_entry(Entry *e) {
    if (e->pc) precond_destroy(e->pc);
    if (e->op) vie_destroy(e->op);
    delete e;
}

// Free idle cache entries (least recently used first, never `keep`) until `need` more bytes
// fit; true if they do.  Called with the lock held.
bool make_room(vie_server srv, uint64_t need, const Entry *keep) {
    while (srv->committed + need > srv->budget) {
        Entry *victim = nullptr;
        for (Entry *e : srv->cache)
            if (e->users == 0 && e->ready && e != keep && (!victim || e->last < victim->last)) victim = e;
        if (!victim) return false;
        srv->cache.remove(victim);
        srv->committed -= victim->bytes;
        destroy_entry(victim);
        srv->n_evicted++;
    }
    return true;
}

// The operator keeps a complex64 copy: complex64 products (mixed mode) or bfloat16 factors.
bool op_c64(const Req *r) {
    return r->so.mode == VIE_MODE_MIXED || (r->precond && r->pco.factor_prec == VIE_BF16C);
}

// Admit the first admissible queued request (with the requests merged into it).  Lock held.
bool pick(vie_server srv, Batch *b) {
    for (size_t qi = 0; qi < srv->queue.size(); ++qi) {
        Req *r = srv->queue[qi];
        // merge later requests with the same batch key
        std::vector<size_t> idx{qi};
        int R = r->nrhs;
        for (size_t qj = qi + 1; qj < srv->queue.size(); ++qj) {
            Req *o = srv->queue[qj];
            if (o->batch_key == r->batch_key && R + o->nrhs <= srv->max_rhs) {
                idx.push_back(qj);
                R += o->nrhs;
            }
        }
        Entry *ent = nullptr;
        for (Entry *e : srv->cache)
            if (e->key == r->key) ent = e;
        if (ent && !ent->ready) continue;  // another worker is building it: later requests may go
        // Merged requests are dropped from the end while the batch could not fit even with every
        // idle entry evicted: the head alone always fits an empty server (checked on submit), so
        // a merge never holds it back for good.
        uint64_t evictable = 0;
        for (Entry *e : srv->cache)
            if (e->users == 0 && e->ready && e != ent) evictable += e->bytes;
        const uint64_t avail = srv->budget + evictable > srv->committed ? srv->budget + evictable - srv->committed : 0;
        uint64_t resident = 0, build = 0, run = 0, need = 0;
        for (;;) {
            if (request_footprint(r->grid, op_c64(r), r->precond ? &r->pco : nullptr, R, &r->so, &resident, &build,
                                  &run) != VIE_OK)
                resident = build = run = 0;  // arguments were checked on submit
            need = run + (ent ? 0 : resident + build);
            if (need <= avail || idx.size() == 1) break;
            R -= srv->queue[idx.back()]->nrhs;
            idx.pop_back();
        }
        if (make_room(srv, need, ent)) {
            // released buffers cached for reuse hold device memory too: past the budget the worker
            // returns them to the driver (outside this lock), so the runtime's own allocations at
            // launch (kernel scratch) still fit
            b->trim = srv->committed + need + pool_cached_bytes() > srv->budget;
            srv->n_trims += b->trim ? 1 : 0;
            commit(srv, need);
            b->reqs.clear();
            for (size_t k : idx) b->reqs.push_back(srv->queue[k]);
            b->key = r->key;
            b->batch_key = r->batch_key;
            b->n_total = (int)idx.size();
            for (size_t k = idx.size(); k-- > 0;) srv->queue.erase(srv->queue.begin() + (long)idx[k]);
            for (size_t k = 0; k < qi; ++k) srv->queue[k]->overtaken++;
            b->build = ent == nullptr;
            if (!ent) {  // listed now, so requests for it wait for this build instead of repeating it
                ent = new Entry();
                ent->key = r->key;
                ent->bytes = resident;
                srv->cache.push_back(ent);
            }
            if (ent->users > 0) srv->n_shared++;
            ent->users++;
            b->entry = ent;
            b->R = R;
            b->build_bytes = b->build ? build : 0;
            b->run = run;
            return true;
        }
        if (r->overtaken >= SERVE_MAX_OVERTAKE) return false;  // the head waits for memory
    }
    return false;
}

// Mark request r complete (lock held): timings, status, waiter woken; r leaves the batch's
// list, since its waiter may free it from now on.
void complete_locked(vie_server srv, Req *r, Batch *b, vie_status st, const std::string &err) {
    b->reqs.erase(std::remove(b->reqs.begin(), b->reqs.end(), r), b->reqs.end());
    r->t_end = Clock::now();
    r->cache_hit = !b->build || r->joined;
    r->merged = b->n_total;
    if (st < 0) {
        r->status = st;
        r->err = err;
    }
    r->done = true;
    srv->n_completed++;
    srv->cv_done.notify_all();
}

// The slots of one running solve (see the header): completes requests whose columns have all
// ended and lets queued requests of the same batch key join the freed slots.
struct SlotHook : SolveHook {
    vie_server srv;
    Batch *batch;
    vie_op op;
    long long n3;
    c128 *e;                    // device incident fields, one column per slot
    std::vector<Req *> owner;   // slot -> request
    std::vector<int> owner_col; // slot -> column of that request
    std::vector<int> free_slots;

    vie_status boundary(const std::vector<int> &ended, const vie_solve_stats *stats, const c128 *x, c128 *b,
                        hipStream_t s, std::vector<int> *refill) override {
        // requests whose last column ended: copy their columns out, then complete them
        std::vector<Req *> fin;
        for (int q : ended) {
            Req *r = owner[q];
            if (!r) continue;
            r->st_out[owner_col[q]] = stats[q];
            if (stats[q].status != VIE_OK) r->status = VIE_NOT_CONVERGED;
            if (--r->cols_left == 0) fin.push_back(r);
        }
        for (Req *r : fin)
            for (int q = 0; q < (int)owner.size(); ++q)
                if (owner[q] == r) {
                    VIE_HIP(hipMemcpyAsync(r->x_out + 2 * n3 * owner_col[q], x + n3 * q, sizeof(c128) * n3,
                                           hipMemcpyDeviceToHost, s));
                    owner[q] = nullptr;
                    free_slots.push_back(q);
                }
        if (!fin.empty()) VIE_HIP(hipStreamSynchronize(s));
        std::vector<Req *> join;
        {
            std::lock_guard<std::mutex> lk(srv->mu);
            // queued requests of this batch key that fit the free slots join, in queue order
            if (!free_slots.empty() && !srv->stop) {
                int nfree = (int)free_slots.size();
                for (size_t qi = 0; qi < srv->queue.size() && nfree > 0;) {
                    Req *r = srv->queue[qi];
                    if (r->batch_key == batch->batch_key && r->nrhs <= nfree) {
                        srv->queue.erase(srv->queue.begin() + (long)qi);
                        nfree -= r->nrhs;
                        r->joined = 1;
                        r->t_start = Clock::now();
                        batch->reqs.push_back(r);
                        batch->n_total++;
                        srv->n_hits++;
                        join.push_back(r);
                    } else {
                        ++qi;
                    }
                }
            }
            // the requests of the solve's last boundary are completed by the worker, together
            // with the end of the solve
            const bool last = join.empty() && (int)free_slots.size() == (int)owner.size();
            for (Req *r : fin) {
                r->finished = true;
                if (!last) complete_locked(srv, r, batch, VIE_OK, std::string());
            }
        }
        for (Req *r : join) {
            r->cols_left = r->nrhs;
            r->status = VIE_OK;
            for (int i = 0; i < r->nrhs; ++i) {
                const int q = free_slots.back();
                free_slots.pop_back();
                owner[q] = r;
                owner_col[q] = i;
                VIE_HIP(hipMemcpyAsync(e + n3 * q, r->e.data() + 2 * n3 * i, sizeof(c128) * n3,
                                       hipMemcpyHostToDevice, s));
                VIE_CHECK(vie_rhs(op, e + n3 * q, b + n3 * q, 1, s));
                refill->push_back(q);
            }
        }
        return VIE_OK;
    }
};

// Build (or take from the cache) the operator and preconditioner and solve the merged
// right-hand sides as slots of one batched GMRES (SlotHook completes the requests and takes
// joiners).  Runs without the lock.
// Build the entry's operator and preconditioner (the admitting worker, without the lock), then
// publish them; on failure the entry leaves the cache.
vie_status build_entry(vie_server srv, Batch *b, hipStream_t s) {
    Req *r0 = b->reqs[0];
    vie_op op = nullptr;
    vie_pc pc = nullptr;
    vie_create_opts co{};
    co.build_c64 = op_c64(r0);
    vie_status st = vie_create(r0->grid, r0->delta, r0->kb, r0->chi.data(), &co, s, &op);
    if (st >= 0 && r0->precond) st = precond_setup(op, &r0->pco, s, &pc);
    std::lock_guard<std::mutex> lk(srv->mu);
    srv->committed -= b->build_bytes;  // the build's transient bytes are released
    b->build_bytes = 0;
    Entry *e = b->entry;
    if (st < 0) {
        if (pc) precond_destroy(pc);
        if (op) vie_destroy(op);
        srv->cache.remove(e);
        srv->committed -= e->bytes;
        delete e;
        b->entry = nullptr;
    } else {
        e->op = op;
        e->pc = pc;
        e->ready = true;
    }
    srv->cv_work.notify_all();  // requests waiting for this entry
    return st;
}

vie_status run_batch(vie_server srv, Batch *b, hipStream_t s) {
    StreamScope scope(s);  // the batch's buffers are reused once this worker's stream is past them
    Req *r0 = b->reqs[0];
    const long long N = (long long)r0->grid[0] * r0->grid[1] * r0->grid[2];
    const long long n3 = 3 * N;
    if (b->build) VIE_CHECK(build_entry(srv, b, s));
    vie_op op = b->entry->op;
    vie_pc pc = b->entry->pc;
    // this stream's scratch of the shared handles goes back to the cache of released blocks when
    // the solve ends (it is part of the solve's accounted bytes, not the entry's)
    struct WsDrop {
        vie_op op;
        vie_pc pc;
        hipStream_t s;
        ~WsDrop() {
            op_drop_ws(op, s);
            pc_drop_ws(pc, s);
        }
    } ws_drop{op, pc, s};
    DevBuf e, bb, x;
    VIE_CHECK(e.ensure(sizeof(c128) * n3 * b->R));
    VIE_CHECK(bb.ensure(sizeof(c128) * n3 * b->R));
    VIE_CHECK(x.ensure(sizeof(c128) * n3 * b->R));
    SlotHook hook;
    hook.srv = srv;
    hook.batch = b;
    hook.op = op;
    hook.n3 = n3;
    hook.e = e.as<c128>();
    hook.owner.assign(b->R, nullptr);
    hook.owner_col.assign(b->R, 0);
    long long off = 0;
    int slot = 0;
    for (Req *r : b->reqs) {
        VIE_HIP(hipMemcpyAsync(e.as<c128>() + off, r->e.data(), sizeof(c128) * n3 * r->nrhs, hipMemcpyHostToDevice, s));
        off += n3 * r->nrhs;
        r->cols_left = r->nrhs;
        r->status = VIE_OK;
        for (int i = 0; i < r->nrhs; ++i, ++slot) {
            hook.owner[slot] = r;
            hook.owner_col[slot] = i;
        }
    }
    VIE_CHECK(vie_rhs(op, e.p, bb.p, b->R, s));
    VIE_HIP(hipMemsetAsync(x.p, 0, sizeof(c128) * n3 * b->R, s));
    std::vector<vie_solve_stats> st(b->R);
    vie_solve_opts so = r0->so;
    so.x0_given = 0;
    const vie_status ss = solve_gmres(op, pc, bb.as<c128>(), x.as<c128>(), b->R, &so, st.data(), s, &hook);
    if (ss < 0) return ss;
    VIE_HIP(hipStreamSynchronize(s));
    return VIE_OK;
}

void worker(vie_server srv) {
    (void)hipSetDevice(srv->device);
    hipStream_t s = nullptr;
    const bool have_stream = hipStreamCreateWithFlags(&s, hipStreamNonBlocking) == hipSuccess;
    std::unique_lock<std::mutex> lk(srv->mu);
    for (;;) {
        Batch b;
        while (!pick(srv, &b)) {
            if (srv->stop && srv->queue.empty()) break;
            srv->cv_work.wait(lk);
        }
        if (b.reqs.empty()) break;
        srv->running++;
        lk.unlock();
        const Clock::time_point t0 = Clock::now();
        for (Req *r : b.reqs) r->t_start = t0;
        const size_t n_admitted = b.reqs.size();  // later joiners are counted when they join
        if (b.trim) pool_trim_cached();
        vie_status st = have_stream ? run_batch(srv, &b, s) : VIE_EDEVICE;
        if (!have_stream) vie_set_error("vie_server: hipStreamCreate failed");
        const std::string err = st < 0 ? std::string(vie_last_error()) : std::string();
        lk.lock();
        srv->running--;
        srv->committed -= b.run;
        srv->n_solves++;
        if (b.entry && !b.entry->ready) {  // admitted to build it but never ran (no stream)
            srv->committed -= b.build_bytes + b.entry->bytes;
            srv->cache.remove(b.entry);
            delete b.entry;
            b.entry = nullptr;
        }
        if (b.entry) {
            b.entry->users--;
            b.entry->last = ++srv->tick;
            if (!b.build) srv->n_hits += (int64_t)n_admitted;
        }
        const std::vector<Req *> left = b.reqs;  // finished at the last boundary, or the solve failed
        for (Req *r : left) {
            if (r->finished && st >= 0) complete_locked(srv, r, &b, VIE_OK, std::string());
            else complete_locked(srv, r, &b, st < 0 ? st : VIE_EDEVICE, st < 0 ? err : "solve ended early");
        }
        srv->cv_done.notify_all();
        srv->cv_work.notify_all();
    }
    lk.unlock();
    if (have_stream) {
        (void)hipStreamSynchronize(s);
        pool_stream_retired(s);
        (void)hipStreamDestroy(s);
    }
}
}  // namespace

extern "C" vie_status vie_server_create(const vie_server_opts *opts, vie_server *out) {
    if (!out) {
        vie_set_error("vie_server_create: out is NULL");
        return VIE_EARG;
    }
    *out = nullptr;
    vie_server_opts o{};
    if (opts) o = *opts;
    if (o.workers < 0 || o.workers > 16 || o.max_batch_rhs < 0) {
        vie_set_error("vie_server_create: workers must be in [0, 16] and max_batch_rhs >= 0");
        return VIE_EARG;
    }
    vie_server srv = new (std::nothrow) vie_server_s();
    if (!srv) return VIE_EOOM;
    srv->workers_n = o.workers ? o.workers : 4;
    srv->max_rhs = o.max_batch_rhs ? o.max_batch_rhs : 64;
    if (hipGetDevice(&srv->device) != hipSuccess) {
        delete srv;
        vie_set_error("vie_server_create: no HIP device");
        return VIE_EDEVICE;
    }
    srv->budget = o.hbm_budget;
    if (!srv->budget) {
        size_t fr = 0, tot = 0;
        if (hipMemGetInfo(&fr, &tot) != hipSuccess) {
            delete srv;
            vie_set_error("vie_server_create: hipMemGetInfo failed");
            return VIE_EDEVICE;
        }
        srv->budget = (uint64_t)(0.9 * (double)fr);
    }
    for (int i = 0; i < srv->workers_n; ++i) srv->threads.emplace_back(worker, srv);
    *out = srv;
    return VIE_OK;
}

extern "C" vie_status vie_server_submit(vie_server srv, const vie_request *req, double *x_out,
                                        vie_solve_stats *stats_out, int64_t *id) {
    if (!srv || !req || !x_out || !stats_out || !id) {
        vie_set_error("vie_server_submit: NULL argument");
        return VIE_EARG;
    }
    for (int a = 0; a < 3; ++a)
        if (req->grid[a] < 1) {
            vie_set_error("vie_server_submit: every grid dimension must be >= 1");
            return VIE_EARG;
        }
    if (!req->chi || !req->e_inc || req->nrhs < 1) {
        vie_set_error("vie_server_submit: chi and e_inc are required and nrhs must be >= 1");
        return VIE_EARG;
    }
    if (req->solve.x0_given) {
        vie_set_error("vie_server_submit: requests start from x = 0 (x0_given must be 0)");
        return VIE_EARG;
    }
    if (req->precond && req->pc.nboxes > 0 && !req->pc.boxes) {
        vie_set_error("vie_server_submit: pc.boxes is NULL");
        return VIE_EARG;
    }
    const long long N = (long long)req->grid[0] * req->grid[1] * req->grid[2];
    Req *r = new (std::nothrow) Req();
    if (!r) return VIE_EOOM;
    std::copy(req->grid, req->grid + 3, r->grid);
    r->delta = req->voxel_size;
    r->kb = req->k_background;
    r->chi.assign(req->chi, req->chi + 2 * N);
    r->e.assign(req->e_inc, req->e_inc + 6 * N * req->nrhs);
    r->nrhs = req->nrhs;
    r->precond = req->precond != 0;
    r->pco = req->pc;
    r->pco.boxes = nullptr;
    r->pco.box_levels = r->pco.box_homog = nullptr;
    if (r->precond && req->pc.nboxes > 0) {
        const int nb = req->pc.nboxes;
        r->boxes.assign(req->pc.boxes, req->pc.boxes + 6 * nb);
        r->pco.boxes = r->boxes.data();
        if (req->pc.box_levels) {
            r->box_levels.assign(req->pc.box_levels, req->pc.box_levels + nb);
            r->pco.box_levels = r->box_levels.data();
        }
        if (req->pc.box_homog) {
            r->box_homog.assign(req->pc.box_homog, req->pc.box_homog + nb);
            r->pco.box_homog = r->box_homog.data();
        }
    }
    r->so = req->solve;
    r->x_out = x_out;
    r->st_out = stats_out;
    const vie_status vs = solve_opts_check("vie_server_submit", r->so);
    if (vs < 0) {
        delete r;
        return vs;
    }
    uint64_t resident = 0, build = 0, run = 0;
    const vie_status fs = request_footprint(r->grid, op_c64(r), r->precond ? &r->pco : nullptr, r->nrhs, &r->so,
                                            &resident, &build, &run);
    if (fs < 0) {
        delete r;
        return fs;
    }
    if (resident + build + run > srv->budget) {
        delete r;
        vie_set_error("vie_server_submit: the request needs " + std::to_string(resident + build + run) +
                      " device bytes, above the budget of " + std::to_string(srv->budget));
        return VIE_EBUDGET;
    }
    char buf[256];
    const uint64_t hchi = fnv1a(r->chi.data(), sizeof(double) * r->chi.size());
    snprintf(buf, sizeof buf, "%dx%dx%d|%a|%a|%016llx|%d|%d", r->grid[0], r->grid[1], r->grid[2], r->delta, r->kb,
             (unsigned long long)hchi, r->precond, (int)op_c64(r));
    r->key = buf;
    if (r->precond) {
        const vie_pc_opts &p = r->pco;
        uint64_t hb = fnv1a(r->boxes.data(), sizeof(int32_t) * r->boxes.size());
        hb = fnv1a(r->box_levels.data(), sizeof(int32_t) * r->box_levels.size(), hb);
        hb = fnv1a(r->box_homog.data(), sizeof(int32_t) * r->box_homog.size(), hb);
        snprintf(buf, sizeof buf, "|pc %d %d %016llx %d %a %d %d %d %d %d %a %d", p.homog, p.nboxes,
                 (unsigned long long)hb, p.reduce, p.reduce ? p.reduce_tol : 0.0, p.factor_prec, p.proxy,
                 p.refine_steps, p.keep_zero_rows, p.levels, p.share_tol, p.no_mirror);
        r->key += buf;
    }
    snprintf(buf, sizeof buf, "|so %a %d %d %d", r->so.tol, r->so.restart, r->so.maxit, r->so.mode);
    r->batch_key = r->key + buf;
    std::lock_guard<std::mutex> lk(srv->mu);
    if (srv->stop) {
        delete r;
        vie_set_error("vie_server_submit: the server is shutting down");
        return VIE_EARG;
    }
    r->id = srv->next_id++;
    r->t_submit = Clock::now();
    srv->queue.push_back(r);
    srv->reqs[r->id] = r;
    srv->n_submitted++;
    *id = r->id;
    srv->cv_work.notify_one();
    return VIE_OK;
}

extern "C" vie_status vie_server_wait(vie_server srv, int64_t id, vie_request_times *times) {
    if (!srv) {
        vie_set_error("vie_server_wait: NULL server");
        return VIE_EARG;
    }
    std::unique_lock<std::mutex> lk(srv->mu);
    auto it = srv->reqs.find(id);
    if (it == srv->reqs.end()) {
        vie_set_error("vie_server_wait: unknown request id " + std::to_string(id));
        return VIE_EARG;
    }
    Req *r = it->second;
    srv->cv_done.wait(lk, [&] { return r->done; });
    if (times) {
        times->queue_ms = ms_between(r->t_submit, r->t_start);
        times->run_ms = ms_between(r->t_start, r->t_end);
        times->total_ms = ms_between(r->t_submit, r->t_end);
        times->cache_hit = r->cache_hit;
        times->merged = r->merged;
        times->joined = r->joined;
    }
    const vie_status st = r->status;
    if (st < 0) vie_set_error("vie_server_wait: request " + std::to_string(id) + " failed: " + r->err);
    srv->reqs.erase(it);
    delete r;
    return st;
}

extern "C" vie_status vie_server_query(vie_server srv, int64_t id, int32_t *done) {
    if (!srv || !done) {
        vie_set_error("vie_server_query: NULL argument");
        return VIE_EARG;
    }
    std::lock_guard<std::mutex> lk(srv->mu);
    auto it = srv->reqs.find(id);
    if (it == srv->reqs.end()) {
        vie_set_error("vie_server_query: unknown request id " + std::to_string(id));
        return VIE_EARG;
    }
    *done = it->second->done ? 1 : 0;
    return VIE_OK;
}

extern "C" vie_status vie_server_info_get(vie_server srv, vie_server_info *info) {
    if (!srv || !info) {
        vie_set_error("vie_server_info_get: NULL argument");
        return VIE_EARG;
    }
    std::lock_guard<std::mutex> lk(srv->mu);
    info->submitted = srv->n_submitted;
    info->completed = srv->n_completed;
    info->solves = srv->n_solves;
    info->cache_hits = srv->n_hits;
    info->evictions = srv->n_evicted;
    info->cached_entries = (int32_t)srv->cache.size();
    info->queued = (int32_t)srv->queue.size();
    info->running = srv->running;
    info->committed_bytes = srv->committed;
    info->peak_committed_bytes = srv->peak;
    info->budget_bytes = srv->budget;
    info->shared_runs = srv->n_shared;
    info->cache_trims = srv->n_trims;
    return VIE_OK;
}

extern "C" vie_status vie_server_destroy(vie_server srv) {
    if (!srv) return VIE_OK;
    {
        std::lock_guard<std::mutex> lk(srv->mu);
        srv->stop = true;
    }
    srv->cv_work.notify_all();
    for (auto &t : srv->threads) t.join();
    for (Entry *e : srv->cache) destroy_entry(e);
    for (auto &kv : srv->reqs) delete kv.second;
    delete srv;
    return VIE_OK;
}
