// Serving pool of libfdtd (declared and documented in include/fdtd.h).
//
// A persistent host thread runs the request loop:
//   admit    queued requests (FIFO, optionally backfilled) whose state fits
//            the free space of the pool's HBM arena (first-fit sub-allocator);
//            their fields are initialised on the compute stream, in order
//            before their first sweep
//   launch   one batched temporal sweep over the tiles of every active
//            request (grouped only by steps-per-sweep and coefficient kind),
//            through a small ring of request tables whose events bound the
//            launches in flight
//   retire   a request whose last sweep is enqueued records a completion
//            event; its memory returns to the allocator at once (stream order
//            keeps the next user of the range behind the last sweep) unless
//            the caller keeps the result for fetching
// Each request's arithmetic is the single-solve tile code on its own buffers,
// so its bits do not depend on what else is in the batch.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <condition_variable>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <deque>
#include <map>
#include <memory>
#include <mutex>
#include <string>
#include <thread>
#include <unordered_set>
#include <vector>

#include "fdtd.h"
#include "fdtd_internal.h"

using fdtd::BatchEntry;
using fdtd::Geom;
using fdtd::Plan;

namespace {

constexpr uint32_t kPoolMagic = 0xFD7DB001u;
constexpr uint32_t kPoolDead = 0xDEADB001u;
constexpr int kRing = 4;  // request tables (and batched launches) in flight

std::mutex g_pools_mu;
std::unordered_set<const void *> g_pools;

int pfail(int status, const char *fmt, ...) __attribute__((format(printf, 2, 3)));
int pfail(int status, const char *fmt, ...)
{
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    fdtd::set_last_error(buf);
    return status;
}

// First-fit allocator over [0, size) with coalescing of free ranges.
class RangeAlloc {
public:
    explicit RangeAlloc(size_t size) { free_[0] = size; }
    bool alloc(size_t bytes, size_t *off)
    {
        for (auto it = free_.begin(); it != free_.end(); ++it) {
            if (it->second < bytes)
                continue;
            *off = it->first;
            const size_t rest = it->second - bytes, at = it->first + bytes;
            free_.erase(it);
            if (rest)
                free_[at] = rest;
            used_ += bytes;
            peak_ = std::max(peak_, used_);
            return true;
        }
        return false;
    }
    void release(size_t off, size_t bytes)
    {
        used_ -= bytes;
        auto it = free_.emplace(off, bytes).first;
        auto next = std::next(it);
        if (next != free_.end() && it->first + it->second == next->first) {
            it->second += next->second;
            free_.erase(next);
        }
        if (it != free_.begin()) {
            auto prev = std::prev(it);
            if (prev->first + prev->second == it->first) {
                prev->second += it->second;
                free_.erase(it);
            }
        }
    }
    size_t used() const { return used_; }
    size_t peak() const { return peak_; }

private:
    size_t used_ = 0, peak_ = 0;
    std::map<size_t, size_t> free_;
};

using Clock = std::chrono::steady_clock;

double seconds_since(Clock::time_point t0) { return std::chrono::duration<double>(Clock::now() - t0).count(); }

struct Req {
    long long id;
    int nx, ny, nz;
    double dx, dt;
    long long steps, remaining;
    unsigned long long seed;
    bool keep, aux, ce_arr, ch_arr, host_fields;
    std::vector<double> eps, mu;    // host copies, dropped at completion
    std::vector<double> fields[6];  // host initial state (FP64 copy); empty for the seeded state
    int state;                      // fdtd_request_state
    double t_submit, t_admit, t_done;
    Plan plan;
    size_t off, bytes;
    bool region_held;
    float *fld[2][6];
    float *ce[3], *ch[3];
    void *staging;
    int cur;
    hipEvent_t done_ev;
    bool ev_live;  // done_ev created and not yet destroyed
    int fetching;  // fdtd_pool_fetch calls reading this request's memory now (release refuses)
};

bool finite_pos(double v) { return std::isfinite(v) && v > 0.0; }

// z-split of one batched launch. A launch ends with its longest workgroup, so
// every request is cut into z-chunks of about the same length (pool_chunk() planes;
// each chunk recomputes 2*tb-1 planes); a launch with fewer than kTargetTiles
// workgroups halves the length once to fill more CUs. The split never changes
// a request's bits.
constexpr int kChunkDefault = 64;
constexpr int kTargetTiles = 512;

// FDTD_POOL_CHUNK overrides the chunk length (planes, 8..4096; read once).
int pool_chunk()
{
    static const int v = [] {
        const char *e = getenv("FDTD_POOL_CHUNK");
        const int c = (e && *e) ? atoi(e) : kChunkDefault;
        return c < 8 ? 8 : (c > 4096 ? 4096 : c);
    }();
    return v;
}

int zsplit(const Geom &g, int len)
{
    const int zc = (g.nz + len / 2) / len;
    return zc < 1 ? 1 : zc;
}

bool request_aux(const fdtd_request &r) { return r.eps_r || r.mu_r || r.fields || r.keep; }

Plan request_plan(const fdtd_request &r)
{
    return fdtd::make_plan(r.nx, r.ny, r.nz, 4, r.eps_r != nullptr, r.mu_r != nullptr, request_aux(r));
}

size_t request_bytes(const Plan &pl) { return (pl.total + 255) / 256 * 256; }

}  // namespace

struct fdtd_pool {
    uint32_t magic;
    int device, tb, max_active, backfill;
    hipStream_t stream, fetch_stream;
    bool own_stream;
    char *arena, *base;
    bool own_arena;
    size_t budget;
    std::unique_ptr<RangeAlloc> alloc;
    BatchEntry *host_tab[kRing];
    BatchEntry *dev_tab[kRing];
    unsigned *dev_queue;  // tile-queue counters of the batched sweeps (zero between launches)
    hipEvent_t ring_ev[kRing];
    bool ring_busy[kRing];
    int ring_next;
    Clock::time_point t0;

    std::mutex mu;
    std::condition_variable cv_loop, cv_done;
    std::vector<std::unique_ptr<Req>> reqs;  // by id; Req objects never move
    std::deque<Req *> queue;
    std::vector<Req *> active;     // admitted, sweeps left to enqueue
    std::vector<Req *> finishing;  // all sweeps enqueued, completion not yet observed
    long long epoch, seen_epoch;   // bumped by submit / release / stop
    bool stop, failed;
    std::string fail_msg;
    std::thread loop;

    long long launches, request_sweeps, completed;
    double cell_updates;
    int peak_active;
};

namespace {

int pcheck(fdtd_pool_t p)
{
    std::lock_guard<std::mutex> lk(g_pools_mu);
    if (!p || !g_pools.count(p) || p->magic != kPoolMagic)
        return pfail(FDTD_E_STATE, "invalid or destroyed pool handle");
    return FDTD_OK;
}

// Record a device failure: every unfinished request fails and waiters wake.
void fail_pool(fdtd_pool_t p, const char *what, hipError_t e)
{
    std::lock_guard<std::mutex> lk(p->mu);
    if (!p->failed) {
        p->failed = true;
        p->fail_msg = std::string(what) + ": " + hipGetErrorString(e);
    }
    for (auto &r : p->reqs)
        if (r->state == FDTD_REQ_QUEUED || r->state == FDTD_REQ_ACTIVE)
            r->state = FDTD_REQ_FAILED;
    p->queue.clear();
    p->active.clear();
    p->finishing.clear();
    p->cv_done.notify_all();
}

// Enqueue the initial state of an admitted request on the compute stream.
hipError_t init_request(fdtd_pool_t p, Req &r)
{
    const Geom &g = r.plan.g;
    hipError_t e = hipMemsetAsync(p->base + r.off, 0, r.plan.total, p->stream);
    for (int which = 0; which < 2 && e == hipSuccess; ++which) {
        const std::vector<double> &m = which == 0 ? r.eps : r.mu;
        if (m.empty())
            continue;
        e = hipMemcpyAsync(r.staging, m.data(), m.size() * sizeof(double), hipMemcpyHostToDevice, p->stream);
        if (e != hipSuccess)
            break;
        float *ce[3] = {nullptr, nullptr, nullptr}, *ch[3] = {nullptr, nullptr, nullptr};
        for (int f = 0; f < 3; ++f) (which == 0 ? ce : ch)[f] = which == 0 ? r.ce[f] : r.ch[f];
        e = fdtd::launch_coef<float>(g, r.dx, r.dt, which == 0 ? (const double *)r.staging : nullptr,
                                     which == 1 ? (const double *)r.staging : nullptr, ce, ch, p->stream);
    }
    if (e != hipSuccess)
        return e;
    if (r.host_fields) {
        for (int f = 0; f < 6 && e == hipSuccess; ++f) {
            e = hipMemcpyAsync(r.staging, r.fields[f].data(), r.fields[f].size() * sizeof(double),
                               hipMemcpyHostToDevice, p->stream);
            if (e == hipSuccess)
                e = fdtd::launch_pack<double, float>(g, f, (const double *)r.staging, r.fld[0][f], r.fld[1][f],
                                                     p->stream);
        }
        return e;
    }
    return fdtd::launch_init_random<float>(g, r.seed, r.fld[0], r.fld[1], p->stream);
}

// Admit queued requests that fit. Returns false after a device failure.
bool admit(fdtd_pool_t p)
{
    std::vector<Req *> admitted;
    {
        std::lock_guard<std::mutex> lk(p->mu);
        p->seen_epoch = p->epoch;
        for (auto it = p->queue.begin(); it != p->queue.end();) {
            if ((int)p->active.size() >= p->max_active)
                break;
            Req &r = **it;
            size_t off;
            if (!p->alloc->alloc(r.bytes, &off)) {
                if (!p->backfill)
                    break;  // FIFO: nobody passes the head of the queue
                ++it;
                continue;
            }
            r.off = off;
            r.region_held = true;
            r.state = FDTD_REQ_ACTIVE;
            r.t_admit = seconds_since(p->t0);
            admitted.push_back(&r);
            it = p->queue.erase(it);
            // listed as active in the same critical section that takes it off the queue, so a
            // waiter never sees it in neither list; only this thread launches, after the init below
            p->active.push_back(&r);
        }
        p->peak_active = std::max(p->peak_active, (int)p->active.size());
    }
    for (Req *rp : admitted) {
        Req &r = *rp;
        char *b = p->base + r.off;
        const size_t guard = (size_t)fdtd::kGuardElems * sizeof(float);
        for (int s = 0; s < 2; ++s)
            for (int f = 0; f < 6; ++f) r.fld[s][f] = (float *)(b + r.plan.off_fields[s][f] + guard);
        for (int f = 0; f < 3; ++f) {
            r.ce[f] = r.ce_arr ? (float *)(b + r.plan.off_ce[f] + guard) : nullptr;
            r.ch[f] = r.ch_arr ? (float *)(b + r.plan.off_ch[f] + guard) : nullptr;
        }
        r.staging = r.aux ? (void *)(b + r.plan.off_staging) : nullptr;
        r.cur = 0;
        hipError_t e = init_request(p, r);
        if (e == hipSuccess) {
            e = hipEventCreateWithFlags(&r.done_ev, hipEventDisableTiming);
            r.ev_live = e == hipSuccess;
        }
        if (e != hipSuccess) {
            fail_pool(p, "admission", e);
            return false;
        }
    }
    return true;
}

// Mark requests whose completion event has fired. Returns false after a device failure.
bool poll_done(fdtd_pool_t p)
{
    std::vector<Req *> fin;
    {
        std::lock_guard<std::mutex> lk(p->mu);
        fin = p->finishing;
    }
    std::vector<Req *> done;
    for (Req *r : fin) {
        hipError_t e = hipEventQuery(r->done_ev);
        if (e == hipSuccess)
            done.push_back(r);
        else if (e != hipErrorNotReady) {
            fail_pool(p, "request execution", e);
            return false;
        }
    }
    if (done.empty())
        return true;
    const double t = seconds_since(p->t0);
    std::lock_guard<std::mutex> lk(p->mu);
    for (Req *r : done) {
        (void)hipEventDestroy(r->done_ev);
        r->ev_live = false;
        r->state = FDTD_REQ_DONE;
        r->t_done = t;
        std::vector<double>().swap(r->eps);
        std::vector<double>().swap(r->mu);
        for (auto &v : r->fields) std::vector<double>().swap(v);
        p->completed += 1;
        p->finishing.erase(std::find(p->finishing.begin(), p->finishing.end(), r));
    }
    p->cv_done.notify_all();
    return true;
}

// Wait for the launch in ring slot s. Returns false after a device failure.
bool wait_slot(fdtd_pool_t p, int s)
{
    hipError_t e = hipEventSynchronize(p->ring_ev[s]);
    if (e != hipSuccess) {
        fail_pool(p, "batched sweep", e);
        return false;
    }
    p->ring_busy[s] = false;
    return poll_done(p);
}

// One round: every active request advances by min(tb, remaining) steps, one
// launch per (steps, Ce kind, Ch kind) group.
bool launch_round(fdtd_pool_t p)
{
    std::vector<Req *> act;
    {
        std::lock_guard<std::mutex> lk(p->mu);
        act = p->active;
    }
    std::map<int, std::vector<Req *>> groups;
    std::vector<Req *> last;
    for (Req *r : act) {
        if (r->remaining == 0) {
            last.push_back(r);
            continue;
        }
        // requests with per-node Ch take at most 3 steps per sweep (a fourth stage spills
        // registers there); the steps per sweep never change an FP32 request's bits
        const int ts = (int)std::min<long long>(r->ch_arr ? std::min(p->tb, 3) : p->tb, r->remaining);
        groups[ts * 4 + (r->ce_arr ? 2 : 0) + (r->ch_arr ? 1 : 0)].push_back(r);
    }
    for (auto &kv : groups) {
        const int ts = kv.first / 4;
        const bool cea = (kv.first & 2) != 0, cha = (kv.first & 1) != 0;
        const int slot = p->ring_next;
        if (p->ring_busy[slot] && !wait_slot(p, slot))
            return false;
        p->ring_next = (slot + 1) % kRing;
        BatchEntry *tab = p->host_tab[slot];
        int ntiles = 0, n = 0;
        double cells = 0;
        long long tiles_at_chunk = 0;
        for (Req *r : kv.second) {
            int kc, ntx, nty, nt;
            fdtd::temporal_tiling(r->plan.g, ts, zsplit(r->plan.g, pool_chunk()), &kc, &ntx, &nty, &nt);
            tiles_at_chunk += nt;
        }
        const int len = tiles_at_chunk < kTargetTiles ? pool_chunk() / 2 : pool_chunk();
        for (Req *r : kv.second) {
            BatchEntry &e = tab[n++];
            e.g = r->plan.g;
            for (int f = 0; f < 6; ++f) {
                e.src.f[f] = r->fld[r->cur][f];
                e.dst.f[f] = r->fld[1 - r->cur][f];
            }
            for (int f = 0; f < 3; ++f) {
                e.c.ce[f] = r->ce[f];
                e.c.ch[f] = r->ch[f];
            }
            e.c.ce_s = (float)(r->dt / r->dx);
            e.c.ch_s = (float)(r->dt / r->dx);
            fdtd::temporal_tiling(r->plan.g, ts, zsplit(r->plan.g, len), &e.kchunk, &e.ntx, &e.nty, &e.ntiles);
            e.tile_begin = ntiles;
            ntiles += e.ntiles;
            cells += (double)r->nx * r->ny * r->nz * ts;
        }
        hipError_t e = hipMemcpyAsync(p->dev_tab[slot], tab, (size_t)n * sizeof(BatchEntry), hipMemcpyHostToDevice,
                                      p->stream);
        if (e == hipSuccess)
            e = fdtd::launch_temporal_batch(p->dev_tab[slot], n, ntiles, ts, cea, cha, p->stream, p->dev_queue);
        if (e == hipSuccess)
            e = hipEventRecord(p->ring_ev[slot], p->stream);
        if (e != hipSuccess) {
            fail_pool(p, "batched sweep launch", e);
            return false;
        }
        p->ring_busy[slot] = true;
        std::lock_guard<std::mutex> lk(p->mu);
        p->launches += 1;
        p->request_sweeps += n;
        p->cell_updates += cells;
        for (Req *r : kv.second) {
            r->cur = 1 - r->cur;
            r->remaining -= ts;
            if (r->remaining == 0)
                last.push_back(r);
        }
    }
    // last sweep enqueued: completion event, and the range goes back to the
    // allocator unless the result is kept
    for (Req *r : last) {
        hipError_t e = hipEventRecord(r->done_ev, p->stream);
        if (e != hipSuccess) {
            fail_pool(p, "completion event", e);
            return false;
        }
        std::lock_guard<std::mutex> lk(p->mu);
        p->active.erase(std::find(p->active.begin(), p->active.end(), r));
        p->finishing.push_back(r);
        if (!r->keep) {
            p->alloc->release(r->off, r->bytes);
            r->region_held = false;
        }
    }
    return true;
}

// The oldest busy ring slot, or -1.
int oldest_busy(fdtd_pool_t p)
{
    for (int q = 0; q < kRing; ++q) {
        const int s = (p->ring_next + q) % kRing;
        if (p->ring_busy[s])
            return s;
    }
    return -1;
}

void loop_main(fdtd_pool_t p)
{
    hipError_t e0 = hipSetDevice(p->device);
    if (e0 != hipSuccess) {
        fail_pool(p, "hipSetDevice", e0);
        return;
    }
    for (;;) {
        bool queued, have_work, pending;
        {
            std::lock_guard<std::mutex> lk(p->mu);
            if (p->stop || p->failed)
                return;
            queued = !p->queue.empty();
        }
        if (queued && !admit(p))
            return;
        {
            std::lock_guard<std::mutex> lk(p->mu);
            have_work = !p->active.empty();
            pending = !p->finishing.empty();
        }
        if (have_work) {
            if (!launch_round(p) || !poll_done(p))
                return;
            continue;
        }
        // nothing to launch: let in-flight work finish, observing completions
        const int s = oldest_busy(p);
        if (s >= 0) {
            if (!wait_slot(p, s))
                return;
            continue;
        }
        if (pending) {
            // completion events recorded after the last launch
            hipError_t e = hipStreamSynchronize(p->stream);
            if (e != hipSuccess) {
                fail_pool(p, "request execution", e);
                return;
            }
            if (!poll_done(p))
                return;
            continue;
        }
        // idle: sleep until a submit or release changes what admission could do
        std::unique_lock<std::mutex> lk(p->mu);
        if (p->stop)
            return;
        if (!p->queue.empty() && p->epoch != p->seen_epoch)
            continue;
        const long long seen = p->epoch;
        p->cv_loop.wait_for(lk, std::chrono::milliseconds(50), [&] { return p->stop || p->epoch != seen; });
    }
}

void bump(fdtd_pool_t p)
{
    p->epoch += 1;
    p->cv_loop.notify_all();
}

void free_pool(fdtd_pool_t p)
{
    for (int s = 0; s < kRing; ++s) {
        if (p->ring_ev[s]) (void)hipEventDestroy(p->ring_ev[s]);
        if (p->host_tab[s]) (void)hipHostFree(p->host_tab[s]);
        if (p->dev_tab[s]) (void)hipFree(p->dev_tab[s]);
    }
    if (p->dev_queue) (void)hipFree(p->dev_queue);
    if (p->own_arena && p->arena) (void)hipFree(p->arena);
    if (p->fetch_stream) (void)hipStreamDestroy(p->fetch_stream);
    if (p->own_stream && p->stream) (void)hipStreamDestroy(p->stream);
}

template <typename S>
hipError_t fetch_fields(fdtd_pool_t p, Req &r, void *const host[6])
{
    for (int f = 0; f < 6; ++f) {
        int X, Y, Z;
        fdtd::extents(r.plan.g, f, X, Y, Z);
        const size_t bytes = (size_t)X * Y * Z * sizeof(S);
        hipError_t e = fdtd::launch_unpack<float, S>(r.plan.g, f, r.fld[r.cur][f], (S *)r.staging, p->fetch_stream);
        if (e == hipSuccess)
            e = hipMemcpyAsync(host[f], r.staging, bytes, hipMemcpyDeviceToHost, p->fetch_stream);
        if (e == hipSuccess)
            e = hipStreamSynchronize(p->fetch_stream);
        if (e != hipSuccess)
            return e;
    }
    return hipSuccess;
}

Req *find_req(fdtd_pool_t p, long long id)
{
    if (id < 0 || id >= (long long)p->reqs.size())
        return nullptr;
    return p->reqs[id].get();
}

}  // namespace

extern "C" {

int fdtd_pool_opts_default(fdtd_pool_opts *o)
{
    if (!o)
        return pfail(FDTD_E_ARG, "NULL opts");
    memset(o, 0, sizeof *o);
    o->tb_steps = 4;
    o->max_active = 256;
    return FDTD_OK;
}

int fdtd_pool_request_bytes(const fdtd_request *r, size_t *out)
{
    if (!r || !out)
        return pfail(FDTD_E_ARG, "NULL argument");
    if (r->nx < 2 || r->ny < 2 || r->nz < 2)
        return pfail(FDTD_E_ARG, "dims must be >= 2 (got %d %d %d)", r->nx, r->ny, r->nz);
    *out = request_bytes(request_plan(*r));
    return FDTD_OK;
}

int fdtd_pool_create(const fdtd_pool_opts *opts, fdtd_pool_t *out)
{
    if (!opts || !out)
        return pfail(FDTD_E_ARG, "NULL argument");
    if (opts->hbm_budget < (1u << 20) && !opts->arena)
        return pfail(FDTD_E_ARG, "hbm_budget must be >= 1 MiB (got %zu)", opts->hbm_budget);
    if (opts->arena && opts->hbm_budget == 0)
        return pfail(FDTD_E_ARG, "arena given with hbm_budget = 0");
    const int tb = opts->tb_steps ? opts->tb_steps : 4;
    if (tb < 1 || tb > 4)
        return pfail(FDTD_E_ARG, "tb_steps must be 1..4 (0: 4), got %d", opts->tb_steps);
    const int max_active = opts->max_active ? opts->max_active : 256;
    if (max_active < 1 || max_active > 65536)
        return pfail(FDTD_E_ARG, "max_active must be 1..65536, got %d", opts->max_active);
    hipError_t e = hipSetDevice(opts->device);
    if (e != hipSuccess)
        return pfail(FDTD_E_DEVICE, "hipSetDevice(%d): %s", opts->device, hipGetErrorString(e));

    fdtd_pool *p = new fdtd_pool();
    p->magic = kPoolMagic;
    p->device = opts->device;
    p->tb = tb;
    p->max_active = max_active;
    p->backfill = opts->backfill != 0;
    p->budget = opts->hbm_budget / 256 * 256;
    p->t0 = Clock::now();
    auto bail = [&](int st, const char *what, hipError_t err) {
        free_pool(p);
        delete p;
        return pfail(st, "%s: %s", what, hipGetErrorString(err));
    };
    if (opts->stream) {
        p->stream = (hipStream_t)opts->stream;
    } else {
        if ((e = hipStreamCreateWithFlags(&p->stream, hipStreamNonBlocking)) != hipSuccess)
            return bail(FDTD_E_DEVICE, "hipStreamCreate", e);
        p->own_stream = true;
    }
    if ((e = hipStreamCreateWithFlags(&p->fetch_stream, hipStreamNonBlocking)) != hipSuccess)
        return bail(FDTD_E_DEVICE, "hipStreamCreate", e);
    if (opts->arena) {
        p->arena = (char *)opts->arena;
        p->base = (char *)(((uintptr_t)p->arena + 255) / 256 * 256);
        const size_t lost = (size_t)(p->base - p->arena);
        p->budget = opts->hbm_budget > lost ? (opts->hbm_budget - lost) / 256 * 256 : 0;
    } else {
        void *mem = nullptr;
        if ((e = hipMalloc(&mem, p->budget)) != hipSuccess) {
            (void)hipGetLastError();
            return bail(FDTD_E_NOMEM, "hipMalloc(hbm_budget)", e);
        }
        p->arena = p->base = (char *)mem;
        p->own_arena = true;
    }
    p->alloc.reset(new RangeAlloc(p->budget));
    for (int s = 0; s < kRing; ++s) {
        const size_t tb_bytes = (size_t)max_active * sizeof(BatchEntry);
        if ((e = hipHostMalloc((void **)&p->host_tab[s], tb_bytes, hipHostMallocDefault)) != hipSuccess ||
            (e = hipMalloc((void **)&p->dev_tab[s], tb_bytes)) != hipSuccess ||
            (e = hipEventCreateWithFlags(&p->ring_ev[s], hipEventDisableTiming)) != hipSuccess)
            return bail(FDTD_E_NOMEM, "request tables", e);
    }
    if ((e = hipMalloc((void **)&p->dev_queue, 256)) != hipSuccess ||
        (e = hipMemsetAsync(p->dev_queue, 0, 256, p->stream)) != hipSuccess)
        return bail(FDTD_E_NOMEM, "tile queue", e);
    {
        std::lock_guard<std::mutex> lk(g_pools_mu);
        g_pools.insert(p);
    }
    p->loop = std::thread(loop_main, p);
    *out = p;
    return FDTD_OK;
}

int fdtd_pool_submit(fdtd_pool_t p, const fdtd_request *r, long long *id)
{
    if (int st = pcheck(p))
        return st;
    if (!r || !id)
        return pfail(FDTD_E_ARG, "NULL argument");
    if (r->nx < 2 || r->ny < 2 || r->nz < 2)
        return pfail(FDTD_E_ARG, "dims must be >= 2 (got %d %d %d)", r->nx, r->ny, r->nz);
    if ((long long)r->nx * r->ny * r->nz > (1LL << 31))
        return pfail(FDTD_E_ARG, "request grid too large");
    if (((long long)r->nx + 1 + 63) / 64 * 64 * (r->ny + 1) * 4 >= (1LL << 31))
        return pfail(FDTD_E_ARG, "request x-y plane too large (planes must stay below 2^31 bytes)");
    if (!finite_pos(r->dx) || !finite_pos(r->dt))
        return pfail(FDTD_E_ARG, "dx and dt must be finite and > 0 (got %g, %g)", r->dx, r->dt);
    if (r->steps < 0)
        return pfail(FDTD_E_ARG, "negative step count %lld", r->steps);
    if (r->fields) {
        if (r->fields_dtype != FDTD_F32 && r->fields_dtype != FDTD_F64)
            return pfail(FDTD_E_ARG, "unsupported fields dtype %d", r->fields_dtype);
        for (int f = 0; f < 6; ++f)
            if (!r->fields[f])
                return pfail(FDTD_E_ARG, "NULL pointer for field %d", f);
    }
    std::unique_ptr<Req> q(new Req());
    const size_t ncell = (size_t)r->nx * r->ny * r->nz;
    double mins[2] = {1.0, 1.0};
    for (int which = 0; which < 2; ++which) {
        const double *m = which == 0 ? r->eps_r : r->mu_r;
        if (!m)
            continue;
        double lo = INFINITY;
        for (size_t c = 0; c < ncell; ++c) {
            if (!finite_pos(m[c]))
                return pfail(FDTD_E_ARG, "%s[%zu] = %g is not finite and > 0", which ? "mu_r" : "eps_r", c, m[c]);
            lo = std::min(lo, m[c]);
        }
        mins[which] = lo;
        (which == 0 ? q->eps : q->mu).assign(m, m + ncell);
    }
    const double courant = r->dt * std::sqrt(3.0) / r->dx;
    if (!(courant < std::sqrt(mins[0] * mins[1])))
        return pfail(FDTD_E_CFL, "dt*sqrt(3)/dx = %.17g violates the Courant limit %.17g", courant,
                     std::sqrt(mins[0] * mins[1]));
    q->plan = request_plan(*r);
    q->bytes = request_bytes(q->plan);
    if (q->bytes > p->budget)
        return pfail(FDTD_E_NOMEM, "request needs %zu bytes, more than the pool budget %zu", q->bytes, p->budget);
    if (r->fields) {
        for (int f = 0; f < 6; ++f) {
            int X, Y, Z;
            fdtd::extents(q->plan.g, f, X, Y, Z);
            const size_t n = (size_t)X * Y * Z;
            q->fields[f].resize(n);
            if (r->fields_dtype == FDTD_F64)
                memcpy(q->fields[f].data(), r->fields[f], n * sizeof(double));
            else
                for (size_t c = 0; c < n; ++c) q->fields[f][c] = ((const float *)r->fields[f])[c];
        }
    }
    q->nx = r->nx;
    q->ny = r->ny;
    q->nz = r->nz;
    q->dx = r->dx;
    q->dt = r->dt;
    q->steps = q->remaining = r->steps;
    q->seed = r->seed;
    q->keep = r->keep != 0;
    q->aux = request_aux(*r);
    q->ce_arr = r->eps_r != nullptr;
    q->ch_arr = r->mu_r != nullptr;
    q->host_fields = r->fields != nullptr;
    q->t_admit = q->t_done = -1.0;
    std::lock_guard<std::mutex> lk(p->mu);
    if (p->failed)
        return pfail(FDTD_E_DEVICE, "pool failed: %s", p->fail_msg.c_str());
    q->id = (long long)p->reqs.size();
    q->state = FDTD_REQ_QUEUED;
    q->t_submit = seconds_since(p->t0);
    p->queue.push_back(q.get());
    *id = q->id;
    p->reqs.push_back(std::move(q));
    bump(p);
    return FDTD_OK;
}

int fdtd_pool_wait(fdtd_pool_t p, long long id, double timeout_s)
{
    if (int st = pcheck(p))
        return st;
    std::unique_lock<std::mutex> lk(p->mu);
    Req *r = nullptr;
    if (id >= 0 && !(r = find_req(p, id)))
        return pfail(FDTD_E_ARG, "unknown request id %lld", id);
    auto settled = [&] {
        if (p->failed)
            return true;
        if (r)
            return r->state != FDTD_REQ_QUEUED && r->state != FDTD_REQ_ACTIVE;
        return p->queue.empty() && p->active.empty() && p->finishing.empty();
    };
    if (timeout_s < 0)
        p->cv_done.wait(lk, settled);
    else if (!p->cv_done.wait_for(lk, std::chrono::duration<double>(timeout_s), settled))
        return pfail(FDTD_E_TIMEOUT, "wait timed out after %g s", timeout_s);
    if (p->failed || (r && r->state == FDTD_REQ_FAILED))
        return pfail(FDTD_E_DEVICE, "pool failed: %s", p->fail_msg.c_str());
    return FDTD_OK;
}

int fdtd_pool_info(fdtd_pool_t p, long long id, fdtd_request_info *out)
{
    if (int st = pcheck(p))
        return st;
    if (!out)
        return pfail(FDTD_E_ARG, "NULL out");
    std::lock_guard<std::mutex> lk(p->mu);
    Req *r = find_req(p, id);
    if (!r)
        return pfail(FDTD_E_ARG, "unknown request id %lld", id);
    out->state = r->state;
    out->t_submit = r->t_submit;
    out->t_admit = r->t_admit;
    out->t_done = r->t_done;
    out->steps = r->steps;
    out->bytes = r->bytes;
    return FDTD_OK;
}

int fdtd_pool_fetch(fdtd_pool_t p, long long id, void *const host[6], int host_dtype)
{
    if (int st = pcheck(p))
        return st;
    if (!host)
        return pfail(FDTD_E_ARG, "NULL field array");
    for (int f = 0; f < 6; ++f)
        if (!host[f])
            return pfail(FDTD_E_ARG, "NULL pointer for field %d", f);
    if (host_dtype != FDTD_F32 && host_dtype != FDTD_F64)
        return pfail(FDTD_E_ARG, "unsupported buffer dtype %d", host_dtype);
    Req *r;
    {
        std::lock_guard<std::mutex> lk(p->mu);
        r = find_req(p, id);
        if (!r)
            return pfail(FDTD_E_ARG, "unknown request id %lld", id);
        if (!r->keep)
            return pfail(FDTD_E_STATE, "request %lld was not submitted with keep = 1", id);
        if (r->state != FDTD_REQ_DONE)
            return pfail(FDTD_E_STATE, "request %lld is not done (state %d)", id, r->state);
        // pinned while its memory is read outside the lock: a concurrent release refuses
        r->fetching += 1;
    }
    hipError_t e = hipSetDevice(p->device);
    if (e == hipSuccess)
        e = host_dtype == FDTD_F32 ? fetch_fields<float>(p, *r, host) : fetch_fields<double>(p, *r, host);
    {
        std::lock_guard<std::mutex> lk(p->mu);
        r->fetching -= 1;
    }
    if (e != hipSuccess)
        return pfail(FDTD_E_DEVICE, "fetch: %s", hipGetErrorString(e));
    return FDTD_OK;
}

int fdtd_pool_release(fdtd_pool_t p, long long id)
{
    if (int st = pcheck(p))
        return st;
    std::lock_guard<std::mutex> lk(p->mu);
    Req *r = find_req(p, id);
    if (!r)
        return pfail(FDTD_E_ARG, "unknown request id %lld", id);
    if (r->state == FDTD_REQ_ACTIVE)
        return pfail(FDTD_E_STATE, "request %lld is running", id);
    if (r->fetching > 0)
        return pfail(FDTD_E_STATE, "request %lld is being fetched", id);
    if (r->state == FDTD_REQ_QUEUED)
        p->queue.erase(std::find(p->queue.begin(), p->queue.end(), r));
    if (r->region_held) {
        p->alloc->release(r->off, r->bytes);
        r->region_held = false;
    }
    if (r->state != FDTD_REQ_FAILED)
        r->state = FDTD_REQ_RELEASED;
    std::vector<double>().swap(r->eps);
    std::vector<double>().swap(r->mu);
    for (auto &v : r->fields) std::vector<double>().swap(v);
    bump(p);
    p->cv_done.notify_all();
    return FDTD_OK;
}

int fdtd_pool_stats(fdtd_pool_t p, fdtd_pool_counters *out)
{
    if (int st = pcheck(p))
        return st;
    if (!out)
        return pfail(FDTD_E_ARG, "NULL out");
    std::lock_guard<std::mutex> lk(p->mu);
    out->submitted = (long long)p->reqs.size();
    out->completed = p->completed;
    out->queued = (long long)p->queue.size();
    out->active = (long long)(p->active.size() + p->finishing.size());
    out->launches = p->launches;
    out->request_sweeps = p->request_sweeps;
    out->cell_updates = p->cell_updates;
    out->bytes_used = p->alloc->used();
    out->bytes_peak = p->alloc->peak();
    out->budget = p->budget;
    out->peak_active = p->peak_active;
    out->failed = p->failed;
    return FDTD_OK;
}

int fdtd_pool_destroy(fdtd_pool_t p)
{
    {
        std::lock_guard<std::mutex> lk(g_pools_mu);
        if (!p || g_pools.erase(p) == 0)
            return pfail(FDTD_E_STATE, "invalid or destroyed pool handle");
    }
    {
        std::lock_guard<std::mutex> lk(p->mu);
        p->stop = true;
        bump(p);
    }
    p->loop.join();
    (void)hipSetDevice(p->device);
    hipError_t e = hipStreamSynchronize(p->stream);
    for (auto &r : p->reqs)
        if (r->ev_live)
            (void)hipEventDestroy(r->done_ev);
    free_pool(p);
    p->magic = kPoolDead;
    delete p;
    if (e != hipSuccess)
        return pfail(FDTD_E_DEVICE, "destroy: pending work failed: %s", hipGetErrorString(e));
    return FDTD_OK;
}

}  // extern "C"
