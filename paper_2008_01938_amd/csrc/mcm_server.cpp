// Request server: continuous batching of matrix-chain solves on one device.
//
// Requests queue in arrival order.  A scheduler thread admits them while a
// slot and arena memory are free, then runs iterations: every admitted,
// unfinished request advances by one tile-diagonal, all of them in the same
// three tiled launches (diagonal tiles, bulk, closure), each request at its
// own tile-diagonal.  Up to kMaxInflight iterations are enqueued ahead of
// the device; an event after each iteration marks the requests whose last
// tile-diagonal it held as complete.
#include <hip/hip_runtime.h>

#include <atomic>
#include <chrono>
#include <condition_variable>
#include <deque>
#include <map>
#include <mutex>
#include <new>
#include <string.h>
#include <thread>
#include <unordered_map>
#include <unordered_set>
#include <vector>

#include "mcm_internal.h"

namespace mcm {
namespace {

constexpr int kMaxInflight = 2;
constexpr size_t kAlign = 256;

double now_s()
{
    return std::chrono::duration<double>(std::chrono::steady_clock::now().time_since_epoch())
        .count();
}

size_t align_up(size_t v) { return (v + kAlign - 1) / kAlign * kAlign; }

// First-fit allocator over [0, size) with coalescing of free ranges.
class Arena {
public:
    explicit Arena(size_t size) { free_[0] = size; }
    // Offset of a new block of `bytes` (aligned), or SIZE_MAX if none fits.
    size_t alloc(size_t bytes)
    {
        bytes = align_up(bytes);
        for (auto it = free_.begin(); it != free_.end(); ++it) {
            if (it->second < bytes) continue;
            const size_t off = it->first, left = it->second - bytes;
            free_.erase(it);
            if (left) free_[off + bytes] = left;
            used_ += bytes;
            return off;
        }
        return SIZE_MAX;
    }
    void release(size_t off, size_t bytes)
    {
        bytes = align_up(bytes);
        used_ -= bytes;
        auto it = free_.emplace(off, bytes).first;
        auto nx = std::next(it);
        if (nx != free_.end() && it->first + it->second == nx->first) {
            it->second += nx->second;
            free_.erase(nx);
        }
        if (it != free_.begin()) {
            auto pv = std::prev(it);
            if (pv->first + pv->second == it->first) {
                pv->second += it->second;
                free_.erase(it);
            }
        }
    }
    size_t used() const { return used_; }

private:
    std::map<size_t, size_t> free_;
    size_t used_ = 0;
};

struct Request {
    uint64_t tag = 0;
    ChainInfo ci;
    std::vector<int32_t> p;
    bool tiled = false;
    int NT = 0, D = 0;
    // Arena block: [p int32 | pd fp64 | m int64 | s int32 | partial minima],
    // each aligned.  The partial region holds two tile-diagonals (by parity)
    // of part_half uint64 each.
    size_t off = SIZE_MAX, bytes = 0, p_at = 0, pd_at = 0, m_at = 0, s_at = 0, part_at = 0;
    size_t part_half = 0;
    BulkLayout lay, lay_next;  // bulk layouts of tile-diagonals D and D+1
    int32_t status = MCM_OK;
    double t_submit = 0, t_admit = 0, t_done = 0;
};

void layout(Request &r)
{
    const size_t np = (size_t)r.ci.n + 1, nn = (size_t)r.ci.n * (size_t)r.ci.n;
    r.p_at = 0;
    r.pd_at = align_up(np * sizeof(int32_t));
    r.m_at = r.pd_at + align_up(np * sizeof(double));
    r.s_at = r.m_at + align_up(nn * sizeof(int64_t));
    r.part_at = r.s_at + align_up(nn * sizeof(int32_t));
    r.part_half = 0;
    if (r.tiled) {
        int32_t kb = 53 - r.ci.cost_bits;
        if (kb > 20) kb = 20;
        r.part_half = bulk_part_max(64, r.NT, kb);
    }
    r.bytes = r.part_at + align_up(2 * r.part_half * sizeof(uint64_t));
}

struct Inflight {
    hipEvent_t ev;
    std::vector<Request *> finishing;
};

}  // namespace

struct Server {
    int device = 0;
    hipStream_t stream = nullptr;
    size_t budget = 0;
    int32_t max_slots = 1;
    char *arena_dev = nullptr;
    Arena arena{0};

    std::mutex mu;
    std::condition_variable cv;
    std::deque<Request *> queue;                     // submitted, not admitted
    std::vector<Request *> active;                   // admitted, work left to enqueue
    std::deque<Inflight> inflight;                   // enqueued iterations
    std::deque<Request *> done;                      // complete, not yet polled
    std::unordered_map<uint64_t, Request *> polled;  // polled, not yet released
    std::unordered_set<uint64_t> live;               // tags submitted, not yet released
    int64_t slots_used = 0, completed = 0, iterations = 0;
    bool stop = false;
    std::thread th;

    void loop();
    void admit_locked();
    bool launch_iteration();
    void retire();
};

void Server::admit_locked()
{
    while (!queue.empty() && slots_used < max_slots) {
        Request *r = queue.front();
        const size_t off = arena.alloc(r->bytes);
        if (off == SIZE_MAX) break;  // first-come first-served: wait for memory
        queue.pop_front();
        r->off = off;
        r->t_admit = now_s();
        slots_used += 1;
        active.push_back(r);
    }
}

bool Server::launch_iteration()
{
    std::vector<Request *> batch;
    {
        std::lock_guard<std::mutex> lk(mu);
        admit_locked();
        if (active.empty() || (int)inflight.size() >= kMaxInflight) return false;
        batch = active;
    }
    int32_t *p_i32 = (int32_t *)arena_dev;
    double *p_f64 = (double *)arena_dev;
    int64_t *m_i64 = (int64_t *)arena_dev;
    int32_t *s_i32 = (int32_t *)arena_dev;
    mcm_status st = MCM_OK;
    // Upload the dims of requests starting this iteration.
    for (Request *r : batch) {
        if (r->D != 0 || st != MCM_OK) continue;
        const size_t np = r->p.size();
        st = upload_to(stream, arena_dev + r->off, r->pd_at + np * sizeof(double), [&](char *h) {
            memcpy(h + r->p_at, r->p.data(), np * sizeof(int32_t));
            double *hd = (double *)(h + r->pd_at);
            for (size_t t = 0; t < np; ++t) hd[t] = (double)r->p[t];
        });
    }
    // Interior chunking of this iteration: when the requests' tiles alone do
    // not fill the device's bulk slots, cut each request's interior into more
    // chunks, in proportion to its share of the iteration's interior work.
    const int64_t slots = (int64_t)device_cus() * bulk_blocks_per_cu();
    double work = 0.0;
    int64_t tiles_all = 0;
    for (Request *r : batch) {
        const int E = r->D + 1;
        if (!r->tiled || r->D < 1 || E < 3 || E >= r->NT) continue;
        work += (double)(r->NT - E) * ((E - 3) * 64 + 1);
        tiles_all += r->NT - E;
    }
    TiledPlan plan;
    std::vector<ChainStep> steps;
    for (Request *r : batch) {
        if (!r->tiled) continue;
        ChainStep cs;
        cs.chain = plan_add_chain(plan, r->ci, (int64_t)((r->off + r->m_at) / sizeof(int64_t)),
                                  (int64_t)((r->off + r->s_at) / sizeof(int32_t)),
                                  (int64_t)((r->off + r->p_at) / sizeof(int32_t)),
                                  (int64_t)((r->off + r->pd_at) / sizeof(double)));
        cs.D = r->D;
        const int64_t part0 = (int64_t)((r->off + r->part_at) / sizeof(uint64_t));
        cs.part_cur = part0 + (int64_t)((r->D & 1) * r->part_half);
        cs.part_next = part0 + (int64_t)(((r->D + 1) & 1) * r->part_half);
        const int E = r->D + 1;
        int32_t nch = 1;
        if (tiles_all < slots && work > 0.0 && r->D >= 1 && E >= 3 && E < r->NT) {
            const double tiles = (double)(r->NT - E);
            const double share = (double)slots * tiles * ((E - 3) * 64 + 1) / work;
            nch = (int32_t)((share + tiles - 1.0) / tiles);
        }
        cs.cur = r->lay;
        cs.next = bulk_layout_chunks(64, r->NT, E, plan.chains[cs.chain].kb, nch);
        r->lay_next = cs.next;
        steps.push_back(cs);
    }
    if (st == MCM_OK && !steps.empty()) {
        plan_add_iteration(plan, steps);
        st = run_tiled_plan(plan, p_i32, p_f64, m_i64, s_i32, (uint64_t *)arena_dev, stream);
    }
    for (Request *r : batch) {
        if (r->tiled || st != MCM_OK) continue;
        DeviceChain dc;
        dc.p = p_i32 + (r->off + r->p_at) / sizeof(int32_t);
        dc.pd = p_f64 + (r->off + r->pd_at) / sizeof(double);
        st = run_wavefront(dc, r->ci, m_i64 + (r->off + r->m_at) / sizeof(int64_t),
                           s_i32 + (r->off + r->s_at) / sizeof(int32_t), stream);
    }
    Inflight fl;
    fl.ev = nullptr;
    if (hipEventCreateWithFlags(&fl.ev, hipEventDisableTiming) != hipSuccess ||
        hipEventRecord(fl.ev, stream) != hipSuccess) {
        if (fl.ev) (void)hipEventDestroy(fl.ev);
        fl.ev = nullptr;
        if (st == MCM_OK) st = MCM_ERR_DEVICE;
    }
    std::lock_guard<std::mutex> lk(mu);
    std::vector<Request *> still;
    for (Request *r : batch) {
        bool fin;
        if (st != MCM_OK) {
            r->status = st;
            fin = true;
        } else if (r->tiled) {
            r->D += 1;
            r->lay = r->lay_next;
            fin = r->D >= r->NT;
        } else {
            fin = true;
        }
        if (fin)
            fl.finishing.push_back(r);
        else
            still.push_back(r);
    }
    // Keep requests admitted meanwhile (none: admission happens here only).
    active.swap(still);
    iterations += 1;
    inflight.push_back(std::move(fl));
    return true;
}

void Server::retire()
{
    for (;;) {
        Inflight fl;
        {
            std::lock_guard<std::mutex> lk(mu);
            if (inflight.empty()) return;
            Inflight &front = inflight.front();
            if (front.ev) {
                const hipError_t q = hipEventQuery(front.ev);
                if (q == hipErrorNotReady) return;
                if (q != hipSuccess)
                    for (Request *r : front.finishing) r->status = MCM_ERR_DEVICE;
            }
            fl = std::move(front);
            inflight.pop_front();
            const double t = now_s();
            for (Request *r : fl.finishing) {
                r->t_done = t;
                done.push_back(r);
                completed += 1;
            }
        }
        if (fl.ev) (void)hipEventDestroy(fl.ev);
        cv.notify_all();
    }
}

void Server::loop()
{
    (void)hipSetDevice(device);
    for (;;) {
        {
            std::lock_guard<std::mutex> lk(mu);
            if (stop) break;
        }
        retire();
        if (!launch_iteration()) {
            std::unique_lock<std::mutex> lk(mu);
            if (stop) break;
            cv.wait_for(lk, std::chrono::microseconds(20));
        }
    }
    (void)hipStreamSynchronize(stream);
    retire();
}

}  // namespace mcm

using namespace mcm;

struct mcm_server : Server {};

extern "C" {

double mcm_clock_now(void) { return now_s(); }

mcm_status mcm_server_create(size_t mem_budget, int32_t max_slots, hipStream_t stream,
                             mcm_server **out)
{
    if (out == nullptr || mem_budget == 0 || max_slots < 1) return MCM_ERR_INVALID_ARG;
    *out = nullptr;
    mcm_server *srv = new (std::nothrow) mcm_server;
    if (!srv) return MCM_ERR_NO_MEMORY;
    if (hipGetDevice(&srv->device) != hipSuccess) {
        delete srv;
        return MCM_ERR_DEVICE;
    }
    srv->budget = mem_budget / kAlign * kAlign;
    if (hipMalloc((void **)&srv->arena_dev, srv->budget) != hipSuccess) {
        delete srv;
        return MCM_ERR_NO_MEMORY;
    }
    srv->arena = Arena(srv->budget);
    // Device queries and the library's aux stream are set up here, once, so
    // that the first iterations do not pay for them.
    StreamSet warm;
    if (device_cus() <= 0 || bulk_blocks_per_cu() <= 0 || acquire_streams(0, &warm) != MCM_OK) {
        (void)hipFree(srv->arena_dev);
        delete srv;
        return MCM_ERR_DEVICE;
    }
    release_streams(warm);
    srv->stream = stream;
    srv->max_slots = max_slots;
    srv->th = std::thread([srv] { srv->loop(); });
    *out = srv;
    return MCM_OK;
}

mcm_status mcm_server_submit(mcm_server *srv, const int32_t *p, int32_t n, uint64_t tag)
{
    if (srv == nullptr) return MCM_ERR_INVALID_ARG;
    ChainInfo ci;
    mcm_status st = check_chain(p, n, &ci);
    if (st != MCM_OK) return st;
    Request *r = new (std::nothrow) Request;
    if (!r) return MCM_ERR_NO_MEMORY;
    r->tag = tag;
    r->ci = ci;
    r->p.assign(p, p + n + 1);
    r->tiled = tiled_accepts(ci);
    r->NT = tiled_nt(n);
    layout(*r);
    if (align_up(r->bytes) > srv->budget) {
        delete r;
        return MCM_ERR_NO_MEMORY;
    }
    {
        std::lock_guard<std::mutex> lk(srv->mu);
        // A tag names one request until it is released: a second request
        // under a live tag could never be released on its own.
        if (!srv->live.insert(tag).second) {
            delete r;
            return MCM_ERR_INVALID_ARG;
        }
        r->t_submit = now_s();
        srv->queue.push_back(r);
    }
    srv->cv.notify_all();
    return MCM_OK;
}

mcm_status mcm_server_poll(mcm_server *srv, mcm_request_info *out, int32_t cap, int32_t *count)
{
    if (srv == nullptr || count == nullptr || cap < 0 || (cap > 0 && out == nullptr))
        return MCM_ERR_INVALID_ARG;
    std::lock_guard<std::mutex> lk(srv->mu);
    int32_t k = 0;
    while (k < cap && !srv->done.empty()) {
        Request *r = srv->done.front();
        srv->done.pop_front();
        mcm_request_info &o = out[k++];
        o.tag = r->tag;
        o.n = r->ci.n;
        o.status = r->status;
        o.m = (int64_t *)(srv->arena_dev + r->off + r->m_at);
        o.s = (int32_t *)(srv->arena_dev + r->off + r->s_at);
        o.t_submit = r->t_submit;
        o.t_admit = r->t_admit;
        o.t_done = r->t_done;
        srv->polled[r->tag] = r;
    }
    *count = k;
    return MCM_OK;
}

size_t mcm_server_request_bytes(const int32_t *p, int32_t n)
{
    ChainInfo ci;
    if (check_chain(p, n, &ci) != MCM_OK) return 0;
    Request r;
    r.ci = ci;
    r.tiled = tiled_accepts(ci);
    r.NT = tiled_nt(n);
    layout(r);
    return align_up(r.bytes);
}

mcm_status mcm_server_release(mcm_server *srv, uint64_t tag)
{
    if (srv == nullptr) return MCM_ERR_INVALID_ARG;
    Request *r = nullptr;
    {
        std::lock_guard<std::mutex> lk(srv->mu);
        auto it = srv->polled.find(tag);
        if (it == srv->polled.end()) return MCM_ERR_INVALID_ARG;
        r = it->second;
        srv->polled.erase(it);
        srv->live.erase(tag);
        srv->arena.release(r->off, r->bytes);
        srv->slots_used -= 1;
    }
    delete r;
    srv->cv.notify_all();
    return MCM_OK;
}

mcm_status mcm_server_stats(mcm_server *srv, int64_t *queued, int64_t *active, int64_t *completed,
                            int64_t *iterations, int64_t *bytes_in_use)
{
    if (srv == nullptr) return MCM_ERR_INVALID_ARG;
    std::lock_guard<std::mutex> lk(srv->mu);
    if (queued) *queued = (int64_t)srv->queue.size();
    if (active) *active = srv->slots_used;
    if (completed) *completed = srv->completed;
    if (iterations) *iterations = srv->iterations;
    if (bytes_in_use) *bytes_in_use = (int64_t)srv->arena.used();
    return MCM_OK;
}

void mcm_server_destroy(mcm_server *srv)
{
    if (!srv) return;
    {
        std::lock_guard<std::mutex> lk(srv->mu);
        srv->stop = true;
    }
    srv->cv.notify_all();
    if (srv->th.joinable()) srv->th.join();
    for (Request *r : srv->queue) delete r;
    for (Request *r : srv->active) delete r;
    for (Inflight &fl : srv->inflight) {
        for (Request *r : fl.finishing) delete r;
        if (fl.ev) (void)hipEventDestroy(fl.ev);
    }
    for (Request *r : srv->done) delete r;
    for (auto &kv : srv->polled) delete kv.second;
    (void)hipFree(srv->arena_dev);
    delete srv;
}

}  // extern "C"
