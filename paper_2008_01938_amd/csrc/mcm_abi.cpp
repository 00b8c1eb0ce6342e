// C ABI layer: validation, chain upload, path selection, workspace and the
// kernel-level profiler.  Every entry point validates its host arguments
// before making any HIP call, so invalid input never touches the device.
#include <hip/hip_runtime.h>

#include <atomic>
#include <mutex>
#include <new>
#include <string.h>
#include <unordered_map>
#include <vector>

#include "mcm_internal.h"

namespace mcm {

// ------------------------------------------------------------------------
// Validation.
// ------------------------------------------------------------------------
mcm_status check_chain(const int32_t *p, int32_t n, ChainInfo *ci)
{
    if (p == nullptr || n < 1) return MCM_ERR_INVALID_ARG;
    int32_t pmin = INT32_MAX, pmax = 0;
    for (int32_t t = 0; t <= n; ++t) {  // branch-free, so it vectorises
        pmin = p[t] < pmin ? p[t] : pmin;
        pmax = p[t] > pmax ? p[t] : pmax;
    }
    if (pmin < 1) return MCM_ERR_INVALID_ARG;
    unsigned __int128 bound = (unsigned __int128)(uint64_t)pmax * (uint64_t)pmax;
    bound *= (uint64_t)pmax;
    bound *= (uint64_t)(n - 1);
    if (bound >= ((unsigned __int128)1 << 63)) return MCM_ERR_OVERFLOW;
    int32_t bits = 0;
    for (unsigned __int128 v = bound; v; v >>= 1) ++bits;
    if (ci) {
        ci->n = n;
        ci->pmax = pmax;
        ci->cost_bits = bits;
    }
    return MCM_OK;
}

namespace {

// ------------------------------------------------------------------------
// Pinned staging for the host chain: a grow-only pool of pinned buffers,
// each guarded by an event recorded after its upload; a buffer is reused
// once its event has completed.
// ------------------------------------------------------------------------
struct StagingBuf {
    void *host = nullptr;
    size_t bytes = 0;
    hipEvent_t done = nullptr;
    int device = -1;
    bool claimed = false;
};

std::mutex g_stage_mu;
std::vector<StagingBuf *> g_stage;

StagingBuf *stage_acquire(size_t bytes, int device)
{
    std::lock_guard<std::mutex> lk(g_stage_mu);
    for (StagingBuf *b : g_stage) {
        if (b->claimed || b->device != device || b->bytes < bytes) continue;
        if (hipEventQuery(b->done) != hipSuccess) continue;
        b->claimed = true;
        return b;
    }
    size_t cap = 64 * 1024;
    while (cap < bytes) cap <<= 1;
    StagingBuf *b = new (std::nothrow) StagingBuf;
    if (!b) return nullptr;
    if (hipHostMalloc(&b->host, cap, hipHostMallocDefault) != hipSuccess) {
        delete b;
        return nullptr;
    }
    if (hipEventCreateWithFlags(&b->done, hipEventDisableTiming) != hipSuccess) {
        (void)hipHostFree(b->host);
        delete b;
        return nullptr;
    }
    b->bytes = cap;
    b->device = device;
    b->claimed = true;
    g_stage.push_back(b);
    return b;
}

void stage_release(StagingBuf *b)
{
    std::lock_guard<std::mutex> lk(g_stage_mu);
    b->claimed = false;
}

// ------------------------------------------------------------------------
// Stream-ordered workspace: hipMallocAsync from the device's default pool,
// with the pool told to keep freed memory cached.
// ------------------------------------------------------------------------
std::mutex g_pool_mu;
std::unordered_map<int, bool> g_pool_ready;

void pool_setup(int device)
{
    std::lock_guard<std::mutex> lk(g_pool_mu);
    if (g_pool_ready[device]) return;
    hipMemPool_t pool;
    if (hipDeviceGetDefaultMemPool(&pool, device) == hipSuccess) {
        uint64_t thr = UINT64_MAX;
        (void)hipMemPoolSetAttribute(pool, hipMemPoolAttrReleaseThreshold, &thr);
    }
    g_pool_ready[device] = true;
}

// ------------------------------------------------------------------------
// Profiler state.
// ------------------------------------------------------------------------
struct ProfRecord {
    int cls;
    hipEvent_t start, stop;
    double evals;
};
std::atomic<int> g_prof_on{0};
std::mutex g_prof_mu;
std::vector<ProfRecord> g_prof_pending;
double g_prof_ms[KC_COUNT];
int64_t g_prof_launches[KC_COUNT];
double g_prof_evals[KC_COUNT];

void prof_clear_locked()
{
    for (auto &r : g_prof_pending) {
        (void)hipEventDestroy(r.start);
        (void)hipEventDestroy(r.stop);
    }
    g_prof_pending.clear();
    for (int c = 0; c < KC_COUNT; ++c) {
        g_prof_ms[c] = 0.0;
        g_prof_launches[c] = 0;
        g_prof_evals[c] = 0.0;
    }
}

void prof_drain_locked()
{
    for (auto &r : g_prof_pending) {
        float ms = 0.f;
        if (hipEventSynchronize(r.stop) == hipSuccess &&
            hipEventElapsedTime(&ms, r.start, r.stop) == hipSuccess) {
            g_prof_ms[r.cls] += ms;
            g_prof_launches[r.cls] += 1;
            g_prof_evals[r.cls] += r.evals;
        }
        (void)hipEventDestroy(r.start);
        (void)hipEventDestroy(r.stop);
    }
    g_prof_pending.clear();
}

mcm_status upload_chain(const int32_t *p, int32_t n, hipStream_t stream, void **dev_block,
                        DeviceChain *dc)
{
    // Layout: n+1 int32 (padded to 8 bytes), then n+1 doubles.
    const size_t np = (size_t)n + 1;
    const size_t off_d = (np * sizeof(int32_t) + 7) / 8 * 8;
    const size_t bytes = off_d + np * sizeof(double);
    void *dev = nullptr;
    mcm_status st = upload_blob(stream, &dev, bytes, [&](char *h) {
        memcpy(h, p, np * sizeof(int32_t));
        double *hd = (double *)(h + off_d);
        for (size_t t = 0; t < np; ++t) hd[t] = (double)p[t];
    });
    if (st != MCM_OK) return st;
    *dev_block = dev;
    dc->p = (const int32_t *)dev;
    dc->pd = (const double *)((char *)dev + off_d);
    return MCM_OK;
}

}  // namespace

mcm_status upload_to(hipStream_t stream, void *dst, size_t bytes,
                     const std::function<void(char *)> &fill)
{
    int device = 0;
    if (hipGetDevice(&device) != hipSuccess) return MCM_ERR_DEVICE;
    StagingBuf *sb = stage_acquire(bytes, device);
    if (!sb) return MCM_ERR_NO_MEMORY;
    fill((char *)sb->host);
    hipError_t e = hipMemcpyAsync(dst, sb->host, bytes, hipMemcpyHostToDevice, stream);
    if (e == hipSuccess) e = hipEventRecord(sb->done, stream);
    stage_release(sb);
    return e == hipSuccess ? MCM_OK : MCM_ERR_DEVICE;
}

mcm_status upload_blob(hipStream_t stream, void **dev_out, size_t bytes,
                       const std::function<void(char *)> &fill)
{
    int device = 0;
    if (hipGetDevice(&device) != hipSuccess) return MCM_ERR_DEVICE;
    pool_setup(device);
    StagingBuf *sb = stage_acquire(bytes, device);
    if (!sb) return MCM_ERR_NO_MEMORY;
    fill((char *)sb->host);
    void *dev = nullptr;
    if (ws_alloc(&dev, bytes, stream) != hipSuccess) {
        stage_release(sb);
        return MCM_ERR_NO_MEMORY;
    }
    hipError_t e = hipMemcpyAsync(dev, sb->host, bytes, hipMemcpyHostToDevice, stream);
    if (e == hipSuccess) e = hipEventRecord(sb->done, stream);
    stage_release(sb);
    if (e != hipSuccess) {
        ws_free(dev, stream);
        return MCM_ERR_DEVICE;
    }
    *dev_out = dev;
    return MCM_OK;
}

namespace {
// Library aux streams and pooled events, per device.  Streams live until
// the process ends.
std::mutex g_streams_mu;
std::unordered_map<int, hipStream_t> g_aux;
std::unordered_map<int, std::vector<hipEvent_t>> g_event_pool;
std::unordered_map<int, int> g_cus;
}  // namespace

int device_cus()
{
    int device = 0;
    if (hipGetDevice(&device) != hipSuccess) return 0;
    std::lock_guard<std::mutex> lk(g_streams_mu);
    int &n = g_cus[device];
    if (n == 0 && hipDeviceGetAttribute(&n, hipDeviceAttributeMultiprocessorCount, device) !=
                      hipSuccess)
        n = 0;
    return n;
}

mcm_status acquire_streams(int count, StreamSet *out)
{
    int device = 0;
    if (hipGetDevice(&device) != hipSuccess) return MCM_ERR_DEVICE;
    std::lock_guard<std::mutex> lk(g_streams_mu);
    hipStream_t &aux = g_aux[device];
    if (!aux && hipStreamCreateWithFlags(&aux, hipStreamNonBlocking) != hipSuccess) {
        aux = nullptr;
        return MCM_ERR_DEVICE;
    }
    out->aux = aux;
    out->events.clear();
    std::vector<hipEvent_t> &pool = g_event_pool[device];
    while ((int)out->events.size() < count) {
        hipEvent_t e = nullptr;
        if (!pool.empty()) {
            e = pool.back();
            pool.pop_back();
        } else if (hipEventCreateWithFlags(&e, hipEventDisableTiming) != hipSuccess) {
            for (hipEvent_t x : out->events) pool.push_back(x);
            out->events.clear();
            return MCM_ERR_DEVICE;
        }
        out->events.push_back(e);
    }
    return MCM_OK;
}

void release_streams(StreamSet &ss)
{
    int device = 0;
    (void)hipGetDevice(&device);
    std::lock_guard<std::mutex> lk(g_streams_mu);
    std::vector<hipEvent_t> &pool = g_event_pool[device];
    for (hipEvent_t e : ss.events) pool.push_back(e);
    ss.events.clear();
}

hipError_t ws_alloc(void **ptr, size_t bytes, hipStream_t stream)
{
    return hipMallocAsync(ptr, bytes ? bytes : 1, stream);
}

void ws_free(void *ptr, hipStream_t stream)
{
    if (ptr) (void)hipFreeAsync(ptr, stream);
}

ProfileScope::ProfileScope(int cls, hipStream_t stream, double evals)
    : cls_(cls), stream_(stream), evals_(evals)
{
    if (!g_prof_on.load(std::memory_order_relaxed)) return;
    if (hipEventCreate(&start_) != hipSuccess) {
        start_ = nullptr;
        return;
    }
    if (hipEventRecord(start_, stream_) != hipSuccess) {
        (void)hipEventDestroy(start_);
        start_ = nullptr;
    }
}

ProfileScope::~ProfileScope()
{
    if (!start_) return;
    hipEvent_t stop = nullptr;
    if (hipEventCreate(&stop) != hipSuccess || hipEventRecord(stop, stream_) != hipSuccess) {
        if (stop) (void)hipEventDestroy(stop);
        (void)hipEventDestroy(start_);
        return;
    }
    std::lock_guard<std::mutex> lk(g_prof_mu);
    g_prof_pending.push_back({cls_, start_, stop, evals_});
}

}  // namespace mcm

using namespace mcm;

extern "C" {

const char *mcm_status_string(int32_t status)
{
    switch (status) {
    case MCM_OK: return "ok";
    case MCM_ERR_INVALID_ARG: return "invalid argument";
    case MCM_ERR_OVERFLOW: return "costs may overflow int64: (n-1)*max(p)^3 >= 2^63";
    case MCM_ERR_NO_MEMORY: return "out of memory";
    case MCM_ERR_DEVICE: return "HIP device error";
    case MCM_ERR_UNSUPPORTED: return "the requested kernel path does not accept this input";
    default: return "unknown status";
    }
}

int32_t mcm_version(void) { return 100; }

mcm_status mcm_check_chain(const int32_t *p, int32_t n) { return check_chain(p, n, nullptr); }

int32_t mcm_select_algo(const int32_t *p, int32_t n)
{
    ChainInfo ci;
    mcm_status st = check_chain(p, n, &ci);
    if (st != MCM_OK) return -(int32_t)st;
    return tiled_accepts(ci) ? MCM_ALGO_TILED : MCM_ALGO_WAVEFRONT;
}

}  // extern "C"

namespace {

// Host-side argument checks shared by the solve entry points; no HIP call.
mcm_status check_outputs(const ChainInfo &ci, int64_t *m_out, int32_t *s_out, int32_t *algo)
{
    if (m_out == nullptr || s_out == nullptr) return MCM_ERR_INVALID_ARG;
    if (((uintptr_t)m_out & 7) != 0 || ((uintptr_t)s_out & 3) != 0) return MCM_ERR_INVALID_ARG;
    if (*algo == MCM_ALGO_AUTO) *algo = tiled_accepts(ci) ? MCM_ALGO_TILED : MCM_ALGO_WAVEFRONT;
    if (*algo != MCM_ALGO_WAVEFRONT && *algo != MCM_ALGO_TILED && *algo != MCM_ALGO_PIPELINE)
        return MCM_ERR_INVALID_ARG;
    if (*algo == MCM_ALGO_TILED && !tiled_accepts(ci)) return MCM_ERR_UNSUPPORTED;
    if (*algo == MCM_ALGO_PIPELINE && ci.n > kPipeMaxN) return MCM_ERR_UNSUPPORTED;
    return MCM_OK;
}

mcm_status run_algo(const DeviceChain &dc, const ChainInfo &ci, int32_t algo, int64_t *m_out,
                    int32_t *s_out, hipStream_t stream)
{
    if (algo == MCM_ALGO_TILED) return run_tiled(dc, ci, m_out, s_out, stream);
    if (algo == MCM_ALGO_PIPELINE) return run_pipeline_solve(dc.p, ci.n, m_out, s_out, stream);
    return run_wavefront(dc, ci, m_out, s_out, stream);
}

}  // namespace

struct mcm_chain {
    ChainInfo ci;
    DeviceChain dc;
    void *block = nullptr;
};

extern "C" {

mcm_status mcm_solve_algo(const int32_t *p, int32_t n, int64_t *m_out, int32_t *s_out,
                          int32_t algo, hipStream_t stream)
{
    ChainInfo ci;
    mcm_status st = check_chain(p, n, &ci);
    if (st != MCM_OK) return st;
    st = check_outputs(ci, m_out, s_out, &algo);
    if (st != MCM_OK) return st;

    if (hipGetLastError() != hipSuccess) return MCM_ERR_DEVICE;
    void *chain_block = nullptr;
    DeviceChain dc;
    st = upload_chain(p, n, stream, &chain_block, &dc);
    if (st != MCM_OK) return st;
    st = run_algo(dc, ci, algo, m_out, s_out, stream);
    ws_free(chain_block, stream);
    return st;
}

mcm_status mcm_solve_batched(int32_t count, const int32_t *n, const int64_t *p_off,
                             const int32_t *p_all, const int64_t *tab_off, int64_t *m_all,
                             int32_t *s_all, hipStream_t stream)
{
    if (count < 0) return MCM_ERR_INVALID_ARG;
    if (count == 0) return MCM_OK;
    if (!n || !p_off || !p_all || !tab_off || !m_all || !s_all) return MCM_ERR_INVALID_ARG;
    if (((uintptr_t)m_all & 7) != 0 || ((uintptr_t)s_all & 3) != 0) return MCM_ERR_INVALID_ARG;
    std::vector<ChainInfo> ci((size_t)count);
    int64_t p_len = 0;
    for (int32_t b = 0; b < count; ++b) {
        if (p_off[b] < 0 || tab_off[b] < 0 || n[b] < 1) return MCM_ERR_INVALID_ARG;
        mcm_status st = check_chain(p_all + p_off[b], n[b], &ci[b]);
        if (st != MCM_OK) return st;
        if (p_off[b] + n[b] + 1 > p_len) p_len = p_off[b] + n[b] + 1;
    }
    if (hipGetLastError() != hipSuccess) return MCM_ERR_DEVICE;

    // All dims in one upload of p_len int32 (padded to 8 bytes); their fp64
    // copies are made on the device, after it.
    const size_t np = (size_t)p_len;
    const size_t off_d = (np * sizeof(int32_t) + 7) / 8 * 8;
    void *dev = nullptr;
    mcm_status st = upload_blob(stream, &dev, off_d, [&](char *h) {
        memcpy(h, p_all, np * sizeof(int32_t));
    });
    if (st != MCM_OK) return st;
    double *pd_own = nullptr;
    if (ws_alloc((void **)&pd_own, np * sizeof(double), stream) != hipSuccess) {
        ws_free(dev, stream);
        return MCM_ERR_NO_MEMORY;
    }
    const int32_t *p_dev = (const int32_t *)dev;
    const double *pd_dev = pd_own;
    st = widen_dims(p_dev, pd_own, np, stream);
    if (st != MCM_OK) {
        ws_free(pd_own, stream);
        ws_free(dev, stream);
        return st;
    }

    TiledPlan plan;
    std::vector<int> ids;
    int maxNT = 0;
    for (int32_t b = 0; b < count; ++b) {
        if (!tiled_accepts(ci[b])) continue;
        const int c = plan_add_chain(plan, ci[b], tab_off[b], tab_off[b], p_off[b], p_off[b]);
        ids.push_back(c);
        if (plan.NT[c] > maxNT) maxNT = plan.NT[c];
    }
    (void)maxNT;
    plan_lockstep(plan, ids);
    st = run_tiled_plan(plan, p_dev, pd_dev, m_all, s_all, nullptr, stream);
    for (int32_t b = 0; b < count && st == MCM_OK; ++b) {
        if (tiled_accepts(ci[b])) continue;
        DeviceChain dc;
        dc.p = p_dev + p_off[b];
        dc.pd = pd_dev + p_off[b];
        st = run_wavefront(dc, ci[b], m_all + tab_off[b], s_all + tab_off[b], stream);
    }
    ws_free(pd_own, stream);
    ws_free(dev, stream);
    return st;
}

mcm_status mcm_chain_create(const int32_t *p, int32_t n, hipStream_t stream, mcm_chain **out)
{
    if (out == nullptr) return MCM_ERR_INVALID_ARG;
    *out = nullptr;
    ChainInfo ci;
    mcm_status st = check_chain(p, n, &ci);
    if (st != MCM_OK) return st;
    if (hipGetLastError() != hipSuccess) return MCM_ERR_DEVICE;
    mcm_chain *c = new (std::nothrow) mcm_chain;
    if (!c) return MCM_ERR_NO_MEMORY;
    c->ci = ci;
    st = upload_chain(p, n, stream, &c->block, &c->dc);
    if (st != MCM_OK) {
        delete c;
        return st;
    }
    *out = c;
    return MCM_OK;
}

mcm_status mcm_chain_solve(const mcm_chain *chain, int32_t algo, int64_t *m_out, int32_t *s_out,
                           hipStream_t stream)
{
    if (chain == nullptr) return MCM_ERR_INVALID_ARG;
    mcm_status st = check_outputs(chain->ci, m_out, s_out, &algo);
    if (st != MCM_OK) return st;
    if (hipGetLastError() != hipSuccess) return MCM_ERR_DEVICE;
    return run_algo(chain->dc, chain->ci, algo, m_out, s_out, stream);
}

int32_t mcm_chain_n(const mcm_chain *chain) { return chain ? chain->ci.n : 0; }

void mcm_chain_destroy(mcm_chain *chain, hipStream_t stream)
{
    if (!chain) return;
    ws_free(chain->block, stream);
    delete chain;
}

mcm_status mcm_solve(const int32_t *p, int32_t n, int64_t *m_out, int32_t *s_out,
                     hipStream_t stream)
{
    return mcm_solve_algo(p, n, m_out, s_out, MCM_ALGO_AUTO, stream);
}

void mcm_profile_enable(int32_t on)
{
    std::lock_guard<std::mutex> lk(g_prof_mu);
    prof_clear_locked();
    g_prof_on.store(on ? 1 : 0);
}

mcm_status mcm_profile_read(int32_t kernel_class, double *total_ms, int64_t *launches,
                            double *split_evals)
{
    if (kernel_class < 0 || kernel_class >= KC_COUNT) return MCM_ERR_INVALID_ARG;
    std::lock_guard<std::mutex> lk(g_prof_mu);
    prof_drain_locked();
    if (total_ms) *total_ms = g_prof_ms[kernel_class];
    if (launches) *launches = g_prof_launches[kernel_class];
    if (split_evals) *split_evals = g_prof_evals[kernel_class];
    return MCM_OK;
}

}  // extern "C"
