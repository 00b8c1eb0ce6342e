// C ABI layer: validation, chain upload, path selection, workspace and the
// kernel-level profiler.  Every entry point validates its host arguments
// before making any HIP call, so invalid input never touches the device.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <map>
#include <memory>
#include <mutex>
#include <new>
#include <string>
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
    return chain_bound(n, pmax, ci);
}

mcm_status chain_bound(int32_t n, int32_t pmax, ChainInfo *ci)
{
    if (n < 1 || pmax < 1) return MCM_ERR_INVALID_ARG;
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

bool ranges_disjoint(int32_t count, const int32_t *n, const int64_t *off, bool square)
{
    std::vector<std::pair<int64_t, int64_t>> r;
    r.reserve((size_t)count);
    for (int32_t b = 0; b < count; ++b) {
        const int64_t len = square ? (int64_t)n[b] * n[b] : (int64_t)n[b] - 1;
        if (len > 0) r.emplace_back(off[b], off[b] + len);
    }
    std::sort(r.begin(), r.end());
    for (size_t u = 1; u < r.size(); ++u)
        if (r[u].first < r[u - 1].second) return false;
    return true;
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
std::atomic<uint32_t> g_prof_mask{0};  // bit c: kernel class c is timed
std::atomic<bool> g_prof_serial{false};  // MCM_PROFILE_SERIAL
std::mutex g_prof_mu;
std::vector<ProfRecord> g_prof_pending;
std::vector<hipEvent_t> g_prof_free;  // recycled events (creation is a host cost per launch)
double g_prof_ms[KC_COUNT];
int64_t g_prof_launches[KC_COUNT];
double g_prof_evals[KC_COUNT];

hipEvent_t prof_event_take()
{
    {
        std::lock_guard<std::mutex> lk(g_prof_mu);
        if (!g_prof_free.empty()) {
            hipEvent_t e = g_prof_free.back();
            g_prof_free.pop_back();
            return e;
        }
    }
    hipEvent_t e = nullptr;
    return hipEventCreate(&e) == hipSuccess ? e : nullptr;
}

void prof_event_give_locked(hipEvent_t e)
{
    if (e) g_prof_free.push_back(e);
}

void prof_clear_locked()
{
    // Pending events may still be in flight: wait for them before reuse.
    for (auto &r : g_prof_pending) {
        (void)hipEventSynchronize(r.stop);
        prof_event_give_locked(r.start);
        prof_event_give_locked(r.stop);
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
        prof_event_give_locked(r.start);
        prof_event_give_locked(r.stop);
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

// Per-device signal word written only by the aux stream, with increasing
// tokens (the write is enqueued under g_streams_mu, so the aux stream
// executes the writes in token order): a wait for "word >= token" on another
// stream ends once the aux work before that token has finished.
struct AuxSignal {
    uint64_t *word = nullptr;
    uint64_t next = 0;
    bool tried = false, ok = false;
};
std::unordered_map<int, AuxSignal> g_aux_sig;
}  // namespace

uint64_t aux_signal_write(hipStream_t aux)
{
    int device = 0;
    if (hipGetDevice(&device) != hipSuccess) return 0;
    std::lock_guard<std::mutex> lk(g_streams_mu);
    AuxSignal &sig = g_aux_sig[device];
    if (!sig.tried) {
        sig.tried = true;
        int can = 0;
        if (hipDeviceGetAttribute(&can, hipDeviceAttributeCanUseStreamWaitValue, device) ==
                hipSuccess &&
            can &&
            hipExtMallocWithFlags((void **)&sig.word, sizeof(uint64_t), hipMallocSignalMemory) ==
                hipSuccess) {
            // Start from zero before any token is handed out (the allocation
            // is not cleared); kept until the process ends.
            sig.ok = hipStreamWriteValue64(aux, sig.word, 0, 0) == hipSuccess &&
                     hipStreamSynchronize(aux) == hipSuccess;
        }
    }
    if (!sig.ok) return 0;
    const uint64_t token = sig.next + 1;
    if (hipStreamWriteValue64(aux, sig.word, token, 0) != hipSuccess) return 0;
    sig.next = token;
    return token;
}

const uint64_t *aux_signal_word()
{
    int device = 0;
    if (hipGetDevice(&device) != hipSuccess) return nullptr;
    std::lock_guard<std::mutex> lk(g_streams_mu);
    const AuxSignal &sig = g_aux_sig[device];
    return sig.ok ? sig.word : nullptr;
}

hipError_t aux_signal_wait(hipStream_t stream, uint64_t token)
{
    int device = 0;
    hipError_t e = hipGetDevice(&device);
    if (e != hipSuccess) return e;
    uint64_t *word = nullptr;
    {
        std::lock_guard<std::mutex> lk(g_streams_mu);
        word = g_aux_sig[device].word;
    }
    if (!word) return hipErrorInvalidValue;
    return hipStreamWaitValue64(stream, word, token, hipStreamWaitValueGte, ~(uint64_t)0);
}

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

bool profile_serial() { return g_prof_serial.load(std::memory_order_relaxed); }

ProfileScope::ProfileScope(int cls, hipStream_t stream, double evals)
    : cls_(cls), stream_(stream), evals_(evals)
{
    if (!((g_prof_mask.load(std::memory_order_relaxed) >> cls) & 1u)) return;
    // Launches recorded into a graph are not timed.
    hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
    if (hipStreamIsCapturing(stream_, &cs) != hipSuccess || cs != hipStreamCaptureStatusNone)
        return;
    start_ = prof_event_take();
    if (start_ && hipEventRecord(start_, stream_) != hipSuccess) {
        std::lock_guard<std::mutex> lk(g_prof_mu);
        prof_event_give_locked(start_);
        start_ = nullptr;
    }
}

ProfileScope::~ProfileScope()
{
    if (!start_) return;
    hipEvent_t stop = prof_event_take();
    const bool ok = stop && hipEventRecord(stop, stream_) == hipSuccess;
    std::lock_guard<std::mutex> lk(g_prof_mu);
    if (!ok) {
        prof_event_give_locked(stop);
        prof_event_give_locked(start_);
        return;
    }
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
    return MCM_ALGO_TILED;
}

}  // extern "C"

namespace {

// Host-side argument checks shared by the solve entry points; no HIP call.
mcm_status check_outputs(const ChainInfo &ci, int64_t *m_out, int32_t *s_out, int32_t *algo)
{
    if (m_out == nullptr || s_out == nullptr) return MCM_ERR_INVALID_ARG;
    if (((uintptr_t)m_out & 7) != 0 || ((uintptr_t)s_out & 3) != 0) return MCM_ERR_INVALID_ARG;
    if (*algo == MCM_ALGO_AUTO) *algo = MCM_ALGO_TILED;
    if (*algo != MCM_ALGO_WAVEFRONT && *algo != MCM_ALGO_TILED && *algo != MCM_ALGO_PIPELINE)
        return MCM_ERR_INVALID_ARG;
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

// One tile edge's schedule of a batched plan, its tables in device memory.
struct PlanVariant {
    TiledPlan tp;
    void *tables = nullptr;  // device: TileChain records, then TileSeg from seg_off
    size_t seg_off = 0;
};

// A configuration a batched plan can run: tile edge and closure-shape
// threshold (64-edge tiles: launches with more tiles use two per CU).
struct PlanConfig {
    int T = 64;
    int pair_min = 0;  // 0: the device's CU count
};

namespace {

// Largest tiled chain for which a plan also builds the 32-edge schedule.
constexpr int32_t kSmallTileMaxN = 1024;

// Tuning cache: the configuration the last autotune chose for a batch shape
// bucket on a device architecture, used by later plans and one-shot batched
// solves of the same bucket.
std::mutex g_tune_mu;
std::map<std::string, PlanConfig> g_tune;

std::string device_arch(int device)
{
    hipDeviceProp_t prop;
    if (hipGetDeviceProperties(&prop, device) != hipSuccess) return "unknown";
    return prop.gcnArchName;
}

int32_t ceil_log2(int64_t v)
{
    int32_t b = 0;
    while (((int64_t)1 << b) < v) ++b;
    return b;
}

// Bucket of a batch: the architecture, ceil(log2) of its largest tiled
// chain and of its number of tiled chains.
std::string tune_key(int device, int32_t max_n, int64_t count)
{
    return device_arch(device) + "/n" + std::to_string(ceil_log2(max_n)) + "/c" +
           std::to_string(ceil_log2(count));
}

bool tune_lookup(const std::string &key, PlanConfig *out)
{
    std::lock_guard<std::mutex> lk(g_tune_mu);
    auto it = g_tune.find(key);
    if (it == g_tune.end()) return false;
    *out = it->second;
    return true;
}

}  // namespace

struct mcm_plan {
    int32_t count = 0, max_dim = 0;
    int device = -1;
    std::vector<int32_t> n;
    std::vector<int64_t> p_off, tab_off;
    std::vector<ChainInfo> ci;     // per chain, from n and max_dim
    PlanVariant wide;               // chains beyond the fp64 keys' range: int64 kernels
    bool has_wide = false;
    int64_t p_len = 0;              // dims read: p_all[0 .. p_len)
    PlanVariant var[2];             // [0]: 64-edge tiles; [1]: 32-edge tiles (small chains only)
    bool has_var[2] = {false, false};
    PlanConfig cfg;                 // the configuration solves use
    int32_t source = MCM_PLAN_DEFAULT;
    std::string key;                // tuning-cache bucket
    std::vector<PlanConfig> cands;  // configurations the plan can run
    std::vector<float> cand_ms;     // their times in the last autotune (-1: not timed)
    // Graph form (mcm_plan_graph_create): the captured schedule and the
    // device buffers it reads: dims, their fp64 copies, partial minima.
    hipGraph_t graph = nullptr;
    hipGraphExec_t gexec = nullptr;
    hipStream_t gaux = nullptr;     // the captured schedule's second stream
    void *gmem = nullptr;
    int32_t *g_dims = nullptr;
    ~mcm_plan() { release(); }
    void release_graph()
    {
        if (gexec) (void)hipGraphExecDestroy(gexec);
        if (graph) (void)hipGraphDestroy(graph);
        if (gmem) (void)hipFree(gmem);
        if (gaux) (void)hipStreamDestroy(gaux);
        gexec = nullptr;
        graph = nullptr;
        gmem = nullptr;
        gaux = nullptr;
        g_dims = nullptr;
    }
    void release()
    {
        release_graph();
        for (PlanVariant &v : var)
            if (v.tables) (void)hipFree(v.tables);
        if (wide.tables) (void)hipFree(wide.tables);
        for (PlanVariant &v : var) v.tables = nullptr;
        wide.tables = nullptr;
    }
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
    // Overlapping tables would race between concurrent tiles.
    if (!ranges_disjoint(count, n, tab_off, true)) return MCM_ERR_INVALID_ARG;
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

    // The configuration the tuning cache holds for this batch's bucket (see
    // mcm_plan_autotune), else 64-edge tiles.
    int32_t max_n = 1;
    int64_t tiled_count = 0;
    for (int32_t b = 0; b < count; ++b) {
        if (!tiled_accepts(ci[b])) continue;
        max_n = n[b] > max_n ? n[b] : max_n;
        tiled_count += 1;
    }
    PlanConfig cfg;
    int device = 0;
    if (tiled_count > 0 && hipGetDevice(&device) == hipSuccess)
        (void)tune_lookup(tune_key(device, max_n, tiled_count), &cfg);
    if (max_n > kSmallTileMaxN) cfg.T = 64;
    TiledPlan plan;
    plan.T = cfg.T;
    plan.pair_min_blocks = cfg.pair_min;
    std::vector<int> ids;
    for (int32_t b = 0; b < count; ++b) {
        if (!tiled_accepts(ci[b])) continue;
        ids.push_back(plan_add_chain(plan, ci[b], tab_off[b], tab_off[b], p_off[b], p_off[b]));
    }
    plan_lockstep(plan, ids);
    st = run_tiled_plan(plan, p_dev, pd_dev, m_all, s_all, nullptr, stream);
    // Chains beyond the fp64 keys' range: the int64 tiled kernels, after.
    TiledPlan wide;
    wide.wide = true;
    std::vector<int> wids;
    for (int32_t b = 0; b < count; ++b) {
        if (tiled_accepts(ci[b])) continue;
        wids.push_back(plan_add_chain(wide, ci[b], tab_off[b], tab_off[b], p_off[b], p_off[b]));
    }
    if (st == MCM_OK && !wids.empty()) {
        plan_lockstep(wide, wids);
        st = run_tiled_plan(wide, p_dev, pd_dev, m_all, s_all, nullptr, stream);
    }
    ws_free(pd_own, stream);
    ws_free(dev, stream);
    return st;
}

mcm_status mcm_plan_create(int32_t count, const int32_t *n, const int64_t *p_off,
                           const int64_t *tab_off, int32_t max_dim, mcm_plan **out)
{
    if (out == nullptr) return MCM_ERR_INVALID_ARG;
    *out = nullptr;
    if (count < 0 || max_dim < 1) return MCM_ERR_INVALID_ARG;
    if (count > 0 && (!n || !p_off || !tab_off)) return MCM_ERR_INVALID_ARG;
    std::unique_ptr<mcm_plan> pl(new (std::nothrow) mcm_plan);
    if (!pl) return MCM_ERR_NO_MEMORY;
    pl->count = count;
    pl->max_dim = max_dim;
    pl->n.assign(n, n + count);
    pl->p_off.assign(p_off, p_off + count);
    pl->tab_off.assign(tab_off, tab_off + count);
    pl->ci.resize((size_t)count);
    for (int32_t b = 0; b < count; ++b) {
        if (p_off[b] < 0 || tab_off[b] < 0 || n[b] < 1) return MCM_ERR_INVALID_ARG;
        const mcm_status st = chain_bound(n[b], max_dim, &pl->ci[b]);
        if (st != MCM_OK) return st;
        if (p_off[b] + n[b] + 1 > pl->p_len) pl->p_len = p_off[b] + n[b] + 1;
    }
    if (!ranges_disjoint(count, n, tab_off, true)) return MCM_ERR_INVALID_ARG;
    if (hipGetLastError() != hipSuccess) return MCM_ERR_DEVICE;
    if (hipGetDevice(&pl->device) != hipSuccess) return MCM_ERR_DEVICE;
    std::vector<int32_t> tiled, wide_ids;
    int32_t max_n = 1;
    for (int32_t b = 0; b < count; ++b) {
        if (!tiled_accepts(pl->ci[b])) {
            wide_ids.push_back(b);
            continue;
        }
        tiled.push_back(b);
        max_n = n[b] > max_n ? n[b] : max_n;
    }
    pl->has_var[0] = !tiled.empty();
    pl->has_var[1] = !tiled.empty() && max_n <= kSmallTileMaxN;
    for (int v = 0; v < 2; ++v) {
        if (!pl->has_var[v]) continue;
        PlanVariant &pv = pl->var[v];
        pv.tp.T = v == 0 ? 64 : 32;
        std::vector<int> ids;
        for (int32_t b : tiled)
            ids.push_back(plan_add_chain(pv.tp, pl->ci[b], tab_off[b], tab_off[b], p_off[b],
                                         p_off[b]));
        plan_lockstep(pv.tp, ids);
        if (pv.tp.launches.empty()) continue;
        const size_t bytes = plan_tables_bytes(pv.tp, &pv.seg_off);
        std::vector<char> host(bytes);
        plan_tables_write(pv.tp, host.data());
        if (hipMalloc(&pv.tables, bytes) != hipSuccess) {
            pv.tables = nullptr;
            return MCM_ERR_NO_MEMORY;
        }
        if (hipMemcpy(pv.tables, host.data(), bytes, hipMemcpyHostToDevice) != hipSuccess)
            return MCM_ERR_DEVICE;
    }
    if (!wide_ids.empty()) {
        PlanVariant &pv = pl->wide;
        pv.tp.wide = true;
        std::vector<int> ids;
        for (int32_t b : wide_ids)
            ids.push_back(plan_add_chain(pv.tp, pl->ci[b], tab_off[b], tab_off[b], p_off[b],
                                         p_off[b]));
        plan_lockstep(pv.tp, ids);
        const size_t bytes = plan_tables_bytes(pv.tp, &pv.seg_off);
        std::vector<char> host(bytes);
        plan_tables_write(pv.tp, host.data());
        if (hipMalloc(&pv.tables, bytes) != hipSuccess) {
            pv.tables = nullptr;
            return MCM_ERR_NO_MEMORY;
        }
        if (hipMemcpy(pv.tables, host.data(), bytes, hipMemcpyHostToDevice) != hipSuccess)
            return MCM_ERR_DEVICE;
        pl->has_wide = true;
    }
    // Candidates: 64-edge tiles at four closure-shape thresholds, then
    // 32-edge tiles.
    const int cus = device_cus();
    if (pl->has_var[0])
        for (int pm : {cus, cus / 2, 2 * cus, 4 * cus}) pl->cands.push_back(PlanConfig{64, pm});
    if (pl->has_var[1]) pl->cands.push_back(PlanConfig{32, 0});
    pl->cand_ms.assign(pl->cands.size(), -1.0f);
    if (!tiled.empty()) {
        pl->key = tune_key(pl->device, max_n, (int64_t)tiled.size());
        PlanConfig c;
        if (tune_lookup(pl->key, &c) && pl->has_var[c.T == 32 ? 1 : 0]) {
            pl->cfg = c;
            pl->source = MCM_PLAN_CACHED;
        }
    }
    *out = pl.release();
    return MCM_OK;
}

}  // extern "C"

namespace {

// Every dimension a chain of the plan reads must lie in [1, max_dim]: the
// plan's key widths were sized for that bound.
bool plan_dims_ok(const mcm_plan *pl, const int32_t *p_all)
{
    for (int32_t b = 0; b < pl->count; ++b) {
        const int32_t *p = p_all + pl->p_off[b];
        int32_t lo = INT32_MAX, hi = 0;
        for (int32_t t = 0; t <= pl->n[b]; ++t) {
            lo = p[t] < lo ? p[t] : lo;
            hi = p[t] > hi ? p[t] : hi;
        }
        if (lo < 1 || hi > pl->max_dim) return false;
    }
    return true;
}

mcm_status plan_solve(const mcm_plan *pl, const int32_t *p_all, int64_t *m_all, int32_t *s_all,
                      hipStream_t stream, const PlanConfig &cfg)
{
    if (pl == nullptr || p_all == nullptr) return MCM_ERR_INVALID_ARG;
    if (pl->count == 0) return MCM_OK;
    if (!m_all || !s_all) return MCM_ERR_INVALID_ARG;
    if (((uintptr_t)m_all & 7) != 0 || ((uintptr_t)s_all & 3) != 0) return MCM_ERR_INVALID_ARG;
    if (!plan_dims_ok(pl, p_all)) return MCM_ERR_INVALID_ARG;
    int dev = -1;
    if (hipGetLastError() != hipSuccess || hipGetDevice(&dev) != hipSuccess)
        return MCM_ERR_DEVICE;
    if (dev != pl->device) return MCM_ERR_INVALID_ARG;

    const size_t np = (size_t)pl->p_len;
    void *dims = nullptr;
    mcm_status st = upload_blob(stream, &dims, np * sizeof(int32_t),
                                [&](char *h) { memcpy(h, p_all, np * sizeof(int32_t)); });
    if (st != MCM_OK) return st;
    double *pd = nullptr;
    if (ws_alloc((void **)&pd, np * sizeof(double), stream) != hipSuccess) {
        ws_free(dims, stream);
        return MCM_ERR_NO_MEMORY;
    }
    const int32_t *p_dev = (const int32_t *)dims;
    st = widen_dims(p_dev, pd, np, stream);
    const PlanVariant &pv = pl->var[cfg.T == 32 && pl->has_var[1] ? 1 : 0];
    if (st == MCM_OK && pv.tables)
        st = exec_tiled_plan(pv.tp, (const TileChain *)pv.tables,
                             (const TileSeg *)((const char *)pv.tables + pv.seg_off), p_dev, pd,
                             m_all, s_all, nullptr, stream, nullptr, cfg.pair_min);
    if (st == MCM_OK && pl->has_wide && pl->wide.tables)
        st = exec_tiled_plan(pl->wide.tp, (const TileChain *)pl->wide.tables,
                             (const TileSeg *)((const char *)pl->wide.tables + pl->wide.seg_off),
                             p_dev, pd, m_all, s_all, nullptr, stream);
    ws_free(pd, stream);
    ws_free(dims, stream);
    return st;
}

}  // namespace

extern "C" {

mcm_status mcm_plan_solve(const mcm_plan *plan, const int32_t *p_all, int64_t *m_all,
                          int32_t *s_all, hipStream_t stream)
{
    if (plan == nullptr) return MCM_ERR_INVALID_ARG;
    return plan_solve(plan, p_all, m_all, s_all, stream, plan->cfg);
}

mcm_status mcm_plan_autotune(mcm_plan *plan, const int32_t *p_all, int64_t *m_all,
                             int32_t *s_all, hipStream_t stream, int32_t *choice)
{
    if (plan == nullptr) return MCM_ERR_INVALID_ARG;
    if (plan->count == 0 || plan->cands.empty()) {
        if (choice) *choice = -1;
        return MCM_OK;
    }
    // Every candidate runs once untimed, then kTuneReps times, each timed
    // with events on the caller's stream; the fastest run counts.
    constexpr int kTuneReps = 3;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    if (hipEventCreate(&e0) != hipSuccess) return MCM_ERR_DEVICE;
    if (hipEventCreate(&e1) != hipSuccess) {
        (void)hipEventDestroy(e0);
        return MCM_ERR_DEVICE;
    }
    mcm_status st = MCM_OK;
    int best = 0;
    for (size_t c = 0; c < plan->cands.size() && st == MCM_OK; ++c) {
        st = plan_solve(plan, p_all, m_all, s_all, stream, plan->cands[c]);
        float fastest = -1.0f;
        for (int r = 0; r < kTuneReps && st == MCM_OK; ++r) {
            if (hipEventRecord(e0, stream) != hipSuccess) st = MCM_ERR_DEVICE;
            if (st == MCM_OK) st = plan_solve(plan, p_all, m_all, s_all, stream, plan->cands[c]);
            if (st == MCM_OK && hipEventRecord(e1, stream) != hipSuccess) st = MCM_ERR_DEVICE;
            float ms = 0.f;
            if (st == MCM_OK && (hipEventSynchronize(e1) != hipSuccess ||
                                 hipEventElapsedTime(&ms, e0, e1) != hipSuccess))
                st = MCM_ERR_DEVICE;
            if (st == MCM_OK && (fastest < 0.f || ms < fastest)) fastest = ms;
        }
        plan->cand_ms[c] = fastest;
        if (st == MCM_OK && fastest < plan->cand_ms[(size_t)best]) best = (int)c;
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (st != MCM_OK) return st;
    plan->cfg = plan->cands[(size_t)best];
    plan->source = MCM_PLAN_TUNED;
    {
        std::lock_guard<std::mutex> lk(g_tune_mu);
        g_tune[plan->key] = plan->cfg;
    }
    if (choice) *choice = best;
    return MCM_OK;
}

mcm_status mcm_plan_config(const mcm_plan *plan, int32_t *tile_edge, int32_t *pair_min_blocks,
                           int32_t *source)
{
    if (plan == nullptr) return MCM_ERR_INVALID_ARG;
    if (tile_edge) *tile_edge = plan->cfg.T;
    if (pair_min_blocks) *pair_min_blocks = plan->cfg.pair_min > 0 ? plan->cfg.pair_min
                                                                   : device_cus();
    if (source) *source = plan->source;
    return MCM_OK;
}

mcm_status mcm_plan_set_config(mcm_plan *plan, int32_t tile_edge, int32_t pair_min_blocks)
{
    if (plan == nullptr || pair_min_blocks < 0) return MCM_ERR_INVALID_ARG;
    if (tile_edge != 64 && tile_edge != 32) return MCM_ERR_INVALID_ARG;
    if (plan->count > 0 && !plan->has_var[tile_edge == 32 ? 1 : 0] && !plan->cands.empty())
        return MCM_ERR_UNSUPPORTED;
    plan->cfg = PlanConfig{tile_edge, pair_min_blocks};
    plan->source = MCM_PLAN_TUNED;
    if (!plan->key.empty()) {
        std::lock_guard<std::mutex> lk(g_tune_mu);
        g_tune[plan->key] = plan->cfg;
    }
    return MCM_OK;
}

mcm_status mcm_plan_candidates(const mcm_plan *plan, int32_t cap, int32_t *tile_edge,
                               int32_t *pair_min_blocks, float *ms, int32_t *count)
{
    if (plan == nullptr || count == nullptr || cap < 0) return MCM_ERR_INVALID_ARG;
    const int32_t k = (int32_t)plan->cands.size() < cap ? (int32_t)plan->cands.size() : cap;
    for (int32_t c = 0; c < k; ++c) {
        if (tile_edge) tile_edge[c] = plan->cands[(size_t)c].T;
        if (pair_min_blocks) pair_min_blocks[c] = plan->cands[(size_t)c].pair_min;
        if (ms) ms[c] = plan->cand_ms[(size_t)c];
    }
    *count = (int32_t)plan->cands.size();
    return MCM_OK;
}

mcm_status mcm_plan_graph_create(mcm_plan *plan, int64_t *m_all, int32_t *s_all,
                                 hipStream_t stream)
{
    if (plan == nullptr || !m_all || !s_all) return MCM_ERR_INVALID_ARG;
    if (((uintptr_t)m_all & 7) != 0 || ((uintptr_t)s_all & 3) != 0) return MCM_ERR_INVALID_ARG;
    if (stream == nullptr) return MCM_ERR_INVALID_ARG;  // the null stream cannot be captured
    int dev = -1;
    if (hipGetLastError() != hipSuccess || hipGetDevice(&dev) != hipSuccess)
        return MCM_ERR_DEVICE;
    if (dev != plan->device) return MCM_ERR_INVALID_ARG;
    plan->release_graph();
    const PlanVariant &pv = plan->var[plan->cfg.T == 32 && plan->has_var[1] ? 1 : 0];
    // Device buffers the graph reads: dims, fp64 dims, partial minima of the
    // configured schedule and of the int64 one.
    const size_t np = (size_t)(plan->p_len > 0 ? plan->p_len : 1);
    const size_t at_pd = (np * sizeof(int32_t) + 255) / 256 * 256;
    const size_t at_part = at_pd + (np * sizeof(double) + 255) / 256 * 256;
    const size_t part1 = (pv.tables ? pv.tp.part_elems : 0) * sizeof(uint64_t);
    const size_t at_wide = at_part + (part1 + 255) / 256 * 256;
    const size_t part2 = (plan->has_wide ? plan->wide.tp.part_elems : 0) * sizeof(uint64_t);
    if (hipMalloc(&plan->gmem, at_wide + part2 + 256) != hipSuccess) {
        plan->gmem = nullptr;
        return MCM_ERR_NO_MEMORY;
    }
    if (hipStreamCreateWithFlags(&plan->gaux, hipStreamNonBlocking) != hipSuccess) {
        plan->gaux = nullptr;
        plan->release_graph();
        return MCM_ERR_DEVICE;
    }
    char *base = (char *)plan->gmem;
    plan->g_dims = (int32_t *)base;
    double *pd = (double *)(base + at_pd);
    // Warm the library's stream set (events) before capturing.
    StreamSet warm;
    if (acquire_streams(0, &warm) != MCM_OK) {
        plan->release_graph();
        return MCM_ERR_DEVICE;
    }
    release_streams(warm);
    mcm_status st = MCM_OK;
    if (hipStreamBeginCapture(stream, hipStreamCaptureModeThreadLocal) != hipSuccess) {
        plan->release_graph();
        return MCM_ERR_DEVICE;
    }
    st = widen_dims(plan->g_dims, pd, np, stream);
    if (st == MCM_OK && pv.tables)
        st = exec_tiled_plan(pv.tp, (const TileChain *)pv.tables,
                             (const TileSeg *)((const char *)pv.tables + pv.seg_off),
                             plan->g_dims, pd, m_all, s_all, (uint64_t *)(base + at_part), stream,
                             nullptr, plan->cfg.pair_min, plan->gaux, true);
    if (st == MCM_OK && plan->has_wide && plan->wide.tables)
        st = exec_tiled_plan(plan->wide.tp, (const TileChain *)plan->wide.tables,
                             (const TileSeg *)((const char *)plan->wide.tables +
                                               plan->wide.seg_off),
                             plan->g_dims, pd, m_all, s_all, (uint64_t *)(base + at_wide),
                             stream, nullptr, -1, plan->gaux, true);
    hipGraph_t g = nullptr;
    const hipError_t ec = hipStreamEndCapture(stream, &g);
    if (st == MCM_OK && (ec != hipSuccess || g == nullptr)) st = MCM_ERR_DEVICE;
    plan->graph = g;
    if (st == MCM_OK && hipGraphInstantiate(&plan->gexec, g, nullptr, nullptr, 0) != hipSuccess) {
        plan->gexec = nullptr;
        st = MCM_ERR_DEVICE;
    }
    if (st != MCM_OK) plan->release_graph();
    return st;
}

mcm_status mcm_plan_graph_solve(const mcm_plan *plan, const int32_t *p_all, hipStream_t stream)
{
    if (plan == nullptr || p_all == nullptr || plan->gexec == nullptr) return MCM_ERR_INVALID_ARG;
    if (!plan_dims_ok(plan, p_all)) return MCM_ERR_INVALID_ARG;
    if (hipGetLastError() != hipSuccess) return MCM_ERR_DEVICE;
    const size_t np = (size_t)plan->p_len;
    if (np > 0) {
        const mcm_status st = upload_to(stream, plan->g_dims, np * sizeof(int32_t),
                                        [&](char *h) { memcpy(h, p_all, np * sizeof(int32_t)); });
        if (st != MCM_OK) return st;
    }
    return hipGraphLaunch(plan->gexec, stream) == hipSuccess ? MCM_OK : MCM_ERR_DEVICE;
}

void mcm_plan_destroy(mcm_plan *plan)
{
    delete plan;
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

void mcm_profile_enable_mask(uint32_t mask)
{
    std::lock_guard<std::mutex> lk(g_prof_mu);
    prof_clear_locked();
    g_prof_mask.store(mask & ((1u << KC_COUNT) - 1u));
    g_prof_serial.store((mask & MCM_PROFILE_SERIAL) != 0);
}

void mcm_profile_enable(int32_t on)
{
    mcm_profile_enable_mask(on ? (1u << KC_COUNT) - 1u : 0u);
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
