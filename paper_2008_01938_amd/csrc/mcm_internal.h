// Library-internal declarations shared by the C ABI layer and the kernel
// translation units.  Not part of the public ABI.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <functional>
#include <vector>

#include "../../include/mcm.h"

namespace mcm {

// Kernel classes for the profiler (must match mcm_profile_read's doc).
enum KernelClass { KC_SETUP = 0, KC_BULK = 1, KC_CLOSE = 2, KC_WAVE = 3, KC_BATCH = 4, KC_COUNT = 5 };

// Host-side facts about a chain, computed once per call.
struct ChainInfo {
    int32_t n = 0;
    int32_t pmax = 0;
    // bit length of (n-1) * pmax^3 (the largest possible candidate cost).
    int32_t cost_bits = 0;
};

// Launch bracket for the profiler: records an event pair around the launch
// when profiling is enabled, and accounts the split evaluations.
struct ProfileScope {
    ProfileScope(int cls, hipStream_t stream, double evals);
    ~ProfileScope();
    int cls_;
    hipStream_t stream_;
    double evals_;
    hipEvent_t start_ = nullptr;
};

// True while MCM_PROFILE_SERIAL is set: single-chain tiled solves use the
// serial schedule (one stream, chunking fitted to the whole device).
bool profile_serial();

// Device copies of the chain, in the forms the kernels read.
struct DeviceChain {
    const int32_t *p = nullptr;   // n+1 int32
    const double *pd = nullptr;   // n+1 doubles (exact copies of p)
};

// Host validation of a chain (no device call); fills ci on success.
mcm_status check_chain(const int32_t *p, int32_t n, ChainInfo *ci);
// The facts of any chain of n matrices whose dims are at most pmax.
mcm_status chain_bound(int32_t n, int32_t pmax, ChainInfo *ci);
// True when the ranges [off[b], off[b] + len(b)) of the `count` entries are
// pairwise disjoint (len(b) = n[b]^2 when square, else n[b] - 1); entries
// with an empty range never conflict.  Host only.
bool ranges_disjoint(int32_t count, const int32_t *n, const int64_t *off, bool square);

// Enqueue a copy of `bytes` host bytes, written by `fill` into pinned
// staging memory, to the existing device buffer `dst` on `stream`.
mcm_status upload_to(hipStream_t stream, void *dst, size_t bytes,
                     const std::function<void(char *)> &fill);

// Stream-ordered workspace allocation (hipMallocAsync on the call's stream).
hipError_t ws_alloc(void **ptr, size_t bytes, hipStream_t stream);
void ws_free(void *ptr, hipStream_t stream);

// Allocate `bytes` of stream-ordered device memory and enqueue its upload:
// `fill` writes the contents into pinned staging memory, which is copied to
// the device on `stream`.  The caller frees *dev with ws_free.
mcm_status upload_blob(hipStream_t stream, void **dev, size_t bytes,
                       const std::function<void(char *)> &fill);

// ------------------------------------------------------------------------
// Tiled launches are driven by tables in device memory, so one launch can
// serve many chains, each at its own tile-diagonal.
// ------------------------------------------------------------------------
struct TileChain {      // one chain of a tiled launch
    int64_t m_off;      // element offset of its n*n int64 m table in m_all
    int64_t s_off;      // element offset of its n*n int32 s table in s_all
    int64_t p_off;      // element offset of its p[0] in the int32 dimension array
    int64_t pd_off;     // element offset of its p[0] in the fp64 dimension array
    int32_t n;          // matrices
    int32_t kb;         // fp64 key: bits below the cost (53 - cost bits, <= 20)
    int32_t kbits;      // bits of a split index in packed partial minima
    int32_t pad;
};

struct TileSeg {        // consecutive workgroups of one launch working on one chain
    int64_t part_off;   // element offset of the chain's packed partial minima
    int32_t first;      // first workgroup index of the segment
    int32_t chain;      // index into the TileChain table
    int32_t D;          // tile-diagonal
    int32_t role;       // k_step: SEG_CLOSE or SEG_BULK
    int32_t KS;         // bulk: splits per chunk
    int32_t nch;        // bulk: chunks per tile in this range
    int32_t groups;     // bulk: workgroups per tile (4 chunks each)
    int32_t koff;       // bulk: range start, offset from (I+1)T-1
    int32_t klen;       // bulk: range length
    int32_t slot0;      // bulk: partial slot of the range's first chunk
    int32_t PT;         // partial slots per tile (bulk: stride; closure: count)
    int32_t pad;
};

enum SegRole { SEG_CLOSE = 0, SEG_BULK = 1 };
enum TiledKernel { TK_TRI = 0, TK_BULK = 1, TK_CLOSE = 2 };

struct TiledLaunch {    // one kernel launch of a tiled plan
    int kind;           // TiledKernel
    int seg_begin;      // first TileSeg of the launch in the plan's table
    int nseg;
    int blocks;         // workgroups
    double evals;       // split evaluations the launch performs
    int stream = 0;     // 0: the caller's stream; 1: the library's aux stream
    int wait = -1;      // launch (on another stream) that must finish first
    bool record = false;  // another launch waits for this one
    int fold = -1;      // lone end blocks: aux launch whose token an extra
                        // workgroup of this launch waits for, so that the
                        // closure after it on this stream needs no stream wait
};

// The library's second stream on the current device (non-blocking, default
// priority, created once) and `count` events (timing disabled) from a pool.
struct StreamSet {
    hipStream_t aux = nullptr;
    std::vector<hipEvent_t> events;
};
mcm_status acquire_streams(int count, StreamSet *out);
// Enqueue on the aux stream a write of the next token of the device's aux
// signal word and return the token (0: no signal word on this device; use an
// event instead).  aux_signal_wait enqueues on `stream` a wait until the word
// holds at least `token`.
uint64_t aux_signal_write(hipStream_t aux);
hipError_t aux_signal_wait(hipStream_t stream, uint64_t token);
// The current device's aux signal word (device-readable), or null before
// the first token or on a device without one.
const uint64_t *aux_signal_word();
// Returns the events once every wait on them has been enqueued.
void release_streams(StreamSet &ss);
// Enqueue a pause of about 4 microseconds (one 64-thread workgroup waiting
// on the wall clock) on `stream`: work behind it on that stream reaches the
// CUs after work another stream has just dispatched.
mcm_status launch_delay(hipStream_t stream);
// Compute units of the current device, and resident k_bulk workgroups per CU.
int device_cus();
int bulk_blocks_per_cu();

// Chunking of the bulk range of one tile-diagonal E of a chain: the
// interior chunks fill partial slots [0, int_nch), the end-block chunks
// the slots after them.  For a lone chain the chunk counts are fitted to
// the workgroup slots the launch finds free: the interior runs beside the
// closure of E-1, which holds NT-E+1 CUs; the end blocks run on those CUs
// after it.
struct BulkLayout {
    int32_t int_ks = 0, int_nch = 0;       // interior: splits per chunk, chunks per tile
    int32_t int_len = 0;                   // ... covering the first int_len interior splits
    int32_t int2_ks = 0, int2_nch = 0;     // lone: shorter chunks for the rest, launched after
    int32_t end_ks = 0, end_nch = 0;       // each end block: splits per chunk, chunks
    int32_t n_end_ranges = 0;              // 1 (E == 2) or 2
    int32_t PT = 0;                        // partial slots per tile
    size_t elems = 0;                      // partial-minima elements (uint64) of all tiles
    bool fold = false;  // lone, two streams: the interior is expected to end before
                        // the end blocks, which then fit the whole device and carry
                        // the closure's wait for the interior
};

// pd[t] = p[t] for t < count, on the device.
mcm_status widen_dims(const int32_t *p, double *pd, size_t count, hipStream_t stream);

// ------------------------------------------------------------------------
// Optimal order read back from split tables (k_paren.hip).
// ------------------------------------------------------------------------
struct ParenChain {     // one chain of a read-back launch
    int64_t s_off;      // element offset of its n*n split table in s_all
    int64_t p_off;      // element offset of its p[0] in the dims, -1 for none
    int64_t g_off;      // element offset of its n-1 node entries in lo/hi
    int64_t q_off;      // element offset of its n-1 task slots in the queue
    int32_t n;          // matrices
    int32_t cost_idx;   // its entry in cost_all, -1 for none
};

// Node intervals lo/hi (and the tree cost when cost_all is given) of every
// chain; one workgroup per chain.  queue_all: sum of (n-1) int64 slots.
// counts (one chain only, or null): 2n int32, receives per matrix the number
// of nodes starting there, then the number ending there.
mcm_status run_paren(const ParenChain *chains, int count, int max_n, const int32_t *s_all,
                     const int32_t *p_all, int32_t *lo_all, int32_t *hi_all, int64_t *cost_all,
                     int64_t *queue_all, int32_t *counts, hipStream_t stream);

// Parenthesized text of one chain from its intervals and the counts run_paren
// wrote (text: its exact length plus a NUL).
mcm_status run_paren_text(const int32_t *lo, int n, const int32_t *counts, char *text,
                          hipStream_t stream);

// ------------------------------------------------------------------------
// Simplified DP (k_sdp.hip).
// ------------------------------------------------------------------------
enum { SDP_MIN = 0, SDP_MAX = 1, SDP_ADD = 2 };

struct SdpPlan {
    int32_t n = 0, a1 = 0;        // table size, largest offset
    int32_t B = 0;                // block of elements per far/near launch pair
    const int32_t *a = nullptr;   // device, k offsets descending
    const int2 *chunks = nullptr; // device, (j0, j1) offset chunks of the far kernel
    int32_t nchunks = 0, chunk_max = 0, span_max = 0;
    int32_t nchunks_old = 0;      // the first chunks, every offset >= 2B (see run_sdp)
    const int32_t *near_a = nullptr;     // device, offsets < B ascending
    int32_t kn = 0;
    const int32_t *cnt_le = nullptr;     // device, B prefix counts of near_a
    const uint64_t *seq_mask = nullptr;  // device, 64 masks of offsets < 64
    int32_t *part = nullptr;      // device workspace, n partial folds
};

mcm_status run_sdp(const SdpPlan &plan, int op, int32_t *st, hipStream_t stream);

// Optimal-BST weights for the tiled kernels (device pointers, one chain of
// L = n+1 gaps): W(i, j) = hi[j] - lo[i] (int64 and exact fp64 copies) and
// the gap weights q on the diagonal.
struct ObstWeights {
    const int64_t *hi = nullptr, *lo = nullptr;
    const double *hid = nullptr, *lod = nullptr;
    const int32_t *q = nullptr;
};

// The optimal BST on the tiled kernels: p_zero / pd_zero hold L+1 zeros (no
// product term); split receives the split k of each cell (-1 at and below
// the diagonal).
mcm_status run_tiled_obst(const ChainInfo &ci, const int32_t *p_zero, const double *pd_zero,
                          const ObstWeights &ob, int64_t *e, int32_t *split, hipStream_t stream);

// Optimal binary search tree over L = n+1 gaps (k_interval.hip): q (L
// int32), W(a, b) = hi_w[b] - lo_w[a]; e and root are L x L.
mcm_status run_obst(const int32_t *q, const int64_t *hi_w, const int64_t *lo_w, int32_t L,
                    int64_t *e, int32_t *root, hipStream_t stream);
// Splits (k) to root keys (k + 1) in place; -1 entries stay.
mcm_status run_obst_root(int32_t *root, int32_t L, hipStream_t stream);

// The pipeline of Fig. 8 with stalls (k_pipeline.hip), an ablation: one
// workgroup, n <= 1025.  Device pointers; inv[u] = the element started at
// step u (or -1), elem[x] = i | d << 16, st / sk the linear table.
struct PipePlan {
    const int32_t *inv = nullptr;
    int64_t S = 0, steps = 0;
    const int32_t *elem = nullptr;
    int64_t *st = nullptr;
    int32_t *sk = nullptr;
};
constexpr int32_t kPipeMaxN = 1025;
mcm_status run_pipeline(const PipePlan &plan, const int32_t *p, int32_t n, int64_t *m,
                        int32_t *s, hipStream_t stream);
// Host schedule of the stalled pipeline: sigma-ordered element table (inv),
// element codes, and the step count.
void pipeline_schedule(int32_t n, std::vector<int32_t> &inv, std::vector<int32_t> &elem,
                       int64_t &steps);
mcm_status run_pipeline_solve(const int32_t *p_dev, int32_t n, int64_t *m, int32_t *s,
                              hipStream_t stream);

// Wavefront path (int64, any valid input).
mcm_status run_wavefront(const DeviceChain &dc, const ChainInfo &ci, int64_t *m, int32_t *s,
                         hipStream_t stream);

// Tiled path.  tiled_accepts: the chain fits the fp64-key kernels (exact
// integers carried in fp64); other chains run the int64 tiled kernels.
bool tiled_accepts(const ChainInfo &ci);
mcm_status run_tiled(const DeviceChain &dc, const ChainInfo &ci, int64_t *m, int32_t *s,
                     hipStream_t stream);

// A sequence of tiled launches over several chains.
struct TiledPlan {
    int T = 64;                        // tile edge: 64, or 32 (batches of small chains;
                                       // no optimal-BST weights)
    std::vector<TileChain> chains;
    std::vector<int32_t> NT;           // tiles per side of each chain
    std::vector<TileSeg> segs;
    std::vector<TiledLaunch> launches;
    size_t part_elems = 0;             // partial-minima buffer (uint64) the plan needs
    bool lone = false;                 // one chain: fit bulk chunks to the GPU's slots
    bool serial = false;               // lone: one stream, chunks fitted to the whole device
    bool wide = false;                 // exact int64 kernels (chains beyond the fp64
                                       // keys' range); 64-edge tiles, no weights
    int chunk_target = 0;              // > 0: about this many interior chunks per
                                       // tile-diagonal (bulk_layout_chunks), device-independent
    int cus = 0;                       // lone: compute units of the device
    int slots_per_cu = 0;              // lone: resident k_bulk workgroups per CU
    int pair_min_blocks = 0;           // closures with more workgroups use the paired
                                       // shape; 0: the device's CU count
    int32_t pmax = 0;                  // largest dimension of any chain
    int32_t cost_bits = 0;             // largest cost_bits of any chain
    bool uses_aux = false;             // some launch runs on the aux stream
    int last_main = -1;                // latest launch on the caller's stream
    int last_close = -1;               // latest closure launch
    int last_interior = -1;            // latest interior-bulk launch (aux stream)
};

// One chain's place in an iteration: it advances from tile-diagonal D to
// D+1.  part_cur: offset of the partial minima of D (read by the closure,
// laid out as `cur`); part_next: offset of those of D+1 (written by its
// bulk, laid out as `next`).
struct ChainStep {
    int chain = 0;
    int D = 0;
    int64_t part_cur = 0;
    int64_t part_next = 0;
    BulkLayout cur, next;
};

int32_t tiled_nt(int32_t n, int32_t T = 64);
// Every launch of a lone plan on the caller's stream, in plan order (which
// already follows every dependency).
void plan_make_serial(TiledPlan &plan);
// lone: cus / slots_per_cu describe the device (TiledPlan); else ignored.
// T: tile edge (64 or 32).  serial: the launches run alone on the device
// (every CU free).  wide: the exact int64 kernels (another rate estimate).
BulkLayout bulk_layout(int32_t T, int32_t NT, int32_t E, int32_t kb, bool lone, int cus = 0,
                       int slots_per_cu = 0, bool serial = false, bool wide = false);
// Interior cut into `nch` chunks per tile (clamped to [1, kMaxChunks] and
// to chunks of at least 64 splits), end blocks in chunks of 64 splits.
BulkLayout bulk_layout_chunks(int32_t T, int32_t NT, int32_t E, int32_t kb, int32_t nch);
// Largest partial-minima buffer (uint64) any tile-diagonal of the chain
// needs under bulk_layout_chunks.
size_t bulk_part_max(int32_t T, int32_t NT, int32_t kb);
constexpr int32_t kMaxChunks = 32;
// Add a chain (offsets as in TileChain); returns its index.
int plan_add_chain(TiledPlan &plan, const ChainInfo &ci, int64_t m_off, int64_t s_off,
                   int64_t p_off, int64_t pd_off);
// Append one iteration: each listed chain advances by one tile-diagonal
// (D = 0 runs its diagonal tiles; D >= 1 closes D and computes the bulk of
// D+1).  Launches: diagonal tiles, closure of D, interior bulk of D+1 (aux
// stream, concurrent with the closure), end blocks of D+1.
void plan_add_iteration(TiledPlan &plan, const std::vector<ChainStep> &steps);
// All chains advance together from D = 0 to their last tile-diagonal, with
// partial minima in one plan-owned buffer (plan.part_elems).
void plan_lockstep(TiledPlan &plan, const std::vector<int> &ids);
// Execute a plan on `stream`: p (int32) and pd (fp64) hold every chain's
// dimensions at its p_off / pd_off; m_all / s_all its tables at m_off /
// s_off.  part_ext: base of the partial minima, or NULL for a buffer of
// plan.part_elems allocated here.
mcm_status run_tiled_plan(const TiledPlan &plan, const int32_t *p, const double *pd,
                          int64_t *m_all, int32_t *s_all, uint64_t *part_ext,
                          hipStream_t stream,
                          const ObstWeights *ob = nullptr);
// The device tables of a plan: TileChain records, then (from *seg_offset,
// 256-byte aligned) TileSeg records.  plan_tables_write fills that layout.
size_t plan_tables_bytes(const TiledPlan &plan, size_t *seg_offset);
void plan_tables_write(const TiledPlan &plan, char *dst);
// run_tiled_plan with the plan's tables already on the device.
// pair_min_blocks >= 0 overrides the plan's closure-shape threshold.
// aux_stream: the second stream to use instead of the library's (whose
// signal tokens are then not used either); events_only: cross-stream edges
// as events only (what a stream capture records).
mcm_status exec_tiled_plan(const TiledPlan &plan, const TileChain *chains, const TileSeg *segs,
                           const int32_t *p, const double *pd, int64_t *m_all, int32_t *s_all,
                           uint64_t *part_ext, hipStream_t stream,
                           const ObstWeights *ob = nullptr, int pair_min_blocks = -1,
                           hipStream_t aux_stream = nullptr, bool events_only = false);

// ------------------------------------------------------------------------
// The no-allocation solve (mcm_noalloc.hip): scratch layout of one call, in
// bytes from the fixed array's base (256-byte aligned regions).
// ------------------------------------------------------------------------
struct NoallocLayout {
    size_t p_off = 0;      // int32 dims, n+1
    size_t pd_off = 0;     // fp64 dims, n+1
    size_t tab_off = 0;    // TileChain records, then TileSeg from tab_off + seg_rel
    size_t seg_rel = 0;
    size_t tab_bytes = 0;
    size_t part_off = 0;   // packed partial minima, plan.part_elems uint64
    size_t total = 0;      // bytes of the array the call uses
};
// The serial single-chain plan of the no-allocation solve and its layout:
// bulk chunking fitted to the device (cus, slots_per_cu) if it fits in
// `cap` bytes, else fewer chunks per tile-diagonal until it does.  False if
// even one chunk per tile does not fit.  Host only.
bool noalloc_plan(const ChainInfo &ci, int cus, int slots_per_cu, size_t cap, TiledPlan &plan,
                  NoallocLayout &lay);

}  // namespace mcm
