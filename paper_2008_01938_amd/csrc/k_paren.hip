// Optimal product order read back from a split table.
//
// The paper takes the MCM problem from the textbook formulation it cites in
// Section IV, where the order is recovered from s by recursion: the product
// of matrices i..j splits at k = s[i][j] into i..k and k+1..j.  The tree
// has n-1 internal nodes, one per split k (the node joining matrices k and
// k+1), so the output is, per split k, the node's interval lo[k]..hi[k].
//
// Done as a recursion the walk is n-1 dependent table reads, each a trip to
// HBM.  Here it is cut into spines.  All nodes that share a left end i are
// nested left children of each other, so they are found by walking row i
// of s downwards (x -> s[i][x]); likewise the nodes sharing a right end j
// are found by walking column j upwards (y -> s[y][j] + 1).  A task walks
// one spine: an L task starts at a node and follows left children, each
// right child it passes starting an R task, and an R task the mirror.
// Every internal node is visited once, and the tasks a task starts can run
// at once, so the walk is as deep as the largest number of direction
// changes on a root-to-leaf path, not as deep as the tree.
//
// One workgroup per chain; its waves share a task queue, and a wave goes
// on with the last task its own walk spawned rather than queueing it.  A
// task stages the part of its row or column it will walk into a per-wave
// LDS window with coalesced (row) or gathered (column) loads, and walks it
// 64 positions at a time: each lane holds one position of the sub-window and
// its split, and pointer doubling over the lanes finds the whole stretch of
// the path inside the sub-window in six rounds of lane permutes, instead of
// one dependent step per node.  Every lane on the path then writes its node
// and the spawned tasks are queued, all lanes at once.
//
// For the parenthesized text, the walk also counts per matrix t the nodes
// that start at t (its "(") and end at t (its ")"); a second kernel places
// every character from those counts with a prefix sum.
#include "mcm_internal.h"

namespace mcm {
namespace {

constexpr int kTextBlock = 1024;
constexpr int kSpinLimit = 1 << 22;   // bounded wait for a queue entry

// Queue entries: a task (start node [a, b], direction) packed into 63 bits;
// -1 marks a slot not yet written.
constexpr int kDirL = 0, kDirR = 1;
__device__ __forceinline__ int64_t task_enc(int32_t a, int32_t b, int dir)
{
    return ((int64_t)a << 32) | (int64_t)(uint32_t)b | ((int64_t)dir << 31);
}

__device__ __forceinline__ int64_t load_entry(const int64_t *q)
{
    return __hip_atomic_load(q, __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_WORKGROUP);
}

// The queue loop keeps the whole wave on one path: no branch in it depends
// on the lane.  Counters are read as wave-uniform values, and updates that
// one lane should make are made by every lane with the others adding zero,
// instead of under `if (lane == 0)`.  (A lane-0 branch lets the compiler
// route the other lanes around the slot claim, and the claimed slot, read
// back with a cross-lane read, is then not lane 0's.)
__device__ __forceinline__ int lds_load(int *x)
{
    return __builtin_amdgcn_readfirstlane(
        __hip_atomic_load(x, __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_WORKGROUP));
}

__device__ __forceinline__ int64_t uniform64(int64_t v)
{
    return ((int64_t)__builtin_amdgcn_readfirstlane((int)(v >> 32)) << 32) |
           (uint32_t)__builtin_amdgcn_readfirstlane((int)v);
}

// Adds `v` once for the wave (lane 0's operand; the other lanes add zero)
// and returns the counter's previous value, wave-uniform.
__device__ __forceinline__ int wave_fetch_add(int *x, int v, int lane, int order)
{
    int old = 0;
    if (order == __ATOMIC_RELEASE)
        old = __hip_atomic_fetch_add(x, lane == 0 ? v : 0, __ATOMIC_RELEASE,
                                     __HIP_MEMORY_SCOPE_WORKGROUP);
    else
        old = __hip_atomic_fetch_add(x, lane == 0 ? v : 0, __ATOMIC_RELAXED,
                                     __HIP_MEMORY_SCOPE_WORKGROUP);
    return __builtin_amdgcn_readfirstlane(old);
}

// win[t] = src[t * stride] for t in [0, len), with up to 16 loads per lane
// in flight before the LDS writes.
__device__ __forceinline__ void stage(int *win, const int32_t *__restrict__ src, int64_t stride,
                                      int len, int lane)
{
    for (int t0 = 0; t0 < len; t0 += 64 * 16) {
        int vals[16];
#pragma unroll
        for (int u = 0; u < 16; ++u) {
            const int t = t0 + u * 64 + lane;
            vals[u] = t < len ? src[(int64_t)t * stride] : 0;
        }
#pragma unroll
        for (int u = 0; u < 16; ++u) {
            const int t = t0 + u * 64 + lane;
            if (t < len) win[t] = vals[u];
        }
    }
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

struct WalkOut {
    int32_t *lo, *hi;
    int32_t *opens, *closes;   // per-matrix parenthesis counts, or null
    int64_t *q;         // this chain's queue
    int qcap;           // slots in q
    int *q_tail;        // LDS
    int *err;           // LDS
};

// Emits the nodes a walk visited in one register sub-window and publishes
// the tasks they spawn.  Lane l holds position sbase + l of the walked row
// (L) or column (R) and its split v; bit l of `visited` marks the positions
// on the walk, so the walk itself only sets bits and the per-node work is
// done here, one lane per node.  With `keep`, the task spawned last (the
// deepest) is returned through it instead of being published.
// `fixed` is the node end shared by the walk (a for L, b for R).
__device__ __forceinline__ void flush(uint64_t visited, int v, int sbase, int fixed, int dir,
                                      const WalkOut &O, int lane, int64_t *keep)
{
    if (visited == 0) return;
    const bool on = (visited >> lane) & 1;
    const int pos = sbase + lane;
    if (on) {
        O.lo[v] = dir == kDirL ? fixed : pos;
        O.hi[v] = dir == kDirL ? pos : fixed;
    }
    if (O.opens) {
        // Matrix t gets one "(" per node starting at t and one ")" per node
        // ending at t.  The walk's shared end takes all its nodes in one
        // add; the other ends are distinct lanes.
        const int cnt = __builtin_popcountll(visited);
        int32_t *shared_end = dir == kDirL ? O.opens + fixed : O.closes + fixed;
        int32_t *own_end = dir == kDirL ? O.closes + pos : O.opens + pos;
        atomicAdd(shared_end, lane == 0 ? cnt : 0);
        if (on) atomicAdd(own_end, 1);
    }
    // L: the right child [v+1, pos]; R: the left child [pos, v].
    const bool spawn = on && (dir == kDirL ? v + 1 < pos : pos < v);
    uint64_t S = __ballot(spawn);
    if (keep && S) {
        // The walk runs down a row and up a column: the last spawn is the
        // lowest position of an L walk and the highest of an R walk.
        const int c = dir == kDirL ? __builtin_ctzll(S) : 63 - __builtin_clzll(S);
        const int vc = __builtin_amdgcn_readlane(v, c);
        *keep = dir == kDirL ? task_enc(vc + 1, sbase + c, kDirR)
                             : task_enc(sbase + c, vc, kDirL);
        S &= ~(1ull << c);
    }
    const int cnt = __builtin_popcountll(S);
    if (cnt == 0) return;
    const int base = wave_fetch_add(O.q_tail, cnt, lane, __ATOMIC_RELAXED);
    if (base + cnt > O.qcap) {
        // Cannot happen for a tree (at most n-2 tasks are spawned);
        // guarded so a broken invariant ends in an error, not a fault.
        atomicOr(O.err, 2);
        return;
    }
    if ((S >> lane) & 1) {
        const int rank = __builtin_amdgcn_mbcnt_hi((uint32_t)(S >> 32),
                                                   __builtin_amdgcn_mbcnt_lo((uint32_t)S, 0));
        const int64_t t = dir == kDirL ? task_enc(v + 1, pos, kDirR) : task_enc(pos, v, kDirL);
        __hip_atomic_store(O.q + base + rank, t, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_WORKGROUP);
    }
}

// The path through one register sub-window, found by pointer doubling
// instead of one dependent step at a time.  Lane l's successor on the walk
// is lane `nxt` (or none: `nxt` < 0 when the walk leaves the sub-window or
// ends there); `own` says whether lane l's node is a real node (its table
// entry is a split of its cell).  Six rounds of lane permutes give every
// lane the set of lanes on its path and the path's last lane; the walk
// reads both at its entry lane e.  Returns the visited mask; *last gets
// the final lane.
__device__ __forceinline__ uint64_t path_from(int e, int nxt, bool own, int lane, int *last)
{
    int J = nxt >= 0 ? nxt : lane;       // the last lane points at itself
    uint32_t mlo = own && lane < 32 ? 1u << lane : 0u;
    uint32_t mhi = own && lane >= 32 ? 1u << (lane - 32) : 0u;
#pragma unroll
    for (int r = 0; r < 6; ++r) {        // 2^6 = 64 lanes: any path fits
        const int addr = J << 2;
        const uint32_t olo = (uint32_t)__builtin_amdgcn_ds_bpermute(addr, (int)mlo);
        const uint32_t ohi = (uint32_t)__builtin_amdgcn_ds_bpermute(addr, (int)mhi);
        J = __builtin_amdgcn_ds_bpermute(addr, J);
        mlo |= olo;
        mhi |= ohi;
    }
    *last = __builtin_amdgcn_readlane(J, e);
    return ((uint64_t)(uint32_t)__builtin_amdgcn_readlane((int)mhi, e) << 32) |
           (uint32_t)__builtin_amdgcn_readlane((int)mlo, e);
}

// L task: nodes [a, x] for x = b, s[a][b], ... down to a; row a of s.  The
// row is staged into the LDS window, 64 positions the first time (many
// walks end there), W after that.  Returns the task to run next, or -1.
__device__ int64_t walk_left(const int32_t *__restrict__ s, int64_t n, int a, int b, int *win,
                             int W, const WalkOut &O, int lane)
{
    const int32_t *row = s + (int64_t)a * n;
    int x = b;
    int wlo = x + 1;         // LDS window holds row positions [wlo, x at staging]
    int wn = 64;
    int64_t next = -1;
    while (x > a) {
        if (x < wlo) {
            const int whi = x;
            wlo = max(a + 1, x - wn + 1);
            wn = W;
            stage(win, row + wlo, 1, whi - wlo + 1, lane);
        }
        // Sub-window [sbase, x]: lane l is position sbase + l.
        const int sbase = max(wlo, x - 63);
        const int pos = min(sbase + lane, x);
        const int v = win[pos - wlo];
        const bool own = v >= a && v < pos;
        const int nxt = own && v >= sbase ? v - sbase : -1;
        int c = 0;
        const uint64_t visited = path_from(x - sbase, nxt, own, lane, &c);
        const int vc = __builtin_amdgcn_readlane(v, c);
        const bool bad = (unsigned)(vc - a) >= (unsigned)(sbase + c - a);
        if (bad) atomicOr(O.err, 1);
        x = bad ? a : vc;
        flush(visited, v, sbase, a, kDirL, O, lane, x > a ? nullptr : &next);
    }
    return next;
}

// R task: nodes [y, b] for y = a, s[a][b]+1, ... up to b; column b of s.
__device__ int64_t walk_right(const int32_t *__restrict__ s, int64_t n, int a, int b, int *win,
                              int W, const WalkOut &O, int lane)
{
    int y = a;
    int whi = y - 1;         // LDS window holds column rows [wlo, whi]
    int wlo = y;
    int wn = 64;
    int64_t next = -1;
    while (y < b) {
        if (y > whi) {
            wlo = y;
            whi = min(b - 1, y + wn - 1);
            wn = W;
            stage(win, s + (int64_t)wlo * n + b, n, whi - wlo + 1, lane);
        }
        // Sub-window [y, send]: lane l is row y + l.
        const int sbase = y;
        const int send = min(y + 63, whi);
        const int pos = min(sbase + lane, send);
        const int v = win[pos - wlo];
        const bool own = v >= pos && v < b;
        const int nxt = own && v + 1 <= send ? v + 1 - sbase : -1;
        int c = 0;
        const uint64_t visited = path_from(0, nxt, own, lane, &c);
        const int vc = __builtin_amdgcn_readlane(v, c);
        const bool bad = (unsigned)(vc - (sbase + c)) >= (unsigned)(b - (sbase + c));
        if (bad) atomicOr(O.err, 1);
        y = bad ? b : vc + 1;
        flush(visited, v, sbase, b, kDirR, O, lane, y < b ? nullptr : &next);
    }
    return next;
}

template <int NW>
__global__ __launch_bounds__(NW * 64) void k_paren(const ParenChain *__restrict__ chains,
                                                   const int32_t *__restrict__ s_all,
                                                   const int32_t *__restrict__ p_all,
                                                   int32_t *__restrict__ lo_all,
                                                   int32_t *__restrict__ hi_all,
                                                   int64_t *__restrict__ cost_all,
                                                   int64_t *__restrict__ queue_all,
                                                   int32_t *__restrict__ counts, int W)
{
    extern __shared__ int win_all[];
    __shared__ int q_head, q_tail, q_done, err;
    __shared__ unsigned long long cost_acc;

    const ParenChain c = chains[blockIdx.x];
    const int n = c.n;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    int32_t *lo = lo_all + c.g_off;
    int32_t *hi = hi_all + c.g_off;
    int64_t *q = queue_all + c.q_off;
    const int qcap = n > 1 ? n - 1 : 0;

    for (int g = tid; g < n - 1; g += NW * 64) {
        lo[g] = -1;
        hi[g] = -1;
        q[g] = g == 0 ? task_enc(0, n - 1, kDirL) : -1;
    }
    if (counts)
        for (int t = tid; t < 2 * n; t += NW * 64) counts[t] = 0;
    if (tid == 0) {
        q_head = 0;
        q_tail = n > 1 ? 1 : 0;
        q_done = 0;
        err = 0;
        cost_acc = 0;
    }
    __syncthreads();

    WalkOut O;
    O.lo = lo;
    O.hi = hi;
    O.opens = counts;
    O.closes = counts ? counts + n : nullptr;
    O.q = q;
    O.qcap = qcap;
    O.q_tail = &q_tail;
    O.err = &err;
    const int32_t *s = s_all + c.s_off;
    int *win = win_all + wave * W;

    for (;;) {
        const int slot = wave_fetch_add(&q_head, 1, lane, __ATOMIC_RELAXED);
        // Wait until the slot holds a task, or until no task can come: every
        // task pushed so far has finished (pushes precede the pusher's done
        // count) and the slot lies beyond the last one pushed.
        int64_t e = -1;
        for (int spin = 0;; ++spin) {
            if (slot < qcap) {
                e = load_entry(q + slot);
                e = uniform64(e);
                if (e >= 0) break;
            }
            const int d = lds_load(&q_done);
            const int t = lds_load(&q_tail);
            if (d == t && slot >= t) break;
            if (spin >= kSpinLimit) {
                atomicOr(&err, 4);
                break;
            }
            __builtin_amdgcn_s_sleep(2);
        }
        if (e < 0) break;
        // The task, then the tasks it keeps for itself; its done count comes
        // after all of them, so it follows every push they make.
        do {
            const int a = (int)(e >> 32);
            const int b = (int)(e & 0x7fffffff);
            e = uniform64(((e >> 31) & 1) ? walk_right(s, n, a, b, win, W, O, lane)
                                          : walk_left(s, n, a, b, win, W, O, lane));
        } while (e >= 0);
        wave_fetch_add(&q_done, 1, lane, __ATOMIC_RELEASE);
    }

    __syncthreads();
    // Tree cost from the finished intervals (one pass, all threads).
    if (cost_all == nullptr || c.cost_idx < 0) return;
    if (!err && c.p_off >= 0) {
        const int32_t *p = p_all + c.p_off;
        int64_t csum = 0;
        for (int k = tid; k < n - 1; k += NW * 64)
            csum += (int64_t)p[lo[k]] * p[k + 1] * p[hi[k] + 1];
        for (int off = 32; off > 0; off >>= 1) csum += __shfl_xor(csum, off);
        if (lane == 0 && csum) atomicAdd(&cost_acc, (unsigned long long)csum);
        __syncthreads();
    }
    if (tid == 0) cost_all[c.cost_idx] = err ? -1 : (int64_t)cost_acc;
}

__device__ __forceinline__ int dec_digits(int t)
{
    int d = 1;
    while (t >= 10) {
        t /= 10;
        ++d;
    }
    return d;
}

constexpr int kLongRun = 32;     // runs longer than this are block-written
constexpr int kMaxRuns = 512;

struct Run {
    int64_t pos;
    int len;
    char ch;
};

// Queues a run for the block to write; false when the list is full (the
// caller then writes it itself).
__device__ __forceinline__ bool add_run(Run *runs, int *n_runs, int64_t pos, int len, char ch)
{
    const int i = atomicAdd(n_runs, 1);
    if (i >= kMaxRuns) return false;
    runs[i].pos = pos;
    runs[i].len = len;
    runs[i].ch = ch;
    return true;
}

// Parenthesized text of one chain; one workgroup.  counts: the per-matrix
// "(" and ")" counts the walk kernel wrote (n each).  text: parens_length(n)
// + 1 bytes.  An incomplete tree (a walk stopped at an entry that is not a
// split) gives the empty string.
__global__ __launch_bounds__(kTextBlock) void k_paren_text(const int32_t *__restrict__ lo, int n,
                                                           const int32_t *__restrict__ counts,
                                                           char *__restrict__ text)
{
    __shared__ int bad, n_runs;
    __shared__ int64_t part[kTextBlock];
    __shared__ Run runs[kMaxRuns];
    const int tid = threadIdx.x;
    const int32_t *opens = counts, *closes = counts + n;
    if (tid == 0) {
        bad = 0;
        n_runs = 0;
    }
    __syncthreads();
    for (int k = tid; k < n - 1; k += kTextBlock)
        if (lo[k] < 0) bad = 1;
    __syncthreads();
    if (bad) {
        if (tid == 0) text[0] = 0;
        return;
    }
    // Contiguous matrices per thread; exclusive scan of their text lengths.
    const int per = (n + kTextBlock - 1) / kTextBlock;
    const int t0 = min(n, tid * per), t1 = min(n, t0 + per);
    int64_t mine = 0;
    for (int t = t0; t < t1; ++t) mine += opens[t] + 1 + dec_digits(t) + closes[t];
    part[tid] = mine;
    __syncthreads();
    for (int off = 1; off < kTextBlock; off <<= 1) {
        const int64_t add = tid >= off ? part[tid - off] : 0;
        __syncthreads();
        part[tid] += add;
        __syncthreads();
    }
    // Long runs of one parenthesis (a matrix that starts or ends a long
    // spine) are written by the whole block afterwards, not by one thread.
    int64_t pos = part[tid] - mine;
    for (int t = t0; t < t1; ++t) {
        const int o = opens[t], c = closes[t];
        if (o > kLongRun && add_run(runs, &n_runs, pos, o, '(')) {
            pos += o;
        } else {
            for (int r = o; r > 0; --r) text[pos++] = '(';
        }
        text[pos++] = 'A';
        const int d = dec_digits(t);
        int v = t;
        for (int i = d - 1; i >= 0; --i) {
            text[pos + i] = (char)('0' + v % 10);
            v /= 10;
        }
        pos += d;
        if (c > kLongRun && add_run(runs, &n_runs, pos, c, ')')) {
            pos += c;
        } else {
            for (int r = c; r > 0; --r) text[pos++] = ')';
        }
    }
    if (tid == kTextBlock - 1) text[part[tid]] = 0;
    __syncthreads();
    const int nr = min(n_runs, kMaxRuns);
    for (int i = 0; i < nr; ++i) {
        const Run r = runs[i];
        for (int j = tid; j < r.len; j += kTextBlock) text[r.pos + j] = r.ch;
    }
}

}  // namespace

mcm_status run_paren(const ParenChain *chains, int count, int max_n, const int32_t *s_all,
                     const int32_t *p_all, int32_t *lo_all, int32_t *hi_all, int64_t *cost_all,
                     int64_t *queue_all, int32_t *counts, hipStream_t stream)
{
    if (count <= 0) return MCM_OK;
    const int64_t rup = ((int64_t)max_n + 63) / 64 * 64;
    hipError_t e;
    if (count == 1) {
        // One chain: sixteen waves share its tasks.
        const int W = (int)(rup < 2048 ? rup : 2048);
        const size_t lds = (size_t)16 * W * sizeof(int);
        hipLaunchKernelGGL(k_paren<16>, dim3(1), dim3(16 * 64), lds, stream, chains, s_all,
                           p_all, lo_all, hi_all, cost_all, queue_all, counts, W);
    } else {
        const int W = (int)(rup < 1024 ? rup : 1024);
        const size_t lds = (size_t)4 * W * sizeof(int);
        hipLaunchKernelGGL(k_paren<4>, dim3((unsigned)count), dim3(4 * 64), lds, stream, chains,
                           s_all, p_all, lo_all, hi_all, cost_all, queue_all, nullptr, W);
    }
    e = hipGetLastError();
    return e == hipSuccess ? MCM_OK : MCM_ERR_DEVICE;
}

mcm_status run_paren_text(const int32_t *lo, int n, const int32_t *counts, char *text,
                          hipStream_t stream)
{
    hipLaunchKernelGGL(k_paren_text, dim3(1), dim3(kTextBlock), 0, stream, lo, n, counts, text);
    return hipGetLastError() == hipSuccess ? MCM_OK : MCM_ERR_DEVICE;
}

}  // namespace mcm
