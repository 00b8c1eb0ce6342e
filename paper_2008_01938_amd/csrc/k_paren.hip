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
// One workgroup per chain; its waves share a task queue.  A task stages the
// part of its row or column it will walk into a per-wave LDS window with
// coalesced (row) or gathered (column) loads, then walks it from a 64-entry
// register sub-window with lane reads, one dependent step costing a few
// instructions rather than a memory trip.  Results of up to 64 steps are
// written in one vector store.
//
// A second kernel turns the node intervals into the parenthesized text:
// leaf t carries one "(" per node starting at t and one ")" per node ending
// at t, so per-leaf counts and a prefix sum place every character.
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

// `old` with lane `idx` (uniform) replaced by `val`.
__device__ __forceinline__ int set_lane(int old, int val, int idx, int lane)
{
    return lane == idx ? val : old;
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
    int64_t *q;         // this chain's queue
    int qcap;           // slots in q
    int *q_tail;        // LDS
    int *err;           // LDS
};

// Per-wave buffers of a walk: step t of the current sub-window in lane t.
struct WalkBuf {
    int ek = 0, eo = 0;      // split k and the varying end (x or y) of the node
    int sa = 0, sb = 0;      // spawned task start node
    int cnt = 0, spawns = 0; // wave-uniform counts
};

// Write the buffered nodes and publish the spawned tasks.  Nothing here
// waits on memory: the walk never stalls for its own stores.
// `fixed` is the node end shared by the walk (a for L, b for R).
__device__ __forceinline__ void flush(WalkBuf &B, const WalkOut &O, int dir, int fixed,
                                      int lane)
{
    if (B.cnt) {
        if (lane < B.cnt) {
            O.lo[B.ek] = dir == kDirL ? fixed : B.eo;
            O.hi[B.ek] = dir == kDirL ? B.eo : fixed;
        }
        B.cnt = 0;
    }
    if (B.spawns) {
        const int base = wave_fetch_add(O.q_tail, B.spawns, lane, __ATOMIC_RELAXED);
        if (base + B.spawns > O.qcap) {
            // Cannot happen for a tree (at most n-2 tasks are spawned);
            // guarded so a broken invariant ends in an error, not a fault.
            atomicOr(O.err, 2);
        } else if (lane < B.spawns) {
            // The opposite direction of the walk that spawned it.
            __hip_atomic_store(O.q + base + lane, task_enc(B.sa, B.sb, dir ^ 1),
                               __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_WORKGROUP);
        }
        B.spawns = 0;
    }
}

// L task: nodes [a, x] for x = b, s[a][b], ... down to a; row a of s.
__device__ void walk_left(const int32_t *__restrict__ s, int64_t n, int a, int b, int *win,
                          int W, const WalkOut &O, int lane)
{
    const int32_t *row = s + (int64_t)a * n;
    WalkBuf B;
    int x = b;
    int wlo = x + 1;         // LDS window holds row positions [wlo, whi]
    int sbase = x + 1;       // register sub-window holds [sbase, sbase + 63]
    int v = 0;
    while (x > a) {
        if (x < sbase) {
            flush(B, O, kDirL, a, lane);
            if (x < wlo) {
                const int whi = x;
                wlo = max(a + 1, x - W + 1);
                stage(win, row + wlo, 1, whi - wlo + 1, lane);
            }
            sbase = max(wlo, x - 63);
            v = win[min(sbase + lane, x) - wlo];
        }
        const int k = __builtin_amdgcn_readlane(v, x - sbase);
        if (k < a || k >= x) {
            atomicOr(O.err, 1);
            break;
        }
        B.ek = set_lane(B.ek, k, B.cnt, lane);
        B.eo = set_lane(B.eo, x, B.cnt, lane);
        ++B.cnt;
        if (k + 1 < x) {     // right child [k+1, x] is a product: R task
            B.sa = set_lane(B.sa, k + 1, B.spawns, lane);
            B.sb = set_lane(B.sb, x, B.spawns, lane);
            ++B.spawns;
        }
        x = k;
    }
    flush(B, O, kDirL, a, lane);
}

// R task: nodes [y, b] for y = a, s[a][b]+1, ... up to b; column b of s.
__device__ void walk_right(const int32_t *__restrict__ s, int64_t n, int a, int b, int *win,
                           int W, const WalkOut &O, int lane)
{
    WalkBuf B;
    int y = a;
    int whi = y - 1;         // LDS window holds column rows [wlo, whi]
    int wlo = y;
    int sbase = y, send = y - 1;   // register sub-window holds [sbase, send]
    int v = 0;
    while (y < b) {
        if (y > send) {
            flush(B, O, kDirR, b, lane);
            if (y > whi) {
                wlo = y;
                whi = min(b - 1, y + W - 1);
                stage(win, s + (int64_t)wlo * n + b, n, whi - wlo + 1, lane);
            }
            sbase = y;
            send = min(y + 63, whi);
            v = win[min(sbase + lane, send) - wlo];
        }
        const int k = __builtin_amdgcn_readlane(v, y - sbase);
        if (k < y || k >= b) {
            atomicOr(O.err, 1);
            break;
        }
        B.ek = set_lane(B.ek, k, B.cnt, lane);
        B.eo = set_lane(B.eo, y, B.cnt, lane);
        ++B.cnt;
        if (y < k) {         // left child [y, k] is a product: L task
            B.sa = set_lane(B.sa, y, B.spawns, lane);
            B.sb = set_lane(B.sb, k, B.spawns, lane);
            ++B.spawns;
        }
        y = k + 1;
    }
    flush(B, O, kDirR, b, lane);
}

template <int NW>
__global__ __launch_bounds__(NW * 64) void k_paren(const ParenChain *__restrict__ chains,
                                                   const int32_t *__restrict__ s_all,
                                                   const int32_t *__restrict__ p_all,
                                                   int32_t *__restrict__ lo_all,
                                                   int32_t *__restrict__ hi_all,
                                                   int64_t *__restrict__ cost_all,
                                                   int64_t *__restrict__ queue_all, int W)
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
                e = ((int64_t)__builtin_amdgcn_readfirstlane((int)(e >> 32)) << 32) |
                    (uint32_t)__builtin_amdgcn_readfirstlane((int)e);
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
        const int a = (int)(e >> 32);
        const int b = (int)(e & 0x7fffffff);
        if ((e >> 31) & 1)
            walk_right(s, n, a, b, win, W, O, lane);
        else
            walk_left(s, n, a, b, win, W, O, lane);
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

// Parenthesized text from the node intervals of one chain; one workgroup.
// counts: 2n int32 workspace.  text: parens_length(n) + 1 bytes.
__global__ __launch_bounds__(kTextBlock) void k_paren_text(const int32_t *__restrict__ lo,
                                                           const int32_t *__restrict__ hi,
                                                           int n, int32_t *__restrict__ counts,
                                                           char *__restrict__ text)
{
    __shared__ int bad;
    __shared__ int64_t part[kTextBlock];
    const int tid = threadIdx.x;
    int32_t *opens = counts, *closes = counts + n;
    if (tid == 0) bad = 0;
    for (int t = tid; t < n; t += kTextBlock) {
        opens[t] = 0;
        closes[t] = 0;
    }
    __syncthreads();
    for (int k = tid; k < n - 1; k += kTextBlock) {
        const int l = lo[k], h = hi[k];
        if (l < 0 || l > k || h <= k || h >= n) {
            bad = 1;
            continue;
        }
        atomicAdd(opens + l, 1);
        atomicAdd(closes + h, 1);
    }
    __syncthreads();
    if (bad) {
        if (tid == 0) text[0] = 0;
        return;
    }
    // Contiguous leaves per thread; exclusive scan of their text lengths.
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
    int64_t pos = part[tid] - mine;
    for (int t = t0; t < t1; ++t) {
        for (int r = opens[t]; r > 0; --r) text[pos++] = '(';
        text[pos++] = 'A';
        const int d = dec_digits(t);
        int v = t;
        for (int i = d - 1; i >= 0; --i) {
            text[pos + i] = (char)('0' + v % 10);
            v /= 10;
        }
        pos += d;
        for (int r = closes[t]; r > 0; --r) text[pos++] = ')';
    }
    if (tid == kTextBlock - 1) text[part[tid]] = 0;
}

}  // namespace

mcm_status run_paren(const ParenChain *chains, int count, int max_n, const int32_t *s_all,
                     const int32_t *p_all, int32_t *lo_all, int32_t *hi_all, int64_t *cost_all,
                     int64_t *queue_all, hipStream_t stream)
{
    if (count <= 0) return MCM_OK;
    const int64_t rup = ((int64_t)max_n + 63) / 64 * 64;
    hipError_t e;
    if (count == 1) {
        // One chain: sixteen waves share its tasks.
        const int W = (int)(rup < 2048 ? rup : 2048);
        const size_t lds = (size_t)16 * W * sizeof(int);
        hipLaunchKernelGGL(k_paren<16>, dim3(1), dim3(16 * 64), lds, stream, chains, s_all,
                           p_all, lo_all, hi_all, cost_all, queue_all, W);
    } else {
        const int W = (int)(rup < 1024 ? rup : 1024);
        const size_t lds = (size_t)4 * W * sizeof(int);
        hipLaunchKernelGGL(k_paren<4>, dim3((unsigned)count), dim3(4 * 64), lds, stream, chains,
                           s_all, p_all, lo_all, hi_all, cost_all, queue_all, W);
    }
    e = hipGetLastError();
    return e == hipSuccess ? MCM_OK : MCM_ERR_DEVICE;
}

mcm_status run_paren_text(const int32_t *lo, const int32_t *hi, int n, int32_t *counts,
                          char *text, hipStream_t stream)
{
    hipLaunchKernelGGL(k_paren_text, dim3(1), dim3(kTextBlock), 0, stream, lo, hi, n, counts,
                       text);
    return hipGetLastError() == hipSuccess ? MCM_OK : MCM_ERR_DEVICE;
}

}  // namespace mcm
