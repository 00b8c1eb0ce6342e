// The simplified DP problem (S-DP) of Section II-A, Definition 1:
//
//   ST[i] = ST[i - a_1] (x) ST[i - a_2] (x) ... (x) ST[i - a_k],   i >= a_1,
//
// with ST[0..a_1-1] preset, a_1 > ... > a_k > 0, and (x) one of minimum (the
// operator of the paper's Table I), maximum or addition modulo 2^32, on int32.
//
// The computed range [a_1, n) is cut into blocks of B elements.  For an
// element i = t + r of the block starting at t, the offsets a > r reach
// before the block, so once the earlier blocks are final all of those terms
// can be folded at once, across the whole device ("far" kernel).  The rest,
// a <= r, read the block itself; they are folded by one workgroup walking the
// block in sub-blocks of 64 ("near" kernel):
//   - terms whose source lies in an earlier sub-block are folded in parallel
//     (a prefix count table giving each element its range of offsets); those
//     reaching before the previous sub-block run while that sub-block's own
//     chain (below) is in progress, the rest right after it;
//   - terms inside the sub-block (offsets below 64) are folded by one wave
//     whose lane l holds element l: at step r' lane r' is final, and every
//     lane l with l - r' among the offsets folds it in, a register update per
//     step instead of a memory round trip.
// Far terms with offsets of two blocks or more read only elements that were
// final before the previous block's near kernel started, so they are folded
// on a second stream beside it (see sdp_launch); the rest stay on the
// caller's stream between two near launches.
// The paper's pipeline (Fig. 2) instead assigns one thread per offset and
// advances one element per step; that keeps k threads busy, while this
// layout spreads the bulk of the work (the far terms) over all CUs and keeps
// only a 64-wide dependency chain on one wave.
#include "mcm_internal.h"

namespace mcm {
namespace {

constexpr int kFarTile = 256;        // targets per far workgroup (one per thread)
constexpr int kNearThreads = 1024;

template <int OP>
__device__ __forceinline__ int32_t sdp_op(int32_t x, int32_t y)
{
    if constexpr (OP == SDP_MIN) return min(x, y);
    else if constexpr (OP == SDP_MAX) return max(x, y);
    else return (int32_t)((uint32_t)x + (uint32_t)y);
}

template <int OP>
__device__ __forceinline__ int32_t sdp_identity()
{
    if constexpr (OP == SDP_MIN) return INT32_MAX;
    else if constexpr (OP == SDP_MAX) return INT32_MIN;
    else return 0;
}

template <int OP>
__device__ __forceinline__ void sdp_atomic(int32_t *p, int32_t v)
{
    if constexpr (OP == SDP_MIN) atomicMin(p, v);
    else if constexpr (OP == SDP_MAX) atomicMax(p, v);
    else atomicAdd(p, v);
}

// dst[x] = src[x] for x < len, NT threads, eight loads in flight per thread
// before the LDS writes (one load at a time would wait out the memory
// latency on every element).
template <int NT>
__device__ __forceinline__ void stage_lds(int32_t *dst, const int32_t *__restrict__ src, int len,
                                          int tid)
{
    for (int base = 0; base < len; base += NT * 8) {
        int32_t v[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) {
            const int x = base + u * NT + tid;
            v[u] = x < len ? src[x] : 0;
        }
#pragma unroll
        for (int u = 0; u < 8; ++u) {
            const int x = base + u * NT + tid;
            if (x < len) dst[x] = v[u];
        }
    }
}

template <int OP>
__global__ __launch_bounds__(256) void k_sdp_fill(int32_t *__restrict__ part, int64_t count)
{
    for (int64_t x = (int64_t)blockIdx.x * 256 + threadIdx.x; x < count;
         x += (int64_t)gridDim.x * 256)
        part[x] = sdp_identity<OP>();
}

// Far terms of block [t, tend): part[i] (x)= ST[i - a_j] for every a_j > i - t.
// Workgroup (tile, chunk): targets t0 .. t0+255 against offsets a[j0..j1),
// whose sources, a span of at most kFarTile + span_max elements, are staged
// into LDS first.  chunks: (j0, j1) pairs.
template <int OP>
__global__ __launch_bounds__(kFarTile) void k_sdp_far(const int32_t *__restrict__ st,
                                                      int32_t *__restrict__ part,
                                                      const int32_t *__restrict__ a,
                                                      const int2 *__restrict__ chunks,
                                                      int nchunks, int t, int tend)
{
    extern __shared__ int32_t lds[];
    const int tile = blockIdx.x / nchunks;
    const int2 ch = chunks[blockIdx.x % nchunks];
    const int t0 = t + tile * kFarTile;
    if (t0 >= tend) return;
    const int amax = a[ch.x], amin = a[ch.y - 1];
    if (amax <= t0 - t) return;                  // no offset reaches before the block
    const int nj = ch.y - ch.x;
    int32_t *offs = lds;                          // nj offsets, descending
    int32_t *src = lds + ((nj + 3) & ~3);         // ST[lo .. hi]
    const int lo = t0 - amax;
    const int hi = min(t0 + kFarTile, tend) - 1 - amin;
    const int tid = threadIdx.x;
    stage_lds<kFarTile>(offs, a + ch.x, nj, tid);
    stage_lds<kFarTile>(src, st + lo, hi - lo + 1, tid);
    __syncthreads();
    const int i = t0 + tid;
    if (i >= tend) return;
    const int r = i - t;
    const int base = i - lo;
    int32_t acc = sdp_identity<OP>();
    int x = 0;
    // Offsets are descending: the valid ones (a_j > r) are a prefix.
    for (; x + 4 <= nj && offs[x + 3] > r; x += 4) {
        acc = sdp_op<OP>(acc, src[base - offs[x]]);
        acc = sdp_op<OP>(acc, src[base - offs[x + 1]]);
        acc = sdp_op<OP>(acc, src[base - offs[x + 2]]);
        acc = sdp_op<OP>(acc, src[base - offs[x + 3]]);
    }
    for (; x < nj && offs[x] > r; ++x) acc = sdp_op<OP>(acc, src[base - offs[x]]);
    if (x > 0) sdp_atomic<OP>(part + i, acc);
}

// Near terms of block [t, tend) (a_j <= i - t), then the block's final
// values to st.  near_a: the offsets below B, ascending; cnt_le[x]: how many
// of them are <= x (x < B); seq_mask[l]: bit r' set when l - r' is an offset
// (0 <= r' < l < 64).  One workgroup; LDS holds the block.
template <int OP>
__global__ __launch_bounds__(kNearThreads) void k_sdp_near(int32_t *__restrict__ st,
                                                           const int32_t *__restrict__ part,
                                                           const int32_t *__restrict__ near_a,
                                                           int kn,
                                                           const int32_t *__restrict__ cnt_le,
                                                           const uint64_t *__restrict__ seq_mask,
                                                           int t, int tend, int B)
{
    extern __shared__ int32_t lds[];
    int32_t *blk = lds;                   // B values of the block
    int32_t *cle = lds + B;               // B prefix counts
    int32_t *na = lds + 2 * B;            // kn offsets (< B), ascending
    const int tid = threadIdx.x;
    const int len = tend - t;
    stage_lds<kNearThreads>(blk, part + t, len, tid);
    for (int x = len + tid; x < B; x += kNearThreads) blk[x] = sdp_identity<OP>();
    stage_lds<kNearThreads>(cle, cnt_le, B, tid);
    stage_lds<kNearThreads>(na, near_a, kn, tid);
    const int lane = tid & 63;
    const uint64_t gm = tid < 64 ? seq_mask[lane] : 0;
    const uint32_t gm_lo = (uint32_t)gm, gm_hi = (uint32_t)(gm >> 32);
    __syncthreads();
    const int nsub = (len + 63) / 64;
    const int wave = tid >> 6;
    for (int s = 0; s < nsub; ++s) {
        // Here sub-block s holds every term but those whose source lies
        // inside it.
        if (wave == 0) {
            // Sources inside the sub-block: lane r' is final at step r', and
            // every lane l with l - r' among the offsets folds it in.
            int32_t v = blk[64 * s + lane];
#pragma unroll 4
            for (int rp = 0; rp < 32; ++rp) {
                const int32_t w = __builtin_amdgcn_readlane(v, rp);
                v = sdp_op<OP>(v, ((gm_lo >> rp) & 1) ? w : sdp_identity<OP>());
            }
#pragma unroll 4
            for (int rp = 32; rp < 63; ++rp) {
                const int32_t w = __builtin_amdgcn_readlane(v, rp);
                v = sdp_op<OP>(v, ((gm_hi >> (rp - 32)) & 1) ? w : sdp_identity<OP>());
            }
            blk[64 * s + lane] = v;
            if (64 * s + lane < len) st[t + 64 * s + lane] = v;
        } else if (wave >= 8 && s + 1 < nsub) {
            // Meanwhile, sub-block s+1 folds its sources before sub-block s
            // (offsets in [l+65, r]), 8 threads per element.
            const int u = tid - 512, l = u >> 3, g = u & 7;
            const int r = 64 * (s + 1) + l;
            int32_t acc = sdp_identity<OP>();
            const int jend = cle[r];
            int j = cle[l + 64] + g;
            for (; j + 24 < jend; j += 32) {
                const int d0 = na[j], d1 = na[j + 8], d2 = na[j + 16], d3 = na[j + 24];
                acc = sdp_op<OP>(acc, blk[r - d0]);
                acc = sdp_op<OP>(acc, blk[r - d1]);
                acc = sdp_op<OP>(acc, blk[r - d2]);
                acc = sdp_op<OP>(acc, blk[r - d3]);
            }
            for (; j < jend; j += 8) acc = sdp_op<OP>(acc, blk[r - na[j]]);
            for (int off = 4; off > 0; off >>= 1) acc = sdp_op<OP>(acc, __shfl_xor(acc, off, 8));
            if (g == 0) blk[r] = sdp_op<OP>(blk[r], acc);
        }
        __syncthreads();
        if (s + 1 < nsub) {
            // Then its sources in sub-block s, now final (offsets in
            // [l+1, l+64]), 16 threads per element.
            const int l = tid >> 4, g = tid & 15;
            const int r = 64 * (s + 1) + l;
            int32_t acc = sdp_identity<OP>();
            for (int j = cle[l] + g; j < cle[l + 64]; j += 16) acc = sdp_op<OP>(acc, blk[r - na[j]]);
            for (int off = 8; off > 0; off >>= 1) acc = sdp_op<OP>(acc, __shfl_xor(acc, off, 16));
            if (g == 0) blk[r] = sdp_op<OP>(blk[r], acc);
        }
        __syncthreads();
    }
}

template <int OP>
mcm_status sdp_launch(const SdpPlan &pl, int32_t *st, hipStream_t stream)
{
    const int64_t cnt = (int64_t)pl.n - pl.a1;
    {
        const int64_t want = (cnt + 255) / 256;
        const unsigned blocks = (unsigned)(want < 4096 ? (want < 1 ? 1 : want) : 4096);
        hipLaunchKernelGGL(k_sdp_fill<OP>, dim3(blocks), dim3(256), 0, stream, pl.part + pl.a1,
                           cnt);
        if (hipGetLastError() != hipSuccess) return MCM_ERR_DEVICE;
    }
    const size_t far_lds = (size_t)(((pl.chunk_max + 3) & ~3) + kFarTile + pl.span_max) * 4;
    const size_t near_lds = (size_t)(2 * pl.B + pl.kn) * 4;
    const int tiles = (pl.B + kFarTile - 1) / kFarTile;
    const int64_t nblocks = (cnt + pl.B - 1) / pl.B;
    const int nold = pl.nchunks_old, nnew = pl.nchunks - pl.nchunks_old;
    auto far = [&](hipStream_t q, const int2 *ch, int nch, int64_t t, int tend) {
        hipLaunchKernelGGL(k_sdp_far<OP>, dim3((unsigned)(tiles * nch)), dim3(kFarTile), far_lds,
                           q, st, pl.part, pl.a, ch, nch, (int)t, tend);
    };
    auto near = [&](hipStream_t q, int64_t t, int tend) {
        hipLaunchKernelGGL(k_sdp_near<OP>, dim3(1), dim3(kNearThreads), near_lds, q, st,
                           pl.part, pl.near_a, pl.kn, pl.cnt_le, pl.seq_mask, (int)t, tend, pl.B);
    };
    if (nold == 0 || nblocks < 3) {
        for (int64_t t = pl.a1; t < pl.n; t += pl.B) {
            const int tend = (int)(t + pl.B < pl.n ? t + pl.B : pl.n);
            far(stream, pl.chunks, pl.nchunks, t, tend);
            near(stream, t, tend);
            if (hipGetLastError() != hipSuccess) return MCM_ERR_DEVICE;
        }
        return MCM_OK;
    }
    // Two streams.  The old terms of block b (offsets >= 2B) read elements
    // before block b-1, final once near(b-2) is done, so they are folded on
    // the library's aux stream while near(b-1) runs; the caller's stream
    // runs the new terms of b, waits for the old ones, then near(b).
    //   - far_old(b) waits for the launch before near(b-1) (which follows
    //     near(b-2)), then a short pause, so near(b-1) reaches a CU first;
    //   - near asks for LDS enough that no far workgroup fits beside it
    //     (a latency-bound workgroup sharing its CU runs markedly slower).
    StreamSet ss;
    if (acquire_streams((int)(2 * nblocks + 2), &ss) != MCM_OK) return MCM_ERR_DEVICE;
    hipEvent_t *ev_old = ss.events.data() + 2, *ev_pre = ev_old + nblocks;
    const size_t lds_cu = 163840;
    const size_t near_excl = far_lds < lds_cu ? lds_cu - far_lds + 1024 : near_lds;
    const size_t near_lds2 = near_excl > near_lds && near_excl <= lds_cu ? near_excl : near_lds;
    mcm_status rc = MCM_OK;
    if (hipEventRecord(ss.events[0], stream) != hipSuccess ||
        hipStreamWaitEvent(ss.aux, ss.events[0], 0) != hipSuccess)
        rc = MCM_ERR_DEVICE;
    const bool forked = rc == MCM_OK;
    for (int64_t b = 0; b < nblocks && rc == MCM_OK; ++b) {
        const int64_t t = pl.a1 + b * pl.B;
        const int tend = (int)(t + pl.B < pl.n ? t + pl.B : pl.n);
        if (b >= 1) {
            if (hipStreamWaitEvent(ss.aux, ev_pre[b - 1], 0) != hipSuccess ||
                launch_delay(ss.aux) != MCM_OK) {
                rc = MCM_ERR_DEVICE;
                break;
            }
        }
        far(ss.aux, pl.chunks, nold, t, tend);
        // The old terms are handed to the caller's stream as an aux signal
        // token when the device has one (a shorter hop), else an event.
        if (hipGetLastError() != hipSuccess) {
            rc = MCM_ERR_DEVICE;
            break;
        }
        const uint64_t token = aux_signal_write(ss.aux);
        if (!token && hipEventRecord(ev_old[b], ss.aux) != hipSuccess) {
            rc = MCM_ERR_DEVICE;
            break;
        }
        if (nnew > 0) far(stream, pl.chunks + nold, nnew, t, tend);
        if (hipGetLastError() != hipSuccess ||
            (token ? aux_signal_wait(stream, token)
                   : hipStreamWaitEvent(stream, ev_old[b], 0)) != hipSuccess ||
            hipEventRecord(ev_pre[b], stream) != hipSuccess) {
            rc = MCM_ERR_DEVICE;
            break;
        }
        hipLaunchKernelGGL(k_sdp_near<OP>, dim3(1), dim3(kNearThreads), near_lds2, stream, st,
                           pl.part, pl.near_a, pl.kn, pl.cnt_le, pl.seq_mask, (int)t, tend, pl.B);
        if (hipGetLastError() != hipSuccess) rc = MCM_ERR_DEVICE;
    }
    if (forked) {
        // Join: the caller's stream continues after everything on aux.
        if (hipEventRecord(ss.events[1], ss.aux) != hipSuccess ||
            hipStreamWaitEvent(stream, ss.events[1], 0) != hipSuccess)
            rc = MCM_ERR_DEVICE;
    }
    release_streams(ss);
    return rc;
}

}  // namespace

mcm_status run_sdp(const SdpPlan &pl, int op, int32_t *st, hipStream_t stream)
{
    if (pl.a1 >= pl.n) return MCM_OK;
    switch (op) {
    case SDP_MIN: return sdp_launch<SDP_MIN>(pl, st, stream);
    case SDP_MAX: return sdp_launch<SDP_MAX>(pl, st, stream);
    case SDP_ADD: return sdp_launch<SDP_ADD>(pl, st, stream);
    default: return MCM_ERR_INVALID_ARG;
    }
}

}  // namespace mcm
