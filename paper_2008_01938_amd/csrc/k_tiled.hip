// Tiled MCM table fill for gfx950.
//
// The table is cut into T x T tiles; tile (I, J), I <= J, holds cells
// i in [I*T, I*T+T), j in [J*T, J*T+T).  Tiles are processed in
// tile-diagonal order D = J - I, the block analogue of the diagonal order
// of the paper's Fig. 5.  For an off-diagonal tile the splits k of a cell
// fall into three ranges:
//
//   (a) k in [i, (I+1)T-2]     left operand in diagonal tile (I,I),
//                              right operand in the tile itself (below);
//   bulk k in [(I+1)T-1, JT-1] both operands in tiles of earlier
//                              tile-diagonals -- the same range for every
//                              cell of the tile;
//   (b) k in [JT, j-1]         left operand in the tile itself (to the
//                              left), right operand in diagonal tile (J,J).
//
// The bulk range splits once more.  Its two end blocks, k in
// [(I+1)T-1, (I+2)T-2] and [(J-1)T, JT-1], read tiles of tile-diagonal
// D-1; the interior between them reads only tiles of diagonals <= D-2.
//
// k_tri_rows fills the diagonal tiles (all their splits stay inside the
// tile) on fp64 keys in row groups, as the closure sweeps (k_tri_key, lanes
// per cell and a shuffle tree, for many 64-edge tiles at once); k_tri<true>
// does it in int64 with the optimal-BST weights.
// k_bulk: a min-plus-like reduction over a chunk of a tile's bulk range.
//         The A panel (rows of I, columns k) and the B panel (rows k+1,
//         columns of J) are staged through LDS; each thread keeps a 4 x 4
//         register microtile of running minima; each workgroup writes packed
//         (cost, k) partial minima.
// k_close: merges a tile's partials, then adds the (a) and (b) splits.
//         Cell (r, c) (local row/column) needs the cells below it in its
//         column and left of it in its row, so the tile is swept in local
//         anti-diagonals w = (T-1-r) + c, one barrier per step, in LDS.
// The closure of tile-diagonal D is long and latency-bound, and the interior
// bulk of D+1 does not depend on it, so the two run concurrently on two
// streams; the end blocks of D+1 follow the closure of D.
//
// Exact integers in fp64.  A candidate cost of cell (i, j) is at most
// (j-i) * pmax^3 < 2^cost_bits.  The kernels carry
// key = cost * 2^kb + k_local as a double with kb = 53 - cost_bits, so
// every key, and every partial sum that forms it (all integers), is below
// 2^53 and therefore exact; one fp64 min then picks the smallest cost and,
// among equal costs, the smallest k_local -- the smallest k when k_local
// increases with k.  A split evaluation is fma + add + min.
#include <hip/hip_ext.h>
#include <math.h>
#include <string.h>

#include <mutex>
#include <type_traits>
#include <unordered_map>

#include "mcm_internal.h"

namespace mcm {
namespace {

// Tile edges: 64 for lone chains and large batches, 32 for batches of small
// chains (half the closure splits per cell, 63 closure steps per tile).
constexpr int KC = 16;         // k values staged per LDS round (bulk)
constexpr int NTH = 256;       // k_tri and k_tri_key threads
constexpr double kPad = 4611686018427387904.0;  // 2^62: never wins a min

typedef uint32_t u32x2 __attribute__((ext_vector_type(2)));

// x * 2^kb as a double for a table entry x in [0, 2^52), given as its two
// 32-bit halves: setting the exponent field of 2^52 over x's bits gives the
// double 2^52 + x exactly, and one fma scales it and removes the 2^52 with a
// single, exact rounding (the result is below 2^53).
__device__ __forceinline__ double cost_key(u32x2 x, double scale)
{
    const double t = __builtin_bit_cast(double, (u32x2){x.x, x.y | 0x43300000u});
    return fma(t, scale, -4503599627370496.0 * scale);
}

// Wave issue priority 0..3 (s_setprio takes an immediate).
__device__ __forceinline__ void set_prio(int p)
{
    if (p >= 3)
        __builtin_amdgcn_s_setprio(3);
    else if (p == 2)
        __builtin_amdgcn_s_setprio(2);
    else if (p == 1)
        __builtin_amdgcn_s_setprio(1);
    else
        __builtin_amdgcn_s_setprio(0);
}

// The segment of a launch that workgroup b belongs to (segments are sorted
// by their first workgroup; every thread of the workgroup agrees).
__device__ __forceinline__ int find_seg(const TileSeg *__restrict__ seg, int nseg, int b)
{
    int lo = 0, hi = nseg - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (seg[mid].first <= b)
            lo = mid;
        else
            hi = mid - 1;
    }
    return lo;
}

// ------------------------------------------------------------------------
// Diagonal tiles (I, I): every split of a cell inside the tile uses two
// cells of the same tile.  Local diagonals dd = 1..nI-1 in order.  The
// nI - dd cells of diagonal dd share the 256 lanes: L lanes per cell, L the
// largest power of two in [4, 64] with cells * L <= 256, so a cell's lanes
// lie in one wave and the longest scan is about 4 splits per lane.  Each
// lane keeps a (cost, k) minimum over its splits; a shuffle tree over the L
// lanes takes the lexicographic minimum.  int64 arithmetic.
// ------------------------------------------------------------------------
// OB: the optimal-BST weights (one chain; p_all then holds zeros): the
// diagonal holds the gap weights q and every cell gains W(i, j) = hi[j] -
// lo[i] after its minimum.
template <int T, bool OB>
__global__ __launch_bounds__(NTH) void k_tri(const TileChain *__restrict__ chains,
                                             const TileSeg *__restrict__ segs, int nseg,
                                             const int32_t *__restrict__ p_all,
                                             int64_t *__restrict__ m_all,
                                             int32_t *__restrict__ s_all,
                                             const int64_t *__restrict__ ob_hi,
                                             const int64_t *__restrict__ ob_lo,
                                             const int32_t *__restrict__ ob_q)
{
    __shared__ int64_t tv[T][T + 1];
    __shared__ uint8_t sv[T][T + 4];  // local split (0..T-2) of cell (r, c), r < c
    __shared__ int64_t ps[T + 1];
    const int tid = threadIdx.x;
    const TileSeg sg = segs[find_seg(segs, nseg, blockIdx.x)];
    const TileChain ch = chains[sg.chain];
    const int32_t n = ch.n;
    const int32_t *__restrict__ p = p_all + ch.p_off;
    int64_t *__restrict__ m = m_all + ch.m_off;
    int32_t *__restrict__ s = s_all + ch.s_off;
    const int base = (blockIdx.x - sg.first) * T;
    const int nI = min(T, n - base);
    for (int q = tid; q <= nI; q += NTH) ps[q] = p[base + q];
    for (int r = tid; r < T; r += NTH) tv[r][r] = OB && r < nI ? (int64_t)ob_q[base + r] : 0;
    __syncthreads();

    for (int dd = 1; dd < nI; ++dd) {
        const int cells = nI - dd;
        int lg = 2;  // log2 L, uniform across the workgroup
        while (lg < 6 && (cells << (lg + 1)) <= NTH) ++lg;
        const int L = 1 << lg;
        const int r = tid >> lg, g = tid & (L - 1);
        const int c = r + dd;
        int64_t best = INT64_MAX;
        int32_t arg = INT32_MAX;
        if (r < cells) {
            const int64_t prc = ps[r] * ps[c + 1];
            for (int kl = r + g; kl < c; kl += L) {
                const int64_t v = tv[r][kl] + tv[kl + 1][c] + prc * ps[kl + 1];
                if (v < best) {
                    best = v;
                    arg = kl;
                }
            }
        }
        // xor partners stay inside the L-aligned lane group of the cell.
        for (int off = 1; off < L; off <<= 1) {
            const int64_t ov = __shfl_xor(best, off, 64);
            const int32_t oa = __shfl_xor(arg, off, 64);
            if (ov < best || (ov == best && oa < arg)) {
                best = ov;
                arg = oa;
            }
        }
        if (r < cells && g == 0) {
            tv[r][c] = OB ? best + (ob_hi[base + c] - ob_lo[base + r]) : best;
            sv[r][c] = (uint8_t)arg;
        }
        __syncthreads();
    }

    for (int idx = tid; idx < T * T; idx += NTH) {
        const int rr = idx / T, cc = idx % T;
        if (rr < nI && cc < nI) {
            const size_t o = (size_t)(base + rr) * n + base + cc;
            m[o] = rr <= cc ? tv[rr][cc] : tv[cc][rr];
            s[o] = rr < cc ? base + (int32_t)sv[rr][cc] : -1;
        }
    }
}

// The same diagonal tiles with the exact fp64 keys of the bulk and closure
// kernels (no weights): a split kl of cell (r, c) is the integer
//   (m[r][kl] + m[kl+1][c] + p[r] p[kl+1] p[c+1]) * 2^kb + kl  <  2^53,
// since every candidate cost is below 2^cost_bits and kb <= 53 - cost_bits
// (and kl < T <= 2^kb), so every fma, add and min on it is exact and one
// fmin picks the smallest cost, then the smallest kl.
template <int T>
__global__ __launch_bounds__(NTH) void k_tri_key(const TileChain *__restrict__ chains,
                                                 const TileSeg *__restrict__ segs, int nseg,
                                                 const double *__restrict__ pd_all,
                                                 int64_t *__restrict__ m_all,
                                                 int32_t *__restrict__ s_all)
{
    __shared__ double tv[T][T + 1];   // cost * 2^kb of cell (r, c), r <= c
    __shared__ uint8_t sv[T][T + 4];  // local split (0..T-2) of cell (r, c), r < c
    __shared__ double ps[T + 1];
    const int tid = threadIdx.x;
    const TileSeg sg = segs[find_seg(segs, nseg, blockIdx.x)];
    const TileChain ch = chains[sg.chain];
    const int32_t n = ch.n;
    const double *__restrict__ pd = pd_all + ch.pd_off;
    int64_t *__restrict__ m = m_all + ch.m_off;
    int32_t *__restrict__ s = s_all + ch.s_off;
    const double scale = ldexp(1.0, ch.kb), inv_scale = ldexp(1.0, -ch.kb);
    const int base = (blockIdx.x - sg.first) * T;
    const int nI = min(T, n - base);
    for (int q = tid; q <= nI; q += NTH) ps[q] = pd[base + q];
    for (int r = tid; r < T; r += NTH) tv[r][r] = 0.0;
    __syncthreads();

    for (int dd = 1; dd < nI; ++dd) {
        const int cells = nI - dd;
        int lg = 2;  // log2 L, lanes per cell as in k_tri
        while (lg < 6 && (cells << (lg + 1)) <= NTH) ++lg;
        const int L = 1 << lg;
        const int r = tid >> lg, g = tid & (L - 1);
        const int c = r + dd;
        double best = kPad;
        if (r < cells) {
            const double prc = ps[r] * ps[c + 1] * scale;
            for (int kl = r + g; kl < c; kl += L)
                best = fmin(best, fma(prc, ps[kl + 1], (double)kl) + tv[r][kl] + tv[kl + 1][c]);
        }
        for (int off = 1; off < L; off <<= 1) best = fmin(best, __shfl_xor(best, off, 64));
        if (r < cells && g == 0) {
            const double cost = floor(best * inv_scale);
            tv[r][c] = cost * scale;
            sv[r][c] = (uint8_t)(int)fma(-cost, scale, best);
        }
        __syncthreads();
    }

    for (int idx = tid; idx < T * T; idx += NTH) {
        const int rr = idx / T, cc = idx % T;
        if (rr < nI && cc < nI) {
            const size_t o = (size_t)(base + rr) * n + base + cc;
            m[o] = (int64_t)((rr <= cc ? tv[rr][cc] : tv[cc][rr]) * inv_scale);
            s[o] = rr < cc ? base + (int32_t)sv[rr][cc] : -1;
        }
    }
}

// ------------------------------------------------------------------------
// Shared memory and launch shapes.
// ------------------------------------------------------------------------
// Paired closure: column stride (doubles) of its LDS tables; T + 8 is
// 8 (mod 16) for both tile edges.
template <int T>
constexpr int cstr() { return T + 8; }

// Closure shapes: G lanes per row group, T rows.  (T, G) = (64, 16): one
// tile per CU (16 waves, column-major DJ table).  (64, 8): a tile in 8 waves
// with a packed DJ table, small enough that two closure workgroups share a
// CU.  (32, 8): a 32-edge tile in 4 waves with the packed table.
template <int T, int G>
struct CloseShape {
    static constexpr int CG = G;          // lanes per row group
    static constexpr int CTH = T * G;     // threads
    static constexpr int CS = T / G;      // register slots per lane
    static constexpr int CROWS = 64 / G;  // rows per wave
};
constexpr int CG_LONE = 16;
constexpr int CG_PAIR = 8;

// Packed DJ table: column c holds DJ[q][c], q = 1..c, from base c; bases
// step by c plus padding so that consecutive columns start 8 doubles apart
// modulo 16 (the two row groups of a 16-lane LDS pass then hit disjoint
// banks).  Reads past a column's length land in later columns or padding:
// finite values whose terms lose anyway (see close_step).
constexpr int dj_packed_base(int c)
{
    // c(c-1)/2 plus the paddings (8 - x) & 15 for x < c: 120 per 16 columns
    // and a closed-form prefix for the rest.
    const int q = c >> 4, rem = c & 15;
    const int pre = rem <= 9 ? 8 * rem - rem * (rem - 1) / 2
                             : 36 + 24 * (rem - 9) - ((rem - 1) * rem / 2 - 36);
    return c * (c - 1) / 2 + 120 * q + pre;
}
static_assert(dj_packed_base(1) == 8 && dj_packed_base(9) == 72 && dj_packed_base(16) == 240 &&
                  dj_packed_base(63) == 2424,
              "packed DJ bases");
template <int T>
constexpr int dj_packed_size() { return dj_packed_base(T - 1) + T; }

template <int T>
struct BulkLds {
    double As[2][KC][T + 1];  // As[kk][r] = m[row0+r][k] * 2^kb + (k - k0)
    double Bs[2][KC][T];      // Bs[kk][c] = m[k+1][col0+c] * 2^kb
    double Ps[2][KC];         // p[k+1]
};

// Closure LDS.  Xt and the full DJ table are column-major with a column
// stride of CSTR doubles.  LDS has 32 banks of 4 bytes, so a 64-bit read is
// conflict-free when the 16 lanes served together touch distinct 8-byte
// words modulo 16: with G = 16 those are one row group reading consecutive
// rows of one column (any stride; the full layout takes an odd one, T + 1,
// so that the prologue's and epilogue's passes along a row, lanes a column
// apart, are conflict-free as well); with G = 8 two row groups reading
// adjacent columns, whose starts differ by CSTR = 8 (mod 16) doubles.  Row T
// is a spare so slot addresses never need clamping.
// The full layout also keeps every cell's final key (Fk), so the sweep
// writes one value per cell and the split is read off in the epilogue; the
// packed one records a split found by the sweep in Ks as its complement
// (negative), resolved in the epilogue, and has no room for the keys.
// The sweep reads column cc of the DJ table through its base offset, which a
// lane advances as its cc grows by one (dj_next), so no per-step multiply.
template <int T>
struct CloseLdsFull {
    static constexpr int CSTR = T + 1;  // odd: a column-strided pass is conflict-free too
    double DJt[T][CSTR];   // DJt[c][q] = DJ[q][c] * 2^kb + T + q - 1 (1 <= q <= c), else 0
    double Xt[T][CSTR];    // Xt[c][q]: bulk key, then final cost * 2^kb of cell (q, c)
    double Fk[T][CSTR];    // Fk[c][q]: final key of cell (q, c) (cost * 2^kb + k_local)
    int32_t Ks[T][T + 1];  // bulk split
    double pJs[T + 1];     // p[col0 + q]
    static constexpr bool kFinalKeys = true;
    __device__ double &dj(int q, int c) { return DJt[c][q]; }
    // Base of column c is c * CSTR (the same as Xt's); DJ[j+1][c] sits at
    // base + j + 1.
    static constexpr bool kPacked = false;
    __device__ static int dj_next(int base, int) { return base + CSTR; }
    __device__ double dj_at_base(int base, int j) const { return (&DJt[0][0])[base + j + 1]; }
};
template <int T>
struct CloseLdsPacked {
    static constexpr int CSTR = cstr<T>();
    double DJp[dj_packed_size<T>()];  // column c from dj_packed_base(c): DJ[q][c] at q - 1
    double Xt[T][CSTR];
    int32_t Ks[T][T + 1];  // bulk split, or ~k_local of a split the sweep found
    double pJs[T + 1];
    static constexpr bool kFinalKeys = false;
    __device__ double &dj(int q, int c) { return DJp[dj_packed_base(c) + q - 1]; }
    // dj_packed_base(c + 1) = dj_packed_base(c) + c + ((8 - c) & 15).
    static constexpr bool kPacked = true;
    __device__ static int dj_next(int base, int c) { return base + c + ((8 - c) & 15); }
    __device__ double dj_at_base(int base, int j) const { return DJp[base + j]; }
};

// ------------------------------------------------------------------------
// Bulk: workgroup b of a segment takes tile b / nch and chunk b % nch of
// the segment's split range; thread (tx, ty) owns the cells rows ty + TW*a,
// columns tx + TW*b (a, b = 0..3, TW = T/4) of the tile: a 4 x 4 register
// microtile, (T/4)^2 threads (256 for T = 64, one wave for T = 32).
// ------------------------------------------------------------------------
template <int T>
constexpr int bulk_threads() { return (T / 4) * (T / 4); }

// __builtin_amdgcn_sched_barrier mask: only scalar ALU instructions may be
// scheduled across the barrier.
constexpr int kSchedScalarOnly = 0x0004;

// With a wait word, a bulk launch's last workgroup computes nothing: its
// first wave waits until the word holds at least `token` (written on
// another stream once the interior beside the launch is complete), so the
// launch ends no earlier than that interior.  The wait is bounded by
// `ticks` of the constant-rate clock.  True for that workgroup.
__device__ __forceinline__ bool bulk_waiter(const uint64_t *word, uint64_t token, long long ticks)
{
    if (word == nullptr || blockIdx.x != gridDim.x - 1) return false;
    if (threadIdx.x < 64) {
        const long long t0 = wall_clock64();
        while (__hip_atomic_load(word, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM) < token &&
               wall_clock64() - t0 < ticks)
            __builtin_amdgcn_s_sleep(1);
    }
    return true;
}

// 64-edge tiles: held to three waves per SIMD (at most 168 VGPRs), which
// the kernel fits without spills; the 32-edge form runs at two.
template <int T>
__global__ __launch_bounds__(bulk_threads<T>()) __attribute__((amdgpu_waves_per_eu(T == 64 ? 3 : 2)))
void k_bulk(const TileChain *__restrict__ chains, const TileSeg *__restrict__ segs, int nseg,
            const int64_t *__restrict__ m_all, const double *__restrict__ pd_all,
            uint64_t *__restrict__ part_all, int paced, const uint64_t *wait_word,
            uint64_t wait_token, long long wait_ticks)
{
    if (bulk_waiter(wait_word, wait_token, wait_ticks)) return;
    constexpr int BTH = bulk_threads<T>();
    constexpr int TW = T / 4;            // threads per microtile row
    constexpr int RA = BTH / KC;         // A rows staged apart per thread
    constexpr int RB = BTH / T;          // B splits staged apart per thread
    constexpr int V = T * KC / BTH;      // elements of each block per thread
    static_assert(BTH % KC == 0 && BTH % T == 0 && RA * V == T && RB * V == KC && BTH >= KC,
                  "staging map");
    __shared__ BulkLds<T> L;
    const TileSeg sg = segs[find_seg(segs, nseg, blockIdx.x)];
    const TileChain ch = chains[sg.chain];
    const int local = blockIdx.x - sg.first;
    const int32_t n = ch.n, D = sg.D, KS = sg.KS, kb = ch.kb, kbits = ch.kbits;
    const int64_t *__restrict__ m = m_all + ch.m_off;
    const double *__restrict__ pd = pd_all + ch.pd_off;
    const int tid = threadIdx.x;
    const int tile = local / sg.nch;
    const int chunk = local - tile * sg.nch;
    const int I = tile, J = tile + D;
    const int row0 = I * T, col0 = J * T;
    const int kbase = (I + 1) * T - 1 + sg.koff;
    const int k0 = kbase + chunk * KS;
    const int kend = min(k0 + KS, kbase + sg.klen);  // exclusive
    const int rounds = (kend - k0 + KC - 1) / KC;
    const int nJ = min(T, n - col0);
    const double scale = ldexp(1.0, kb);
    const double inv_scale = ldexp(1.0, -kb);
    const int tx = tid % TW, ty = tid / TW;

    // The eight dims are loaded together (column indices clamped into the
    // table, the products past the last column then zeroed) so that the
    // prologue waits for memory once, not once per conditional load.
    double pi4[4], pc4[4];
#pragma unroll
    for (int a = 0; a < 4; ++a) pi4[a] = pd[row0 + ty + TW * a];
#pragma unroll
    for (int b = 0; b < 4; ++b) pc4[b] = pd[col0 + min(tx + TW * b, nJ - 1) + 1];
    double pj[4][4], best[4][4];
#pragma unroll
    for (int a = 0; a < 4; ++a) {
#pragma unroll
        for (int b = 0; b < 4; ++b) {
            const double v = pi4[a] * scale * pc4[b];
            pj[a][b] = tx + TW * b < nJ ? v : 0.0;
            best[a][b] = __builtin_inf();
        }
    }

    // Staging: the A block is T rows x KC columns, the B block KC rows x T
    // columns.  Thread tid stages A rows ar + RA*v at split akk and B splits
    // bkk + RB*v at column bc (v < V).  Only the round's base moves, so on a
    // table under 2 GiB the loads take 32-bit byte offsets from a uniform
    // base.  In a round that passes kend, splits at or past it are staged
    // from split kend-1 (inside the table) and masked.  (Raw buffer loads
    // with the same offsets measured slower.)
    const int akk = tid % KC, ar = tid / KC;
    const int bcol = tid % T, bc = min(bcol, nJ - 1), bkk = tid / T;
    const bool narrow = (size_t)n * (size_t)n * sizeof(int64_t) < ((size_t)1 << 31);
    uint32_t oa[V], ob[V];
#pragma unroll
    for (int v = 0; v < V; ++v) {
        oa[v] = (uint32_t)(((size_t)(row0 + ar + RA * v) * n + akk) * sizeof(int64_t));
        ob[v] = (uint32_t)(((size_t)(bkk + RB * v + 1) * n + col0 + bc) * sizeof(int64_t));
    }
    // Table entries as two 32-bit halves; every entry staged is a cost of a
    // final cell, below 2^46, which the store turns into a key exactly.
    u32x2 ra[V], rb[V];
    double rp = 0.0;
    auto load = [&](int kc) {
        if (kc + KC <= kend && narrow) {
            const char *ba = (const char *)(m + kc);
            const char *bb = (const char *)(m + (size_t)kc * n);
#pragma unroll
            for (int v = 0; v < V; ++v) {
                ra[v] = *(const u32x2 *)(ba + oa[v]);
                rb[v] = *(const u32x2 *)(bb + ob[v]);
            }
        } else {
#pragma unroll
            for (int v = 0; v < V; ++v) {
                const int ka = min(kc + akk, kend - 1);
                ra[v] = __builtin_bit_cast(u32x2, m[(size_t)(row0 + ar + RA * v) * n + ka]);
                const int kb2 = min(kc + bkk + RB * v, kend - 1);
                rb[v] = __builtin_bit_cast(u32x2, m[(size_t)(kb2 + 1) * n + col0 + bc]);
            }
        }
        if (tid < KC) rp = (kc + tid < kend) ? pd[kc + tid + 1] : 0.0;
    };
    // The A side carries the split's offset from k0 (one split per thread
    // and round: akk), so A keys are cost * 2^kb + (k - k0) and B keys
    // cost * 2^kb; their sum is the same key.
    auto store = [&](int kc, int buf) {
        const double koff = (double)(kc + akk - k0);
        if (kc + KC <= kend) {
#pragma unroll
            for (int v = 0; v < V; ++v)
                L.As[buf][akk][ar + RA * v] = cost_key(ra[v], scale) + koff;
        } else {
#pragma unroll
            for (int v = 0; v < V; ++v)
                L.As[buf][akk][ar + RA * v] =
                    kc + akk < kend ? cost_key(ra[v], scale) + koff : kPad;
        }
#pragma unroll
        for (int v = 0; v < V; ++v) L.Bs[buf][bkk + RB * v][bcol] = cost_key(rb[v], scale);
        if (tid < KC) L.Ps[buf][tid] = rp;
    };

    load(k0);
    store(k0, 0);
    __syncthreads();
    int buf = 0;
    for (int rd = 0; rd < rounds; ++rd) {
        const int kc = k0 + rd * KC;
        const bool more = rd + 1 < rounds;
        // paced: issue priority falls as the chunk progresses (3 in its
        // first quarter, 0 in its last).  The workgroups sharing a CU would
        // otherwise be served oldest first and finish one after another,
        // the last alone on the CU with little to hide its latencies.  Not
        // for launches that share CUs with closures (batched plans).
        if (paced) set_prio(3 - (4 * rd) / rounds);
        if (more) load(kc + KC);
        if constexpr (T == 64) {
#pragma unroll 4
            for (int kk = 0; kk < KC; ++kk) {
                double av[4], bv[4];
#pragma unroll
                for (int a = 0; a < 4; ++a) av[a] = L.As[buf][kk][ty + TW * a];
#pragma unroll
                for (int b = 0; b < 4; ++b) bv[b] = L.Bs[buf][kk][tx + TW * b];
                const double pk = L.Ps[buf][kk];
#pragma unroll
                for (int a = 0; a < 4; ++a)
#pragma unroll
                    for (int b = 0; b < 4; ++b)
                        best[a][b] = fmin(best[a][b], fma(pj[a][b], pk, bv[b]) + av[a]);
            }
        } else {
            // 32-edge tiles run two waves per SIMD, too few to hide a cell's
            // dependent fma -> add -> min when the compiler emits the cells
            // one after another.  Here the next split's operands are read
            // first and the row's four cells go through each stage together;
            // scheduling barriers that let only scalar instructions cross
            // keep that order.
            double av[4], bv[4], pk;
#pragma unroll
            for (int a = 0; a < 4; ++a) av[a] = L.As[buf][0][ty + TW * a];
#pragma unroll
            for (int b = 0; b < 4; ++b) bv[b] = L.Bs[buf][0][tx + TW * b];
            pk = L.Ps[buf][0];
#pragma unroll 4
            for (int kk = 0; kk < KC; ++kk) {
                const int kn = min(kk + 1, KC - 1);  // the last split reads itself again
                double nav[4], nbv[4];
#pragma unroll
                for (int b = 0; b < 4; ++b) nbv[b] = L.Bs[buf][kn][tx + TW * b];
                const double npk = L.Ps[buf][kn];
#pragma unroll
                for (int a = 0; a < 4; ++a) nav[a] = L.As[buf][kn][ty + TW * a];
                __builtin_amdgcn_sched_barrier(kSchedScalarOnly);
#pragma unroll
                for (int a = 0; a < 4; ++a) {
                    double t[4];
#pragma unroll
                    for (int b = 0; b < 4; ++b) t[b] = fma(pj[a][b], pk, bv[b]);
                    __builtin_amdgcn_sched_barrier(kSchedScalarOnly);
#pragma unroll
                    for (int b = 0; b < 4; ++b) t[b] = t[b] + av[a];
                    __builtin_amdgcn_sched_barrier(kSchedScalarOnly);
#pragma unroll
                    for (int b = 0; b < 4; ++b) best[a][b] = fmin(best[a][b], t[b]);
                    __builtin_amdgcn_sched_barrier(kSchedScalarOnly);
                }
#pragma unroll
                for (int a = 0; a < 4; ++a) av[a] = nav[a];
#pragma unroll
                for (int b = 0; b < 4; ++b) bv[b] = nbv[b];
                pk = npk;
            }
        }
        if (more) store(kc + KC, buf ^ 1);
        __syncthreads();
        buf ^= 1;
    }

    uint64_t *out = part_all + sg.part_off + ((size_t)tile * sg.PT + sg.slot0 + chunk) * T * T;
#pragma unroll
    for (int a = 0; a < 4; ++a) {
#pragma unroll
        for (int b = 0; b < 4; ++b) {
            const int r = ty + TW * a, c = tx + TW * b;
            uint64_t packed = UINT64_MAX;
            if (c < nJ) {
                const double key = best[a][b];
                const double cost = floor(key * inv_scale);
                const int kl = (int)fma(-cost, scale, key);
                packed = ((uint64_t)cost << kbits) | (uint64_t)(k0 + kl);
            }
            out[r * T + c] = packed;
        }
    }
}

// ------------------------------------------------------------------------
// Closure role: one workgroup per tile (I, I+D), D >= 1.
//
// Row group r (CG lanes) owns local row r.  At local anti-diagonal step w
// it finalises cell (r, c), c = w - (T-1-r), from the bulk result and the
// closure splits:
//   (a) q in [r, T-2]:  DI[r][q] + X[q+1][c] + p_i p[row0+q+1] p_{j+1}
//   (b) c' in [0, c-1]: X[r][c'] + DJ[c'+1][c] + p_i p[col0+c'+1] p_{j+1}
// DI[r][.] never changes and X[r][c'] was finalised by this same group, so
// lane g keeps the entries with q = g (mod CG) and c' = g (mod CG) in
// registers (slot t holds index t*CG + g); only X[q+1][c] (other rows) and
// DJ[c'+1][c] come from LDS.  Slots that do not apply hold 2^62 in their
// register operand, so their terms never win and need no select.  The
// rows of wave h use (a) slots >= (h*CROWS)/CG only, so the step body is
// instantiated per first slot.  All LDS reads of a step are issued before
// the first use; the row group's minimum is formed with DPP lane
// permutations; one barrier per step publishes the new cells.
// ------------------------------------------------------------------------
template <int CTRL>
__device__ __forceinline__ double dpp_perm(double v)
{
    const int2 b = __builtin_bit_cast(int2, v);
    int2 o;
    o.x = __builtin_amdgcn_mov_dpp(b.x, CTRL, 0xF, 0xF, false);
    o.y = __builtin_amdgcn_mov_dpp(b.y, CTRL, 0xF, 0xF, false);
    return __builtin_bit_cast(double, o);
}

// Minimum over each aligned group of G lanes (all lanes active).
template <int G>
__device__ __forceinline__ double min_group(double v)
{
    v = fmin(v, dpp_perm<0xB1>(v));                     // quad_perm [1,0,3,2]: lane ^ 1
    v = fmin(v, dpp_perm<0x4E>(v));                     // quad_perm [2,3,0,1]: lane ^ 2
    if constexpr (G >= 8) v = fmin(v, dpp_perm<0x141>(v));   // row_half_mirror: i <-> 7-i
    if constexpr (G >= 16) v = fmin(v, dpp_perm<0x140>(v));  // row_mirror: i <-> 15-i
    return v;
}

template <int T, int G>
struct CloseRegs {
    double DIr[CloseShape<T, G>::CS], PIr[CloseShape<T, G>::CS], PJr[CloseShape<T, G>::CS],
        Xrow[CloseShape<T, G>::CS];
};

// Minimum of v[Lo..Hi) as a balanced tree (Hi > Lo, both compile-time).
template <int Lo, int Hi>
__device__ __forceinline__ double range_min(const double *v)
{
    if constexpr (Hi - Lo == 1) {
        return v[Lo];
    } else {
        constexpr int M = (Lo + Hi) / 2;
        return fmin(range_min<Lo, M>(v), range_min<M, Hi>(v));
    }
}

// One step of a row group: the minimum over its (a) and (b) splits of cell
// (r, cc).  T0: the first (a) slot any row of the wave uses.  A (b) slot
// whose cell is not final yet still holds Xrow = 2^62, so whatever DJ value
// it meets, its term loses.  (Bounding the (b) slots per wave as well, by
// instantiating the step per bound, measured slower: the larger code costs
// more than the skipped slots save.)
template <int T, int G, int T0, class Lds>
__device__ __forceinline__ double close_step(const CloseRegs<T, G> &R, const Lds &L, int xo,
                                             int djb, int g, double pJc)
{
    constexpr int CS = CloseShape<T, G>::CS;
    double xa[CS], xb[CS], va[CS], vb[CS];
    const double *__restrict__ xcol = &L.Xt[0][0] + xo;  // column cc of Xt
#pragma unroll
    for (int t = T0; t < CS; ++t) xa[t] = xcol[t * G + g + 1];
#pragma unroll
    for (int t = 0; t < CS; ++t) xb[t] = L.dj_at_base(djb, t * G + g);
    // Independent terms, then balanced min trees.
#pragma unroll
    for (int t = T0; t < CS; ++t) va[t] = fma(pJc, R.PIr[t], R.DIr[t]) + xa[t];
#pragma unroll
    for (int t = 0; t < CS; ++t) vb[t] = fma(pJc, R.PJr[t], xb[t]) + R.Xrow[t];
    return min_group<G>(fmin(range_min<T0, CS>(va), range_min<0, CS>(vb)));
}

// close_step with its first (a) slot t0 (wave-uniform) as a template
// argument.
template <int T, int G, int T0, class Lds>
__device__ __forceinline__ double close_step_at(int t0, const CloseRegs<T, G> &R, const Lds &L,
                                                int xo, int djb, int g, double pJc)
{
    if constexpr (T0 + 1 < CloseShape<T, G>::CS) {
        if (t0 > T0) return close_step_at<T, G, T0 + 1>(t0, R, L, xo, djb, g, pJc);
    }
    return close_step<T, G, T0>(R, L, xo, djb, g, pJc);
}

// Cells a thread of a 32-edge paired closure moves between global memory
// and the packed LDS tables (column stride 8 mod 16 doubles, so lanes a
// column apart hit 2 banks in 16): the tile in 8 x 8 blocks of 64 flat
// indices, each 16 consecutive indices 2 columns x 8 rows (16 distinct
// banks), a wave's 64 covering 8 consecutive columns of 8 rows (64-byte
// runs in global memory).  Thread tid's u-th cell (index tid + CTH*u, with
// CTH / 64 == T / 8) is (rr0 + 8u, cc0).
template <int T>
__device__ __forceinline__ void blocked_cell(int tid, int &rr0, int &cc0)
{
    const int b = tid >> 6, l = tid & 63, j = l & 15;
    rr0 = ((b / (T / 8)) << 3) + (j >> 1);
    cc0 = ((b % (T / 8)) << 3) + ((l >> 4) << 1) + (j & 1);
}

// OB: the optimal-BST weights (pd_all then holds zeros, so every product
// term vanishes): a cell gains W(i, j) = ob_hi[j] - ob_lo[i] once its
// minimum is known.  pJs then carries ob_hi of the tile's columns.
template <int T, int G, class Lds, bool OB>
__device__ __forceinline__ void close_tile(Lds &L, const TileChain *__restrict__ chains,
                                           const TileSeg *__restrict__ segs, int nseg,
                                           int64_t *__restrict__ m_all,
                                           int32_t *__restrict__ s_all,
                                           const double *__restrict__ pd_all,
                                           const uint64_t *__restrict__ part_all,
                                           const double *__restrict__ ob_hi,
                                           const double *__restrict__ ob_lo)
{
    constexpr int CTH = CloseShape<T, G>::CTH, CS = CloseShape<T, G>::CS;
    constexpr int CROWS = CloseShape<T, G>::CROWS;
    constexpr int CSTR = Lds::CSTR;
    const TileSeg sg = segs[find_seg(segs, nseg, blockIdx.x)];
    const TileChain ch = chains[sg.chain];
    const int local = blockIdx.x - sg.first;
    const int tid = threadIdx.x;
    const int32_t n = ch.n, D = sg.D, PT = sg.PT, kb = ch.kb, kbits = ch.kbits;
    int64_t *__restrict__ m = m_all + ch.m_off;
    int32_t *__restrict__ s = s_all + ch.s_off;
    const double *__restrict__ pd = pd_all + ch.pd_off;
    const uint64_t *__restrict__ part = part_all + sg.part_off;
    const int I = local, J = I + D;
    const int row0 = I * T, col0 = J * T;
    const int nJ = min(T, n - col0);
    const double scale = ldexp(1.0, kb);
    const double inv_scale = ldexp(1.0, -kb);
    const uint64_t kmask = (((uint64_t)1) << kbits) - 1;

    const int r = tid / G, g = tid % G;
    // 32-edge packed tables: prologue and epilogue in blocked cells (the
    // 64-edge ones keep row-major cells: the map cost them registers that
    // two workgroups per CU cannot spare).
    constexpr bool BLK = Lds::kPacked && T == 32;
    static_assert(!BLK || CTH / 64 == T / 8, "blocked cells");
    int rr0 = 0, cc0 = 0;
    if constexpr (BLK) blocked_cell<T>(tid, rr0, cc0);
    const int h = __builtin_amdgcn_readfirstlane(tid / 64);  // rows CROWS*h ..
    // Register operands.  Every load is issued unconditionally (indices
    // clamped into the table) and the slots that do not apply are replaced
    // afterwards, so the prologue -- on the solve's critical path -- waits
    // for memory once instead of once per conditional load.
    CloseRegs<T, G> R;
    const double pi_s = pd[row0 + r] * scale;
    {
        double dm[CS], dpi[CS], dpj[CS];
#pragma unroll
        for (int t = 0; t < CS; ++t) {
            const int q = t * G + g;
            const int qa = min(q, T - 2);
            dm[t] = (double)m[(size_t)(row0 + r) * n + row0 + qa];
            dpi[t] = pd[row0 + qa + 1];
            dpj[t] = pd[col0 + min(q, nJ - 1) + 1];
        }
#pragma unroll
        for (int t = 0; t < CS; ++t) {
            const int q = t * G + g;  // (a) split column q; (b) split column c' = q
            const bool qa = q >= r && q <= T - 2;
            R.DIr[t] = qa ? fma(dm[t], scale, (double)q) : kPad;
            R.PIr[t] = qa ? pi_s * dpi[t] : 0.0;
            R.PJr[t] = q < nJ ? pi_s * dpj[t] : 0.0;
            R.Xrow[t] = kPad;  // until cell (r, q) is final
        }
    }

    if constexpr (OB) {
        for (int q = tid; q <= T; q += CTH)
            L.pJs[q] = q >= 1 && q <= nJ ? ob_hi[col0 + q - 1] : 0.0;
    } else {
        for (int q = tid; q <= T; q += CTH) L.pJs[q] = q <= nJ ? pd[col0 + q] : 0.0;
    }
    const double w_row = OB ? ob_lo[row0 + r] : 0.0;
    {
        double *z = &L.Xt[0][0];
        for (int idx = tid; idx < T * CSTR; idx += CTH) z[idx] = 0.0;
        if constexpr (!Lds::kPacked) {
            double *zd = &L.dj(0, 0);
            for (int idx = tid; idx < T * CSTR; idx += CTH) zd[idx] = 0.0;
        } else {
            double *zd = &L.dj(1, 0);
            for (int idx = tid; idx < dj_packed_size<T>(); idx += CTH) zd[idx] = 0.0;
        }
    }
    __syncthreads();
    // DJ[q][c], 1 <= q <= c < nJ, read row-major (coalesced); every
    // thread's loads are issued together (indices clamped into the table)
    // and only the entries that apply are stored.
    {
        constexpr int DPT = T * T / CTH;  // entries per thread
        double dv[DPT];
#pragma unroll
        for (int u = 0; u < DPT; ++u) {
            const int idx = tid + CTH * u;
            int qq = idx / T, c = idx % T;
            if constexpr (BLK) {
                qq = rr0 + 8 * u;
                c = cc0;
            }
            qq = min(qq, nJ - 1);
            c = min(c, nJ - 1);
            dv[u] = (double)m[(size_t)(col0 + qq) * n + col0 + c];
        }
#pragma unroll
        for (int u = 0; u < DPT; ++u) {
            const int idx = tid + CTH * u;
            const int qq = BLK ? rr0 + 8 * u : idx / T, c = BLK ? cc0 : idx % T;
            if (qq >= 1 && qq <= c && c < nJ) L.dj(qq, c) = fma(dv[u], scale, (double)(T + qq - 1));
        }
    }
    // Bulk result per cell: the minimum of the PT packed (cost << kbits | k)
    // partials, or for D == 1 the single bulk split k = (I+1)T-1 whose
    // operands both lie in the diagonal tiles.
    constexpr int CPT = T * T / CTH;  // cells per thread
    uint64_t key[CPT];
#pragma unroll
    for (int u = 0; u < CPT; ++u) key[u] = UINT64_MAX;
    if (D == 1) {
        const int k = row0 + T - 1;
#pragma unroll
        for (int u = 0; u < CPT; ++u) {
            const int idx = tid + CTH * u;
            const int rr = BLK ? rr0 + 8 * u : idx / T, c = BLK ? cc0 : idx % T;
            if (c < nJ) {
                const int64_t cost = m[(size_t)(row0 + rr) * n + k] +
                                     m[(size_t)(k + 1) * n + col0 + c] +
                                     (int64_t)pd[row0 + rr] * (int64_t)pd[k + 1] *
                                         (int64_t)pd[col0 + c + 1];
                key[u] = ((uint64_t)cost << kbits) | (uint64_t)k;
            }
        }
    } else {
        // SPR slots' loads in flight per round trip (16 loads per thread); a
        // last partial group re-reads its final slot, which changes no
        // minimum.
        constexpr int SPR = 16 / CPT;
        const uint64_t *src = part + ((size_t)I * PT) * T * T;
        for (int sl = 0; sl < PT; sl += SPR) {
            uint64_t v[SPR][CPT];
#pragma unroll
            for (int e = 0; e < SPR; ++e) {
                const size_t so = (size_t)min(sl + e, PT - 1) * T * T;
#pragma unroll
                for (int u = 0; u < CPT; ++u) {
                    if constexpr (BLK) v[e][u] = src[so + (rr0 + 8 * u) * T + cc0];
                    else v[e][u] = src[so + tid + CTH * u];
                }
            }
#pragma unroll
            for (int e = 0; e < SPR; ++e)
#pragma unroll
                for (int u = 0; u < CPT; ++u) key[u] = v[e][u] < key[u] ? v[e][u] : key[u];
        }
    }
#pragma unroll
    for (int u = 0; u < CPT; ++u) {
        const int idx = tid + CTH * u;
        const int rr = BLK ? rr0 + 8 * u : idx / T, c = BLK ? cc0 : idx % T;
        if (c < nJ) {
            L.Xt[c][rr] = fma((double)(int64_t)(key[u] >> kbits), scale, (double)(T - 1));
            L.Ks[rr][c] = (int32_t)(key[u] & kmask);
        }
    }
    __syncthreads();

    // The sweep is the critical path of the solve.  A row's clamped column
    // cc grows by at most one per step the wave runs (those steps are
    // consecutive and the first has every cc = 0), so the packed DJ column
    // base advances by addition instead of its closed form.
    __builtin_amdgcn_s_setprio(3);
    const int wmax = (T - 1) + (nJ - 1);
    int cc_run = 0, djb = 0;
    for (int w = 0; w <= wmax; ++w) {
        const int c = w - (T - 1 - r);
        const int c_lo = w - (T - 1 - CROWS * h);  // c of the wave's first row
        const int c_hi = c_lo + CROWS - 1;         // ... and of its last row
        if (c_hi >= 0 && c_lo < nJ) {              // wave-uniform
            const int cc = min(max(c, 0), nJ - 1);
            const int xo = __mul24(cc, CSTR);  // column cc of Xt
            if constexpr (Lds::kPacked) {
                djb = cc != cc_run ? Lds::dj_next(djb, cc_run) : djb;
                cc_run = cc;
            } else {
                djb = xo;
            }
            const double pJc = L.pJs[cc + 1];
            const double xbulk = (&L.Xt[0][0])[xo + r];
            const double best = close_step_at<T, G, 0>((h * CROWS) / G, R, L, xo, djb, g, pJc);
            const double fin = fmin(best, xbulk);
            const double base = floor(fin * inv_scale);
            const double cost = OB ? base + (pJc - w_row) : base;
            const double xv = cost * scale;
            if (c >= 0 && c < nJ) {
#pragma unroll
                for (int t = 0; t < CS; ++t)
                    if (t * G + g == c) R.Xrow[t] = xv;
                if (g == 0) {
                    (&L.Xt[0][0])[xo + r] = xv;
                    if constexpr (Lds::kFinalKeys) {
                        (&L.Fk[0][0])[xo + r] = fin;  // the split is read off at the end
                    } else {
                        const int kl = (int)fma(-base, scale, fin);
                        if (kl != T - 1) L.Ks[r][c] = ~kl;  // a local split, resolved at the end
                    }
                }
            }
        }
        __syncthreads();
    }

    for (int idx = tid; idx < T * T; idx += CTH) {
        const int rr = BLK ? rr0 + 8 * ((idx - tid) / CTH) : idx / T, c = BLK ? cc0 : idx % T;
        if (c < nJ) {
            const size_t o = (size_t)(row0 + rr) * n + col0 + c;
            m[o] = (int64_t)(L.Xt[c][rr] * inv_scale);
            if constexpr (Lds::kFinalKeys) {
                const double f = L.Fk[c][rr];
                const int kl = (int)fma(-floor(f * inv_scale), scale, f);
                s[o] = kl == T - 1 ? L.Ks[rr][c] : kl < T - 1 ? row0 + kl : col0 + (kl - T);
            } else {
                const int code = L.Ks[rr][c];
                const int kl = ~code;
                s[o] = code >= 0 ? code : kl < T - 1 ? row0 + kl : col0 + (kl - T);
            }
        }
    }
    for (int idx = tid; idx < T * T; idx += CTH) {
        const int c = idx / T, rr = idx % T;
        if (c < nJ) {
            const size_t o = (size_t)(col0 + c) * n + row0 + rr;
            m[o] = (int64_t)(L.Xt[c][rr] * inv_scale);
            s[o] = -1;
        }
    }
}

// Diagonal tiles in row groups (fp64 keys): G lanes own local row r; at
// step d (local diagonal, 1 .. nI-1) the group finalises cell (r, r + d)
// from the splits k in [r, r + d - 1]: X[r][k] (its own row, final at an
// earlier step, kept in registers with k added: lane g holds k = t*G + g in
// slot t) + X[k+1][c] (column c, rows below, from LDS) + p_r p_{k+1}
// p_{c+1}.  Slots whose left cell is not final (k >= c) or not a cell
// (k < r) hold 2^62 and lose.  One barrier per step publishes the new
// cells; the split is read off each cell's final key at the end.  Every
// split is evaluated once per slot, as in the closure, instead of lanes per
// cell and a shuffle tree (k_tri_key's form, kept for launches of many
// 64-edge tiles).
template <int T, int G>
__global__ __launch_bounds__(T * G) void k_tri_rows(const TileChain *__restrict__ chains,
                                                    const TileSeg *__restrict__ segs, int nseg,
                                                    const double *__restrict__ pd_all,
                                                    int64_t *__restrict__ m_all,
                                                    int32_t *__restrict__ s_all)
{
    constexpr int CTH = T * G, CS = T / G, ROWS = 64 / G;  // rows per wave
    // Column stride: odd for 16-lane rows (any stride serves one row group's
    // 16-lane LDS pass; odd also the epilogue's); 8 (mod 16) for 8-lane rows,
    // whose two row groups per pass read adjacent columns.
    constexpr int TS = G == 16 ? T + 1 : T + 8;
    __shared__ double Xt[T][TS];  // Xt[c][q]: final cost * 2^kb of cell (q, c)
    __shared__ double Fk[T][TS];  // Fk[c][q]: its final key (cost * 2^kb + k_local)
    __shared__ double ps[T + 1];
    const int tid = threadIdx.x;
    const TileSeg sg = segs[find_seg(segs, nseg, blockIdx.x)];
    const TileChain ch = chains[sg.chain];
    const int32_t n = ch.n;
    const double *__restrict__ pd = pd_all + ch.pd_off;
    int64_t *__restrict__ m = m_all + ch.m_off;
    int32_t *__restrict__ s = s_all + ch.s_off;
    const double scale = ldexp(1.0, ch.kb), inv_scale = ldexp(1.0, -ch.kb);
    const int base = (blockIdx.x - sg.first) * T;
    const int nI = min(T, n - base);
    const int r = tid / G, g = tid % G;
    const int h = __builtin_amdgcn_readfirstlane(tid / 64);

    for (int q = tid; q <= T; q += CTH) ps[q] = q <= nI ? pd[base + min(q, nI)] : 0.0;
    for (int idx = tid; idx < T * TS; idx += CTH) (&Xt[0][0])[idx] = 0.0;
    __syncthreads();
    // Own-row operands: slot t of lane g is split k = t*G + g.
    double Xk[CS], PR[CS];
    const double pr = ps[r] * scale;
#pragma unroll
    for (int t = 0; t < CS; ++t) {
        const int k = t * G + g;
        Xk[t] = k == r ? (double)k : kPad;  // cell (r, r) costs 0
        PR[t] = pr * ps[min(k + 1, T)];
    }

    for (int d = 1; d < nI; ++d) {
        if (ROWS * h + d < nI) {  // wave-uniform: some row of the wave is active
            const int c = min(r + d, nI - 1);
            const double pc = ps[c + 1];
            const double *__restrict__ col = &Xt[c][0];
            double v[CS];
#pragma unroll
            for (int t = 0; t < CS; ++t) v[t] = fma(PR[t], pc, col[t * G + g + 1]) + Xk[t];
            const double best = min_group<G>(range_min<0, CS>(v));
            const double cost = floor(best * inv_scale);
            const double xv = cost * scale;
            if (r + d < nI) {
#pragma unroll
                for (int t = 0; t < CS; ++t)
                    if (t * G + g == c) Xk[t] = xv + (double)c;
                if (g == 0) {
                    Xt[c][r] = xv;
                    Fk[c][r] = best;
                }
            }
        }
        __syncthreads();
    }

    for (int idx = tid; idx < T * T; idx += CTH) {
        const int rr = idx / T, cc = idx % T;
        if (rr < nI && cc < nI) {
            const size_t o = (size_t)(base + rr) * n + base + cc;
            m[o] = (int64_t)((rr <= cc ? Xt[cc][rr] : Xt[rr][cc]) * inv_scale);
            if (rr < cc) {
                const double f = Fk[cc][rr];
                s[o] = base + (int32_t)fma(-floor(f * inv_scale), scale, f);
            } else {
                s[o] = -1;
            }
        }
    }
}

// One tile per CU (lone chains: the closure is their critical path).
__global__ __launch_bounds__((CloseShape<64, CG_LONE>::CTH)) void k_close(
    const TileChain *__restrict__ chains, const TileSeg *__restrict__ segs, int nseg,
    int64_t *__restrict__ m_all, int32_t *__restrict__ s_all, const double *__restrict__ pd_all,
    const uint64_t *__restrict__ part_all)
{
    __shared__ CloseLdsFull<64> L;
    close_tile<64, CG_LONE, CloseLdsFull<64>, false>(L, chains, segs, nseg, m_all, s_all, pd_all,
                                                     part_all, nullptr, nullptr);
}

// Two tiles per CU (many chains: closure throughput matters); the same
// shape serves the 32-edge tiles of batches of small chains, several per CU:
// held to six waves per SIMD there (at most 80 VGPRs; a few spill around the
// sweep), which measured 3% faster on a batch of 4096 chains than the five
// its 88 VGPRs allowed; seven spilled more and gained nothing.
template <int T>
__global__ __launch_bounds__((CloseShape<T, CG_PAIR>::CTH))
__attribute__((amdgpu_waves_per_eu(T == 32 ? 6 : 1))) void k_close_pair(
    const TileChain *__restrict__ chains, const TileSeg *__restrict__ segs, int nseg,
    int64_t *__restrict__ m_all, int32_t *__restrict__ s_all, const double *__restrict__ pd_all,
    const uint64_t *__restrict__ part_all)
{
    __shared__ CloseLdsPacked<T> L;
    close_tile<T, CG_PAIR, CloseLdsPacked<T>, false>(L, chains, segs, nseg, m_all, s_all, pd_all,
                                                     part_all, nullptr, nullptr);
}

// The same closures with the optimal-BST weights.
__global__ __launch_bounds__((CloseShape<64, CG_LONE>::CTH)) void k_close_ob(
    const TileChain *__restrict__ chains, const TileSeg *__restrict__ segs, int nseg,
    int64_t *__restrict__ m_all, int32_t *__restrict__ s_all, const double *__restrict__ pd_all,
    const uint64_t *__restrict__ part_all, const double *__restrict__ ob_hi,
    const double *__restrict__ ob_lo)
{
    __shared__ CloseLdsFull<64> L;
    close_tile<64, CG_LONE, CloseLdsFull<64>, true>(L, chains, segs, nseg, m_all, s_all, pd_all,
                                                    part_all, ob_hi, ob_lo);
}

// Four waves per SIMD: without the bound the weight terms take it past the
// 128 VGPRs that two workgroups per CU allow.
__global__ __launch_bounds__((CloseShape<64, CG_PAIR>::CTH), 4) void k_close_pair_ob(
    const TileChain *__restrict__ chains, const TileSeg *__restrict__ segs, int nseg,
    int64_t *__restrict__ m_all, int32_t *__restrict__ s_all, const double *__restrict__ pd_all,
    const uint64_t *__restrict__ part_all, const double *__restrict__ ob_hi,
    const double *__restrict__ ob_lo)
{
    __shared__ CloseLdsPacked<64> L;
    close_tile<64, CG_PAIR, CloseLdsPacked<64>, true>(L, chains, segs, nseg, m_all, s_all, pd_all,
                                                      part_all, ob_hi, ob_lo);
}

static_assert(2 * sizeof(CloseLdsPacked<64>) <= 163840, "two paired closures per CU");

// Dynamic LDS requested on top of CloseLdsFull by every lone closure launch,
// so that no bulk workgroup fits beside it on a CU (160 KB per CU): the
// sweep is latency-bound and slows down several-fold next to a bulk
// workgroup.
constexpr size_t kCloseExtraLds =
    163840 - sizeof(CloseLdsFull<64>) - sizeof(BulkLds<64>) + 1024;
static_assert(sizeof(CloseLdsFull<64>) + kCloseExtraLds <= 163840, "closure LDS exceeds a CU");

// ------------------------------------------------------------------------
// Exact int64 arithmetic for chains beyond the fp64 keys' range
// ((n-1) max(p)^3 >= 2^46, up to the int64 limit): the same decomposition,
// chunking and schedule on 64-edge tiles, with costs and splits carried
// apart and compared as (cost, split) pairs.  Every sum formed is a real
// candidate cost (< 2^63 by the host's bound), so nothing can overflow:
// splits that do not apply are skipped, never padded.  The diagonal tiles
// use k_tri<64, false>.  Partial minima take two words per cell: the cost
// block (T*T int64) of a slot, then its split block.
// ------------------------------------------------------------------------
constexpr int WT = 64;

struct BulkLdsWide {
    int64_t As[2][KC][WT + 1];  // m[row0+r][k]
    int64_t Bs[2][KC][WT];      // m[k+1][col0+c]
    uint32_t Ps[2][KC];         // p[k+1] (a dimension: positive int32)
};

// Chains past the fp64 keys' range whose costs still stay below 2^53
// ((n-1) max(p)^3 < 2^53): every cost, product term and partial sum is an
// exact fp64 integer, but no bits remain below the cost for the split, so
// each thread carries the split of its minima beside them (a compare and a
// select more per evaluation than k_bulk; still no integer multiply).  The
// same tiles, chunks and staging as k_bulk; writes the (cost, split) pairs
// of k_bulk_wide, which the int64 closure merges.
__device__ __forceinline__ double cost53(u32x2 x)
{
    // x < 2^53: both halves convert exactly, and so does their sum.
    return fma((double)x.y, 4294967296.0, (double)x.x);
}

__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(3)))
void k_bulk_mid(const TileChain *__restrict__ chains, const TileSeg *__restrict__ segs, int nseg,
                const int64_t *__restrict__ m_all, const double *__restrict__ pd_all,
                int64_t *__restrict__ part_all, int paced, const uint64_t *wait_word,
                uint64_t wait_token, long long wait_ticks)
{
    if (bulk_waiter(wait_word, wait_token, wait_ticks)) return;
    constexpr int T = 64, TW = 16, RA = 16, RB = 4, V = 4;  // 256 threads, as k_bulk<64>
    __shared__ BulkLds<64> L;  // As, Bs: costs; Ps: p[k+1]
    const TileSeg sg = segs[find_seg(segs, nseg, blockIdx.x)];
    const TileChain ch = chains[sg.chain];
    const int local = blockIdx.x - sg.first;
    const int32_t n = ch.n, D = sg.D, KS = sg.KS;
    const int64_t *__restrict__ m = m_all + ch.m_off;
    const double *__restrict__ pd = pd_all + ch.pd_off;
    const int tid = threadIdx.x;
    const int tile = local / sg.nch;
    const int chunk = local - tile * sg.nch;
    const int I = tile, J = tile + D;
    const int row0 = I * T, col0 = J * T;
    const int kbase = (I + 1) * T - 1 + sg.koff;
    const int k0 = kbase + chunk * KS;
    const int kend = min(k0 + KS, kbase + sg.klen);  // exclusive
    const int rounds = (kend - k0 + KC - 1) / KC;
    const int nJ = min(T, n - col0);
    const int tx = tid % TW, ty = tid / TW;

    double pi4[4], pc4[4];
#pragma unroll
    for (int a = 0; a < 4; ++a) pi4[a] = pd[row0 + ty + TW * a];
#pragma unroll
    for (int b = 0; b < 4; ++b) pc4[b] = pd[col0 + min(tx + TW * b, nJ - 1) + 1];
    double pj[4][4], best[4][4];
    int32_t bk[4][4];
#pragma unroll
    for (int a = 0; a < 4; ++a) {
#pragma unroll
        for (int b = 0; b < 4; ++b) {
            pj[a][b] = tx + TW * b < nJ ? pi4[a] * pc4[b] : 0.0;
            best[a][b] = __builtin_inf();
            bk[a][b] = k0;
        }
    }
    // Staging as in k_bulk (same per-thread map, 32-bit offsets on a table
    // under 2 GiB); splits at or past kend are staged from kend-1 and padded
    // with 2^62 on the A side, so they never win.
    const int akk = tid % KC, ar = tid / KC;
    const int bcol = tid % T, bc = min(bcol, nJ - 1), bkk = tid / T;
    const bool narrow = (size_t)n * (size_t)n * sizeof(int64_t) < ((size_t)1 << 31);
    uint32_t oa[V], ob[V];
#pragma unroll
    for (int v = 0; v < V; ++v) {
        oa[v] = (uint32_t)(((size_t)(row0 + ar + RA * v) * n + akk) * sizeof(int64_t));
        ob[v] = (uint32_t)(((size_t)(bkk + RB * v + 1) * n + col0 + bc) * sizeof(int64_t));
    }
    u32x2 ra[V], rb[V];
    double rp = 0.0;
    auto load = [&](int kc) {
        if (kc + KC <= kend && narrow) {
            const char *ba = (const char *)(m + kc);
            const char *bb = (const char *)(m + (size_t)kc * n);
#pragma unroll
            for (int v = 0; v < V; ++v) {
                ra[v] = *(const u32x2 *)(ba + oa[v]);
                rb[v] = *(const u32x2 *)(bb + ob[v]);
            }
        } else {
#pragma unroll
            for (int v = 0; v < V; ++v) {
                const int ka = min(kc + akk, kend - 1);
                ra[v] = __builtin_bit_cast(u32x2, m[(size_t)(row0 + ar + RA * v) * n + ka]);
                const int kb2 = min(kc + bkk + RB * v, kend - 1);
                rb[v] = __builtin_bit_cast(u32x2, m[(size_t)(kb2 + 1) * n + col0 + bc]);
            }
        }
        if (tid < KC) rp = (kc + tid < kend) ? pd[kc + tid + 1] : 0.0;
    };
    auto store = [&](int kc, int buf) {
        const bool full = kc + KC <= kend;
#pragma unroll
        for (int v = 0; v < V; ++v) {
            L.As[buf][akk][ar + RA * v] = (full || kc + akk < kend) ? cost53(ra[v]) : kPad;
            L.Bs[buf][bkk + RB * v][bcol] = cost53(rb[v]);
        }
        if (tid < KC) L.Ps[buf][tid] = rp;
    };

    load(k0);
    store(k0, 0);
    __syncthreads();
    int buf = 0;
    for (int rd = 0; rd < rounds; ++rd) {
        const int kc = k0 + rd * KC;
        const bool more = rd + 1 < rounds;
        if (paced) set_prio(3 - (4 * rd) / rounds);  // as in k_bulk
        if (more) load(kc + KC);
#pragma unroll 4
        for (int kk = 0; kk < KC; ++kk) {
            double av[4], bv[4];
#pragma unroll
            for (int a = 0; a < 4; ++a) av[a] = L.As[buf][kk][ty + TW * a];
#pragma unroll
            for (int b = 0; b < 4; ++b) bv[b] = L.Bs[buf][kk][tx + TW * b];
            const double pk = L.Ps[buf][kk];
            // Splits arrive in increasing k, so a strict < keeps the smallest.
#pragma unroll
            for (int a = 0; a < 4; ++a)
#pragma unroll
                for (int b = 0; b < 4; ++b) {
                    const double v = fma(pj[a][b], pk, bv[b]) + av[a];
                    bk[a][b] = v < best[a][b] ? kc + kk : bk[a][b];
                    best[a][b] = fmin(best[a][b], v);
                }
        }
        if (more) store(kc + KC, buf ^ 1);
        __syncthreads();
        buf ^= 1;
    }

    int64_t *out = part_all + sg.part_off + ((size_t)tile * sg.PT + sg.slot0 + chunk) * 2 * T * T;
#pragma unroll
    for (int a = 0; a < 4; ++a) {
#pragma unroll
        for (int b = 0; b < 4; ++b) {
            const int r = ty + TW * a, c = tx + TW * b;
            out[r * T + c] = c < nJ ? (int64_t)best[a][b] : INT64_MAX;
            out[T * T + r * T + c] = bk[a][b];
        }
    }
}

// PJ32: every dimension is below 2^16, so p_i p_j fits 32 bits and the
// product term p_i p_j p[k+1] is one 32 x 32 -> 64-bit multiply.
template <bool PJ32>
__global__ __launch_bounds__(256) void k_bulk_wide(const TileChain *__restrict__ chains,
                                                  const TileSeg *__restrict__ segs, int nseg,
                                                  const int64_t *__restrict__ m_all,
                                                  const int32_t *__restrict__ p_all,
                                                  int64_t *__restrict__ part_all, int paced,
                                                  const uint64_t *wait_word, uint64_t wait_token,
                                                  long long wait_ticks)
{
    if (bulk_waiter(wait_word, wait_token, wait_ticks)) return;
    constexpr int T = WT, TW = 16, RA = 16, RB = 4, V = 4;
    __shared__ BulkLdsWide L;
    const TileSeg sg = segs[find_seg(segs, nseg, blockIdx.x)];
    const TileChain ch = chains[sg.chain];
    const int local = blockIdx.x - sg.first;
    const int32_t n = ch.n, D = sg.D, KS = sg.KS;
    const int64_t *__restrict__ m = m_all + ch.m_off;
    const int32_t *__restrict__ p = p_all + ch.p_off;
    const int tid = threadIdx.x;
    const int tile = local / sg.nch;
    const int chunk = local - tile * sg.nch;
    const int I = tile, J = tile + D;
    const int row0 = I * T, col0 = J * T;
    const int kbase = (I + 1) * T - 1 + sg.koff;
    const int k0 = kbase + chunk * KS;
    const int kend = min(k0 + KS, kbase + sg.klen);  // exclusive
    const int rounds = (kend - k0 + KC - 1) / KC;
    const int nJ = min(T, n - col0);
    const int tx = tid % TW, ty = tid / TW;

    // Dims loaded together (clamped column indices), as in k_bulk.
    int64_t pi4[4], pc4[4];
#pragma unroll
    for (int a = 0; a < 4; ++a) pi4[a] = p[row0 + ty + TW * a];
#pragma unroll
    for (int b = 0; b < 4; ++b) pc4[b] = p[col0 + min(tx + TW * b, nJ - 1) + 1];
    using PJ = typename std::conditional<PJ32, uint32_t, uint64_t>::type;
    PJ pj[4][4];
    int64_t best[4][4];
    int32_t bk[4][4];
#pragma unroll
    for (int a = 0; a < 4; ++a) {
#pragma unroll
        for (int b = 0; b < 4; ++b) {
            pj[a][b] = tx + TW * b < nJ ? (PJ)(pi4[a] * pc4[b]) : (PJ)0;
            best[a][b] = INT64_MAX;
            bk[a][b] = k0;
        }
    }
    // Staging as in k_bulk; splits at or past kend are staged from kend-1
    // (inside the table) and never evaluated.
    const int akk = tid % KC, ar = tid / KC;
    const int bcol = tid % T, bc = min(bcol, nJ - 1), bkk = tid / T;
    int64_t ra[V], rb[V];
    uint32_t rp = 0;
    auto load = [&](int kc) {
#pragma unroll
        for (int v = 0; v < V; ++v) {
            const int ka = min(kc + akk, kend - 1);
            ra[v] = m[(size_t)(row0 + ar + RA * v) * n + ka];
            const int kb2 = min(kc + bkk + RB * v, kend - 1);
            rb[v] = m[(size_t)(kb2 + 1) * n + col0 + bc];
        }
        if (tid < KC) rp = (uint32_t)p[min(kc + tid, kend - 1) + 1];
    };
    auto store = [&](int buf) {
#pragma unroll
        for (int v = 0; v < V; ++v) {
            L.As[buf][akk][ar + RA * v] = ra[v];
            L.Bs[buf][bkk + RB * v][bcol] = rb[v];
        }
        if (tid < KC) L.Ps[buf][tid] = rp;
    };

    load(k0);
    store(0);
    __syncthreads();
    int buf = 0;
    for (int rd = 0; rd < rounds; ++rd) {
        const int kc = k0 + rd * KC;
        const bool more = rd + 1 < rounds;
        const int kn = min(KC, kend - kc);  // splits of this round (uniform)
        if (paced) set_prio(3 - (4 * rd) / rounds);  // as in k_bulk
        if (more) load(kc + KC);
        for (int kk = 0; kk < kn; ++kk) {
            int64_t av[4], bv[4];
#pragma unroll
            for (int a = 0; a < 4; ++a) av[a] = L.As[buf][kk][ty + TW * a];
#pragma unroll
            for (int b = 0; b < 4; ++b) bv[b] = L.Bs[buf][kk][tx + TW * b];
            // p[k+1] fits 32 bits, so the product term is a 64 x 32-bit
            // multiply, or 32 x 32 with PJ32 (integer multiplies are quarter
            // rate).
            const uint64_t pk = L.Ps[buf][kk];
            // Splits arrive in increasing k, so a strict < keeps the smallest.
#pragma unroll
            for (int a = 0; a < 4; ++a)
#pragma unroll
                for (int b = 0; b < 4; ++b) {
                    const int64_t c = (int64_t)((uint64_t)pj[a][b] * pk) + bv[b] + av[a];
                    if (c < best[a][b]) {
                        best[a][b] = c;
                        bk[a][b] = kc + kk;
                    }
                }
        }
        if (more) store(buf ^ 1);
        __syncthreads();
        buf ^= 1;
    }

    int64_t *out = part_all + sg.part_off + ((size_t)tile * sg.PT + sg.slot0 + chunk) * 2 * T * T;
#pragma unroll
    for (int a = 0; a < 4; ++a) {
#pragma unroll
        for (int b = 0; b < 4; ++b) {
            const int r = ty + TW * a, c = tx + TW * b;
            out[r * T + c] = c < nJ ? best[a][b] : INT64_MAX;
            out[T * T + r * T + c] = bk[a][b];
        }
    }
}

// (cost, split) pair order: the smaller cost, then the smaller split.
__device__ __forceinline__ bool pair_less(int64_t c1, int32_t k1, int64_t c0, int32_t k0)
{
    return c1 < c0 || (c1 == c0 && k1 < k0);
}

template <int CTRL>
__device__ __forceinline__ void dpp_pair_min(int64_t &c, int32_t &k)
{
    const int2 b = __builtin_bit_cast(int2, c);
    int2 o;
    o.x = __builtin_amdgcn_mov_dpp(b.x, CTRL, 0xF, 0xF, false);
    o.y = __builtin_amdgcn_mov_dpp(b.y, CTRL, 0xF, 0xF, false);
    const int32_t ok = __builtin_amdgcn_mov_dpp(k, CTRL, 0xF, 0xF, false);
    const int64_t oc = __builtin_bit_cast(int64_t, o);
    if (pair_less(oc, ok, c, k)) {
        c = oc;
        k = ok;
    }
}

// Minimum of a 64-bit key with the same lane's key in the DPP pattern.
template <int CTRL>
__device__ __forceinline__ int64_t dpp_key_min(int64_t v)
{
    const int2 b = __builtin_bit_cast(int2, v);
    int2 o;
    o.x = __builtin_amdgcn_mov_dpp(b.x, CTRL, 0xF, 0xF, false);
    o.y = __builtin_amdgcn_mov_dpp(b.y, CTRL, 0xF, 0xF, false);
    const int64_t ov = __builtin_bit_cast(int64_t, o);
    return ov < v ? ov : v;
}

struct CloseLdsWide {
    int64_t DJ[WT][WT + 1];  // DJ[c][q] = m[col0+q][col0+c] (1 <= q <= c)
    int64_t X[WT][WT + 1];   // X[c][q]: bulk minimum, then final cost of cell (q, c)
    int32_t K[WT][WT + 1];   // its split
    uint32_t pJ[WT + 1];     // p[col0 + q] (a dimension: positive int32)
};

// The closure of one 64-edge tile on int64: row group r (16 lanes) sweeps
// its row in local anti-diagonal order as in close_tile.  A lane scans its
// (a) splits, then (lane 0) the bulk minimum, then its (b) splits, in
// increasing split order with a strict <, so its pair is the lexicographic
// minimum of its splits; four DPP steps combine the 16 lanes.
// PJ32: as in k_bulk_wide, p_i p[k+1] fits 32 bits and every product term
// is one 32 x 32 -> 64-bit multiply on the sweep's critical path.
// KEYED: every cost is below 2^54, so the sweep carries int64 keys
// cost * 2^7 + k_local as the fp64 closure does (k_local: q for (a) splits,
// T-1 for the bulk, T + c' for (b) splits, increasing with k), and one
// 64-bit min replaces the (cost, split) pair comparison; slots that do not
// apply hold 2^62 (above every key, and two keys plus it stay below 2^63).
template <bool PJ32, bool KEYED>
__global__ __launch_bounds__(1024) void k_close_wide(const TileChain *__restrict__ chains,
                                                    const TileSeg *__restrict__ segs, int nseg,
                                                    int64_t *__restrict__ m_all,
                                                    int32_t *__restrict__ s_all,
                                                    const int32_t *__restrict__ p_all,
                                                    const int64_t *__restrict__ part_all)
{
    constexpr int T = WT, G = 16, CS = T / G, CTH = T * G, CROWS = 64 / G;
    __shared__ CloseLdsWide L;
    const TileSeg sg = segs[find_seg(segs, nseg, blockIdx.x)];
    const TileChain ch = chains[sg.chain];
    const int local = blockIdx.x - sg.first;
    const int tid = threadIdx.x;
    const int32_t n = ch.n, D = sg.D, PT = sg.PT;
    int64_t *__restrict__ m = m_all + ch.m_off;
    int32_t *__restrict__ s = s_all + ch.s_off;
    const int32_t *__restrict__ p = p_all + ch.p_off;
    const int64_t *__restrict__ part = part_all + sg.part_off;
    const int I = local, J = I + D;
    const int row0 = I * T, col0 = J * T;
    const int nJ = min(T, n - col0);
    const int r = tid / G, g = tid % G;
    const int h = __builtin_amdgcn_readfirstlane(tid / 64);

    // Lane g of row r holds the (a) splits q = t*G + g (r <= q <= T-2) and
    // the (b) splits c' = t*G + g.
    using PP = typename std::conditional<PJ32, uint32_t, uint64_t>::type;
    constexpr int KB = 7;                                // key bits below the cost
    constexpr int64_t kKeyPad = (int64_t)1 << 62;
    int64_t DIr[CS], Xrow[CS];
    PP PIr[CS], PJr[CS];
    const int64_t pi = p[row0 + r];
#pragma unroll
    for (int t = 0; t < CS; ++t) {
        const int q = t * G + g;
        const bool qa = q >= r && q <= T - 2;
        const int64_t dm = m[(size_t)(row0 + r) * n + row0 + min(q, T - 2)];
        if constexpr (KEYED)
            DIr[t] = qa ? (dm << KB) + q : kKeyPad;
        else
            DIr[t] = qa ? dm : 0;
        PIr[t] = qa ? (PP)(pi * (int64_t)p[row0 + q + 1]) : (PP)0;
        PJr[t] = q < nJ ? (PP)(pi * (int64_t)p[col0 + q + 1]) : (PP)0;
        Xrow[t] = KEYED ? kKeyPad : 0;
    }
    for (int q = tid; q <= T; q += CTH) L.pJ[q] = q <= nJ ? (uint32_t)p[col0 + q] : 0u;
    if constexpr (KEYED) {
        // Every entry a keyed sweep may read, including those whose terms
        // lose, holds a key below 2^61: no sum can overflow.
        for (int idx = tid; idx < T * (T + 1); idx += CTH) {
            (&L.DJ[0][0])[idx] = 0;
            (&L.X[0][0])[idx] = 0;
        }
        __syncthreads();
    }
    for (int idx = tid; idx < T * T; idx += CTH) {
        const int qq = idx / T, c = idx % T;
        if (qq >= 1 && qq <= c && c < nJ)
            L.DJ[c][qq] = m[(size_t)(col0 + qq) * n + col0 + c] << (KEYED ? KB : 0);
    }
    // Bulk minimum per cell: the lexicographic minimum of the PT partial
    // pairs, or for D == 1 the single split k = (I+1)T-1.
    constexpr int CPT = T * T / CTH;
#pragma unroll
    for (int u = 0; u < CPT; ++u) {
        const int idx = tid + CTH * u;
        const int rr = idx / T, c = idx % T;
        int64_t bc = INT64_MAX;
        int32_t bkk = INT32_MAX;
        if (c < nJ) {
            if (D == 1) {
                const int k = row0 + T - 1;
                bc = m[(size_t)(row0 + rr) * n + k] + m[(size_t)(k + 1) * n + col0 + c] +
                     (int64_t)p[row0 + rr] * (int64_t)p[k + 1] * (int64_t)p[col0 + c + 1];
                bkk = k;
            } else {
                const int64_t *src = part + (size_t)I * PT * 2 * T * T;
                for (int sl = 0; sl < PT; ++sl) {
                    const int64_t pc = src[(size_t)sl * 2 * T * T + idx];
                    const int32_t pk = (int32_t)src[(size_t)sl * 2 * T * T + T * T + idx];
                    if (pair_less(pc, pk, bc, bkk)) {
                        bc = pc;
                        bkk = pk;
                    }
                }
            }
            L.X[c][rr] = KEYED ? (bc << KB) + (T - 1) : bc;
            L.K[c][rr] = bkk;
        }
    }
    __syncthreads();

    __builtin_amdgcn_s_setprio(3);
    const int wmax = (T - 1) + (nJ - 1);
    if constexpr (KEYED) {
        for (int w = 0; w <= wmax; ++w) {
            const int c = w - (T - 1 - r);
            const int c_lo = w - (T - 1 - CROWS * h);
            const int c_hi = c_lo + CROWS - 1;
            if (c_hi >= 0 && c_lo < nJ) {  // wave-uniform
                const int cc = min(max(c, 0), nJ - 1);
                const uint64_t pJc = L.pJ[cc + 1];
                int64_t best = L.X[cc][r];  // the bulk key (every lane of the row)
#pragma unroll
                for (int t = 0; t < CS; ++t) {  // (a) splits
                    const int64_t v = DIr[t] + L.X[cc][t * G + g + 1] +
                                      (int64_t)(((uint64_t)PIr[t] * pJc) << KB);
                    best = v < best ? v : best;
                }
#pragma unroll
                for (int t = 0; t < CS; ++t) {  // (b) splits
                    const int64_t v = Xrow[t] + L.DJ[cc][t * G + g + 1] +
                                      (int64_t)(((uint64_t)PJr[t] * pJc) << KB);
                    best = v < best ? v : best;
                }
                best = dpp_key_min<0xB1>(best);   // lane ^ 1
                best = dpp_key_min<0x4E>(best);   // lane ^ 2
                best = dpp_key_min<0x141>(best);  // i <-> 7 - i
                best = dpp_key_min<0x140>(best);  // i <-> 15 - i
                if (c >= 0 && c < nJ) {
                    const int64_t xv = best >> KB << KB;  // the final cost as a key
                    const int kl = (int)(best - xv);
#pragma unroll
                    for (int t = 0; t < CS; ++t)
                        if (t * G + g == c) Xrow[t] = xv + T + c;
                    if (g == 0) {
                        L.X[c][r] = xv;
                        if (kl != T - 1) L.K[c][r] = kl < T - 1 ? row0 + kl : col0 + (kl - T);
                    }
                }
            }
            __syncthreads();
        }
    }
    for (int w = 0; w <= (KEYED ? -1 : wmax); ++w) {
        const int c = w - (T - 1 - r);
        const int c_lo = w - (T - 1 - CROWS * h);
        const int c_hi = c_lo + CROWS - 1;
        if (c_hi >= 0 && c_lo < nJ) {  // wave-uniform
            const int cc = min(max(c, 0), nJ - 1);
            const uint64_t pJc = L.pJ[cc + 1];
            int64_t best = INT64_MAX;
            int32_t bk = INT32_MAX;
#pragma unroll
            for (int t = 0; t < CS; ++t) {  // (a): k = row0 + q, increasing in t
                const int q = t * G + g;
                if (q >= r && q <= T - 2) {
                    const int64_t v = DIr[t] + L.X[cc][q + 1] + (int64_t)((uint64_t)PIr[t] * pJc);
                    if (v < best) {
                        best = v;
                        bk = row0 + q;
                    }
                }
            }
            if (g == 0) {  // the bulk splits lie between (a) and (b)
                const int64_t v = L.X[cc][r];
                if (v < best) {
                    best = v;
                    bk = L.K[cc][r];
                }
            }
#pragma unroll
            for (int t = 0; t < CS; ++t) {  // (b): k = col0 + c', increasing in t
                const int cp = t * G + g;
                if (cp < cc) {
                    const int64_t v = Xrow[t] + L.DJ[cc][cp + 1] + (int64_t)((uint64_t)PJr[t] * pJc);
                    if (v < best) {
                        best = v;
                        bk = col0 + cp;
                    }
                }
            }
            dpp_pair_min<0xB1>(best, bk);   // lane ^ 1
            dpp_pair_min<0x4E>(best, bk);   // lane ^ 2
            dpp_pair_min<0x141>(best, bk);  // i <-> 7 - i
            dpp_pair_min<0x140>(best, bk);  // i <-> 15 - i
            if (c >= 0 && c < nJ) {
#pragma unroll
                for (int t = 0; t < CS; ++t)
                    if (t * G + g == c) Xrow[t] = best;
                if (g == 0) {
                    L.X[c][r] = best;
                    L.K[c][r] = bk;
                }
            }
        }
        __syncthreads();
    }

    for (int idx = tid; idx < T * T; idx += CTH) {
        const int rr = idx / T, c = idx % T;
        if (c < nJ) {
            const size_t o = (size_t)(row0 + rr) * n + col0 + c;
            m[o] = L.X[c][rr] >> (KEYED ? KB : 0);
            s[o] = L.K[c][rr];
        }
    }
    for (int idx = tid; idx < T * T; idx += CTH) {
        const int c = idx / T, rr = idx % T;
        if (c < nJ) {
            const size_t o = (size_t)(col0 + c) * n + row0 + rr;
            m[o] = L.X[c][rr] >> (KEYED ? KB : 0);
            s[o] = -1;
        }
    }
}

// The same reservation for the int64 closure of a lone chain.
constexpr size_t kCloseWideExtraLds =
    163840 - sizeof(CloseLdsWide) - sizeof(BulkLdsWide) + 1024;
static_assert(sizeof(CloseLdsWide) + kCloseWideExtraLds <= 163840, "closure LDS exceeds a CU");

// A bounded pause (constant-rate wall clock) on the stream it runs on.
__global__ __launch_bounds__(64) void k_delay(long long ticks)
{
    const long long t0 = wall_clock64();
    while (wall_clock64() - t0 < ticks) __builtin_amdgcn_s_sleep(8);
}

// The constant-rate clock's ticks per millisecond.
long long clock_khz_for_device()
{
    int device = 0, khz = 0;
    if (hipGetDevice(&device) != hipSuccess ||
        hipDeviceGetAttribute(&khz, hipDeviceAttributeWallClockRate, device) != hipSuccess ||
        khz <= 0)
        khz = 100000;
    return khz;
}

// Ticks of a pause (launch_delay): about 4 microseconds.
long long delay_ticks_for_device() { return clock_khz_for_device() * 4 / 1000; }

// Bound of an end-block launch's wait for an interior token: 2 seconds,
// far beyond any interior (the wait ends when the token lands).
long long wait_ticks_for_device() { return clock_khz_for_device() * 2000; }

}  // namespace

mcm_status launch_delay(hipStream_t stream)
{
    hipLaunchKernelGGL(k_delay, dim3(1), dim3(64), 0, stream, delay_ticks_for_device());
    return hipGetLastError() == hipSuccess ? MCM_OK : MCM_ERR_DEVICE;
}

namespace {

// ------------------------------------------------------------------------
// Host planning.
// ------------------------------------------------------------------------
int32_t bitlen_u64(uint64_t v)
{
    int32_t b = 0;
    while (v) {
        ++b;
        v >>= 1;
    }
    return b;
}

double tri_evals(int32_t n, int32_t NT, int32_t T)
{
    double ev = 0.0;
    for (int32_t I = 0; I < NT; ++I) {
        const double nI = (double)((n - I * T) < T ? (n - I * T) : T);
        ev += (nI * nI * nI - nI) / 6.0;
    }
    return ev;
}

// Valid cells of the NT - D tiles of tile-diagonal D (the last tile column
// may be ragged).
double diag_cells(int32_t n, int32_t NT, int32_t D, int32_t T)
{
    const int32_t nlast = n - (NT - 1) * T;
    return (double)(NT - D - 1) * T * T + (double)T * nlast;
}

}  // namespace

namespace {
// Estimated duration, in split units, of `units` equal workgroups of `ks`
// splits each on `slots` resident workgroup slots: whole waves of
// workgroups, each paying about one staged round of fixed cost.
// When a lone chain's closure CUs take up bulk work again, in split times
// of a bulk workgroup.  The sweep itself takes about 250 of them; 192
// (tier-2 chunks planned to start somewhat early, so somewhat longer)
// measured best, 2.2% faster at n = 8192 than 256, with 224 within noise
// and 128 3% slower.
constexpr int32_t kCloseSplits = 192;

// Lone chains (two streams): where the interior of E is expected to end
// before the end blocks of E (the first and last tile-diagonals), the
// closure of E does not wait for it with a stream wait (a runtime kernel
// between two kernel boundaries, about 11 us): one extra workgroup of the
// end-block launch waits for the interior's token instead, and the end
// blocks' chunks fit the whole device (the interior no longer holds CUs).
// In the middle tile-diagonals the interior is the longer branch, and the
// next interior waits for the end-block launch, so there the stream wait
// stays.  The estimate: bulk at about 2.9e4 split evaluations per us on each
// CU it holds, a closure sweep of about 80 us (exact int64 kernels: 1.6e4
// and 130 us), and about 14 us from the interior's end to its token.
constexpr double kBulkEvalsPerUsCu = 2.9e4;
constexpr double kSweepUs = 80.0;
constexpr double kWideBulkEvalsPerUsCu = 1.6e4;
constexpr double kWideSweepUs = 130.0;
constexpr double kTokenHopUs = 14.0;

bool interior_ends_first(int32_t T, int32_t tiles, int32_t E, int held, int free_cus, bool wide)
{
    if (E < 3 || held <= 0 || free_cus <= 0) return false;
    const double rate = wide ? kWideBulkEvalsPerUsCu : kBulkEvalsPerUsCu;
    const double sweep = wide ? kWideSweepUs : kSweepUs;
    const double cells = (double)tiles * T * T;
    const double t_int = cells * ((E - 3) * T + 1) / (rate * (double)free_cus);
    const double t_end = cells * (2.0 * T) / (rate * (double)held);
    return t_int + kTokenHopUs < sweep + t_end;
}

double wave_cost(int64_t units, int32_t ks, int64_t slots)
{
    const int64_t waves = (units + slots - 1) / slots;
    return (double)waves * (double)(ks + KC);
}

}  // namespace

BulkLayout bulk_layout(int32_t T, int32_t NT, int32_t E, int32_t kb, bool lone, int cus,
                       int slots_per_cu, bool serial, bool wide)
{
    BulkLayout bl{};
    if (E < 2 || E >= NT) return bl;
    const int32_t tiles = NT - E;
    int32_t cap = kb >= 30 ? (1 << 30) : (1 << kb);
    cap = cap / KC * KC;
    const bool fit = lone && cus >= 64 && slots_per_cu > 0;
    int64_t slots_int = 0, slots_end = 0;
    if (fit && serial) {
        // Serial schedule: every launch has the whole device.
        slots_int = slots_end = (int64_t)slots_per_cu * cus;
    } else if (fit) {
        // The closure of E-1 holds one CU per tile (NT-E+1) while the
        // interior runs; the end blocks follow the closure on those CUs.
        int64_t held = NT - E + 1;
        if (held > cus - cus / 4) held = cus - cus / 4;
        slots_int = (int64_t)slots_per_cu * (cus - held);
        slots_end = (int64_t)slots_per_cu * held;
        bl.fold = T == 64 && interior_ends_first(T, tiles, E, (int)held, (int)(cus - held), wide);
    }
    // The end blocks' slots: the closure's CUs, or the whole device once the
    // interior is expected to be done (fold).
    const int64_t slots_endblk = bl.fold ? (int64_t)slots_per_cu * cus : slots_end;
    // End blocks: E == 2 has a single range of T+1 splits, E >= 3 two of T.
    const int32_t end_len = E == 2 ? T + 1 : T;
    bl.n_end_ranges = E == 2 ? 1 : 2;
    int32_t end_ks = (end_len + KC - 1) / KC * KC;  // one chunk per range
    if (fit) {
        double best = 0.0;
        for (int32_t ks = KC; ks <= end_len + KC - 1; ks += KC) {
            const int32_t nch = (end_len + ks - 1) / ks;
            const double c = wave_cost((int64_t)tiles * bl.n_end_ranges * nch, ks, slots_endblk);
            if (ks == KC || c < best) {
                best = c;
                end_ks = ks;
            }
        }
    }
    // A lone chain's end blocks run on the closure's CUs right after it,
    // one or two workgroups per CU: chunks of at most 32 splits halve each
    // workgroup's latency-bound run (measured faster than the model's pick
    // of one 64-split chunk per range).
    if (fit && !serial && end_ks > 2 * KC) end_ks = 2 * KC;
    if (end_ks > cap) end_ks = cap;
    bl.end_ks = end_ks;
    bl.end_nch = (end_len + end_ks - 1) / end_ks;
    // Interior, E >= 3: (E-3)T + 1 splits.
    if (E >= 3) {
        const int32_t L = (E - 3) * T + 1;
        int32_t ks = (L + KC - 1) / KC * KC;
        if (fit) {
            // Chunks per tile (at most 32 partial slots) that minimise the
            // estimated duration on the interior's slots.
            double best = 0.0;
            // Where the interior has slack (fold), chunks of at least 192
            // splits: a short interior cut finer than that ran slower (and
            // left more partial minima for the closure to merge).
            int32_t most = kMaxChunks;
            if (bl.fold && L / 192 < most) most = L / 192 > 1 ? L / 192 : 1;
            for (int32_t want = 1; want <= most && (want - 1) * KC < L; ++want) {
                int32_t k = (L + want - 1) / want;
                k = (k + KC - 1) / KC * KC;
                const int32_t nch = (L + k - 1) / k;
                const double c = wave_cost((int64_t)tiles * nch, k, slots_int);
                if (want == 1 || c < best) {
                    best = c;
                    ks = k;
                }
            }
        }
        if (ks > cap) ks = cap;
        bl.int_ks = ks;
        bl.int_nch = (L + ks - 1) / ks;
        bl.int_len = L;
        if (fit && !serial) {
            // Alternative: one wave of long chunks on the interior's slots,
            // then short chunks that start on the closure's CUs once the
            // closure is done (kCloseSplits); both tiers should end
            // together.  The short tier gets one and a third chunks per
            // closure-CU slot: those slots also run the end blocks, which
            // are short, and a queue a third deep keeps them busy after.
            // (Half a chunk per slot, the first choice, left the closure
            // CUs idle for most of a middle tile-diagonal's interior:
            // 17.5 -> 16.9 ms at n = 8192 with this and kCloseSplits.)
            const double single = wave_cost((int64_t)tiles * bl.int_nch, ks, slots_int);
            const int64_t nb64 = slots_int / tiles;
            const int64_t ns64 = (slots_end + slots_end / 3) / tiles;
            const int32_t nb = (int32_t)(nb64 < kMaxChunks ? nb64 : kMaxChunks);
            const int32_t ns = (int32_t)(ns64 < kMaxChunks - nb ? ns64 : kMaxChunks - nb);
            if (nb >= 1 && ns >= 1) {
                const int32_t xs = (L - nb * kCloseSplits) / (nb + ns) / KC * KC;
                if (xs >= 2 * KC && xs <= cap) {
                    const int32_t lb = L - ns * xs;
                    const int32_t xb = ((lb + nb - 1) / nb + KC - 1) / KC * KC;
                    const double two = xb + KC > kCloseSplits + xs + KC ? xb + KC
                                                                         : kCloseSplits + xs + KC;
                    if (xb <= cap && two < single) {
                        bl.int_ks = xb;
                        bl.int_nch = (lb + xb - 1) / xb;
                        bl.int_len = lb;
                        bl.int2_ks = xs;
                        bl.int2_nch = ns;
                    }
                }
            }
        }
    }
    bl.PT = bl.int_nch + bl.int2_nch + bl.n_end_ranges * bl.end_nch;
    bl.elems = (size_t)tiles * bl.PT * T * T;
    return bl;
}

BulkLayout bulk_layout_chunks(int32_t T, int32_t NT, int32_t E, int32_t kb, int32_t nch)
{
    BulkLayout bl = bulk_layout(T, NT, E, kb, false);
    if (E < 3 || E >= NT) return bl;
    const int32_t L = (E - 3) * T + 1;
    int32_t cap = kb >= 30 ? (1 << 30) : (1 << kb);
    cap = cap / KC * KC;
    int32_t most = (L + 63) / 64;
    if (most > kMaxChunks) most = kMaxChunks;
    if (nch > most) nch = most;
    if (nch < 1) nch = 1;
    int32_t ks = ((L + nch - 1) / nch + KC - 1) / KC * KC;
    if (ks > cap) ks = cap;
    bl.int_ks = ks;
    bl.int_nch = (L + ks - 1) / ks;
    bl.int_len = L;
    bl.int2_ks = bl.int2_nch = 0;
    bl.PT = bl.int_nch + bl.n_end_ranges * bl.end_nch;
    bl.elems = (size_t)(NT - E) * bl.PT * T * T;
    return bl;
}

size_t bulk_part_max(int32_t T, int32_t NT, int32_t kb)
{
    size_t most = 0;
    for (int32_t E = 2; E < NT; ++E) {
        const size_t e = bulk_layout_chunks(T, NT, E, kb, kMaxChunks).elems;
        if (e > most) most = e;
    }
    return most;
}

int bulk_blocks_per_cu()
{
    int device = 0;
    if (hipGetDevice(&device) != hipSuccess) return 0;
    static std::mutex mu;
    static std::unordered_map<int, int> cache;
    std::lock_guard<std::mutex> lk(mu);
    int &nb = cache[device];
    if (nb == 0 && hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, k_bulk<64>,
                                                                 bulk_threads<64>(), 0) !=
                       hipSuccess)
        nb = 0;
    return nb;
}

bool tiled_accepts(const ChainInfo &ci)
{
    const int32_t kbits = bitlen_u64((uint64_t)(ci.n > 1 ? ci.n - 1 : 1));
    return ci.cost_bits + 7 <= 53 && ci.cost_bits + kbits <= 64;
}

int32_t tiled_nt(int32_t n, int32_t T) { return (n + T - 1) / T; }

int plan_add_chain(TiledPlan &plan, const ChainInfo &ci, int64_t m_off, int64_t s_off,
                   int64_t p_off, int64_t pd_off)
{
    TileChain c{};
    c.m_off = m_off;
    c.s_off = s_off;
    c.p_off = p_off;
    c.pd_off = pd_off;
    c.n = ci.n;
    // fp64 keys: bits below the cost.  The int64 kernels carry splits apart,
    // so a chunk's split count is not bounded by key bits there.
    c.kb = plan.wide ? 30 : 53 - ci.cost_bits;
    if (!plan.wide && c.kb > 20) c.kb = 20;
    c.kbits = bitlen_u64((uint64_t)(ci.n > 1 ? ci.n - 1 : 1));
    if (ci.pmax > plan.pmax) plan.pmax = ci.pmax;
    if (ci.cost_bits > plan.cost_bits) plan.cost_bits = ci.cost_bits;
    plan.chains.push_back(c);
    plan.NT.push_back(tiled_nt(ci.n, plan.T));
    return (int)plan.chains.size() - 1;
}

// The end blocks carry the closure's wait for the interior beside them
// where the layout expects the interior to end first (BulkLayout::fold).
bool fold_closure_wait(const TiledPlan &plan, const std::vector<ChainStep> &steps)
{
    if (!plan.lone || plan.serial || plan.T != 64) return false;
    bool any = false;
    for (const ChainStep &cs : steps) {
        const int E = cs.D + 1, NT = plan.NT[cs.chain];
        if (cs.D < 1 || E < 3 || E >= NT) continue;
        if (!cs.next.fold) return false;
        any = true;
    }
    return any;
}

void plan_add_iteration(TiledPlan &plan, const std::vector<ChainStep> &steps)
{
    const int32_t T = plan.T;
    auto push = [&](TiledLaunch L, int wait) {
        L.wait = wait;
        if (wait >= 0) plan.launches[wait].record = true;
        plan.launches.push_back(L);
        const int idx = (int)plan.launches.size() - 1;
        if (L.stream == 0) plan.last_main = idx;
        else plan.uses_aux = true;
        return idx;
    };
    // Diagonal tiles of chains starting now (main stream).
    TiledLaunch tri{TK_TRI, (int)plan.segs.size(), 0, 0, 0.0};
    for (const ChainStep &cs : steps) {
        if (cs.D != 0) continue;
        TileSeg sg{};
        sg.first = tri.blocks;
        sg.chain = cs.chain;
        plan.segs.push_back(sg);
        tri.nseg += 1;
        tri.blocks += plan.NT[cs.chain];
        tri.evals += tri_evals(plan.chains[cs.chain].n, plan.NT[cs.chain], T);
    }
    if (tri.nseg) push(tri, -1);

    // Closure of D (main stream), after the interior bulk of D (aux stream,
    // previous iteration).
    TiledLaunch close{TK_CLOSE, (int)plan.segs.size(), 0, 0, 0.0};
    for (const ChainStep &cs : steps) {
        const int c = cs.chain, D = cs.D, NT = plan.NT[c];
        if (D < 1 || D >= NT) continue;
        const int32_t n = plan.chains[c].n;
        const BulkLayout &bl = cs.cur;
        TileSeg sg{};
        sg.part_off = cs.part_cur;
        sg.first = close.blocks;
        sg.chain = c;
        sg.D = D;
        sg.role = SEG_CLOSE;
        sg.PT = bl.PT;
        plan.segs.push_back(sg);
        close.nseg += 1;
        close.blocks += NT - D;
        // (a) and (b) splits of every cell, plus the single bulk split of
        // D == 1: per tile sum over cells of (T-1-r) + c.
        const int32_t nlast = n - (NT - 1) * T;
        const double per_full = (double)T * T * (T - 1);
        const double per_last =
            (double)nlast * T * (T - 1) / 2.0 + (double)T * nlast * (nlast - 1) / 2.0;
        close.evals += (double)(NT - D - 1) * per_full + per_last;
        if (D == 1) close.evals += diag_cells(n, NT, D, T);
    }
    // The interior bulk of D+1 needs the closure of D-1, complete once the
    // launches before this closure on the caller's stream are.
    const int before_close = plan.last_main;
    if (close.nseg) plan.last_close = push(close, plan.last_interior);
    plan.last_interior = -1;

    auto add_bulk = [&](TiledLaunch &Lc, const ChainStep &cs, int E, int koff, int klen, int KS,
                        int nch, int slot0, int PT) {
        const int c = cs.chain, NT = plan.NT[c];
        TileSeg sg{};
        sg.part_off = cs.part_next;
        sg.first = Lc.blocks;
        sg.chain = c;
        sg.D = E;
        sg.role = SEG_BULK;
        sg.KS = KS;
        sg.nch = nch;
        sg.koff = koff;
        sg.klen = klen;
        sg.slot0 = slot0;
        sg.PT = PT;
        plan.segs.push_back(sg);
        Lc.nseg += 1;
        Lc.blocks += (NT - E) * nch;
        Lc.evals += diag_cells(plan.chains[c].n, NT, E, T) * klen;
    };
    // Interior bulk of D+1 (aux stream): needs tile-diagonals <= D-1 only,
    // so it waits for the previous closure, not this one.
    TiledLaunch inter{TK_BULK, (int)plan.segs.size(), 0, 0, 0.0};
    inter.stream = 1;
    for (const ChainStep &cs : steps) {
        const int c = cs.chain, E = cs.D + 1, NT = plan.NT[c];
        if (cs.D < 1 || E < 3 || E >= NT) continue;
        const BulkLayout &bl = cs.next;
        add_bulk(inter, cs, E, T, bl.int_len, bl.int_ks, bl.int_nch, 0, bl.PT);
        if (bl.int2_nch)
            add_bulk(inter, cs, E, T + bl.int_len, (E - 3) * T + 1 - bl.int_len, bl.int2_ks,
                     bl.int2_nch, bl.int_nch, bl.PT);
    }
    // The interior starts after the launch before the closure (an event
    // wait on the aux stream, whose own latency already lets the closure's
    // workgroups reach their CUs first; a further pause measured slower).
    if (inter.nseg) plan.last_interior = push(inter, before_close);

    // End blocks of D+1 (main stream, after the closure of D).
    TiledLaunch ends{TK_BULK, (int)plan.segs.size(), 0, 0, 0.0};
    for (const ChainStep &cs : steps) {
        const int c = cs.chain, E = cs.D + 1, NT = plan.NT[c];
        if (cs.D < 1 || E < 2 || E >= NT) continue;
        const BulkLayout &bl = cs.next;
        if (E == 2) {
            add_bulk(ends, cs, E, 0, T + 1, bl.end_ks, bl.end_nch, bl.int_nch + bl.int2_nch,
                     bl.PT);
        } else {
            const int32_t s0 = bl.int_nch + bl.int2_nch;
            add_bulk(ends, cs, E, 0, T, bl.end_ks, bl.end_nch, s0, bl.PT);
            add_bulk(ends, cs, E, (E - 2) * T + 1, T, bl.end_ks, bl.end_nch, s0 + bl.end_nch,
                     bl.PT);
        }
    }
    if (ends.nseg && plan.last_interior >= 0 && fold_closure_wait(plan, steps))
        ends.fold = plan.last_interior;
    if (ends.nseg) push(ends, -1);
}

void plan_lockstep(TiledPlan &plan, const std::vector<int> &ids)
{
    // Two partial buffers, by parity of the tile-diagonal they hold.  In
    // lockstep every chain with NT > E writes its layout of E in the
    // iteration before E and reads it in iteration E, always in plan order,
    // so positional offsets agree between writer and reader.
    int maxNT = 0;
    for (int c : ids) maxNT = plan.NT[c] > maxNT ? plan.NT[c] : maxNT;
    // Layouts depend on (NT, kb) only: compute each once (many chains of a
    // batch share them).
    std::unordered_map<int64_t, std::vector<BulkLayout>> cache;
    auto layouts = [&](int c) -> const std::vector<BulkLayout> & {
        const int NT = plan.NT[c], kb = plan.chains[c].kb;
        std::vector<BulkLayout> &v = cache[(int64_t)NT * 64 + kb];
        if (v.empty()) {
            v.resize((size_t)NT + 1);
            for (int E = 0; E <= NT; ++E) {
                if (plan.chunk_target > 0) {
                    const int tiles = NT - E > 1 ? NT - E : 1;
                    int nch = plan.chunk_target / tiles;
                    nch = nch < 1 ? 1 : (nch > kMaxChunks ? kMaxChunks : nch);
                    v[E] = bulk_layout_chunks(plan.T, NT, E, kb, nch);
                } else {
                    v[E] = bulk_layout(plan.T, NT, E, kb, plan.lone, plan.cus,
                                       plan.slots_per_cu, plan.serial, plan.wide);
                }
            }
        }
        return v;
    };
    std::vector<const std::vector<BulkLayout> *> lay(ids.size());
    for (size_t u = 0; u < ids.size(); ++u) lay[u] = &layouts(ids[u]);
    // The int64 kernels keep two words (cost, split) per partial minimum.
    const size_t words = plan.wide ? 2 : 1;
    auto elems = [&](size_t u, int E) {
        return E < (int)lay[u]->size() ? words * (*lay[u])[E].elems : (size_t)0;
    };
    size_t half = 0;
    for (int E = 2; E < maxNT; ++E) {
        size_t used = 0;
        for (size_t u = 0; u < ids.size(); ++u) used += elems(u, E);
        if (used > half) half = used;
    }
    plan.part_elems = 2 * half;
    std::vector<ChainStep> steps;
    steps.reserve(ids.size());
    for (int D = 0; D < maxNT; ++D) {
        size_t used_cur = 0, used_next = 0;
        steps.clear();
        for (size_t u = 0; u < ids.size(); ++u) {
            const int c = ids[u];
            const size_t oc = used_cur, on = used_next;
            used_cur += elems(u, D);
            used_next += elems(u, D + 1);
            if (D >= plan.NT[c]) continue;
            ChainStep cs;
            cs.chain = c;
            cs.D = D;
            cs.part_cur = (int64_t)((D & 1) * half + oc);
            cs.part_next = (int64_t)(((D + 1) & 1) * half + on);
            cs.cur = (*lay[u])[D];
            cs.next = (*lay[u])[D + 1];
            steps.push_back(cs);
        }
        plan_add_iteration(plan, steps);
    }
}

size_t plan_tables_bytes(const TiledPlan &plan, size_t *seg_offset)
{
    const size_t cbytes = plan.chains.size() * sizeof(TileChain);
    const size_t soff = (cbytes + 255) / 256 * 256;
    if (seg_offset) *seg_offset = soff;
    return soff + plan.segs.size() * sizeof(TileSeg);
}

void plan_tables_write(const TiledPlan &plan, char *dst)
{
    size_t soff = 0;
    plan_tables_bytes(plan, &soff);
    memcpy(dst, plan.chains.data(), plan.chains.size() * sizeof(TileChain));
    memcpy(dst + soff, plan.segs.data(), plan.segs.size() * sizeof(TileSeg));
}

mcm_status run_tiled_plan(const TiledPlan &plan, const int32_t *p, const double *pd,
                          int64_t *m_all, int32_t *s_all, uint64_t *part_ext, hipStream_t stream,
                          const ObstWeights *ob)
{
    if (plan.launches.empty()) return MCM_OK;
    // One device block: chain table, then segment table.
    size_t soff = 0;
    const size_t bytes = plan_tables_bytes(plan, &soff);
    void *tables = nullptr;
    mcm_status st =
        upload_blob(stream, &tables, bytes, [&](char *dst) { plan_tables_write(plan, dst); });
    if (st != MCM_OK) return st;
    st = exec_tiled_plan(plan, (const TileChain *)tables,
                         (const TileSeg *)((const char *)tables + soff), p, pd, m_all, s_all,
                         part_ext, stream, ob);
    ws_free(tables, stream);
    return st;
}

namespace {
// A launch whose completion `stop` (if not null) records: the event is the
// dispatch's own completion, with no marker packet after it.
template <typename K, typename... A>
void launch_with_stop(K kernel, unsigned blocks, unsigned threads, hipStream_t q, hipEvent_t stop,
                      A... args)
{
    if (stop)
        hipExtLaunchKernelGGL(kernel, dim3(blocks), dim3(threads), 0, q, nullptr, stop, 0u,
                              args...);
    else
        hipLaunchKernelGGL(kernel, dim3(blocks), dim3(threads), 0, q, args...);
}
}  // namespace

mcm_status exec_tiled_plan(const TiledPlan &plan, const TileChain *chains, const TileSeg *segs,
                           const int32_t *p, const double *pd, int64_t *m_all, int32_t *s_all,
                           uint64_t *part_ext, hipStream_t stream, const ObstWeights *ob,
                           int pair_min_blocks, hipStream_t aux_stream, bool events_only)
{
    if (plan.launches.empty()) return MCM_OK;
    mcm_status st = MCM_OK;
    uint64_t *part = part_ext;
    uint64_t *part_own = nullptr;
    if (!part && plan.part_elems) {
        if (ws_alloc((void **)&part_own, plan.part_elems * sizeof(uint64_t), stream) !=
            hipSuccess)
            return MCM_ERR_NO_MEMORY;
        part = part_own;
    }
    int nrec = 0;
    for (const TiledLaunch &L : plan.launches) nrec += L.record ? 1 : 0;
    const bool aux = plan.uses_aux;
    // Events: one per launch another launch waits for, plus fork and join.
    StreamSet ss;
    if (aux && acquire_streams(nrec + 2, &ss) != MCM_OK) st = MCM_ERR_DEVICE;
    hipStream_t lib_aux = ss.aux;
    if (aux && aux_stream) ss.aux = aux_stream;
    std::vector<hipEvent_t> rec(plan.launches.size(), nullptr);
    // Aux launches the caller's stream waits for hand over a signal token
    // instead of an event when the device has a signal word (a stream wait
    // on a value is a shorter hop than an event wait).
    std::vector<uint64_t> tok(plan.launches.size(), 0);
    // Aux launches whose token a launch on the caller's stream already
    // waited for in-kernel (TiledLaunch::fold): later launches on that
    // stream need no stream wait for them.
    std::vector<char> folded(plan.launches.size(), 0);
    int next_ev = 2;
    bool forked = false;
    if (aux && st == MCM_OK) {
        // Fork: the aux stream starts after everything already on `stream`
        // (the tables upload, and earlier work of the caller).
        if (hipEventRecord(ss.events[0], stream) != hipSuccess ||
            hipStreamWaitEvent(ss.aux, ss.events[0], 0) != hipSuccess)
            st = MCM_ERR_DEVICE;
        forked = st == MCM_OK;
    }
    const int cus = device_cus();
    // Under stream capture a launch's stop event does not become a graph
    // dependency, so captured plans record their events as markers.
    hipStreamCaptureStatus capture = hipStreamCaptureStatusNone;
    if (hipStreamIsCapturing(stream, &capture) != hipSuccess) capture = hipStreamCaptureStatusActive;
    const bool own_events = capture == hipStreamCaptureStatusNone;
    for (size_t li = 0; li < plan.launches.size() && st == MCM_OK; ++li) {
        const TiledLaunch &L = plan.launches[li];
        hipStream_t q = L.stream == 1 ? ss.aux : stream;
        hipError_t e = hipSuccess;
        if (L.wait >= 0 && plan.launches[L.wait].stream != L.stream && !folded[L.wait])
            e = tok[L.wait] ? aux_signal_wait(q, tok[L.wait])
                            : hipStreamWaitEvent(q, rec[L.wait], 0);
        if (e != hipSuccess) {
            st = MCM_ERR_DEVICE;
            break;
        }
        const TileSeg *sg = segs + L.seg_begin;
        // Bulk launches.  End blocks (fold): one extra workgroup waits for
        // the interior's token.  End blocks the next interior waits for:
        // the event is the launch's own completion, so no marker packet
        // sits between it and the closure after it on this stream (about
        // 7 us on that path at the first and last tile-diagonals).
        const uint64_t *ww = nullptr;
        uint64_t wt = 0;
        hipEvent_t stop = nullptr;
        if (L.kind == TK_BULK) {
            if (L.fold >= 0 && L.stream == 0 && plan.launches[L.fold].stream == 1 &&
                tok[L.fold] && plan.T == 64) {
                ww = aux_signal_word();
                wt = ww ? tok[L.fold] : 0;
            }
            if (own_events && aux && L.record && L.stream == 0) {
                rec[li] = ss.events[next_ev++];
                stop = rec[li];
            }
        }
        const long long wticks = ww ? wait_ticks_for_device() : 0LL;
        const unsigned bblocks = (unsigned)L.blocks + (ww ? 1u : 0u);
        if (plan.wide) {
            ProfileScope ps(L.kind == TK_TRI ? KC_SETUP : L.kind == TK_BULK ? KC_BULK : KC_CLOSE,
                            q, L.evals);
            if (L.kind == TK_TRI)
                hipLaunchKernelGGL((k_tri<64, false>), dim3(L.blocks), dim3(NTH), 0, q, chains,
                                   sg, L.nseg, p, m_all, s_all, nullptr, nullptr, nullptr);
            else if (L.kind == TK_BULK && plan.cost_bits <= 53)
                launch_with_stop(k_bulk_mid, bblocks, 256, q, stop, chains, sg, L.nseg, m_all, pd,
                                 (int64_t *)part, plan.lone ? 1 : 0, ww, wt, wticks);
            else if (L.kind == TK_BULK && plan.pmax < 65536)
                launch_with_stop(k_bulk_wide<true>, bblocks, 256, q, stop, chains, sg, L.nseg,
                                 m_all, p, (int64_t *)part, plan.lone ? 1 : 0, ww, wt, wticks);
            else if (L.kind == TK_BULK)
                launch_with_stop(k_bulk_wide<false>, bblocks, 256, q, stop, chains, sg, L.nseg,
                                 m_all, p, (int64_t *)part, plan.lone ? 1 : 0, ww, wt, wticks);
            else if (plan.cost_bits <= 54 && plan.pmax < 65536)
                hipLaunchKernelGGL((k_close_wide<true, true>), dim3(L.blocks), dim3(1024),
                                   plan.lone ? kCloseWideExtraLds : 0, q, chains, sg, L.nseg,
                                   m_all, s_all, p, (const int64_t *)part);
            else if (plan.cost_bits <= 54)
                hipLaunchKernelGGL((k_close_wide<false, true>), dim3(L.blocks), dim3(1024),
                                   plan.lone ? kCloseWideExtraLds : 0, q, chains, sg, L.nseg,
                                   m_all, s_all, p, (const int64_t *)part);
            else if (plan.pmax < 65536)
                hipLaunchKernelGGL((k_close_wide<true, false>), dim3(L.blocks), dim3(1024),
                                   plan.lone ? kCloseWideExtraLds : 0, q, chains, sg, L.nseg,
                                   m_all, s_all, p, (const int64_t *)part);
            else
                hipLaunchKernelGGL((k_close_wide<false, false>), dim3(L.blocks), dim3(1024),
                                   plan.lone ? kCloseWideExtraLds : 0, q, chains, sg, L.nseg,
                                   m_all, s_all, p, (const int64_t *)part);
            e = hipGetLastError();
        } else if (L.kind == TK_TRI) {
            ProfileScope ps(KC_SETUP, q, L.evals);
            if (ob)
                hipLaunchKernelGGL((k_tri<64, true>), dim3(L.blocks), dim3(NTH), 0, q, chains, sg,
                                   L.nseg, p, m_all, s_all, ob->hi, ob->lo, ob->q);
            else if (plan.T == 32)
                hipLaunchKernelGGL((k_tri_rows<32, 8>), dim3(L.blocks), dim3(32 * 8), 0, q,
                                   chains, sg, L.nseg, pd, m_all, s_all);
            else if (!plan.lone && L.blocks > cus)
                // Many 64-edge tiles: the 1024-thread row-group form fits one
                // or two per CU, the 256-thread form more (measured faster
                // on a batch of 4096 chains).
                hipLaunchKernelGGL(k_tri_key<64>, dim3(L.blocks), dim3(NTH), 0, q, chains, sg,
                                   L.nseg, pd, m_all, s_all);
            else
                hipLaunchKernelGGL((k_tri_rows<64, 16>), dim3(L.blocks), dim3(64 * 16), 0, q,
                                   chains, sg, L.nseg, pd, m_all, s_all);
            e = hipGetLastError();
        } else if (L.kind == TK_BULK) {
            ProfileScope ps(KC_BULK, q, L.evals);
            const int paced = plan.lone ? 1 : 0;
            if (plan.T == 32)
                launch_with_stop(k_bulk<32>, bblocks, bulk_threads<32>(), q, stop, chains, sg,
                                 L.nseg, m_all, pd, part, paced, ww, wt, wticks);
            else
                launch_with_stop(k_bulk<64>, bblocks, bulk_threads<64>(), q, stop, chains, sg,
                                 L.nseg, m_all, pd, part, paced, ww, wt, wticks);
            e = hipGetLastError();
        } else if (L.kind == TK_CLOSE) {
            ProfileScope ps(KC_CLOSE, q, L.evals);
            // Paired closures (two per CU, each somewhat slower) only when
            // the launch has more tiles than the device has CUs (or than
            // the plan's tuned threshold).
            const int tuned = pair_min_blocks >= 0 ? pair_min_blocks : plan.pair_min_blocks;
            const int pair_min = tuned > 0 ? tuned : cus;
            const bool lone = plan.lone || L.blocks <= pair_min;
            if (plan.T == 32)
                hipLaunchKernelGGL(k_close_pair<32>, dim3(L.blocks),
                                   dim3(CloseShape<32, CG_PAIR>::CTH), 0, q, chains, sg, L.nseg,
                                   m_all, s_all, pd, part);
            else if (ob && lone)
                hipLaunchKernelGGL(k_close_ob, dim3(L.blocks),
                                   dim3(CloseShape<64, CG_LONE>::CTH), kCloseExtraLds, q, chains,
                                   sg, L.nseg, m_all, s_all, pd, part, ob->hid, ob->lod);
            else if (ob)
                hipLaunchKernelGGL(k_close_pair_ob, dim3(L.blocks),
                                   dim3(CloseShape<64, CG_PAIR>::CTH), 0, q, chains, sg, L.nseg,
                                   m_all, s_all, pd, part, ob->hid, ob->lod);
            else if (lone)
                hipLaunchKernelGGL(k_close, dim3(L.blocks), dim3(CloseShape<64, CG_LONE>::CTH),
                                   kCloseExtraLds, q, chains, sg, L.nseg, m_all, s_all, pd, part);
            else
                hipLaunchKernelGGL(k_close_pair<64>, dim3(L.blocks),
                                   dim3(CloseShape<64, CG_PAIR>::CTH), 0, q, chains, sg, L.nseg,
                                   m_all, s_all, pd, part);
            e = hipGetLastError();
        }
        if (e == hipSuccess && ww) folded[L.fold] = 1;
        if (e == hipSuccess && L.record && aux) {
            if (L.stream == 1 && !events_only && !aux_stream) tok[li] = aux_signal_write(ss.aux);
            if (!tok[li] && !rec[li]) {
                rec[li] = ss.events[next_ev++];
                e = hipEventRecord(rec[li], q);
            }
        }
        if (e != hipSuccess) st = MCM_ERR_DEVICE;
    }
    if (forked) {
        // Join: `stream` continues after everything enqueued on aux.
        if (hipEventRecord(ss.events[1], ss.aux) != hipSuccess ||
            hipStreamWaitEvent(stream, ss.events[1], 0) != hipSuccess)
            st = MCM_ERR_DEVICE;
    }
    ss.aux = lib_aux;
    if (aux) release_streams(ss);
    if (part_own) ws_free(part_own, stream);
    return st;
}

// The serial schedule: the plan's launch order already respects every
// dependency (each launch follows everything it waits for), so one stream
// runs it as is.
void plan_make_serial(TiledPlan &plan)
{
    for (TiledLaunch &L : plan.launches) {
        L.stream = 0;
        L.wait = -1;
        L.record = false;
    }
    plan.uses_aux = false;
    plan.last_interior = -1;
}

mcm_status run_tiled(const DeviceChain &dc, const ChainInfo &ci, int64_t *m, int32_t *s,
                     hipStream_t stream)
{
    TiledPlan plan;
    plan.wide = !tiled_accepts(ci);
    plan.lone = true;
    plan.serial = profile_serial();
    plan.cus = device_cus();
    plan.slots_per_cu = bulk_blocks_per_cu();
    const int c = plan_add_chain(plan, ci, 0, 0, 0, 0);
    plan_lockstep(plan, {c});
    if (plan.serial) plan_make_serial(plan);
    return run_tiled_plan(plan, dc.p, dc.pd, m, s, nullptr, stream, nullptr);
}

mcm_status run_tiled_obst(const ChainInfo &ci, const int32_t *p_zero, const double *pd_zero,
                          const ObstWeights &ob, int64_t *e, int32_t *split, hipStream_t stream)
{
    if (!tiled_accepts(ci)) return MCM_ERR_UNSUPPORTED;
    TiledPlan plan;
    plan.lone = true;
    plan.cus = device_cus();
    plan.slots_per_cu = bulk_blocks_per_cu();
    const int c = plan_add_chain(plan, ci, 0, 0, 0, 0);
    plan_lockstep(plan, {c});
    return run_tiled_plan(plan, p_zero, pd_zero, e, split, nullptr, stream, &ob);
}

}  // namespace mcm
