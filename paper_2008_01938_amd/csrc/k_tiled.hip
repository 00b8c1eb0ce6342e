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
// k_tri fills the diagonal tiles (all their splits stay inside the tile).
// k_bulk evaluates the bulk range of every tile of one tile-diagonal: a
// min-plus-like reduction where the A panel (rows of I, columns k) and the
// B panel (rows k+1, columns of J) are staged through LDS and each thread
// keeps a 4 x 4 register microtile of running minima.  The bulk range is
// cut into chunks spread over workgroups; each writes packed (cost, k)
// partial minima.  k_close merges the partials and then adds the (a) and
// (b) splits, which depend on cells of the same tile: cell (r, c) (local
// row/column) needs the cells below it in its column and left of it in its
// row, so the tile is swept in local anti-diagonals w = (T-1-r) + c, one
// workgroup barrier per anti-diagonal, entirely in LDS.
//
// Exact integers in fp64.  A candidate cost of cell (i, j) is at most
// (j-i) * pmax^3 < 2^cost_bits.  The kernels carry
// key = cost * 2^kb + k_local as a double with kb = 53 - cost_bits, so
// every key, and every partial sum that forms it (all integers), is below
// 2^53 and therefore exact; one fp64 min then picks the smallest cost and,
// among equal costs, the smallest k_local -- the smallest k when k_local
// increases with k.  A split evaluation is fma + add + min.
#include <math.h>

#include "mcm_internal.h"

namespace mcm {
namespace {

constexpr int T = 64;        // tile edge
constexpr int KC = 16;       // k values staged per LDS round in k_bulk
constexpr int NTH = 256;     // threads per workgroup
constexpr double kPad = 4611686018427387904.0;  // 2^62: never wins a min

// ------------------------------------------------------------------------
// Diagonal tiles (I, I): every split of a cell inside the tile uses two
// cells of the same tile.  Local diagonals dd = 1..nI-1 in order; four
// lanes per cell, lexicographic (cost, k) reduction.  int64 arithmetic.
// ------------------------------------------------------------------------
__global__ __launch_bounds__(NTH) void k_tri(const int32_t *__restrict__ p, int32_t n,
                                             int64_t *__restrict__ m, int32_t *__restrict__ s)
{
    __shared__ int64_t tv[T][T + 1];
    __shared__ int32_t sv[T][T + 1];
    __shared__ int64_t ps[T + 1];
    const int tid = threadIdx.x;
    const int base = blockIdx.x * T;
    const int nI = min(T, n - base);
    for (int q = tid; q <= nI; q += NTH) ps[q] = p[base + q];
    for (int r = tid; r < T; r += NTH) tv[r][r] = 0;
    __syncthreads();

    const int r = tid >> 2, g = tid & 3;
    for (int dd = 1; dd < nI; ++dd) {
        const int c = r + dd;
        int64_t best = INT64_MAX;
        int32_t arg = INT32_MAX;
        if (c < nI) {
            const int64_t prc = ps[r] * ps[c + 1];
            for (int kl = r + g; kl < c; kl += 4) {
                const int64_t v = tv[r][kl] + tv[kl + 1][c] + prc * ps[kl + 1];
                if (v < best) {
                    best = v;
                    arg = kl;
                }
            }
        }
#pragma unroll
        for (int off = 1; off < 4; off <<= 1) {
            const int64_t ov = __shfl_xor(best, off, 4);
            const int32_t oa = __shfl_xor(arg, off, 4);
            if (ov < best || (ov == best && oa < arg)) {
                best = ov;
                arg = oa;
            }
        }
        if (c < nI && g == 0) {
            tv[r][c] = best;
            sv[r][c] = base + arg;
        }
        __syncthreads();
    }

    for (int idx = tid; idx < T * T; idx += NTH) {
        const int rr = idx / T, cc = idx % T;
        if (rr < nI && cc < nI) {
            const size_t o = (size_t)(base + rr) * n + base + cc;
            m[o] = rr <= cc ? tv[rr][cc] : tv[cc][rr];
            s[o] = rr < cc ? sv[rr][cc] : -1;
        }
    }
}

// ------------------------------------------------------------------------
// Bulk splits of tile-diagonal D >= 2.  Workgroup b handles tile I = b / P
// (J = I + D) and chunk b % P of its bulk range.  Thread (tx, ty) owns the
// cells rows ty + 16a, columns tx + 16b (a, b = 0..3) of the tile.
// ------------------------------------------------------------------------
__global__ __launch_bounds__(NTH) void k_bulk(const int64_t *__restrict__ m,
                                              const double *__restrict__ pd, int32_t n,
                                              int32_t D, int32_t KS, int32_t P, int32_t kb,
                                              int32_t kbits, uint64_t *__restrict__ part)
{
    __shared__ double As[2][KC][T + 1];  // As[kk][r] = m[row0+r][k] * 2^kb
    __shared__ double Bs[2][KC][T];      // Bs[kk][c] = m[k+1][col0+c] * 2^kb + (k - k0)
    __shared__ double Ps[2][KC];         // p[k+1]

    const int tid = threadIdx.x;
    const int tile = blockIdx.x / P;
    const int chunk = blockIdx.x - tile * P;
    const int I = tile, J = tile + D;
    const int row0 = I * T, col0 = J * T;
    const int k0 = (I + 1) * T - 1 + chunk * KS;
    const int kend = min(k0 + KS, col0);  // exclusive end of this chunk
    const int nJ = min(T, n - col0);
    const double scale = ldexp(1.0, kb);
    const double inv_scale = ldexp(1.0, -kb);
    const int tx = tid & 15, ty = tid >> 4;

    double pj[4][4], best[4][4];
#pragma unroll
    for (int a = 0; a < 4; ++a) {
        const double pi = pd[row0 + ty + 16 * a] * scale;
#pragma unroll
        for (int b = 0; b < 4; ++b) {
            const int c = tx + 16 * b;
            pj[a][b] = c < nJ ? pi * pd[col0 + c + 1] : 0.0;
            best[a][b] = __builtin_inf();
        }
    }

    // Staging: A block is T rows x KC columns, B block KC rows x T columns;
    // 4 elements of each per thread.
    int64_t ra[4], rb[4];
    double rp = 0.0;
    auto load = [&](int kc) {
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            const int e = tid + NTH * u;
            const int r = e / KC, kk = e % KC;
            const int k = kc + kk;
            ra[u] = k < kend ? m[(size_t)(row0 + r) * n + k] : 0;
            const int kk2 = e / T, c = e % T;
            const int k2 = kc + kk2;
            rb[u] = (k2 < kend && c < nJ) ? m[(size_t)(k2 + 1) * n + col0 + c] : 0;
        }
        if (tid < KC) rp = (kc + tid < kend) ? pd[kc + tid + 1] : 0.0;
    };
    auto store = [&](int kc, int buf) {
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            const int e = tid + NTH * u;
            const int r = e / KC, kk = e % KC;
            As[buf][kk][r] = (kc + kk < kend) ? (double)ra[u] * scale : kPad;
            const int kk2 = e / T, c = e % T;
            Bs[buf][kk2][c] = fma((double)rb[u], scale, (double)(kc + kk2 - k0));
        }
        if (tid < KC) Ps[buf][tid] = rp;
    };

    load(k0);
    store(k0, 0);
    __syncthreads();
    int buf = 0;
    for (int kc = k0; kc < kend; kc += KC) {
        const bool more = kc + KC < kend;
        if (more) load(kc + KC);
#pragma unroll 4
        for (int kk = 0; kk < KC; ++kk) {
            double av[4], bv[4];
#pragma unroll
            for (int a = 0; a < 4; ++a) av[a] = As[buf][kk][ty + 16 * a];
#pragma unroll
            for (int b = 0; b < 4; ++b) bv[b] = Bs[buf][kk][tx + 16 * b];
            const double pk = Ps[buf][kk];
#pragma unroll
            for (int a = 0; a < 4; ++a)
#pragma unroll
                for (int b = 0; b < 4; ++b)
                    best[a][b] = fmin(best[a][b], fma(pj[a][b], pk, bv[b]) + av[a]);
        }
        if (more) store(kc + KC, buf ^ 1);
        __syncthreads();
        buf ^= 1;
    }

    uint64_t *out = part + (size_t)blockIdx.x * T * T;
#pragma unroll
    for (int a = 0; a < 4; ++a) {
#pragma unroll
        for (int b = 0; b < 4; ++b) {
            const int r = ty + 16 * a, c = tx + 16 * b;
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
// Closure of tile-diagonal D >= 1: one workgroup per tile (I, I+D).
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
// register operand, so their terms never win and need no select.  Wave h
// covers rows 8h..8h+7, whose (a) splits all lie in slots >= h: the step
// body is instantiated per wave index so that range is static.  Two waves
// per SIMD hide the fp64 issue latency a single wave would expose.  All
// LDS reads of a step are issued before the first use; the row group's
// minimum is formed with DPP lane permutations; one barrier per step
// publishes the new cells to the other rows.
// ------------------------------------------------------------------------
constexpr int CG = 8;               // lanes per row group
constexpr int CTH = T * CG;          // 512 threads = 8 waves, 2 per SIMD
constexpr int CS = T / CG;           // register slots per lane
constexpr int CROWS = 64 / CG;       // rows per wave
constexpr int CSTR = T + 8;          // column stride (doubles) of the closure's LDS tables

template <int CTRL>
__device__ __forceinline__ double dpp_perm(double v)
{
    const int2 b = __builtin_bit_cast(int2, v);
    int2 o;
    o.x = __builtin_amdgcn_update_dpp(0, b.x, CTRL, 0xF, 0xF, false);
    o.y = __builtin_amdgcn_update_dpp(0, b.y, CTRL, 0xF, 0xF, false);
    return __builtin_bit_cast(double, o);
}

// Minimum over each aligned group of CG = 8 lanes (all lanes active).
__device__ __forceinline__ double min_group(double v)
{
    v = fmin(v, dpp_perm<0xB1>(v));   // quad_perm [1,0,3,2]: lane ^ 1
    v = fmin(v, dpp_perm<0x4E>(v));   // quad_perm [2,3,0,1]: lane ^ 2
    v = fmin(v, dpp_perm<0x141>(v));  // row_half_mirror: lane i <-> 7-i
    return v;
}

struct CloseRegs {
    double DIr[CS], PIr[CS], PJr[CS], Xrow[CS];
};

// One anti-diagonal step for wave H (rows 16H..16H+15).  Returns the
// minimum over the closure splits of this lane's cell (before the bulk).
template <int H>
__device__ __forceinline__ double close_step(const CloseRegs &R, const double (*Xt)[CSTR],
                                             const double (*DJt)[CSTR], int cc, int g,
                                             double pJc)
{
    constexpr int T0 = H * (CROWS / CG);  // first (a) slot any row of this wave uses
    double xa[CS], xb[CS];
#pragma unroll
    for (int t = T0; t < CS; ++t) xa[t] = Xt[cc][t * CG + g + 1];
    // All (b) slots are read: DJt is zero outside its triangle, and a slot
    // whose cell is not final yet still holds Xrow = 2^62.
#pragma unroll
    for (int t = 0; t < CS; ++t) xb[t] = DJt[cc][t * CG + g + 1];
    // Independent terms, then a balanced min tree: a single running
    // minimum would make every slot wait for the previous one.
    double v[CS];
#pragma unroll
    for (int t = 0; t < CS; ++t) {
        const double tb = fma(pJc, R.PJr[t], xb[t]) + R.Xrow[t];
        v[t] = t >= T0 ? fmin(tb, fma(pJc, R.PIr[t], R.DIr[t]) + xa[t]) : tb;
    }
#pragma unroll
    for (int span = 1; span < CS; span *= 2)
#pragma unroll
        for (int t = 0; t + span < CS; t += 2 * span) v[t] = fmin(v[t], v[t + span]);
    return min_group(v[0]);
}

__global__ __launch_bounds__(CTH) void k_close(int64_t *__restrict__ m, int32_t *__restrict__ s,
                                               const double *__restrict__ pd, int32_t n,
                                               int32_t D, int32_t P, int32_t kb, int32_t kbits,
                                               const uint64_t *__restrict__ part)
{
    // Column-major with a column stride of CSTR = 72 doubles.  LDS has 32
    // banks of 4 bytes, so a 64-bit read is conflict-free when the 16 lanes
    // served together touch distinct 8-byte words modulo 16.  In a step,
    // lane (i, g) of a wave (row 8h+i) reads row t*CG+g+1 of column c_lo+i:
    // word (c_lo+i)*72 + 8t+g+1 = 8i + g + const (mod 16), distinct for the
    // 16 lanes i = 0..1, g = 0..7 of each group.  Row T is a spare so slot
    // addresses never need clamping.
    __shared__ double DJt[T][CSTR];  // DJt[c][q] = DJ[q][c] * 2^kb + T + q - 1 (1 <= q <= c), else 0
    __shared__ double Xt[T][CSTR];   // Xt[c][q]: bulk key, then final cost * 2^kb of cell (q, c)
    __shared__ int32_t Ks[T][T + 1];  // bulk split, then final split
    __shared__ double pJs[T + 1];     // p[col0 + q]

    const int tid = threadIdx.x;
    const int I = blockIdx.x, J = I + D;
    const int row0 = I * T, col0 = J * T;
    const int nJ = min(T, n - col0);
    const double scale = ldexp(1.0, kb);
    const double inv_scale = ldexp(1.0, -kb);
    const uint64_t kmask = (((uint64_t)1) << kbits) - 1;

    const int r = tid / CG, g = tid % CG;
    const int h = __builtin_amdgcn_readfirstlane(tid / 64);  // rows CROWS*h ..
    CloseRegs R;
    const double pi_s = pd[row0 + r] * scale;
#pragma unroll
    for (int t = 0; t < CS; ++t) {
        const int q = t * CG + g;  // (a) split column q; (b) split column c' = q
        const bool qa = q >= r && q <= T - 2;
        R.DIr[t] = qa ? fma((double)m[(size_t)(row0 + r) * n + row0 + q], scale, (double)q) : kPad;
        R.PIr[t] = qa ? pi_s * pd[row0 + q + 1] : 0.0;
        R.PJr[t] = q < nJ ? pi_s * pd[col0 + q + 1] : 0.0;
        R.Xrow[t] = kPad;  // until cell (r, q) is final
    }

    for (int q = tid; q <= T; q += CTH) pJs[q] = q <= nJ ? pd[col0 + q] : 0.0;
    for (int idx = tid; idx < T * CSTR; idx += CTH) {
        (&DJt[0][0])[idx] = 0.0;
        (&Xt[0][0])[idx] = 0.0;
    }
    __syncthreads();
    // DJ[q][c], 1 <= q <= c < nJ, read row-major (coalesced).
#pragma unroll 4
    for (int idx = tid; idx < T * T; idx += CTH) {
        const int qq = idx / T, c = idx % T;
        if (qq >= 1 && qq <= c && c < nJ)
            DJt[c][qq] = fma((double)m[(size_t)(col0 + qq) * n + col0 + c], scale,
                             (double)(T + qq - 1));
    }
    // Bulk result per cell: the minimum of P packed (cost << kbits | k)
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
            const int rr = idx / T, c = idx % T;
            if (c < nJ) {
                const int64_t cost = m[(size_t)(row0 + rr) * n + k] +
                                     m[(size_t)(k + 1) * n + col0 + c] +
                                     (int64_t)pd[row0 + rr] * (int64_t)pd[k + 1] *
                                         (int64_t)pd[col0 + c + 1];
                key[u] = ((uint64_t)cost << kbits) | (uint64_t)k;
            }
        }
    } else {
        const uint64_t *src = part + ((size_t)I * P) * T * T + tid;
        for (int ch = 0; ch < P; ++ch) {
            uint64_t v[CPT];
#pragma unroll
            for (int u = 0; u < CPT; ++u) v[u] = src[(size_t)ch * T * T + CTH * u];
#pragma unroll
            for (int u = 0; u < CPT; ++u) key[u] = v[u] < key[u] ? v[u] : key[u];
        }
    }
#pragma unroll
    for (int u = 0; u < CPT; ++u) {
        const int idx = tid + CTH * u;
        const int rr = idx / T, c = idx % T;
        if (c < nJ) {
            Xt[c][rr] = fma((double)(int64_t)(key[u] >> kbits), scale, (double)(T - 1));
            Ks[rr][c] = (int32_t)(key[u] & kmask);
        }
    }
    __syncthreads();

    const int wmax = (T - 1) + (nJ - 1);
    for (int w = 0; w <= wmax; ++w) {
        const int c = w - (T - 1 - r);
        const int c_lo = w - (T - 1 - CROWS * h);  // c of the wave's first row
        const int c_hi = c_lo + CROWS - 1;         // ... and of its last row
        if (c_hi >= 0 && c_lo < nJ) {              // wave-uniform
            const int cc = min(max(c, 0), nJ - 1);
            const double pJc = pJs[cc + 1];
            const double xbulk = Xt[cc][r];
            double best;
            switch (h) {
            case 0: best = close_step<0>(R, Xt, DJt, cc, g, pJc); break;
            case 1: best = close_step<1>(R, Xt, DJt, cc, g, pJc); break;
            case 2: best = close_step<2>(R, Xt, DJt, cc, g, pJc); break;
            case 3: best = close_step<3>(R, Xt, DJt, cc, g, pJc); break;
            case 4: best = close_step<4>(R, Xt, DJt, cc, g, pJc); break;
            case 5: best = close_step<5>(R, Xt, DJt, cc, g, pJc); break;
            case 6: best = close_step<6>(R, Xt, DJt, cc, g, pJc); break;
            default: best = close_step<7>(R, Xt, DJt, cc, g, pJc); break;
            }
            const double fin = fmin(best, xbulk);
            const double cost = floor(fin * inv_scale);
            const double xv = cost * scale;
            if (c >= 0 && c < nJ) {
#pragma unroll
                for (int t = 0; t < CS; ++t)
                    if (t * CG + g == c) R.Xrow[t] = xv;
                if (g == 0) {
                    Xt[c][r] = xv;
                    const int kl = (int)fma(-cost, scale, fin);
                    if (kl != T - 1) Ks[r][c] = kl < T - 1 ? row0 + kl : col0 + (kl - T);
                }
            }
        }
        __syncthreads();
    }

    for (int idx = tid; idx < T * T; idx += CTH) {
        const int rr = idx / T, c = idx % T;
        if (c < nJ) {
            const size_t o = (size_t)(row0 + rr) * n + col0 + c;
            m[o] = (int64_t)(Xt[c][rr] * inv_scale);
            s[o] = Ks[rr][c];
        }
    }
    for (int idx = tid; idx < T * T; idx += CTH) {
        const int c = idx / T, rr = idx % T;
        if (c < nJ) {
            const size_t o = (size_t)(col0 + c) * n + row0 + rr;
            m[o] = (int64_t)(Xt[c][rr] * inv_scale);
            s[o] = -1;
        }
    }
}

struct Plan {
    int32_t NT = 0, kb = 0, kbits = 0;
};

// Chunking of the bulk range of tile-diagonal D: P chunks of KS splits.
void bulk_split(int32_t NT, int32_t D, int32_t kb, int32_t *KS, int32_t *P)
{
    const int32_t tiles = NT - D;
    const int32_t L = (D - 1) * T + 1;
    const int32_t target_groups = 1024;
    int32_t want = (target_groups + tiles - 1) / tiles;
    int32_t maxp = (L + 63) / 64;  // at least 64 splits per chunk
    if (maxp > 32) maxp = 32;
    if (want > maxp) want = maxp;
    if (want < 1) want = 1;
    int32_t ks = (L + want - 1) / want;
    ks = (ks + KC - 1) / KC * KC;
    const int32_t cap = kb >= 30 ? (1 << 30) : (1 << kb);
    if (ks > cap) ks = cap / KC * KC;
    *KS = ks;
    *P = (L + ks - 1) / ks;
}

int32_t bitlen_u64(uint64_t v)
{
    int32_t b = 0;
    while (v) {
        ++b;
        v >>= 1;
    }
    return b;
}

}  // namespace

bool tiled_accepts(const ChainInfo &ci)
{
    const int32_t kbits = bitlen_u64((uint64_t)(ci.n > 1 ? ci.n - 1 : 1));
    return ci.cost_bits + 7 <= 53 && ci.cost_bits + kbits <= 64;
}

mcm_status run_tiled(const DeviceChain &dc, const ChainInfo &ci, int64_t *m, int32_t *s,
                     hipStream_t stream)
{
    if (!tiled_accepts(ci)) return MCM_ERR_UNSUPPORTED;
    const int32_t n = ci.n;
    Plan pl;
    pl.NT = (n + T - 1) / T;
    pl.kb = 53 - ci.cost_bits;
    if (pl.kb > 20) pl.kb = 20;
    pl.kbits = bitlen_u64((uint64_t)(n > 1 ? n - 1 : 1));

    // Partial buffer: the largest tile-diagonal.
    size_t part_elems = 0;
    for (int32_t D = 2; D < pl.NT; ++D) {
        int32_t KS, P;
        bulk_split(pl.NT, D, pl.kb, &KS, &P);
        const size_t e = (size_t)(pl.NT - D) * P * T * T;
        if (e > part_elems) part_elems = e;
    }
    uint64_t *part = nullptr;
    if (part_elems) {
        if (ws_alloc((void **)&part, part_elems * sizeof(uint64_t), stream) != hipSuccess)
            return MCM_ERR_NO_MEMORY;
    }
    mcm_status st = MCM_OK;
    {
        // Split evaluations inside the diagonal tiles: sum over tiles of
        // (nI^3 - nI) / 6.
        double ev = 0.0;
        for (int32_t I = 0; I < pl.NT; ++I) {
            const double nI = (double)((n - I * T) < T ? (n - I * T) : T);
            ev += (nI * nI * nI - nI) / 6.0;
        }
        ProfileScope ps(KC_SETUP, stream, ev);
        hipLaunchKernelGGL(k_tri, dim3(pl.NT), dim3(NTH), 0, stream, dc.p, n, m, s);
        if (hipGetLastError() != hipSuccess) st = MCM_ERR_DEVICE;
    }
    for (int32_t D = 1; D < pl.NT && st == MCM_OK; ++D) {
        const int32_t tiles = pl.NT - D;
        const int32_t nlast = n - (pl.NT - 1) * T;  // valid columns of the last tile
        const double cells = (double)(tiles - 1) * T * T + (double)T * nlast;
        int32_t KS = 0, P = 0;
        if (D >= 2) {
            bulk_split(pl.NT, D, pl.kb, &KS, &P);
            const double L = (double)(D - 1) * T + 1;
            ProfileScope ps(KC_BULK, stream, cells * L);
            hipLaunchKernelGGL(k_bulk, dim3(tiles * P), dim3(NTH), 0, stream, m, dc.pd, n, D, KS,
                               P, pl.kb, pl.kbits, part);
            if (hipGetLastError() != hipSuccess) {
                st = MCM_ERR_DEVICE;
                break;
            }
        }
        {
            // Closure evaluations: (a) and (b) splits, plus the single bulk
            // split when D == 1.  Per tile: sum over cells of (T-1-r) + c.
            const double per_full = (double)T * T * (T - 1);
            const double per_last = (double)nlast * T * (T - 1) / 2.0 +
                                    (double)T * nlast * (nlast - 1) / 2.0;
            double ev = (double)(tiles - 1) * per_full + per_last;
            if (D == 1) ev += cells;
            ProfileScope ps(KC_CLOSE, stream, ev);
            hipLaunchKernelGGL(k_close, dim3(tiles), dim3(CTH), 0, stream, m, s, dc.pd, n, D, P,
                               pl.kb, pl.kbits, part);
            if (hipGetLastError() != hipSuccess) st = MCM_ERR_DEVICE;
        }
    }
    if (part) ws_free(part, stream);
    return st;
}

}  // namespace mcm
