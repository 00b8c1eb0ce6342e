// Plain anti-diagonal wavefront for the MCM table, exact int64.
//
// The table is filled diagonal by diagonal (the computation order of the
// paper's Fig. 5): every cell (i, i+d) of diagonal d needs only diagonals
// < d, so all n-d cells of a diagonal run in parallel, one launch per
// diagonal.  A cell's d splits are scanned by a group of G lanes (the
// per-element work the paper spreads over threads, Section II-B), each lane
// keeping a running (cost, k) minimum over its own strided k, and the group
// is then reduced with lane shuffles in the "tournament" fashion the paper
// describes (Section II-B), lexicographically on (cost, k) so the smallest
// split wins ties.
//
// Layout: m is n*n row-major and symmetric.  The left operands m[i][k],
// k = i..j-1, are a contiguous run of row i; the right operands m[k+1][j]
// are read from the mirror m[j][k+1], a contiguous run of row j.  Both
// loads are coalesced across the lanes of a group.
#include "mcm_internal.h"

namespace mcm {
namespace {

constexpr int kBlock = 256;

// pd[t] = p[t]: exact fp64 copies of dimensions (grid-stride).
__global__ __launch_bounds__(kBlock) void k_widen(const int32_t *__restrict__ p,
                                                  double *__restrict__ pd, size_t count)
{
    for (size_t t = (size_t)blockIdx.x * kBlock + threadIdx.x; t < count;
         t += (size_t)gridDim.x * kBlock)
        pd[t] = (double)p[t];
}

__device__ __forceinline__ void lex_min(int64_t &v, int32_t &k, int64_t v2, int32_t k2)
{
    if (v2 < v || (v2 == v && k2 < k)) {
        v = v2;
        k = k2;
    }
}

// Diagonal d >= 1.  G lanes per cell, G divides the wavefront size so a
// group never straddles waves.
template <int G>
__global__ __launch_bounds__(kBlock) void k_wave_diag(const int32_t *__restrict__ p, int32_t n,
                                                      int32_t d, int64_t *__restrict__ m,
                                                      int32_t *__restrict__ s)
{
    const int64_t gid = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    const int32_t i = (int32_t)(gid / G);
    const int32_t lane = (int32_t)(gid % G);
    const bool active = i < n - d;
    int64_t best = INT64_MAX;
    int32_t arg = INT32_MAX;
    if (active) {
        const int32_t j = i + d;
        const int64_t *row_i = m + (size_t)i * n;
        const int64_t *row_j = m + (size_t)j * n;
        const int64_t pij = (int64_t)p[i] * (int64_t)p[j + 1];
        for (int32_t k = i + lane; k < j; k += G) {
            const int64_t c = row_i[k] + row_j[k + 1] + pij * (int64_t)p[k + 1];
            if (c < best) {  // a lane's k increase, so strict < keeps the smallest
                best = c;
                arg = k;
            }
        }
    }
#pragma unroll
    for (int off = G / 2; off > 0; off >>= 1) {
        const int64_t ov = __shfl_xor(best, off, G);
        const int32_t ok = __shfl_xor(arg, off, G);
        lex_min(best, arg, ov, ok);
    }
    if (active && lane == 0) {
        const int32_t j = i + d;
        m[(size_t)i * n + j] = best;
        m[(size_t)j * n + i] = best;
        s[(size_t)i * n + j] = arg;
    }
}

// Base cases: m[i][i] = 0 and s[i][j] = -1 for i >= j.  Upper s and the
// off-diagonal m are written by the diagonal launches.
__global__ __launch_bounds__(kBlock) void k_wave_init(int32_t n, int64_t *__restrict__ m,
                                                      int32_t *__restrict__ s)
{
    const int64_t total = (int64_t)n * n;
    for (int64_t idx = (int64_t)blockIdx.x * kBlock + threadIdx.x; idx < total;
         idx += (int64_t)gridDim.x * kBlock) {
        const int64_t i = idx / n, j = idx % n;
        if (i >= j) s[idx] = -1;
        if (i == j) m[idx] = 0;
    }
}

template <int G>
hipError_t launch_diag(const int32_t *p, int32_t n, int32_t d, int64_t *m, int32_t *s,
                       hipStream_t stream)
{
    const int64_t threads = (int64_t)(n - d) * G;
    const unsigned blocks = (unsigned)((threads + kBlock - 1) / kBlock);
    hipLaunchKernelGGL(k_wave_diag<G>, dim3(blocks), dim3(kBlock), 0, stream, p, n, d, m, s);
    return hipGetLastError();
}

}  // namespace

mcm_status widen_dims(const int32_t *p, double *pd, size_t count, hipStream_t stream)
{
    if (count == 0) return MCM_OK;
    size_t blocks = (count + kBlock - 1) / kBlock;
    if (blocks > 4096) blocks = 4096;
    hipLaunchKernelGGL(k_widen, dim3((unsigned)blocks), dim3(kBlock), 0, stream, p, pd, count);
    return hipGetLastError() == hipSuccess ? MCM_OK : MCM_ERR_DEVICE;
}

mcm_status run_wavefront(const DeviceChain &dc, const ChainInfo &ci, int64_t *m, int32_t *s,
                         hipStream_t stream)
{
    const int32_t n = ci.n;
    {
        const int64_t total = (int64_t)n * n;
        int64_t want = (total + kBlock - 1) / kBlock;
        const unsigned blocks = (unsigned)(want < 4096 ? (want < 1 ? 1 : want) : 4096);
        ProfileScope ps(KC_SETUP, stream, 0.0);
        hipLaunchKernelGGL(k_wave_init, dim3(blocks), dim3(kBlock), 0, stream, n, m, s);
        if (hipGetLastError() != hipSuccess) return MCM_ERR_DEVICE;
    }
    for (int32_t d = 1; d < n; ++d) {
        ProfileScope ps(KC_WAVE, stream, (double)(n - d) * d);
        hipError_t e;
        if (d >= 256)
            e = launch_diag<64>(dc.p, n, d, m, s, stream);
        else if (d >= 32)
            e = launch_diag<16>(dc.p, n, d, m, s, stream);
        else if (d >= 4)
            e = launch_diag<4>(dc.p, n, d, m, s, stream);
        else
            e = launch_diag<1>(dc.p, n, d, m, s, stream);
        if (e != hipSuccess) return MCM_ERR_DEVICE;
    }
    return MCM_OK;
}

}  // namespace mcm
