// Optimal binary search tree: the textbook's other interval DP with the
// split shape of MCM, which the paper (end of Section IV) proposes to carry
// its technique to.  Leaves are the n+1 gaps d_0..d_n between the keys; the
// cell (a, b), a <= b, is the subtree over keys a+1..b:
//
//   e[a][a] = q_a
//   e[a][b] = min_{a <= k < b} e[a][k] + e[k+1][b] + W(a, b),   root key k+1
//   W(a, b) = q_a + ... + q_b + p_{a+1} + ... + p_b
//
// W does not depend on the split, so it is added once after the minimum.
// The table is filled diagonal by diagonal like the MCM wavefront path (the
// order of Fig. 5): one launch per diagonal, a group of lanes per cell
// scanning its splits over row a and the mirrored row b, then a lane
// reduction on (cost, k).  int64 throughout.
#include "mcm_internal.h"

namespace mcm {
namespace {

constexpr int kIvBlock = 256;

__device__ __forceinline__ void iv_lex_min(int64_t &v, int32_t &k, int64_t v2, int32_t k2)
{
    if (v2 < v || (v2 == v && k2 < k)) {
        v = v2;
        k = k2;
    }
}

// hi_w[b] - lo_w[a] = W(a, b).
template <int G>
__global__ __launch_bounds__(kIvBlock) void k_obst_diag(const int64_t *__restrict__ hi_w,
                                                        const int64_t *__restrict__ lo_w,
                                                        int32_t L, int32_t d,
                                                        int64_t *__restrict__ e,
                                                        int32_t *__restrict__ root)
{
    const int64_t gid = (int64_t)blockIdx.x * kIvBlock + threadIdx.x;
    const int32_t a = (int32_t)(gid / G);
    const int32_t lane = (int32_t)(gid % G);
    const bool active = a < L - d;
    int64_t best = INT64_MAX;
    int32_t arg = INT32_MAX;
    if (active) {
        const int32_t b = a + d;
        const int64_t *row_a = e + (size_t)a * L;
        const int64_t *row_b = e + (size_t)b * L;
        for (int32_t k = a + lane; k < b; k += G) {
            const int64_t c = row_a[k] + row_b[k + 1];
            if (c < best) {  // a lane's k increase: strict < keeps the smallest
                best = c;
                arg = k;
            }
        }
    }
#pragma unroll
    for (int off = G / 2; off > 0; off >>= 1) {
        const int64_t ov = __shfl_xor(best, off, G);
        const int32_t ok = __shfl_xor(arg, off, G);
        iv_lex_min(best, arg, ov, ok);
    }
    if (active && lane == 0) {
        const int32_t b = a + d;
        const int64_t v = best + (hi_w[b] - lo_w[a]);
        e[(size_t)a * L + b] = v;
        e[(size_t)b * L + a] = v;
        root[(size_t)a * L + b] = arg + 1;
    }
}

// e[a][a] = q_a; root = -1 on and below the diagonal.
__global__ __launch_bounds__(kIvBlock) void k_obst_init(const int32_t *__restrict__ q, int32_t L,
                                                        int64_t *__restrict__ e,
                                                        int32_t *__restrict__ root)
{
    const int64_t total = (int64_t)L * L;
    for (int64_t idx = (int64_t)blockIdx.x * kIvBlock + threadIdx.x; idx < total;
         idx += (int64_t)gridDim.x * kIvBlock) {
        const int64_t a = idx / L, b = idx % L;
        if (a >= b) root[idx] = -1;
        if (a == b) e[idx] = q[a];
    }
}

// The tiled path writes the split k (a gap index); the root key is k + 1.
__global__ __launch_bounds__(kIvBlock) void k_obst_root(int32_t *__restrict__ root, int64_t total)
{
    for (int64_t idx = (int64_t)blockIdx.x * kIvBlock + threadIdx.x; idx < total;
         idx += (int64_t)gridDim.x * kIvBlock) {
        const int32_t v = root[idx];
        if (v >= 0) root[idx] = v + 1;
    }
}

template <int G>
hipError_t launch_obst(const int64_t *hi_w, const int64_t *lo_w, int32_t L, int32_t d,
                       int64_t *e, int32_t *root, hipStream_t stream)
{
    const int64_t threads = (int64_t)(L - d) * G;
    const unsigned blocks = (unsigned)((threads + kIvBlock - 1) / kIvBlock);
    hipLaunchKernelGGL(k_obst_diag<G>, dim3(blocks), dim3(kIvBlock), 0, stream, hi_w, lo_w, L, d,
                       e, root);
    return hipGetLastError();
}

}  // namespace

mcm_status run_obst(const int32_t *q, const int64_t *hi_w, const int64_t *lo_w, int32_t L,
                    int64_t *e, int32_t *root, hipStream_t stream)
{
    {
        const int64_t total = (int64_t)L * L;
        const int64_t want = (total + kIvBlock - 1) / kIvBlock;
        const unsigned blocks = (unsigned)(want < 4096 ? (want < 1 ? 1 : want) : 4096);
        hipLaunchKernelGGL(k_obst_init, dim3(blocks), dim3(kIvBlock), 0, stream, q, L, e, root);
        if (hipGetLastError() != hipSuccess) return MCM_ERR_DEVICE;
    }
    for (int32_t d = 1; d < L; ++d) {
        hipError_t err;
        if (d >= 256)
            err = launch_obst<64>(hi_w, lo_w, L, d, e, root, stream);
        else if (d >= 32)
            err = launch_obst<16>(hi_w, lo_w, L, d, e, root, stream);
        else if (d >= 4)
            err = launch_obst<4>(hi_w, lo_w, L, d, e, root, stream);
        else
            err = launch_obst<1>(hi_w, lo_w, L, d, e, root, stream);
        if (err != hipSuccess) return MCM_ERR_DEVICE;
    }
    return MCM_OK;
}

}  // namespace mcm

namespace mcm {

mcm_status run_obst_root(int32_t *root, int32_t L, hipStream_t stream)
{
    const int64_t total = (int64_t)L * L;
    const int64_t want = (total + kIvBlock - 1) / kIvBlock;
    const unsigned blocks = (unsigned)(want < 4096 ? (want < 1 ? 1 : want) : 4096);
    hipLaunchKernelGGL(k_obst_root, dim3(blocks), dim3(kIvBlock), 0, stream, root, total);
    return hipGetLastError() == hipSuccess ? MCM_OK : MCM_ERR_DEVICE;
}

}  // namespace mcm
