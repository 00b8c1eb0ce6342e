// The paper's pipeline for MCM (Section IV-B, Fig. 8), kept as an ablation
// of the tiled path.  The table is linearised in the diagonal order of
// Fig. 5: element x = (i, j = i + d) sits at off[d] + i, the n elements of
// diagonal 0 are preset, and element x has k_x = d splits.  Thread j'
// (1 <= j' <= n-1) folds split j' (k = i + j' - 1) of an element into it, so
// an element's splits are folded one step apart by consecutive threads, in
// increasing k, and every step ends with a barrier.
//
// Fig. 8 starts element x at step x.  Run in lockstep that can read an
// operand before its last split has been folded (it happens on the
// diagonals past the middle of the table), so here element x starts at a
// step sigma(x) computed on the host: the earliest step, after its
// predecessor's, at which every operand it reads is final when read.  The
// element order and the one-split-per-thread-per-step shape of Fig. 8 stay;
// stalls are inserted where the printed schedule would read too early.
//
// One workgroup (n <= 1025: n-1 threads).  The linear table lives in global
// memory (n(n+1)/2 int64 values and int32 splits).
#include "mcm_internal.h"

namespace mcm {
namespace {

constexpr int kPipeMaxThreads = 1024;

__global__ __launch_bounds__(kPipeMaxThreads) void k_pipe(
    const int32_t *__restrict__ p, int32_t n, const int32_t *__restrict__ inv, int64_t S,
    int64_t steps, const int32_t *__restrict__ elem, int64_t *__restrict__ st,
    int32_t *__restrict__ sk)
{
    __shared__ int32_t off[kPipeMaxThreads + 2];
    const int tid = threadIdx.x;
    for (int d = tid; d <= n; d += blockDim.x) off[d] = d * n - d * (d - 1) / 2;
    for (int i = tid; i < n; i += blockDim.x) st[i] = 0;  // diagonal 0 is preset
    __syncthreads();
    const int jp = tid + 1;  // thread j'
    for (int64_t t = 0; t < steps; ++t) {
        const int64_t u = t - jp + 1;  // sigma of the element this thread serves now
        const int x = (jp <= n - 1 && u >= 0 && u < S) ? inv[u] : -1;
        if (x >= 0) {
            const int code = elem[x];
            const int i = code & 0xffff, d = code >> 16;
            if (jp <= d) {
                const int k = i + jp - 1, j = i + d;
                const int64_t v = st[off[k - i] + i] + st[off[j - k - 1] + k + 1] +
                                  (int64_t)p[i] * p[k + 1] * p[j + 1];
                // splits arrive in increasing k: strict < keeps the smallest
                if (jp == 1 || v < st[x]) {
                    st[x] = v;
                    sk[x] = k;
                }
            }
        }
        __syncthreads();
    }
}

// Linear table to the square m / s layout.
__global__ __launch_bounds__(256) void k_pipe_unpack(int32_t n, const int64_t *__restrict__ st,
                                                     const int32_t *__restrict__ sk,
                                                     int64_t *__restrict__ m,
                                                     int32_t *__restrict__ s)
{
    const int64_t total = (int64_t)n * n;
    for (int64_t idx = (int64_t)blockIdx.x * 256 + threadIdx.x; idx < total;
         idx += (int64_t)gridDim.x * 256) {
        const int64_t r = idx / n, c = idx % n;
        const int64_t i = r < c ? r : c, j = r < c ? c : r, d = j - i;
        const int64_t x = d * n - d * (d - 1) / 2 + i;
        m[idx] = st[x];
        s[idx] = r < c ? sk[x] : -1;
    }
}

}  // namespace

mcm_status run_pipeline(const PipePlan &pl, const int32_t *p, int32_t n, int64_t *m, int32_t *s,
                        hipStream_t stream)
{
    const int threads = ((n - 1 + 63) / 64) * 64;
    hipLaunchKernelGGL(k_pipe, dim3(1), dim3(threads < 64 ? 64 : threads), 0, stream, p, n,
                       pl.inv, pl.S, pl.steps, pl.elem, pl.st, pl.sk);
    if (hipGetLastError() != hipSuccess) return MCM_ERR_DEVICE;
    const int64_t total = (int64_t)n * n;
    const int64_t want = (total + 255) / 256;
    const unsigned blocks = (unsigned)(want < 4096 ? (want < 1 ? 1 : want) : 4096);
    hipLaunchKernelGGL(k_pipe_unpack, dim3(blocks), dim3(256), 0, stream, n, pl.st, pl.sk, m, s);
    return hipGetLastError() == hipSuccess ? MCM_OK : MCM_ERR_DEVICE;
}

}  // namespace mcm
