// C ABI of the optimal binary search tree solver: validation, the weight
// prefix sums, upload and launch.
#include <cstring>
#include <vector>

#include "mcm.h"
#include "mcm_internal.h"

using namespace mcm;

extern "C" {

mcm_status mcm_obst_solve(const int32_t *p, const int32_t *q, int32_t n, int64_t *e_out,
                          int32_t *root_out, hipStream_t stream)
{
    if (q == nullptr || (n > 0 && p == nullptr) || n < 0 || n > (1 << 30) || e_out == nullptr ||
        root_out == nullptr)
        return MCM_ERR_INVALID_ARG;
    if (((uintptr_t)e_out & 7) != 0 || ((uintptr_t)root_out & 3) != 0) return MCM_ERR_INVALID_ARG;
    const int32_t L = n + 1;
    // Prefix sums: W(a, b) = hi_w[b] - lo_w[a] with hi_w[b] = sum q_0..q_b +
    // sum p_1..p_b and lo_w[a] = sum q_0..q_(a-1) + sum p_1..p_a.
    std::vector<int64_t> hi_w(L), lo_w(L);
    int64_t qs = 0, ps = 0, wmax = 0;
    for (int32_t t = 0; t < L; ++t) {
        if (q[t] < 0 || (t > 0 && p[t - 1] < 0)) return MCM_ERR_INVALID_ARG;
        if (t > 0) ps += p[t - 1];
        lo_w[t] = qs + ps;
        qs += q[t];
        hi_w[t] = qs + ps;
        if (q[t] > wmax) wmax = q[t];
        if (t > 0 && p[t - 1] > wmax) wmax = p[t - 1];
    }
    // Every cost is at most (depth + 1) summed over the 2n+1 weights, depth
    // <= n, and a candidate adds two of them: 2 (n+1) (2n+1) max weight must
    // fit in int64.
    if ((long double)(n + 1) * (long double)(2 * (int64_t)n + 1) * (long double)wmax >=
        4.6e18L)
        return MCM_ERR_OVERFLOW;
    if (hipGetLastError() != hipSuccess) return MCM_ERR_DEVICE;

    const size_t o_hi = 0, o_lo = (size_t)L * 8, o_q = 2 * (size_t)L * 8;
    const size_t bytes = o_q + (size_t)L * 4;
    void *blob = nullptr;
    mcm_status st = upload_blob(stream, &blob, bytes, [&](char *h) {
        memcpy(h + o_hi, hi_w.data(), (size_t)L * 8);
        memcpy(h + o_lo, lo_w.data(), (size_t)L * 8);
        memcpy(h + o_q, q, (size_t)L * 4);
    });
    if (st != MCM_OK) return st;
    const char *b = (const char *)blob;
    st = run_obst((const int32_t *)(b + o_q), (const int64_t *)(b + o_hi),
                  (const int64_t *)(b + o_lo), L, e_out, root_out, stream);
    ws_free(blob, stream);
    return st;
}

}  // extern "C"
