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
    return mcm_obst_solve_algo(p, q, n, e_out, root_out, MCM_ALGO_AUTO, stream);
}

mcm_status mcm_obst_solve_algo(const int32_t *p, const int32_t *q, int32_t n, int64_t *e_out,
                               int32_t *root_out, int32_t algo, hipStream_t stream)
{
    if (algo != MCM_ALGO_AUTO && algo != MCM_ALGO_WAVEFRONT && algo != MCM_ALGO_TILED)
        return MCM_ERR_INVALID_ARG;
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
    // The tiled kernels carry costs in fp64 keys: every candidate must stay
    // below 2^46 (as for MCM chains), with L cells.
    ChainInfo ci;
    ci.n = L;
    ci.pmax = 0;
    {
        const long double bound = 2.0L * (n + 1) * (2.0L * n + 1) * (long double)wmax;
        int bits = 1;
        while (bits < 63 && (long double)(1ULL << bits) <= bound) ++bits;
        ci.cost_bits = bits;
    }
    const bool tiled = algo == MCM_ALGO_TILED || (algo == MCM_ALGO_AUTO && L >= 2 && tiled_accepts(ci));
    if (tiled && (L < 2 || !tiled_accepts(ci))) return MCM_ERR_UNSUPPORTED;
    if (hipGetLastError() != hipSuccess) return MCM_ERR_DEVICE;

    // One upload: int64 and fp64 prefix weights, gap weights, and for the
    // tiled path the zero dimension vectors (no product term).
    const size_t o_hi = 0, o_lo = (size_t)L * 8, o_hid = 2 * (size_t)L * 8,
                 o_lod = 3 * (size_t)L * 8, o_zd = 4 * (size_t)L * 8,
                 o_q = o_zd + ((size_t)L + 1) * 8, o_z = o_q + ((size_t)L * 4 + 7) / 8 * 8;
    const size_t bytes = o_z + ((size_t)L + 1) * 4;
    void *blob = nullptr;
    mcm_status st = upload_blob(stream, &blob, bytes, [&](char *h) {
        memcpy(h + o_hi, hi_w.data(), (size_t)L * 8);
        memcpy(h + o_lo, lo_w.data(), (size_t)L * 8);
        double *hd = (double *)(h + o_hid), *ld = (double *)(h + o_lod);
        for (int32_t t = 0; t < L; ++t) {
            hd[t] = (double)hi_w[t];
            ld[t] = (double)lo_w[t];
        }
        memset(h + o_zd, 0, ((size_t)L + 1) * 8);
        memcpy(h + o_q, q, (size_t)L * 4);
        memset(h + o_z, 0, ((size_t)L + 1) * 4);
    });
    if (st != MCM_OK) return st;
    const char *b = (const char *)blob;
    if (tiled) {
        ObstWeights ob;
        ob.hi = (const int64_t *)(b + o_hi);
        ob.lo = (const int64_t *)(b + o_lo);
        ob.hid = (const double *)(b + o_hid);
        ob.lod = (const double *)(b + o_lod);
        ob.q = (const int32_t *)(b + o_q);
        st = run_tiled_obst(ci, (const int32_t *)(b + o_z), (const double *)(b + o_zd), ob, e_out,
                            root_out, stream);
        if (st == MCM_OK) st = run_obst_root(root_out, L, stream);
    } else {
        st = run_obst((const int32_t *)(b + o_q), (const int64_t *)(b + o_hi),
                      (const int64_t *)(b + o_lo), L, e_out, root_out, stream);
    }
    ws_free(blob, stream);
    return st;
}

}  // extern "C"
