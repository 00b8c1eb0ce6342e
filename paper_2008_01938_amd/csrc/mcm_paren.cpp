// C ABI of the optimal-order read-back: validation, uploads and workspace
// around the k_paren kernels.
#include <cstring>
#include <vector>

#include "mcm.h"
#include "mcm_internal.h"

using namespace mcm;

namespace {

// Workspace allocations of one call, released stream-ordered on exit.
struct Workspace {
    hipStream_t stream;
    std::vector<void *> held;
    explicit Workspace(hipStream_t s) : stream(s) {}
    ~Workspace()
    {
        for (void *p : held) ws_free(p, stream);
    }
    template <typename T>
    T *get(size_t count)
    {
        void *p = nullptr;
        if (ws_alloc(&p, count * sizeof(T), stream) != hipSuccess) return nullptr;
        held.push_back(p);
        return (T *)p;
    }
};

}  // namespace

extern "C" {

int64_t mcm_parens_length(int32_t n)
{
    if (n < 1) return -1;
    int64_t total = 2 * ((int64_t)n - 1);
    // "A" plus the decimal digits of every index 0..n-1.
    int64_t lo = 0, hi = 10;
    for (int digits = 1; lo < n; ++digits, lo = hi, hi *= 10) {
        const int64_t top = hi < n ? hi : n;
        total += (top - lo) * (1 + digits);
    }
    return total;
}

mcm_status mcm_parenthesize(const int32_t *p, int32_t n, const int32_t *s, int32_t *lo,
                            int32_t *hi, int64_t *cost, char *text, hipStream_t stream)
{
    if (n < 1 || s == nullptr || ((uintptr_t)s & 3) != 0) return MCM_ERR_INVALID_ARG;
    if (((uintptr_t)lo & 3) != 0 || ((uintptr_t)hi & 3) != 0 || ((uintptr_t)cost & 7) != 0)
        return MCM_ERR_INVALID_ARG;
    if ((lo == nullptr) != (hi == nullptr)) return MCM_ERR_INVALID_ARG;
    if (cost != nullptr && p == nullptr) return MCM_ERR_INVALID_ARG;
    if (p != nullptr) {
        mcm_status st = check_chain(p, n, nullptr);
        if (st != MCM_OK) return st;
    }
    if (hipGetLastError() != hipSuccess) return MCM_ERR_DEVICE;

    Workspace ws(stream);
    const size_t g = n > 1 ? (size_t)n - 1 : 1;
    if (lo == nullptr) {
        lo = ws.get<int32_t>(g);
        hi = ws.get<int32_t>(g);
        if (!lo || !hi) return MCM_ERR_NO_MEMORY;
    }
    int64_t *queue = ws.get<int64_t>(g);
    if (!queue) return MCM_ERR_NO_MEMORY;

    // One upload: the chain descriptor, then the dims when a cost is wanted.
    const bool with_p = cost != nullptr;
    const size_t dims_at = (sizeof(ParenChain) + 7) / 8 * 8;
    const size_t bytes = dims_at + (with_p ? ((size_t)n + 1) * sizeof(int32_t) : 0);
    void *blob = nullptr;
    mcm_status st = upload_blob(stream, &blob, bytes, [&](char *h) {
        ParenChain c;
        c.s_off = 0;
        c.p_off = with_p ? 0 : -1;
        c.g_off = 0;
        c.q_off = 0;
        c.n = n;
        c.cost_idx = with_p ? 0 : -1;
        memcpy(h, &c, sizeof c);
        if (with_p) memcpy(h + dims_at, p, ((size_t)n + 1) * sizeof(int32_t));
    });
    if (st != MCM_OK) return st;
    ws.held.push_back(blob);
    const ParenChain *chain = (const ParenChain *)blob;
    const int32_t *p_dev = with_p ? (const int32_t *)((char *)blob + dims_at) : nullptr;

    int32_t *counts = nullptr;
    if (text != nullptr && !(counts = ws.get<int32_t>(2 * (size_t)n))) return MCM_ERR_NO_MEMORY;
    st = run_paren(chain, 1, n, s, p_dev, lo, hi, cost, queue, counts, stream);
    if (st != MCM_OK || text == nullptr) return st;
    return run_paren_text(lo, n, counts, text, stream);
}

mcm_status mcm_parenthesize_batched(int32_t count, const int32_t *n, const int64_t *p_off,
                                    const int32_t *p_all, const int64_t *tab_off,
                                    const int32_t *s_all, const int64_t *node_off,
                                    int32_t *lo_all, int32_t *hi_all, int64_t *cost_all,
                                    hipStream_t stream)
{
    if (count < 0) return MCM_ERR_INVALID_ARG;
    if (count == 0) return MCM_OK;
    if (!n || !tab_off || !s_all || !node_off || !lo_all || !hi_all) return MCM_ERR_INVALID_ARG;
    if (((uintptr_t)s_all & 3) != 0 || ((uintptr_t)lo_all & 3) != 0 ||
        ((uintptr_t)hi_all & 3) != 0 || ((uintptr_t)cost_all & 7) != 0)
        return MCM_ERR_INVALID_ARG;
    const bool with_p = cost_all != nullptr;
    if (with_p && (!p_off || !p_all)) return MCM_ERR_INVALID_ARG;
    int64_t p_len = 0, q_len = 0;
    int32_t max_n = 1;
    for (int32_t b = 0; b < count; ++b) {
        if (n[b] < 1 || tab_off[b] < 0 || node_off[b] < 0) return MCM_ERR_INVALID_ARG;
        if (with_p) {
            if (p_off[b] < 0) return MCM_ERR_INVALID_ARG;
            mcm_status st = check_chain(p_all + p_off[b], n[b], nullptr);
            if (st != MCM_OK) return st;
            if (p_off[b] + n[b] + 1 > p_len) p_len = p_off[b] + n[b] + 1;
        }
        q_len += n[b] > 1 ? n[b] - 1 : 0;
        if (n[b] > max_n) max_n = n[b];
    }
    // Overlapping node ranges would be written by two workgroups at once.
    if (!ranges_disjoint(count, n, node_off, false)) return MCM_ERR_INVALID_ARG;
    if (hipGetLastError() != hipSuccess) return MCM_ERR_DEVICE;

    Workspace ws(stream);
    int64_t *queue = ws.get<int64_t>(q_len > 0 ? (size_t)q_len : 1);
    if (!queue) return MCM_ERR_NO_MEMORY;
    const size_t table = (size_t)count * sizeof(ParenChain);
    const size_t dims_at = (table + 7) / 8 * 8;
    const size_t bytes = dims_at + (size_t)p_len * sizeof(int32_t);
    void *blob = nullptr;
    mcm_status st = upload_blob(stream, &blob, bytes, [&](char *h) {
        ParenChain *c = (ParenChain *)h;
        int64_t q = 0;
        for (int32_t b = 0; b < count; ++b) {
            c[b].s_off = tab_off[b];
            c[b].p_off = with_p ? p_off[b] : -1;
            c[b].g_off = node_off[b];
            c[b].q_off = q;
            c[b].n = n[b];
            c[b].cost_idx = with_p ? b : -1;
            q += n[b] > 1 ? n[b] - 1 : 0;
        }
        if (p_len) memcpy(h + dims_at, p_all, (size_t)p_len * sizeof(int32_t));
    });
    if (st != MCM_OK) return st;
    ws.held.push_back(blob);
    const int32_t *p_dev = with_p ? (const int32_t *)((char *)blob + dims_at) : nullptr;
    return run_paren((const ParenChain *)blob, count, max_n, s_all, p_dev, lo_all, hi_all,
                     cost_all, queue, nullptr, stream);
}

}  // extern "C"
