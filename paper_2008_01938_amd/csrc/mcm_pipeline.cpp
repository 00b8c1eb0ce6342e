// Host side of the pipeline ablation (Fig. 8 with stalls): the schedule and
// the launch around k_pipe.
#include <algorithm>
#include <cstring>
#include <vector>

#include "mcm.h"
#include "mcm_internal.h"

namespace mcm {

void pipeline_schedule(int32_t n, std::vector<int32_t> &inv, std::vector<int32_t> &elem,
                       int64_t &steps)
{
    const int64_t N = (int64_t)n * (n + 1) / 2;
    auto off = [n](int64_t d) { return d * n - d * (d - 1) / 2; };
    auto lin = [&](int64_t i, int64_t j) { return off(j - i) + i; };
    elem.assign((size_t)N, 0);
    std::vector<int64_t> sigma((size_t)N, -1);
    // ready[x]: the step at which x's last split is folded; preset elements
    // are ready before the first step.
    std::vector<int64_t> ready((size_t)N, INT64_MIN / 4);
    int64_t prev = -1, last = -1;
    for (int64_t d = 0; d < n; ++d) {
        for (int64_t i = 0; i + d < n; ++i) {
            const int64_t x = off(d) + i;
            elem[(size_t)x] = (int32_t)(i | (d << 16));
            if (d == 0) continue;
            // Split j' is read at step s + j' - 1; its operands must have been
            // folded for the last time at an earlier step.
            int64_t s = prev + 1;
            for (int64_t jp = 1; jp <= d; ++jp) {
                const int64_t k = i + jp - 1;
                s = std::max(s, ready[(size_t)lin(i, k)] - jp + 2);
                s = std::max(s, ready[(size_t)lin(k + 1, i + d)] - jp + 2);
            }
            sigma[(size_t)x] = s;
            ready[(size_t)x] = s + d - 1;
            last = std::max(last, s + d - 1);
            prev = s;
        }
    }
    inv.assign((size_t)(prev + 1 > 0 ? prev + 1 : 1), -1);
    for (int64_t x = n; x < N; ++x) inv[(size_t)sigma[(size_t)x]] = (int32_t)x;
    steps = last + 1;
}

mcm_status run_pipeline_solve(const int32_t *p_dev, int32_t n, int64_t *m, int32_t *s,
                              hipStream_t stream)
{
    if (n > kPipeMaxN) return MCM_ERR_UNSUPPORTED;
    std::vector<int32_t> inv, elem;
    int64_t steps = 0;
    pipeline_schedule(n, inv, elem, steps);
    const int64_t N = (int64_t)n * (n + 1) / 2;
    const size_t o_inv = 0, o_elem = (inv.size() * 4 + 7) / 8 * 8;
    const size_t bytes = o_elem + elem.size() * 4;
    void *blob = nullptr;
    mcm_status st = upload_blob(stream, &blob, bytes, [&](char *h) {
        memcpy(h + o_inv, inv.data(), inv.size() * 4);
        memcpy(h + o_elem, elem.data(), elem.size() * 4);
    });
    if (st != MCM_OK) return st;
    void *tab = nullptr;
    if (ws_alloc(&tab, (size_t)N * 12, stream) != hipSuccess) {
        ws_free(blob, stream);
        return MCM_ERR_NO_MEMORY;
    }
    PipePlan pl;
    pl.inv = (const int32_t *)((char *)blob + o_inv);
    pl.S = (int64_t)inv.size();
    pl.steps = steps;
    pl.elem = (const int32_t *)((char *)blob + o_elem);
    pl.st = (int64_t *)tab;
    pl.sk = (int32_t *)((char *)tab + (size_t)N * 8);
    st = run_pipeline(pl, p_dev, n, m, s, stream);
    ws_free(tab, stream);
    ws_free(blob, stream);
    return st;
}

}  // namespace mcm
