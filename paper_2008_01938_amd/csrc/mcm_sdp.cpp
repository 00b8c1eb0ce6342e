// C ABI of the simplified DP (S-DP) solver: validation, the plan tables the
// kernels read (offset chunks, near-offset tables), upload and workspace.
#include <cstring>
#include <vector>

#include "mcm.h"
#include "mcm_internal.h"

using namespace mcm;

namespace {

constexpr int kSdpBlock = 2048;      // elements per far/near launch pair
constexpr int kChunkMax = 1024;      // offsets per far workgroup (old terms)
constexpr int kChunkMaxNew = 64;     // ... for the terms on the critical path
constexpr int kSpanMax = 8192 - 256; // a[j0] - a[j1-1] within a chunk

size_t align8(size_t x) { return (x + 7) / 8 * 8; }

}  // namespace

extern "C" {

mcm_status mcm_sdp_solve(const int32_t *a, int32_t k, int32_t op, int32_t *st, int32_t n,
                         hipStream_t stream)
{
    if (a == nullptr || st == nullptr || k < 1 || n < 1) return MCM_ERR_INVALID_ARG;
    if (((uintptr_t)st & 3) != 0) return MCM_ERR_INVALID_ARG;
    if (op != MCM_SDP_MIN && op != MCM_SDP_MAX && op != MCM_SDP_ADD) return MCM_ERR_INVALID_ARG;
    if (a[k - 1] < 1 || a[0] > n) return MCM_ERR_INVALID_ARG;
    for (int32_t j = 1; j < k; ++j)
        if (a[j] >= a[j - 1]) return MCM_ERR_INVALID_ARG;
    if (a[0] == n) return MCM_OK;    // every element is preset
    if (hipGetLastError() != hipSuccess) return MCM_ERR_DEVICE;

    const int B = kSdpBlock;
    // Far kernel chunks: runs of consecutive offsets, at most kChunkMax of
    // them spanning at most kSpanMax values (their sources fit in LDS).  No
    // chunk mixes offsets >= 2B with smaller ones: the former ("old" terms)
    // read only elements two blocks back and are folded ahead of time.
    std::vector<int32_t> chunks;
    int chunk_max = 0, span_max = 0, nchunks_old = 0;
    const int32_t old_min = 2 * kSdpBlock;
    for (int32_t j0 = 0; j0 < k;) {
        const bool old = a[j0] >= old_min;
        // A far workgroup's time grows with its offsets, so the new terms,
        // folded between two near launches, come in short chunks.
        const int32_t cmax = old ? kChunkMax : kChunkMaxNew;
        int32_t j1 = j0 + 1;
        while (j1 < k && j1 - j0 < cmax && a[j0] - a[j1] <= kSpanMax &&
               (a[j1] >= old_min) == old)
            ++j1;
        chunks.push_back(j0);
        chunks.push_back(j1);
        if (old) ++nchunks_old;
        if (j1 - j0 > chunk_max) chunk_max = j1 - j0;
        if (a[j0] - a[j1 - 1] > span_max) span_max = a[j0] - a[j1 - 1];
        j0 = j1;
    }
    const int nchunks = (int)chunks.size() / 2;
    // Near tables: offsets below B ascending, their prefix counts, and the
    // in-sub-block masks (offsets below 64).
    std::vector<int32_t> near_a;
    for (int32_t j = k - 1; j >= 0 && a[j] < B; --j) near_a.push_back(a[j]);
    const int kn = (int)near_a.size();

    const size_t o_a = 0;
    const size_t o_chunks = align8(o_a + (size_t)k * 4);
    const size_t o_near = align8(o_chunks + chunks.size() * 4);
    const size_t o_cnt = align8(o_near + (size_t)(kn > 0 ? kn : 1) * 4);
    const size_t o_mask = align8(o_cnt + (size_t)B * 4);
    const size_t bytes = o_mask + 64 * 8;
    void *blob = nullptr;
    mcm_status s = upload_blob(stream, &blob, bytes, [&](char *h) {
        memcpy(h + o_a, a, (size_t)k * 4);
        memcpy(h + o_chunks, chunks.data(), chunks.size() * 4);
        if (kn) memcpy(h + o_near, near_a.data(), (size_t)kn * 4);
        int32_t *cnt = (int32_t *)(h + o_cnt);
        int c = 0;
        for (int x = 0; x < B; ++x) {
            while (c < kn && near_a[c] <= x) ++c;
            cnt[x] = c;
        }
        uint64_t *mask = (uint64_t *)(h + o_mask);
        for (int l = 0; l < 64; ++l) {
            uint64_t m = 0;
            for (int c2 = 0; c2 < kn && near_a[c2] <= l; ++c2) m |= 1ull << (l - near_a[c2]);
            mask[l] = m;
        }
    });
    if (s != MCM_OK) return s;
    int32_t *part = nullptr;
    if (ws_alloc((void **)&part, (size_t)n * 4, stream) != hipSuccess) {
        ws_free(blob, stream);
        return MCM_ERR_NO_MEMORY;
    }
    SdpPlan pl;
    pl.n = n;
    pl.a1 = a[0];
    pl.B = B;
    pl.a = (const int32_t *)((char *)blob + o_a);
    pl.chunks = (const int2 *)((char *)blob + o_chunks);
    pl.nchunks = nchunks;
    pl.nchunks_old = nchunks_old;
    pl.chunk_max = chunk_max;
    pl.span_max = span_max;
    pl.near_a = (const int32_t *)((char *)blob + o_near);
    pl.kn = kn;
    pl.cnt_le = (const int32_t *)((char *)blob + o_cnt);
    pl.seq_mask = (const uint64_t *)((char *)blob + o_mask);
    pl.part = part;
    s = run_sdp(pl, op, st, stream);
    ws_free(part, stream);
    ws_free(blob, stream);
    return s;
}

}  // extern "C"
