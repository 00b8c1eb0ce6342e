// Host-only checks of the library's validation and planning code, built with
// AddressSanitizer and UndefinedBehaviorSanitizer on the host side (the
// device code is compiled but never launched: no GPU is needed).
//
// 1. Every C entry point rejects bad input before any device call.
// 2. ranges_disjoint agrees with a brute-force overlap test.
// 3. Tiled plans (lone chains on the overlapped and serial schedules, fixed
//    chunk counts, and lockstep batches) cover the bulk split range of every
//    tile of every tile-diagonal exactly once, give each chunk its own
//    partial slot, keep every partial inside the plan's buffer, hand each
//    closure the slot count its bulk wrote, and never let a bulk write the
//    partials a closure of the same iteration reads.
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include <algorithm>
#include <array>
#include <map>
#include <random>
#include <set>
#include <tuple>
#include <vector>

#include "../../paper_2008_01938_amd/csrc/mcm_internal.h"

using namespace mcm;

static int g_fail = 0;
#define CHECK(c)                                                               \
    do {                                                                       \
        if (!(c)) {                                                            \
            fprintf(stderr, "check failed: %s (line %d)\n", #c, __LINE__);     \
            ++g_fail;                                                          \
        }                                                                      \
    } while (0)

static void check_rejections()
{
    int64_t m[16];
    int32_t s[16];
    for (int i = 0; i < 16; ++i) m[i] = 7, s[i] = 7;
    int32_t p_bad[3] = {3, 0, 4}, p_ok[3] = {2, 3, 4};
    int32_t p_big[3] = {1 << 21, 1 << 21, 1 << 21};
    CHECK(mcm_check_chain(p_bad, 2) == MCM_ERR_INVALID_ARG);
    CHECK(mcm_check_chain(p_big, 2) == MCM_ERR_OVERFLOW);
    CHECK(mcm_check_chain(nullptr, 2) == MCM_ERR_INVALID_ARG);
    CHECK(mcm_check_chain(p_ok, 0) == MCM_ERR_INVALID_ARG);
    CHECK(mcm_solve(p_bad, 2, m, s, nullptr) == MCM_ERR_INVALID_ARG);
    CHECK(mcm_solve(p_big, 2, m, s, nullptr) == MCM_ERR_OVERFLOW);
    CHECK(mcm_solve(p_ok, 2, nullptr, s, nullptr) == MCM_ERR_INVALID_ARG);
    CHECK(mcm_solve_algo(p_ok, 2, m, s, 9, nullptr) == MCM_ERR_INVALID_ARG);
    // batched: overlapping tables, zero n, negative offsets
    int32_t ns[2] = {2, 2};
    int64_t poff[2] = {0, 0}, toff[2] = {0, 3};
    CHECK(mcm_solve_batched(2, ns, poff, p_ok, toff, m, s, nullptr) == MCM_ERR_INVALID_ARG);
    int32_t ns0[2] = {2, 0};
    int64_t toff2[2] = {0, 4};
    CHECK(mcm_solve_batched(2, ns0, poff, p_ok, toff2, m, s, nullptr) == MCM_ERR_INVALID_ARG);
    CHECK(mcm_solve_batched(-1, ns, poff, p_ok, toff2, m, s, nullptr) == MCM_ERR_INVALID_ARG);
    mcm_plan *plan = nullptr;
    CHECK(mcm_plan_create(2, ns, poff, toff, 8, &plan) == MCM_ERR_INVALID_ARG && !plan);
    CHECK(mcm_plan_create(2, ns, poff, toff2, 0, &plan) == MCM_ERR_INVALID_ARG && !plan);
    int32_t a_bad[2] = {3, 3};
    int32_t st[8];
    CHECK(mcm_sdp_solve(a_bad, 2, 0, st, 8, nullptr) == MCM_ERR_INVALID_ARG);
    int32_t q[4] = {1, 1, -1, 1};
    CHECK(mcm_obst_solve(p_ok, q, 3, m, s, nullptr) == MCM_ERR_INVALID_ARG);
    CHECK(mcm_parens_length(0) == -1 && mcm_parens_length(1) == 2);
    CHECK(mcm_server_request_bytes(p_bad, 2) == 0);
    CHECK(mcm_server_request_bytes(p_ok, 2) >= 2 * 2 * 12);
    for (int i = 0; i < 16; ++i) CHECK(m[i] == 7 && s[i] == 7);
}

static void check_ranges()
{
    std::mt19937_64 rng(7);
    for (int trial = 0; trial < 2000; ++trial) {
        const int count = 1 + (int)(rng() % 6);
        std::vector<int32_t> n(count);
        std::vector<int64_t> off(count);
        for (int b = 0; b < count; ++b) {
            n[b] = 1 + (int32_t)(rng() % 4);
            off[b] = (int64_t)(rng() % 40);
        }
        for (int sq = 0; sq < 2; ++sq) {
            bool overlap = false;
            for (int a = 0; a < count; ++a)
                for (int b = a + 1; b < count; ++b) {
                    const int64_t la = sq ? (int64_t)n[a] * n[a] : n[a] - 1;
                    const int64_t lb = sq ? (int64_t)n[b] * n[b] : n[b] - 1;
                    if (la > 0 && lb > 0 && off[a] < off[b] + lb && off[b] < off[a] + la)
                        overlap = true;
                }
            CHECK(ranges_disjoint(count, n.data(), off.data(), sq != 0) == !overlap);
        }
    }
}

// True when no interval of `a` intersects an interval of `b`, and (when
// `self` is set) the intervals of `a` are pairwise disjoint.
static bool disjoint_sets(std::vector<std::pair<int64_t, int64_t>> a,
                          std::vector<std::pair<int64_t, int64_t>> b, bool self)
{
    std::sort(a.begin(), a.end());
    if (self)
        for (size_t u = 1; u < a.size(); ++u)
            if (a[u].first < a[u - 1].second) return false;
    std::sort(b.begin(), b.end());
    size_t j = 0;
    for (const auto &x : a) {  // b sorted by start: skip those ending before x
        while (j < b.size() && b[j].second <= x.first) ++j;
        for (size_t k = j; k < b.size() && b[k].first < x.second; ++k)
            if (b[k].second > x.first) return false;
    }
    return true;
}

// Coverage and buffer checks of one tiled plan; T is the tile edge the plan
// was built for.
static void check_plan(const TiledPlan &plan, int T, const char *what)
{
    const int fail0 = g_fail;
    const int nchain = (int)plan.chains.size();
    typedef std::pair<int, int> Key;  // (chain, tile-diagonal)
    std::map<Key, std::vector<int>> cover;  // per split offset: chunks covering it
    std::map<Key, std::set<int>> slots;
    std::map<Key, int> pt, close_pt, bulk_iter, close_iter;
    std::map<Key, int64_t> part_bulk, part_close;
    // partial regions read by the closures of D and written by the bulks of
    // D+1, per D (one lockstep iteration)
    std::map<int, std::vector<std::pair<int64_t, int64_t>>> reads, writes;
    const int64_t TT = (int64_t)T * T * (plan.wide ? 2 : 1);  // partial words per slot
    for (size_t li = 0; li < plan.launches.size(); ++li) {
        const TiledLaunch &L = plan.launches[li];
        int blocks = 0;
        for (int u = 0; u < L.nseg; ++u) {
            const TileSeg &sg = plan.segs[(size_t)L.seg_begin + u];
            CHECK(sg.first == blocks);
            CHECK(sg.chain >= 0 && sg.chain < nchain);
            const int NT = plan.NT[sg.chain];
            if (L.kind == TK_TRI) {
                blocks += NT;
                continue;
            }
            const int E = sg.D;
            CHECK(E >= 1 && E < NT);
            const Key key(sg.chain, E);
            if (L.kind == TK_CLOSE) {
                blocks += NT - E;
                CHECK(close_iter.count(key) == 0);
                close_pt[key] = sg.PT;
                part_close[key] = sg.part_off;
                close_iter[key] = (int)li;
                if (E >= 2)
                    reads[E].push_back({sg.part_off, sg.part_off + (NT - E) * sg.PT * TT});
                continue;
            }
            blocks += (NT - E) * sg.nch;
            const int Lb = (E - 1) * T + 1;
            std::vector<int> &cv = cover[key];
            if (cv.empty()) cv.assign((size_t)Lb, 0);
            CHECK(sg.KS > 0 && sg.nch > 0 && sg.klen > 0);
            CHECK(sg.koff >= 0 && sg.koff + sg.klen <= Lb);
            CHECK((sg.nch - 1) * sg.KS < sg.klen && sg.nch * sg.KS >= sg.klen);
            for (int ch = 0; ch < sg.nch; ++ch) {
                const int k0 = sg.koff + ch * sg.KS;
                const int k1 = std::min(k0 + sg.KS, sg.koff + sg.klen);
                for (int k = k0; k < k1; ++k)
                    if (k >= 0 && k < Lb) cv[(size_t)k] += 1;
                CHECK(slots[key].insert(sg.slot0 + ch).second);
                CHECK(sg.slot0 + ch < sg.PT);
            }
            if (pt.count(key)) CHECK(pt[key] == sg.PT);
            if (part_bulk.count(key)) CHECK(part_bulk[key] == sg.part_off);
            pt[key] = sg.PT;
            part_bulk[key] = sg.part_off;
            const int64_t end = sg.part_off + (int64_t)(NT - E) * sg.PT * TT;
            CHECK(sg.part_off >= 0 && (size_t)end <= plan.part_elems);
            bulk_iter[key] = (int)li;
        }
        CHECK(blocks == L.blocks);
    }
    for (int c = 0; c < nchain; ++c) {
        const int NT = plan.NT[c];
        for (int E = 2; E < NT; ++E) {
            const Key key(c, E);
            CHECK(cover.count(key) == 1);
            if (!cover.count(key)) continue;
            for (int v : cover[key]) CHECK(v == 1);
            CHECK((int)slots[key].size() == pt[key]);
            CHECK(close_pt.count(key) && close_pt[key] == pt[key]);
            CHECK(part_close[key] == part_bulk[key]);
            CHECK(close_iter[key] > bulk_iter[key]);
            const int64_t o = part_bulk[key];
            writes[E - 1].push_back({o, o + (NT - E) * pt[key] * TT});
        }
        for (int E = 1; E < NT; ++E) CHECK(close_iter.count(Key(c, E)) == 1);
    }
    // In the iteration that closes D, the bulks of D+1 write partials while
    // the closures of D read theirs: the two sets must not meet, and the
    // writers must not share partials either.
    for (auto &kv : writes) {
        CHECK(disjoint_sets(kv.second, reads[kv.first], true));
    }
    if (g_fail != fail0) fprintf(stderr, "  in plan: %s\n", what);
}

// Static race check of a plan's schedule.  Launches run on two streams (the
// caller's, 0, and the library's second, 1) in plan order per stream, and a
// launch that names another stream's launch in `wait` starts after it
// (event or signal token).  Vector clocks give, for every launch, the last
// launch of each stream that has finished before it starts.  Every read of
// a table tile or a partial slot must then follow the launch that wrote it,
// and every write must follow the earlier reads and writes of the same
// resource (no write-after-read or write-after-write race): the readiness
// that a debug build would assert at run time, proven for the whole plan.
static void check_schedule(const TiledPlan &plan, int T, const char *what)
{
    const int fail0 = g_fail;
    const size_t nl = plan.launches.size();
    std::vector<int> stream(nl), pos(nl);
    std::vector<std::array<int, 2>> vc(nl);
    int count[2] = {0, 0};
    std::array<int, 2> last_vc[2] = {{-1, -1}, {-1, -1}};
    for (size_t li = 0; li < nl; ++li) {
        const TiledLaunch &L = plan.launches[li];
        const int st = L.stream;
        stream[li] = st;
        pos[li] = count[st]++;
        std::array<int, 2> v = last_vc[st];
        v[st] = pos[li];
        if (L.wait >= 0) {
            CHECK(L.wait < (int)li);
            const std::array<int, 2> &w = vc[(size_t)L.wait];
            v[0] = std::max(v[0], w[0]);
            v[1] = std::max(v[1], w[1]);
        }
        vc[li] = v;
        last_vc[st] = v;
    }
    // W finishes before L starts.
    auto before = [&](int W, int L) {
        return W != L && pos[(size_t)W] <= vc[(size_t)L][stream[(size_t)W]] &&
               (stream[(size_t)W] != stream[(size_t)L] || W < L);
    };
    // Resources: tiles (chain, I, J) and partial slots (start element).
    struct Use {
        int writer = -1;
        std::vector<int> readers;
    };
    std::map<std::tuple<int, int, int>, Use> tiles;
    std::map<int64_t, Use> slots;
    const int64_t words = plan.wide ? 2 : 1;
    const int64_t TT = (int64_t)T * T * words;
    auto read = [&](Use &u, int L, const char *kind) {
        if (u.writer < 0 || !before(u.writer, L)) {
            fprintf(stderr, "  %s read by launch %d not ordered after its writer %d\n", kind, L,
                    u.writer);
            CHECK(false);
        }
        u.readers.push_back(L);
    };
    auto write = [&](Use &u, int L, const char *kind) {
        if (u.writer >= 0 && u.writer != L && !before(u.writer, L)) {
            fprintf(stderr, "  %s written by launch %d races its writer %d\n", kind, L,
                    u.writer);
            CHECK(false);
        }
        for (int R : u.readers)
            if (R != L && !before(R, L)) {
                fprintf(stderr, "  %s written by launch %d races its reader %d\n", kind, L, R);
                CHECK(false);
            }
        u.writer = L;
        u.readers.clear();
    };
    for (size_t li = 0; li < nl && g_fail == fail0; ++li) {
        const TiledLaunch &L = plan.launches[li];
        const int l = (int)li;
        for (int u = 0; u < L.nseg; ++u) {
            const TileSeg &sg = plan.segs[(size_t)L.seg_begin + u];
            const int c = sg.chain, NT = plan.NT[c];
            if (L.kind == TK_TRI) {
                for (int I = 0; I < NT; ++I) write(tiles[{c, I, I}], l, "diagonal tile");
                continue;
            }
            const int D = sg.D;
            for (int I = 0; I + D < NT; ++I) {
                const int J = I + D;
                if (L.kind == TK_CLOSE) {
                    read(tiles[{c, I, I}], l, "tile");
                    read(tiles[{c, J, J}], l, "tile");
                    if (D >= 2)
                        for (int sl = 0; sl < sg.PT; ++sl)
                            read(slots[sg.part_off + ((int64_t)I * sg.PT + sl) * TT], l,
                                 "partial");
                    write(tiles[{c, I, J}], l, "tile");
                    continue;
                }
                const int n = plan.chains[c].n;
                const int kbase = (I + 1) * T - 1 + sg.koff;
                for (int ch = 0; ch < sg.nch; ++ch) {
                    const int k0 = kbase + ch * sg.KS;
                    const int k1 = std::min(k0 + sg.KS, kbase + sg.klen);  // exclusive
                    CHECK(k0 < k1 && k1 <= n);
                    for (int K = k0 / T; K <= (k1 - 1) / T; ++K) read(tiles[{c, I, K}], l, "tile");
                    for (int K = (k0 + 1) / T; K <= k1 / T && K <= J; ++K)
                        read(tiles[{c, K, J}], l, "tile");
                    write(slots[sg.part_off + ((int64_t)I * sg.PT + sg.slot0 + ch) * TT], l,
                          "partial");
                }
            }
        }
    }
    if (g_fail != fail0) fprintf(stderr, "  in schedule: %s\n", what);
}

static void check_lone_plans()
{
    const int ns[] = {1, 2, 31, 32, 33, 63, 64, 65, 128, 129, 191, 193, 300, 1000, 2048, 3001,
                      8192, 16384};
    for (int T : {64, 32})
    for (int n : ns) {
        if (T == 32 && n > 3001) continue;
        for (int mode = 0; mode < 4; ++mode) {
            ChainInfo ci;
            CHECK(chain_bound(n, 1024, &ci) == MCM_OK);
            TiledPlan plan;
            plan.T = T;
            plan.wide = T == 64 && (n % 3) == 0;
            plan.lone = mode != 3;
            plan.serial = mode == 1;
            plan.chunk_target = mode == 2 ? 512 : 0;
            plan.cus = 256;
            plan.slots_per_cu = 3;
            const int c = plan_add_chain(plan, ci, 0, 0, 0, 0);
            plan_lockstep(plan, {c});
            if (plan.serial) plan_make_serial(plan);
            char what[64];
            snprintf(what, sizeof what, "lone n=%d mode=%d T=%d", n, mode, T);
            check_plan(plan, T, what);
            check_schedule(plan, T, what);
            size_t seg_off = 0;
            const size_t bytes = plan_tables_bytes(plan, &seg_off);
            std::vector<char> buf(bytes + 1, (char)0x5a);
            plan_tables_write(plan, buf.data());
            CHECK(buf[bytes] == (char)0x5a);
            CHECK(seg_off % 256 == 0);
        }
    }
}

static void check_batch_plans()
{
    std::mt19937_64 rng(3);
    for (int trial = 0; trial < 12; ++trial) {
        TiledPlan plan;
        plan.T = trial % 2 ? 32 : 64;
        plan.wide = trial == 4 || trial == 8;
        std::vector<int> ids;
        const int count = trial >= 10 ? 4096 : 1 + (int)(rng() % 300);
        int64_t off = 0;
        for (int b = 0; b < count; ++b) {
            const int n = 16 + (int)(rng() % 497);
            ChainInfo ci;
            CHECK(chain_bound(n, 256, &ci) == MCM_OK);
            ids.push_back(plan_add_chain(plan, ci, off, off, 0, 0));
            off += (int64_t)n * n;
        }
        plan_lockstep(plan, ids);
        char what[64];
        snprintf(what, sizeof what, "batch trial %d count %d T %d wide %d", trial, count,
                 plan.T, (int)plan.wide);
        check_plan(plan, plan.T, what);
        check_schedule(plan, plan.T, what);
    }
}

// The no-allocation solve: for chains up to MCM_NOALLOC_MAX_N, with keys
// (dims <= 1024) and on the int64 kernels (dims 2^16), a plan is found whose
// dims, tables and partials fit the fixed array in disjoint aligned regions,
// and it passes the same coverage and schedule checks.
static void check_noalloc_plans()
{
    std::vector<int> ns = {1, 2, 3, 63, 64, 65, 127, 128, 129, 1000, 4095, 4096, 4097,
                           8000, MCM_NOALLOC_MAX_N - 1, MCM_NOALLOC_MAX_N};
    for (int n = 5; n < MCM_NOALLOC_MAX_N; n += 397) ns.push_back(n);
    for (int n : ns)
    for (int32_t pmax : {1024, 1 << 16}) {
        ChainInfo ci;
        CHECK(chain_bound(n, pmax, &ci) == MCM_OK);
        for (int slots : {3, 0}) {
            TiledPlan plan;
            NoallocLayout lay;
            const bool ok = noalloc_plan(ci, 256, slots, MCM_NOALLOC_SCRATCH_BYTES, plan, lay);
            CHECK(ok);
            if (!ok) continue;
            CHECK(plan.wide == (pmax > 1024 && n > 1));
            CHECK(!plan.uses_aux);
            CHECK(lay.total <= MCM_NOALLOC_SCRATCH_BYTES);
            CHECK(lay.pd_off >= (size_t)(n + 1) * 4 && lay.pd_off % 256 == 0);
            CHECK(lay.tab_off >= lay.pd_off + (size_t)(n + 1) * 8 && lay.tab_off % 256 == 0);
            CHECK(lay.part_off >= lay.tab_off + lay.tab_bytes && lay.part_off % 256 == 0);
            CHECK(lay.total == lay.part_off + plan.part_elems * sizeof(uint64_t));
            if (n % 397 == 5 && n > 2000) continue;  // coverage on a subset (time)
            char what[64];
            snprintf(what, sizeof what, "noalloc n=%d pmax=%d slots=%d", n, (int)pmax, slots);
            check_plan(plan, 64, what);
            check_schedule(plan, 64, what);
        }
    }
}

int main()
{
    check_rejections();
    check_ranges();
    check_lone_plans();
    check_batch_plans();
    check_noalloc_plans();
    if (g_fail) {
        fprintf(stderr, "%d checks failed\n", g_fail);
        return 1;
    }
    printf("host checks passed\n");
    return 0;
}
