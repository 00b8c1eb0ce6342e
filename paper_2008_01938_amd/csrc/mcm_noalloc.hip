// mcm_solve_noalloc: the single-chain tiled solve with every buffer beyond
// the caller's inputs and outputs in one fixed device array, for callers
// that cannot allocate device memory.
//
// The array (`scratch`, MCM_NOALLOC_SCRATCH_BYTES, 256-byte aligned) is a
// file-scope __device__ object: every device the library runs on holds its
// own copy from code-object load until the process ends.  Host code never
// passes the array's name to a kernel (on the host it is only a stand-in
// symbol); the device address comes from hipGetSymbolAddress, taken once
// per device on the first call with that device current, and every launch
// and copy uses that address.
//
// Layout of one call (256-byte aligned regions):
//   dims int32 [n+1] | dims fp64 [n+1] | TileChain / TileSeg tables |
//   packed partial minima of the bulk (two halves, by tile-diagonal parity)
// The dims and tables reach the array through kernel arguments (k_stage,
// a few KB per launch), so the call needs no staging buffer and no copy
// from pageable memory; the fp64 dims are widened on the device.  The
// launches run on the caller's stream in the serial schedule (no second
// stream, no events).  Nothing in the array has to start at zero: every
// byte a kernel of the call reads was written earlier in the same call.
#include <string.h>

#include <mutex>
#include <vector>

#include "mcm_internal.h"

namespace mcm {
namespace {

__device__ __align__(256) unsigned char scratch[MCM_NOALLOC_SCRATCH_BYTES];

constexpr int kStageWords = 960;  // 3840 bytes of payload per launch
struct StageArgs {
    uint32_t off_words;  // destination, 32-bit words from the array's base
    uint32_t words;      // payload words (<= kStageWords)
    uint32_t data[kStageWords];
};

__global__ __launch_bounds__(256) void k_stage(uint32_t *__restrict__ base, StageArgs a)
{
    for (uint32_t i = threadIdx.x; i < a.words; i += 256) base[a.off_words + i] = a.data[i];
}

constexpr int kMaxDevices = 64;
std::mutex g_mu;
unsigned char *g_base[kMaxDevices] = {};

// The array's device address on the current device (looked up once).
mcm_status scratch_base(unsigned char **out)
{
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kMaxDevices)
        return MCM_ERR_DEVICE;
    std::lock_guard<std::mutex> lk(g_mu);
    if (g_base[dev] == nullptr) {
        void *ptr = nullptr;
        if (hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)) != hipSuccess || ptr == nullptr)
            return MCM_ERR_DEVICE;
        g_base[dev] = (unsigned char *)ptr;
    }
    *out = g_base[dev];
    return MCM_OK;
}

size_t align256(size_t x) { return (x + 255) / 256 * 256; }

}  // namespace

bool noalloc_plan(const ChainInfo &ci, int cus, int slots_per_cu, size_t cap, TiledPlan &plan,
                  NoallocLayout &lay)
{
    // Bulk chunking: first the serial schedule's fit to the whole device,
    // then ever fewer chunks per tile-diagonal until the partials fit.
    static const int kTargets[] = {0, 1024, 512, 256, 128, 64, 32, 16, 8, 4, 2, 1};
    for (int target : kTargets) {
        if (target == 0 && (cus < 64 || slots_per_cu < 1)) continue;
        plan = TiledPlan();
        plan.wide = !tiled_accepts(ci);
        plan.lone = true;
        plan.serial = true;
        plan.cus = cus;
        plan.slots_per_cu = slots_per_cu;
        plan.chunk_target = target;
        const int c = plan_add_chain(plan, ci, 0, 0, 0, 0);
        plan_lockstep(plan, {c});
        plan_make_serial(plan);
        NoallocLayout l{};
        l.p_off = 0;
        l.pd_off = align256((size_t)(ci.n + 1) * sizeof(int32_t));
        l.tab_off = l.pd_off + align256((size_t)(ci.n + 1) * sizeof(double));
        l.tab_bytes = plan_tables_bytes(plan, &l.seg_rel);
        l.part_off = l.tab_off + align256(l.tab_bytes);
        l.total = l.part_off + plan.part_elems * sizeof(uint64_t);
        if (l.total <= cap) {
            lay = l;
            return true;
        }
    }
    return false;
}

}  // namespace mcm

using namespace mcm;

extern "C" mcm_status mcm_solve_noalloc(const int32_t *p, int32_t n, int64_t *m_out,
                                        int32_t *s_out, hipStream_t stream)
{
    ChainInfo ci;
    mcm_status st = check_chain(p, n, &ci);
    if (st != MCM_OK) return st;
    if (m_out == nullptr || s_out == nullptr || ((uintptr_t)m_out & 7) != 0 ||
        ((uintptr_t)s_out & 3) != 0)
        return MCM_ERR_INVALID_ARG;
    if (n > MCM_NOALLOC_MAX_N) return MCM_ERR_UNSUPPORTED;

    TiledPlan plan;
    NoallocLayout lay;
    if (!noalloc_plan(ci, device_cus(), bulk_blocks_per_cu(), MCM_NOALLOC_SCRATCH_BYTES, plan,
                      lay))
        return MCM_ERR_UNSUPPORTED;
    unsigned char *base = nullptr;
    if ((st = scratch_base(&base)) != MCM_OK) return st;

    // Host image of the dims and the tables, staged word by word.
    std::vector<uint32_t> img((lay.tab_off + lay.tab_bytes + 3) / 4, 0u);
    memcpy(img.data(), p, (size_t)(n + 1) * sizeof(int32_t));
    plan_tables_write(plan, (char *)img.data() + lay.tab_off);
    StageArgs a;
    auto stage = [&](size_t w0, size_t w1) -> bool {
        for (size_t w = w0; w < w1; w += kStageWords) {
            a.off_words = (uint32_t)w;
            a.words = (uint32_t)(w1 - w < (size_t)kStageWords ? w1 - w : (size_t)kStageWords);
            memcpy(a.data, img.data() + w, a.words * sizeof(uint32_t));
            hipLaunchKernelGGL(k_stage, dim3(1), dim3(256), 0, stream, (uint32_t *)base, a);
            if (hipGetLastError() != hipSuccess) return false;
        }
        return true;
    };
    if (!stage(0, (size_t)(n + 1)) || !stage(lay.tab_off / 4, img.size())) return MCM_ERR_DEVICE;

    const int32_t *p_dev = (const int32_t *)(base + lay.p_off);
    double *pd_dev = (double *)(base + lay.pd_off);
    if ((st = widen_dims(p_dev, pd_dev, (size_t)n + 1, stream)) != MCM_OK) return st;
    const TileChain *chains = (const TileChain *)(base + lay.tab_off);
    const TileSeg *segs = (const TileSeg *)(base + lay.tab_off + lay.seg_rel);
    return exec_tiled_plan(plan, chains, segs, p_dev, pd_dev, m_out, s_out,
                           (uint64_t *)(base + lay.part_off), stream);
}
