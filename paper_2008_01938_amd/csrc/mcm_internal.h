// Library-internal declarations shared by the C ABI layer and the kernel
// translation units.  Not part of the public ABI.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "../../include/mcm.h"

namespace mcm {

// Kernel classes for the profiler (must match mcm_profile_read's doc).
enum KernelClass { KC_SETUP = 0, KC_BULK = 1, KC_CLOSE = 2, KC_WAVE = 3, KC_BATCH = 4, KC_COUNT = 5 };

// Host-side facts about a chain, computed once per call.
struct ChainInfo {
    int32_t n = 0;
    int32_t pmax = 0;
    // bit length of (n-1) * pmax^3 (the largest possible candidate cost).
    int32_t cost_bits = 0;
};

// Launch bracket for the profiler: records an event pair around the launch
// when profiling is enabled, and accounts the split evaluations.
struct ProfileScope {
    ProfileScope(int cls, hipStream_t stream, double evals);
    ~ProfileScope();
    int cls_;
    hipStream_t stream_;
    double evals_;
    hipEvent_t start_ = nullptr;
};

// Device copies of the chain, in the forms the kernels read.
struct DeviceChain {
    const int32_t *p = nullptr;   // n+1 int32
    const double *pd = nullptr;   // n+1 doubles (exact copies of p)
};

// Stream-ordered workspace allocation (hipMallocAsync on the call's stream).
hipError_t ws_alloc(void **ptr, size_t bytes, hipStream_t stream);
void ws_free(void *ptr, hipStream_t stream);

// Wavefront path (int64, any valid input).
mcm_status run_wavefront(const DeviceChain &dc, const ChainInfo &ci, int64_t *m, int32_t *s,
                         hipStream_t stream);

// Tiled path (exact integers carried in fp64; see can_run_tiled).
bool tiled_accepts(const ChainInfo &ci);
mcm_status run_tiled(const DeviceChain &dc, const ChainInfo &ci, int64_t *m, int32_t *s,
                     hipStream_t stream);

}  // namespace mcm
