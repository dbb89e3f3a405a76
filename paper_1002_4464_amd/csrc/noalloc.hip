// Sorting without any allocation: dsort_sort_noalloc runs the same pipeline as
// dsort_keys / dsort_pairs (automatic plan), with its workspace in a fixed device array of the
// library instead of a caller buffer.  For callers that may not allocate device memory.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <mutex>

#include "dsort_internal.h"

namespace {

// The workspace of every call, one copy per device (held until the process ends).  In host
// code this name is only a handle for hipGetSymbolAddress: its device address is looked up
// once per device and kept in g_scratch.
__device__ __align__(256) unsigned char scratch[DSORT_NOALLOC_SCRATCH_BYTES];

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void *g_scratch[kMaxDevices];

// Device address of `scratch` on the current device, looked up on the first call there.
int scratch_ptr(void **out) {
    int dev = -1;
    if (hipGetDevice(&dev) != hipSuccess) {
        const hipError_t e = hipGetLastError();
        dsort::set_last_error("noalloc_device", hipGetErrorName(e), hipGetErrorString(e));
        return DSORT_E_HIP;
    }
    if (dev < 0 || dev >= kMaxDevices) return DSORT_E_UNSUPPORTED;
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch[dev]) {
        void *p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p) {
            (void)hipGetLastError();
            dsort::set_last_error("noalloc_symbol", hipGetErrorName(e), hipGetErrorString(e));
            return DSORT_E_HIP;
        }
        g_scratch[dev] = p;
    }
    *out = g_scratch[dev];
    return DSORT_OK;
}

}  // namespace

extern "C" int dsort_sort_noalloc(int key_type, int with_values, void *d_keys,
                                  uint32_t *d_values, uint64_t n, void *stream) {
    if (key_type != DSORT_U32 && key_type != DSORT_U64 && key_type != DSORT_F32)
        return DSORT_E_INVALID;
    if (with_values != 0 && with_values != 1) return DSORT_E_INVALID;
    if (n > dsort::kMaxItems) return DSORT_E_INVALID;
    if (n <= 1) return DSORT_OK;
    if (!d_keys || (with_values && !d_values) || (!with_values && d_values))
        return DSORT_E_INVALID;
    if (((uintptr_t)d_keys & (key_type == DSORT_U64 ? 7 : 3)) != 0) return DSORT_E_INVALID;
    if (with_values && ((uintptr_t)d_values & 3) != 0) return DSORT_E_INVALID;
    dsort::Geom g;  // plain host struct: planning allocates nothing
    const dsort_tuning_t automatic{};
    int rc = dsort::make_geom(key_type, with_values != 0, n, automatic, g);
    if (rc != DSORT_OK) return rc;
    if (g.total > (size_t)DSORT_NOALLOC_SCRATCH_BYTES) return DSORT_E_CAPACITY;
    void *ws = nullptr;
    rc = scratch_ptr(&ws);
    if (rc != DSORT_OK) return rc;
    // Every counter and flag the pipeline needs at zero is cleared by its first kernel.
    return dsort::run_pipeline(g, d_keys, d_values, ws, stream, nullptr);
}
