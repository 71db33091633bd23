// Allocation-free variant of cbs_residual (see cbs_residual_noalloc in
// cbs.h).  Its kernels work in a file-scope device array instead of a
// caller workspace: each GPU the library runs on holds its own copy of the
// array from module load until the process ends.  The array's device address
// is looked up once per device, with that device current, on the first call
// there; host code uses only that address, never the array's name.
#include <mutex>

#include "cbs.h"
#include "cbs_internal.h"

namespace cbs {
cbs_status residual_impl(cbs_medium m, const void* s_p, const void* s_u, const void* p, const void* u,
                         int32_t adjoint, int32_t rhs_kind, int32_t ptr_kind, double* rel_residual, void* r_p,
                         void* r_u, void* workspace, size_t ws_bytes, hipStream_t st, bool no_alloc);
size_t residual_workspace_bytes(cbs_medium m);
}  // namespace cbs

namespace {

static __device__ __align__(256) unsigned char scratch[CBS_NOALLOC_SCRATCH_BYTES];

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch[kMaxDevices] = {};   // device address of `scratch` per device

// The current device's copy of the scratch array.
cbs_status scratch_for_current_device(void** out) {
    int dev = -1;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0) return CBS_E_DEVICE;
    if (dev >= kMaxDevices) return CBS_E_UNSUPPORTED;
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (!g_scratch[dev]) {
        void* ptr = nullptr;
        if (hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)) != hipSuccess || !ptr) return CBS_E_DEVICE;
        g_scratch[dev] = ptr;
    }
    *out = g_scratch[dev];
    return CBS_OK;
}

}  // namespace

extern "C" cbs_status cbs_residual_noalloc(cbs_medium m, const void* s_p, const void* s_u, const void* p,
                                           const void* u, int32_t adjoint, int32_t rhs_kind, int32_t ptr_kind,
                                           double* rel_residual, void* r_p, void* r_u, void* hip_stream) {
    if (!m || !s_p || !p) return CBS_E_INVALID;
    if (cbs::residual_workspace_bytes(m) > CBS_NOALLOC_SCRATCH_BYTES) return CBS_E_NOMEM;
    void* ws = nullptr;
    const cbs_status cs = scratch_for_current_device(&ws);
    if (cs != CBS_OK) return cs;
    try {
        return cbs::residual_impl(m, s_p, s_u, p, u, adjoint, rhs_kind, ptr_kind, rel_residual, r_p, r_u, ws,
                                  CBS_NOALLOC_SCRATCH_BYTES, (hipStream_t)hip_stream, true);
    } catch (...) {
        return CBS_E_DEVICE;
    }
}
