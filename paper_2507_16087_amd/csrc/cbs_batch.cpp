// Batched same-shape slots for continuous-batching serving (see cbs.h).
#include "cbs.h"

extern "C" {
cbs_status cbs_batch_workspace_bytes(const cbs_grid*, int32_t, int32_t, size_t*) { return CBS_E_UNSUPPORTED; }
cbs_status cbs_batch_create(const cbs_grid*, int32_t, int32_t, void*, size_t, void*, cbs_batch*) {
    return CBS_E_UNSUPPORTED;
}
cbs_status cbs_batch_destroy(cbs_batch) { return CBS_E_UNSUPPORTED; }
cbs_status cbs_batch_submit(cbs_batch, cbs_medium, const void*, const void*, const cbs_solve_opts*, int32_t*) {
    return CBS_E_UNSUPPORTED;
}
cbs_status cbs_batch_step(cbs_batch, int32_t, uint8_t*) { return CBS_E_UNSUPPORTED; }
cbs_status cbs_batch_retire(cbs_batch, int32_t, void*, void*, int32_t, cbs_solve_info*) { return CBS_E_UNSUPPORTED; }
}
