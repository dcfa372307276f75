// Grouped persistent launch (placeholder until the persistent kernel lands).
#include <hip/hip_runtime.h>

#include "abi_internal.hpp"
#include "mgemm.h"

namespace mg {
int grouped_device_init(DevState *) { return GEMM_OK; }
void grouped_device_free(DevState *) {}
}  // namespace mg

extern "C" {
int gemm_grouped(int64_t, const gemm_problem *, int) { return GEMM_E_UNSUPPORTED; }
int64_t gemm_grouped_capacity(void) { return 0; }
int gemm_grouped_slot_create(void **) { return GEMM_E_UNSUPPORTED; }
int gemm_grouped_slot_write(void *, int64_t, const gemm_problem *, int) { return GEMM_E_UNSUPPORTED; }
int gemm_grouped_slot_launch(void *) { return GEMM_E_UNSUPPORTED; }
void gemm_grouped_slot_destroy(void *) {}
}
