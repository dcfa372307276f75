// gemm_noalloc: gemm() for callers that cannot allocate device memory.  The
// workspace of the configurations that need one (the packed split product's
// bf16 operand pieces, split-K's partial tiles) is a fixed device array of
// this file instead of the calling stream's reservation, so the call never
// reaches an allocator and needs no gemm_init / gemm_reserve_workspace.
#include <hip/hip_runtime.h>

#include <mutex>

#include "abi_internal.hpp"
#include "mgemm.h"

namespace mg {

// Every GPU the library runs on holds its own copy of this array (in the
// loaded code object) until the process ends.
static __device__ __align__(256) char scratch[kNoallocScratchBytes];

// Device address of `scratch` per device.  The array's name in host code
// is a host-side stand-in, never a device address: kernels only ever get
// these pointers.
static void *g_scratch_ptr[kMaxDevices];
static std::mutex g_scratch_mu;

int scratch_device_init(int device)
{
    if (device < 0 || device >= kMaxDevices) return GEMM_E_NOINIT;
    std::lock_guard<std::mutex> g(g_scratch_mu);
    if (g_scratch_ptr[device]) return GEMM_OK;
    int cur = -1;
    hipError_t e = hipGetDevice(&cur);
    if (e == hipSuccess && cur != device) e = hipSetDevice(device);
    void *p = nullptr;
    if (e == hipSuccess) e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (cur >= 0 && cur != device) (void)hipSetDevice(cur);
    if (e != hipSuccess || !p) {
        t_tls.hip_err = (int)e;
        (void)hipGetLastError();
        return GEMM_E_HIP;
    }
    g_scratch_ptr[device] = p;
    return GEMM_OK;
}

}  // namespace mg

using namespace mg;

extern "C" int gemm_noalloc(char transA, char transB, int64_t m, int64_t n, int64_t k,
                            double alpha, const void *A, int64_t lda, const void *B, int64_t ldb,
                            double beta, void *C, int64_t ldc, int dtype)
{
    const int v = validate(transA, transB, m, n, k, alpha, A, lda, B, ldb, beta, C, ldc, dtype);
    if (v != 0) return v;
    if (m == 0 || n == 0) return GEMM_OK;
    if ((alpha == 0.0 || k == 0) && beta == 1.0) return GEMM_OK;
    DevState *d = nullptr;
    int rc = device_state(&d);
    if (rc != GEMM_OK) return rc;
    rc = scratch_device_init(d->device);
    if (rc != GEMM_OK) return rc;
    Workspace w;
    w.ptr = g_scratch_ptr[d->device];
    w.bytes = kNoallocScratchBytes;
    return gemm_ws(transA, transB, m, n, k, alpha, A, lda, B, ldb, beta, C, ldc, dtype, w, true);
}

extern "C" int64_t gemm_noalloc_scratch_bytes(void) { return (int64_t)kNoallocScratchBytes; }
