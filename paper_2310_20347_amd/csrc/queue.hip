// Persistent request-queue kernel (device side of serve_run_queue).
//
// Each workgroup loops: claim the next tile index, wait until the host has
// published it, copy its 128-byte record into LDS, run the tile body of the
// request's dtype class (the same direct-staged and split-at-read tiles as
// the grouped kernel's compact bodies, so a tile's bits equal the standalone
// GEMM's), publish the tile, and count it; the workgroup that finishes a
// request's last tile tells the host.
//
// Every wait is bounded.  The frontier (the workgroup whose claim equals the
// device's copy of the tail) counts consecutive empty polls of the host and,
// past idle_polls or when the host sets stop, sets the device stop word, on
// which every other workgroup leaves.  Those count their own polls as well
// (each about half as long as the frontier's) and leave after sixteen times
// as many without progress, so no wave can wait forever even if the
// frontier is gone.  A workgroup leaves only from the wait, never with a
// published tile in hand, so the host can relaunch the kernel from the
// device's tail.
#include <hip/hip_runtime.h>

#include "abi_internal.hpp"
#include "grouped.hpp"
#include "mgemm.h"
#include "queue.hpp"

namespace mg {
namespace {

// Tile bodies by dtype class (KClass order).
typedef DShape<TF32, 128, 128, 2> QB0;
typedef SDShape<2, 128, 128, 2> QB1;
typedef SDShape<3, 64, 64, 2> QB2;
typedef DShape<TBF16, 128, 128, 2> QB3;
typedef DShape<TF16, 128, 128, 2> QB4;
typedef DShape<TF8, 128, 128, 2> QB5;
typedef DShape<TI8, 128, 128, 2> QB6;
constexpr int kQueueLds =
    cmax(cmax(cmax(QB0::lds, QB1::lds), cmax(QB2::lds, QB3::lds)), cmax(cmax(QB4::lds, QB5::lds), QB6::lds));

__device__ __forceinline__ void run_body(int body, const GemmArgs &p, int tm, int tn, char *lds)
{
    switch (body) {
    case K_F32: QB0::run(p, tm, tn, lds); break;
    case K_SPLIT2: QB1::run(p, tm, tn, lds); break;
    case K_SPLIT3: QB2::run(p, tm, tn, lds); break;
    case K_BF16: QB3::run(p, tm, tn, lds); break;
    case K_F16: QB4::run(p, tm, tn, lds); break;
    case K_F8: QB5::run(p, tm, tn, lds); break;
    default: QB6::run(p, tm, tn, lds); break;
    }
}

// Waits until tile t is published.  Returns true to run it, false to leave.
__device__ bool wait_published(int64_t t, const QCtl *ctl, QDev *dev, int64_t idle_polls)
{
    int64_t polls = 0, seen = -1;
    for (;;) {
        const int64_t dt = __hip_atomic_load(&dev->tail, __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_AGENT);
        if (t < dt) return true;
        if (__hip_atomic_load(&dev->stop, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)) return false;
        if (dt != seen) {
            seen = dt;
            polls = 0;
        }
        if (t == dt) {
            // the frontier: poll the host
            const int64_t ht = __hip_atomic_load(&ctl->tail, __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_SYSTEM);
            if (ht > dt) {
                __hip_atomic_fetch_max(&dev->tail, ht, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
                continue;
            }
            if (__hip_atomic_load(&ctl->stop, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM) ||
                ++polls > idle_polls) {
                __hip_atomic_store(&dev->stop, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                return false;
            }
            __builtin_amdgcn_s_sleep(4);
        } else {
            if (++polls > 16 * idle_polls + 4096) return false;
            __builtin_amdgcn_s_sleep(32);
        }
    }
}

__global__ void __launch_bounds__(256, 2) queue_kernel(const QTile *ring, int64_t ring_mask,
                                                       const QCtl *ctl, int *done, QDev *dev,
                                                       int64_t idle_polls)
{
    __shared__ __attribute__((aligned(16))) char lds[kQueueLds];
    __shared__ __attribute__((aligned(16))) QTile s_tile;
    __shared__ int64_t s_t;
    const int tid = threadIdx.x;
    for (;;) {
        if (tid == 0) {
            const int64_t t = (int64_t)atomicAdd((unsigned long long *)&dev->claim, 1ull);
            s_t = wait_published(t, ctl, dev, idle_polls) ? t : -1;
        }
        __syncthreads();
        const int64_t t = s_t;
        if (t < 0) break;
        // the record and the operands it names were written by other agents
        // (the host; copies) before the tail that published t
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "");
        if (tid < 8) ((u32x4 *)&s_tile)[tid] = ((const u32x4 *)(ring + (t & ring_mask)))[tid];
        __syncthreads();
        const GemmArgs p = s_tile.a;
        const int body = s_tile.body, slot = s_tile.slot, ntiles = s_tile.ntiles;
        const int gen = s_tile.gen;
        int tm, tn;
        raster(s_tile.t, p.tiles_m, p.tiles_n, p.order, p.group, tm, tn);
        run_body(body, p, tm, tn, lds);
        // this workgroup's C stores, visible to the host's copies before the
        // tile is counted
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "");
        __syncthreads();
        if (tid == 0) {
            const int before =
                __hip_atomic_fetch_add(&dev->counters[slot], 1, __ATOMIC_ACQ_REL, __HIP_MEMORY_SCOPE_AGENT);
            if (before == ntiles - 1) {
                __hip_atomic_store(&dev->counters[slot], 0, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                __builtin_amdgcn_fence(__ATOMIC_RELEASE, "");
                __hip_atomic_store(&done[slot], gen, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_SYSTEM);
            }
        }
        __syncthreads();   // s_t and s_tile are rewritten next
    }
}

}  // namespace

int launch_queue_kernel(const QTile *ring, int64_t ring_mask, const QCtl *ctl, int *done, QDev *dev,
                        int64_t idle_polls, int grid, hipStream_t s)
{
    hipLaunchKernelGGL(queue_kernel, dim3(grid), dim3(256), 0, s, ring, ring_mask, ctl, done, dev,
                       idle_polls);
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) {
        t_tls.hip_err = (int)e;
        return GEMM_E_HIP;
    }
    return GEMM_OK;
}

}  // namespace mg
