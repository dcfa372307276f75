// Persistent request-queue kernel (device side of serve_run_queue).
//
// Each workgroup loops: claim the next tile index, wait until the host has
// published it, copy its 144-byte record into LDS, and run it.  A copy tile
// moves one chunk of a request's operands into the arena and counts itself
// in the slot's copy counter.  An output tile waits for that counter to
// reach the request's copy tiles, then runs the tile body of the request's
// dtype class (the same direct-staged and split-at-read tiles as the grouped
// kernel's compact bodies, so a tile's bits equal the standalone GEMM's) and
// counts itself; the workgroup that finishes a request's last output tile
// tells the host.  A request's copy tiles are published before its output
// tiles and claimed in order, so they are running whenever an output tile
// waits for them.
//
// Every wait is bounded.  The frontier (the workgroup whose claim equals the
// device's copy of the tail) counts consecutive empty polls of the host and,
// past idle_polls or when the host sets stop, sets the device stop word, on
// which every other workgroup leaves.  Those count their own polls as well
// (each about half as long as the frontier's) and leave after sixteen times
// as many without progress, so no wave can wait forever even if the
// frontier is gone.  A workgroup leaves only from the wait, never with a
// published tile in hand, so the host can relaunch the kernel from the
// device's tail.  An output tile whose copies do not arrive within a bound
// (which would be a bug) raises the fault word for the host.
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
// The polls are relaxed loads: an acquiring load invalidates the compute
// unit's caches and its L2 at every poll, which the workgroups still
// computing on that XCD would pay for.  One acquire follows the wait.
__device__ bool wait_published(int64_t t, QCtl *ctl, QDev *dev, int64_t idle_polls)
{
    int64_t polls = 0, seen = -1;
    for (;;) {
        const int64_t dt = __hip_atomic_load(&dev->tail, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        if (t < dt) {
            __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
            // claim progress for the host's publication pacing, every 16th
            // tile: the barrier after the claim waits for this store to reach
            // host memory
            if ((t & 15) == 0)
                __hip_atomic_store(&ctl->claimed, t + 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
            return true;
        }
        if (__hip_atomic_load(&dev->stop, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)) return false;
        if (dt != seen) {
            seen = dt;
            polls = 0;
        }
        if (t == dt) {
            // the frontier: poll the host
            const int64_t ht = __hip_atomic_load(&ctl->tail, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
            if (ht > dt) {
                __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "");
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

// One copy tile: `bytes` from src to dst (dst 16-byte aligned; 16-byte
// vectors when src and bytes allow).
__device__ void copy_chunk(const char *src, char *dst, int64_t bytes, int tid)
{
    if ((((uintptr_t)src | (uintptr_t)bytes) & 15) == 0) {
        const u32x4 *s4 = (const u32x4 *)src;
        u32x4 *d4 = (u32x4 *)dst;
        const int64_t n = bytes >> 4;
        int64_t i = tid;
        for (; i + 3 * 256 < n; i += 4 * 256) {
            const u32x4 v0 = s4[i], v1 = s4[i + 256], v2 = s4[i + 512], v3 = s4[i + 768];
            d4[i] = v0;
            d4[i + 256] = v1;
            d4[i + 512] = v2;
            d4[i + 768] = v3;
        }
        for (; i < n; i += 256) d4[i] = s4[i];
    } else {
        for (int64_t i = tid; i < bytes; i += 256) dst[i] = src[i];
    }
}

__global__ void __launch_bounds__(256, 2) queue_kernel(const QTile *ring, int64_t ring_mask,
                                                       QCtl *ctl, int *done, QDev *dev, int slots,
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
        // the record is in fine-grained host memory, read uncached
        if (tid < (int)(sizeof(QTile) / 16))
            ((u32x4 *)&s_tile)[tid] = ((const u32x4 *)(ring + (t & ring_mask)))[tid];
        __syncthreads();
        const GemmArgs p = s_tile.a;
        const int slot = s_tile.slot;
        int *out_count = &dev->counters[slot], *copy_count = &dev->counters[slots + slot];
        if (s_tile.kind == 1) {
            copy_chunk((const char *)p.A, (char *)p.C, p.lda, tid);
            // the chunk, visible to every compute unit before it is counted
            __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
            __syncthreads();
            if (tid == 0) __hip_atomic_fetch_add(copy_count, 1, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
            __syncthreads();   // s_t and s_tile are rewritten next
            continue;
        }
        const int body = s_tile.body, ntiles = s_tile.ntiles, gen = s_tile.gen;
        if (tid == 0) {
            // the request's operands: its copy tiles were claimed before this
            // tile and are running or done
            const int ncopy = s_tile.ncopy;
            int64_t polls = 0;
            while (__hip_atomic_load(copy_count, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) < ncopy) {
                if (++polls > (int64_t)1 << 24) {
                    __hip_atomic_store(&ctl->fault, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
                    break;
                }
                __builtin_amdgcn_s_sleep(2);
            }
        }
        __syncthreads();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
        int tm, tn;
        raster(s_tile.t, p.tiles_m, p.tiles_n, p.order, p.group, tm, tn);
        run_body(body, p, tm, tn, lds);
        // this workgroup's C stores, visible outside its L2 before the tile is
        // counted (the arena is reused by later copies)
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
        __syncthreads();
        if (tid == 0) {
            const int before = __hip_atomic_fetch_add(out_count, 1, __ATOMIC_ACQ_REL, __HIP_MEMORY_SCOPE_AGENT);
            if (before == ntiles - 1) {
                __hip_atomic_store(out_count, 0, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                __hip_atomic_store(copy_count, 0, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                __builtin_amdgcn_fence(__ATOMIC_RELEASE, "");
                __hip_atomic_store(&done[slot], gen, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_SYSTEM);
            }
        }
        __syncthreads();   // s_t and s_tile are rewritten next
    }
}

}  // namespace

int launch_queue_kernel(const QTile *ring, int64_t ring_mask, QCtl *ctl, int *done, QDev *dev,
                        int slots, int64_t idle_polls, int grid, hipStream_t s)
{
    hipLaunchKernelGGL(queue_kernel, dim3(grid), dim3(256), 0, s, ring, ring_mask, ctl, done, dev,
                       slots, idle_polls);
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) {
        t_tls.hip_err = (int)e;
        return GEMM_E_HIP;
    }
    return GEMM_OK;
}

}  // namespace mg
