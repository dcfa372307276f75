// Device-side request queue: the records shared by the host loop
// (serve_run_queue in serve.cpp) and the persistent kernel (queue.hip).
//
// The host publishes work as tiles: a request's copy tiles (its operands
// into the arena), then its output tiles.  Tile records live in a ring in
// pinned, fine-grained host memory; `tail` (also host memory) counts the
// tiles published so far.  Workgroups of the persistent kernel claim tile
// indices in order from a device counter; the one workgroup whose claim
// equals the device's copy of the tail (the frontier) polls the host tail
// and copies it to device memory, so only one workgroup reads across PCIe
// while the queue is empty.  When the last tile of a request is done, its
// workgroup writes the request's generation number to `done[slot]` in host
// memory.  An output tile waits (bounded) for its request's copy tiles,
// which were published, and so claimed, before it.
#pragma once

#include <stdint.h>

#include "device.hpp"

namespace mg {

// One published unit of work (144 bytes, copied into LDS by 9 lanes):
//   kind 1, a copy tile: a.lda bytes from a.A to a.C (a request's operands
//     materialised in the arena at admission, in chunks of kCopyChunk);
//   kind 0, an output tile: the request's arguments and the tile's index in
//     its raster; it starts once the request's ncopy copy tiles are done.
struct QTile {
    GemmArgs a;      // the request (row-major 'N','N', alpha 1, beta 0), or the copy
    int t;           // tile index within the request, 0 .. ntiles-1
    int slot;        // request slot: index into done[] and the device counters
    int ntiles;      // output tiles of the request
    int body;        // tile body: the request's dtype class (KClass)
    int gen;         // value written to done[slot] when the request completes
    int kind;        // 0 output tile, 1 copy tile
    int ncopy;       // copy tiles of the request
    int pad;
};
constexpr int64_t kCopyChunk = 256 << 10;   // bytes per copy tile
static_assert(sizeof(QTile) == 144, "tile records are 144 bytes");

// Control words in pinned host memory: tail and stop written by the host,
// fault and claimed by the kernel.
struct QCtl {
    int64_t tail;      // tiles published
    int32_t stop;      // set by the host when no more work will come
    int32_t fault;     // set by the kernel: an output tile's operands never arrived
    int64_t claimed;   // 1 + a recently claimed tile index, stored for every
                       // 16th tile by the workgroup claiming it (stores land
                       // in any order): fewer than 16 + workgroups behind the
                       // claims; how far the kernel has taken the ring
    int32_t pad[10];
};
static_assert(sizeof(QCtl) == 64, "control words are one 64-byte line");

// Device-memory state of the queue.  claim and tail are reset by the host
// between kernel instances; the per-slot counters reset themselves (the last
// output tile of a request sets both of its slot's counters back to zero).
struct QDev {
    int64_t claim;   // next tile index to hand out
    int64_t tail;    // the device's copy of the published tail
    int32_t stop;    // set by the frontier: every workgroup leaves
    int32_t pad[11];
    int32_t counters[1];   // [2 * slots]: finished output tiles of the slot's request,
                           // then finished copy tiles
};

// Launches the persistent kernel: `grid` workgroups of 256 threads.
// idle_polls bounds the frontier's consecutive empty polls of the host tail
// before the whole kernel leaves (the host relaunches it when work comes).
int launch_queue_kernel(const QTile *ring, int64_t ring_mask, QCtl *ctl, int *done, QDev *dev,
                        int slots, int64_t idle_polls, int grid, hipStream_t s);

}  // namespace mg
