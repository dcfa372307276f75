// Device-side request queue: the records shared by the host loop
// (serve_run_queue in serve.cpp) and the persistent kernel (queue.hip).
//
// The host publishes work as output tiles.  Tile records live in a ring in
// pinned, fine-grained host memory; `tail` (also host memory) counts the
// tiles published so far.  Workgroups of the persistent kernel claim tile
// indices in order from a device counter; the one workgroup whose claim
// equals the device's copy of the tail (the frontier) polls the host tail
// and copies it to device memory, so only one workgroup reads across PCIe
// while the queue is empty.  When the last tile of a request is done, its
// workgroup writes the request's generation number to `done[slot]` in host
// memory.
#pragma once

#include <stdint.h>

#include "device.hpp"

namespace mg {

// One published output tile: the request's arguments and the tile's index
// in its raster (128 bytes, copied into LDS by 8 lanes).
struct QTile {
    GemmArgs a;      // the request (row-major 'N','N', alpha 1, beta 0)
    int t;           // tile index within the request, 0 .. ntiles-1
    int slot;        // request slot: index into done[] and the tile counters
    int ntiles;      // tiles of the request
    int body;        // tile body: the request's dtype class (KClass)
    int gen;         // value written to done[slot] when the request completes
    int pad[3];
};
static_assert(sizeof(QTile) == 128, "tile records are 128 bytes");

// Host-written control words (pinned host memory).
struct QCtl {
    int64_t tail;    // tiles published
    int32_t stop;    // set by the host when no more work will come
    int32_t pad[13];
};

// Device-memory state of the queue.  claim and tail are reset by the host
// between kernel instances; counters reset themselves (the last tile of a
// request sets its slot's counter back to zero).
struct QDev {
    int64_t claim;   // next tile index to hand out
    int64_t tail;    // the device's copy of the published tail
    int32_t stop;    // set by the frontier: every workgroup leaves
    int32_t pad[11];
    int32_t counters[1];   // [slots]: finished tiles of the slot's request
};

// Launches the persistent kernel: `grid` workgroups of 256 threads.
// idle_polls bounds the frontier's consecutive empty polls of the host tail
// before the whole kernel leaves (the host relaunches it when work comes).
int launch_queue_kernel(const QTile *ring, int64_t ring_mask, const QCtl *ctl, int *done,
                        QDev *dev, int64_t idle_polls, int grid, hipStream_t s);

}  // namespace mg
