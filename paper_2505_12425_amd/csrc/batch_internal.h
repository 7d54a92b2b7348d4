// batch_internal.h -- the batched launch's building blocks, shared by the
// batch entry points and the request server.
#pragma once

#include <vector>

#include "tiled.h"
#include "tiled_launch.h"

namespace kr {

// One operation group of a batch, ready to launch.  Its job table lists the
// items bin by bin: bins[k] is the tile range of XCD k, filled by longest
// processing time first (items by estimated bytes, largest first, each into
// the least loaded bin), so that the eight XCDs get equal shares of the work
// while each image's tiles stay on one XCD's L2.
struct BatchGroup {
    int op = OP_RESIZE;
    TileCfg cfg{4, 16, 1, 1, GRID_FULL};
    TileGeom G{0, 0};
    int njobs = 0;
    int ntiles = 0;
    TileBins bins{};
    size_t lds = 0;
    const TiledJob *jobs_dev = nullptr;  // device copy of the job table
};

// Every launch of a batch: one group (one launch) per operation.  Items whose
// source boxes fit the group's tile shape within the batch LDS budget are
// staged through LDS; the tiles of the others read their taps from global
// memory in the same launch.
struct BatchBuild {
    std::vector<BatchGroup> groups;
    std::vector<std::vector<TiledJob>> tables;
    // device bytes of all job tables, each 256-byte aligned
    size_t bytes() const;
    // the tables concatenated at their device offsets (host staging image)
    void pack(uint8_t *host) const;
    // point every group at its table inside a device buffer holding pack()'s image
    void bind(void *dev);
};

// Build the launches of a batch (imgs[0]: resizes, imgs[1]: warps).  force[k]:
// primary configuration of operation k (NULL: tuned for this batch class,
// else the default).
void build_batch(const std::vector<ImageJob> imgs[2], bool f32, int c, const TileCfg *const force[2],
                 BatchBuild &b);

// Launch one group whose job table is already on the device (g.jobs_dev).
hipError_t launch_group(const BatchGroup &g, int c, kr_dtype dt, const Epilogue &e, hipStream_t s);

// Most groups a batch can have.
constexpr int KB_MAX_GROUPS = 4;

// Bytes of n job records, 256-byte multiple.
size_t table_bytes(int n);

}  // namespace kr
