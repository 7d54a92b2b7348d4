// batch_internal.h -- the batched launch's building blocks, shared by the
// batch entry points and the request server.
#pragma once

#include <vector>

#include "tiled.h"
#include "tiled_launch.h"

namespace kr {

// One operation group of a batch, ready to launch.
struct BatchGroup {
    int op = OP_RESIZE;
    TileCfg cfg{4, 16, 1, 1, false};
    TileGeom G{0, 0};
    int njobs = 0;
    int ntiles = 0;
    size_t lds = 0;
    const TiledJob *jobs_dev = nullptr;  // device copy of the job table
};

// Host-side job table of one operation group (tile prefix sums, launch-wide
// LDS geometry).  force: explicit configuration, else the tuned one for this
// batch class, else the default.
void build_group(int op, bool f32, int c, const std::vector<ImageJob> &imgs, BatchGroup &g,
                 std::vector<TiledJob> &table, const TileCfg *force);

// Launch one group whose job table is already on the device (g.jobs_dev).
hipError_t launch_group(const BatchGroup &g, int c, kr_dtype dt, const Epilogue &e, hipStream_t s);

// Bytes of one group's device job table for n images (256-byte multiple).
size_t table_bytes(int n);

}  // namespace kr
