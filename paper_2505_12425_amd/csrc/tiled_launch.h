// tiled_launch.h -- host-side helpers shared by the per-image and batched
// launches of the tiled kernels.
#pragma once

#include "kr_internal.h"

namespace kr {

struct TiledJob;
struct TileGeom;

constexpr size_t KT_LDS_CAP = 64 * 1024;  // dynamic LDS per workgroup

// One tile configuration: runs of PX consecutive pixels per lane, TXT lanes
// per tile row, CPT runs per lane, RPT rows per lane (tile = TXT*PX*CPT wide,
// (256/TXT)*RPT high); persistent or one-tile-per-block grid.
struct TileCfg {
    int px, txt, cpt, rpt;
    bool persistent;
};

int device_cus();
int persistent_grid(int ntiles, int per_cu);
TiledJob make_tiled_job(const ImageJob &j, int op, int tw, int th);
TileGeom tile_geom(const ImageJob &j, int op, int tw, int th);
size_t tile_lds_bytes(const TileGeom &G, int tw, int th);
bool wants_gather(const ImageJob &j, int op);
bool tiled_supported(int c, kr_dtype st);

}  // namespace kr
