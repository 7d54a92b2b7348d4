// tiled_launch.h -- host-side helpers shared by the per-image and batched
// launches of the tiled kernels.
#pragma once

#include "kr_internal.h"

namespace kr {

struct TiledJob;
struct TileGeom;

constexpr size_t KT_LDS_CAP = 64 * 1024;  // dynamic LDS per workgroup

// Grid modes of the tiled kernels: one workgroup per tile, or a persistent
// grid whose workgroups prefetch their next tile.
enum { GRID_FULL = 0, GRID_PERSISTENT = 1 };

// One tile configuration: runs of PX consecutive pixels per lane, TXT lanes
// per tile row, CPT runs per lane, RPT rows per lane (tile = TXT*PX*CPT wide,
// (256/TXT)*RPT high), and the grid mode.
struct TileCfg {
    int px, txt, cpt, rpt;
    int grid;
};

// Compiled tile configurations (PX, TXT, CPT, RPT) per operation: the
// per-image kernels and the batched work-list kernels.
#define KR_WARP_CFGS(X) X(4, 16, 1, 2) X(4, 16, 1, 4) X(4, 8, 1, 1) X(1, 64, 1, 8) X(1, 64, 1, 16)
#define KR_RESIZE_CFGS(X) X(4, 16, 1, 1) X(4, 32, 1, 1) X(4, 32, 1, 2) X(4, 64, 1, 1) X(4, 64, 1, 2) \
    X(1, 64, 2, 4) X(1, 64, 4, 2)
// Channel code of the tiled kernels for a one-channel f32 source (f32
// output): its pixels are staged as 4-byte words, as RGBA u8 pixels are.
constexpr int KT_F32_SOURCE = 5;

// One- and two-channel sources: 4-pixel runs only.
#define KR_WARP_CFGS_NARROW(X) X(4, 16, 1, 2) X(4, 16, 1, 4) X(4, 8, 1, 1)
#define KR_RESIZE_CFGS_NARROW(X) X(4, 16, 1, 1) X(4, 32, 1, 1) X(4, 64, 1, 1)
#define KR_BATCH_WARP_CFGS(X) X(4, 16, 1, 1) X(4, 16, 1, 2) X(4, 8, 1, 1) X(1, 64, 1, 4) X(1, 64, 1, 8)
#define KR_BATCH_RESIZE_CFGS(X) X(4, 16, 1, 1) X(4, 64, 1, 1) X(1, 64, 1, 4) X(1, 64, 2, 4)
#define KR_BATCH_WARP_CFGS_NARROW(X) X(4, 16, 1, 1)
#define KR_BATCH_RESIZE_CFGS_NARROW(X) X(4, 16, 1, 1)

// Launch one image with an explicit configuration; fits = false (nothing
// launched) when its LDS footprint exceeds the per-workgroup budget.
hipError_t launch_tiled_cfg(int op, int c, kr_dtype dt, const TileCfg &cfg, const ImageJob &j, const Epilogue &e,
                            hipStream_t s, bool &fits);

int device_cus();
// Resident workgroups per CU of a kernel at a dynamic LDS size (cached).
int blocks_per_cu(const void *kernel, size_t lds, int threads = 256);
int persistent_grid(int ntiles, int per_cu);
TiledJob make_tiled_job(const ImageJob &j, int op, int tw, int th);
TileGeom tile_geom(const ImageJob &j, int op, int tw, int th);
size_t tile_lds_bytes(const TileGeom &G, int tw, int th);
bool wants_gather(const ImageJob &j, int op);
// u8 sources with 3 or 4 channels: the ones the autotuner takes.
bool tunable_source(int c, kr_dtype st);
// u8 sources with 1-4 channels: the tiled kernels of single images, batches
// and the serving loop (fixed configurations for 1 and 2 channels).
bool tiled_image_supported(int c, kr_dtype st);
// One-channel f32 sources (f32 output): single images on the tiled kernels.
bool tiled_f32_supported(int c, kr_dtype st);

}  // namespace kr
