// tune.h -- autotuned choice of tile configuration (process-wide table).
//
// A key names a class of launches: operation, channels, output type, single
// image or batch, the source-pixels-per-output-pixel class (half-octaves of
// the area ratio) and the output-size class (factors of 4 in pixels).  The
// table maps keys to the configuration the tuner measured fastest; launchers
// try it before their defaults.  KR_AUTOTUNE_CACHE names a text file loaded
// on first use.
#pragma once

#include <functional>
#include <string>
#include <vector>

#include "tiled_launch.h"

namespace kr {

struct TuneKey {
    int op, c, f32, batch, sclass, zclass;
};

TuneKey tune_key_image(int op, int c, bool f32, const ImageJob &j);
TuneKey tune_key_batch(int op, int c, bool f32, const std::vector<ImageJob> &imgs);
bool tune_lookup(const TuneKey &k, TileCfg *cfg);
void tune_store(const TuneKey &k, const TileCfg &cfg);
void tune_clear();
std::string tune_key_string(const TuneKey &k);
std::string tune_cfg_string(const TileCfg &c);
std::string tune_dump();
// 0: merged; 1: malformed (table unchanged); 2: made for another build
// (architecture or kernel sources differ; table unchanged).
int tune_load_text(const std::string &text);
// "<arch> <kernel-source hash>" of this library.
const char *tune_build_key();

// Every compiled configuration of an operation (single image: both grid
// modes; batch: one-tile-per-block and persistent grids).
std::vector<TileCfg> image_candidates(int op);
std::vector<TileCfg> batch_candidates(int op);

// Duration (ms) of one call of `launch` on stream s.  Without a scrub buffer:
// reps calls back to back between one event pair, averaged.  With one: reps
// pairs (copy the buffer's first half over its second, which evicts the
// caller's source from the caches; call) minus reps copies alone, averaged,
// so that the call is charged for its HBM reads and its output's write-back.
// Synchronises s.
hipError_t time_launches(const std::function<hipError_t()> &launch, int reps, void *scrub, size_t scrub_bytes,
                         hipStream_t s, float &ms);

}  // namespace kr
