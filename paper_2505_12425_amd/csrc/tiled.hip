// tiled.hip -- per-image launches of the LDS-tiled kernels (tiled.h): tile
// shape, LDS budget and grid for one image.
#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>

#include "tiled.h"
#include "tiled_launch.h"
#include "tune.h"

namespace kr {

// PERS: persistent grid (each workgroup walks several tiles, prefetching the
// next one); else one workgroup per tile.
template <int OP, int C, bool F32, int PX, int TXT, int CPT, int RPT, int MAXIT, bool PERS>
__global__ __launch_bounds__(KT_THREADS) void k_tiled(TiledJob job, Epilogue e, TileGeom G)
{
    extern __shared__ uint32_t lds[];
    TileSeq seq(blockIdx.x, gridDim.x, job.ntiles);
    run_tiles<OP, C, F32, Layout<PX, TXT, CPT, RPT>, MAXIT, PERS>(G, e, lds, [&](TiledJob &t, int &tile) {
        if (!seq.take(tile))
            return false;
        t = job;
        return true;
    });
}

int device_cus()
{
    static int cus[64] = {0};
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 64)
        return 256;
    if (cus[dev] == 0) {
        int n = 0;
        if (hipDeviceGetAttribute(&n, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || n <= 0)
            n = 256;
        cus[dev] = n;
    }
    return cus[dev];
}

// Resident workgroups per CU for a kernel at a dynamic LDS size, cached per
// kernel and kilobyte of LDS.
template <typename K>
static int blocks_per_cu(K kernel, size_t lds)
{
    static int cache[65] = {0};
    const size_t slot = (lds + 1023) / 1024;
    if (slot > 64)
        return 1;
    if (cache[slot] == 0) {
        int n = 0;
        if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, kernel, KT_THREADS, slot * 1024) != hipSuccess || n < 1)
            n = 1;
        cache[slot] = n;
    }
    return cache[slot];
}

int persistent_grid(int ntiles, int per_cu)
{
    const long resident = (long)per_cu * device_cus();
    if (resident >= ntiles)
        return ntiles;
    int g = (int)resident & ~7;
    return g < 8 ? 8 : g;
}

TiledJob make_tiled_job(const ImageJob &j, int op, int tw, int th)
{
    TiledJob t;
    t.j = j;
    for (int i = 0; i < 6; i++)
        t.m2048[i] = 2048.0 * j.inv[i];
    t.rden_x = 1.0 / (2.0 * (double)j.dw);
    t.rden_y = 1.0 / (2.0 * (double)j.dh);
    t.op = op;
    t.tiles_x = (j.dw + tw - 1) / tw;
    t.ntiles = t.tiles_x * ((j.dh + th - 1) / th);
    t.first_tile = 0;
    return t;
}

// LDS pitch rounded up to 17 (mod 32) dwords: slots then start on banks that
// differ for 32 consecutive slots (staging writes) and neighbouring tap rows
// fall on different banks (gathers).
static int bank_pitch(int pitch) { return pitch + ((17 - pitch % 32) + 32) % 32; }

// Perspective warp: the largest tap box over the tiles whose corners all have
// w > 0 and whose box fits the LDS cap (the others evaluate their pixels from
// global memory), with the device plan's extra pixel per side and one more of
// slack for its rounding.
static TileGeom persp_geom(const ImageJob &j, int tw, int th)
{
    const int tx_n = (j.dw + tw - 1) / tw, ty_n = (j.dh + th - 1) / th;
    int maxw = 0, maxh = 0;
    for (int ty = 0; ty < ty_n; ty++) {
        for (int tx = 0; tx < tx_n; tx++) {
            const int x0 = tx * tw, x1 = std::min(x0 + tw, j.dw) - 1;
            const int y0 = ty * th, y1 = std::min(y0 + th, j.dh) - 1;
            double xmin = 1e300, xmax = -1e300, ymin = 1e300, ymax = -1e300;
            bool ok = true;
            for (int q = 0; q < 4; q++) {
                const double cx = (q & 1) ? x1 : x0, cy = (q & 2) ? y1 : y0;
                const double w = j.proj[0] * cx + j.proj[1] * cy + j.proj[2];
                if (!(w > 0.0)) {
                    ok = false;
                    break;
                }
                const double X = std::fmin(std::fmax((j.inv[0] * cx + j.inv[1] * cy + j.inv[2]) / w, -2.0), j.sw + 1.0);
                const double Y = std::fmin(std::fmax((j.inv[3] * cx + j.inv[4] * cy + j.inv[5]) / w, -2.0), j.sh + 1.0);
                xmin = std::fmin(xmin, X); xmax = std::fmax(xmax, X);
                ymin = std::fmin(ymin, Y); ymax = std::fmax(ymax, Y);
            }
            if (!ok)
                continue;
            const int bw = (int)(std::floor(xmax) - std::floor(xmin)) + 6;
            const int bh = (int)(std::floor(ymax) - std::floor(ymin)) + 6;
            if ((size_t)bank_pitch(bw + 2 * KT_MARGIN) * bh * 4 + (size_t)(2 * tw + 2 * th) * 4 > KT_LDS_CAP)
                continue;
            maxw = std::max(maxw, bw);
            maxh = std::max(maxh, bh);
        }
    }
    TileGeom G;
    G.pitch = maxw > 0 ? bank_pitch(maxw + 2 * KT_MARGIN) : 0;
    G.rows = maxh;
    return G;
}

TileGeom tile_geom(const ImageJob &j, int op, int tw, int th)
{
    TileGeom G;
    if (op == OP_PERSP)
        return persp_geom(j, tw, th);
    if (op == OP_WARP) {
        const double ex = std::fabs(j.inv[0]) * (tw - 1) + std::fabs(j.inv[1]) * (th - 1);
        const double ey = std::fabs(j.inv[3]) * (tw - 1) + std::fabs(j.inv[4]) * (th - 1);
        G.pitch = (int)std::fmin(std::ceil(ex) + 4.0, (double)j.sw + 6.0) + 2 * KT_MARGIN;
        G.rows = (int)std::fmin(std::ceil(ey) + 4.0, (double)j.sh + 6.0);
        G.pitch = bank_pitch(G.pitch);
    } else {
        const double rx = (double)j.sw / (double)j.dw;
        G.pitch = (int)std::fmin(std::ceil(rx * (tw - 1)) + 3.0, (double)j.sw + 4.0) + 2 * KT_MARGIN;
        G.rows = 2 * th;
        G.pitch = bank_pitch(G.pitch);
    }
    return G;
}

// Resizes that shrink by more than 3x along x share no horizontal taps between
// neighbouring outputs: staging buys no reuse, the taps are read directly.
bool wants_gather(const ImageJob &j, int op)
{
    return op == OP_RESIZE && (double)j.sw > 3.0 * (double)j.dw;
}

size_t tile_lds_bytes(const TileGeom &G, int tw, int th)
{
    return (size_t)G.rows * G.pitch * 4 + (size_t)(2 * tw + 2 * th) * 4;
}

template <int OP, int C, bool F32, int PX, int TXT, int CPT, int RPT>
static hipError_t launch_cfg(const ImageJob &j, const Epilogue &e, hipStream_t s, bool persistent, bool gather,
                             bool &fits)
{
    using L = Layout<PX, TXT, CPT, RPT>;
    constexpr int TW = L::TW, TH = L::TH, MAXIT = 3;
    const TiledJob t = make_tiled_job(j, OP, TW, TH);
    TileGeom G = tile_geom(j, OP, TW, TH);
    if (gather || wants_gather(j, OP)) {
        G.pitch = 0;  // no tile fits: every tile reads its taps from global memory
        G.rows = 0;
    }
    const size_t lds = tile_lds_bytes(G, TW, TH);
    fits = lds <= KT_LDS_CAP;
    if (!fits)
        return hipSuccess;
    if (persistent) {
        auto kern = k_tiled<OP, C, F32, PX, TXT, CPT, RPT, MAXIT, true>;
        const int grid = persistent_grid(t.ntiles, blocks_per_cu(kern, lds));
        hipLaunchKernelGGL(kern, dim3(grid), dim3(KT_THREADS), lds, s, t, e, G);
    } else {
        auto kern = k_tiled<OP, C, F32, PX, TXT, CPT, RPT, MAXIT, false>;
        hipLaunchKernelGGL(kern, dim3(t.ntiles), dim3(KT_THREADS), lds, s, t, e, G);
    }
    return hipGetLastError();
}

template <int OP, int C, bool F32>
static hipError_t launch_shape(const TileCfg &cfg, const ImageJob &j, const Epilogue &e, hipStream_t s, bool gather,
                               bool &fits)
{
#define KR_TRY(PX, TXT, CPT, RPT)                                                                        \
    if (cfg.px == PX && cfg.txt == TXT && cfg.cpt == CPT && cfg.rpt == RPT)                              \
        return launch_cfg<OP, C, F32, PX, TXT, CPT, RPT>(j, e, s, cfg.persistent, gather, fits);
    if constexpr (OP != OP_RESIZE) {
        KR_WARP_CFGS(KR_TRY)
    } else {
        KR_RESIZE_CFGS(KR_TRY)
    }
#undef KR_TRY
    fits = false;
    return hipSuccess;
}

// Tile shapes tried in order (the first whose LDS footprint fits is used).
// KR_TILE="PXxTXTxCPTxRPT" and KR_GRID="full"|"persistent" override the
// first choice.
static int default_cfgs(int op, bool f32, TileCfg *out)
{
    int n = 0;
    const char *tile = std::getenv("KR_TILE");
    const char *grid = std::getenv("KR_GRID");
    const bool force_full = grid && std::strcmp(grid, "full") == 0;
    const bool force_pers = grid && std::strcmp(grid, "persistent") == 0;
    int px = 0, txt = 0, cpt = 0, rpt = 0;
    if (tile && std::sscanf(tile, "%dx%dx%dx%d", &px, &txt, &cpt, &rpt) == 4)
        out[n++] = TileCfg{px, txt, cpt, rpt, !force_full};
    auto add = [&](int a, int b, int c, int d, bool pers) {
        out[n++] = TileCfg{a, b, c, d, force_pers ? true : (force_full ? false : pers)};
    };
    // the autotuner's choices on MI355X for 4K sources (3840x2160x3 u8, every
    // source read from HBM): one workgroup per tile beat persistent grids
    if (op != OP_RESIZE) {
        if (f32) {
            add(1, 64, 1, 8, false);
            add(1, 64, 1, 16, false);
        } else {
            add(4, 16, 1, 4, false);
            add(4, 16, 1, 2, false);
        }
        add(1, 64, 1, 8, false);
    } else {
        add(1, 64, 2, 4, false);
        add(4, 16, 1, 1, false);
    }
    return n;
}

template <int OP, int C, bool F32>
static hipError_t launch_c(const ImageJob &j, const Epilogue &e, hipStream_t s)
{
    TileCfg cfgs[8];
    int n = 0;
    TileCfg tuned;
    if (tune_lookup(tune_key_image(OP, C, F32, j), &tuned))
        cfgs[n++] = tuned;
    n += default_cfgs(OP, F32, cfgs + n);
    for (int i = 0; i < n; i++) {
        bool fits = false;
        const hipError_t err = launch_shape<OP, C, F32>(cfgs[i], j, e, s, false, fits);
        if (fits || err != hipSuccess)
            return err;
    }
    bool fits = false;
    return launch_shape<OP, C, F32>(cfgs[n - 1], j, e, s, true, fits);
}

hipError_t launch_tiled_cfg(int op, int c, kr_dtype dt, const TileCfg &cfg, const ImageJob &j, const Epilogue &e,
                            hipStream_t s, bool &fits)
{
    const bool f = dt == KR_F32;
    fits = false;
    if (op == OP_PERSP) {
        if (c == 3)
            return f ? launch_shape<OP_PERSP, 3, true>(cfg, j, e, s, false, fits)
                     : launch_shape<OP_PERSP, 3, false>(cfg, j, e, s, false, fits);
        return f ? launch_shape<OP_PERSP, 4, true>(cfg, j, e, s, false, fits)
                 : launch_shape<OP_PERSP, 4, false>(cfg, j, e, s, false, fits);
    }
    if (op == OP_WARP) {
        if (c == 3)
            return f ? launch_shape<OP_WARP, 3, true>(cfg, j, e, s, false, fits)
                     : launch_shape<OP_WARP, 3, false>(cfg, j, e, s, false, fits);
        return f ? launch_shape<OP_WARP, 4, true>(cfg, j, e, s, false, fits)
                 : launch_shape<OP_WARP, 4, false>(cfg, j, e, s, false, fits);
    }
    if (c == 3)
        return f ? launch_shape<OP_RESIZE, 3, true>(cfg, j, e, s, false, fits)
                 : launch_shape<OP_RESIZE, 3, false>(cfg, j, e, s, false, fits);
    return f ? launch_shape<OP_RESIZE, 4, true>(cfg, j, e, s, false, fits)
             : launch_shape<OP_RESIZE, 4, false>(cfg, j, e, s, false, fits);
}

bool tiled_supported(int c, kr_dtype st) { return st == KR_U8 && (c == 3 || c == 4); }

hipError_t launch_tiled(int op, int c, kr_dtype dt, const ImageJob &j, const Epilogue &e, hipStream_t s)
{
    const bool f = dt == KR_F32;
    if (op == OP_PERSP) {
        if (c == 3)
            return f ? launch_c<OP_PERSP, 3, true>(j, e, s) : launch_c<OP_PERSP, 3, false>(j, e, s);
        return f ? launch_c<OP_PERSP, 4, true>(j, e, s) : launch_c<OP_PERSP, 4, false>(j, e, s);
    }
    if (op == OP_WARP) {
        if (c == 3)
            return f ? launch_c<OP_WARP, 3, true>(j, e, s) : launch_c<OP_WARP, 3, false>(j, e, s);
        return f ? launch_c<OP_WARP, 4, true>(j, e, s) : launch_c<OP_WARP, 4, false>(j, e, s);
    }
    if (c == 3)
        return f ? launch_c<OP_RESIZE, 3, true>(j, e, s) : launch_c<OP_RESIZE, 3, false>(j, e, s);
    return f ? launch_c<OP_RESIZE, 4, true>(j, e, s) : launch_c<OP_RESIZE, 4, false>(j, e, s);
}

}  // namespace kr
