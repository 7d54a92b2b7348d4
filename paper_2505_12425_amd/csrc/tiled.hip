// tiled.hip -- per-image launches of the LDS-tiled kernels (tiled.h): tile
// shape, LDS budget and grid for one image.
#include <algorithm>
#include <atomic>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <map>
#include <mutex>
#include <tuple>

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
    // f32 outputs leave through non-temporal stores (no kernel of the call
    // reads them back)
    constexpr bool SF = C == KT_F32_SOURCE;
    run_tiles<OP, SF ? 1 : C, F32, Layout<PX, TXT, CPT, RPT, true>, MAXIT, PERS, SF>(G, e, lds,
                                                                                     [&](TiledJob &t, int &tile) {
        if (!seq.take(tile))
            return false;
        t = job;
        return true;
    });
}

int device_cus()
{
    static std::atomic<int> cus[64];  // 0 = not queried yet (static storage starts zeroed)
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 64)
        return 256;
    int n = cus[dev].load(std::memory_order_relaxed);
    if (n == 0) {
        if (hipDeviceGetAttribute(&n, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || n <= 0)
            n = 256;
        cus[dev].store(n, std::memory_order_relaxed);
    }
    return n;
}

// Resident workgroups per CU for a kernel at a dynamic LDS size, cached per
// device, kernel and kilobyte of LDS (the kernels share one signature, so the
// key holds the kernel's address).
int blocks_per_cu(const void *kernel, size_t lds, int threads)
{
    static std::mutex mu;
    static std::map<std::tuple<int, const void *, size_t>, int> cache;
    const size_t slot = (lds + 1023) / 1024;
    if (slot > 64)
        return 1;
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess)
        dev = -1;
    const auto key = std::make_tuple(dev, kernel, slot);
    {
        std::lock_guard<std::mutex> g(mu);
        const auto it = cache.find(key);
        if (it != cache.end())
            return it->second;
    }
    int n = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, kernel, threads, slot * 1024) != hipSuccess || n < 1)
        n = 1;
    std::lock_guard<std::mutex> g(mu);
    cache[key] = n;
    return n;
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
    t.rows_contig = op == OP_RESIZE && (double)j.sh <= 2.0 * (double)j.dh;
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
//
// Scanning every tile costs four quotient pairs per tile on the host, more
// than the kernel itself at 4K.  The tiles are therefore grouped into regions
// (at most 16 x 16), each region gets an upper bound on its tiles' boxes, and
// only regions whose bound could raise the running maximum are scanned.  The
// bound is the smaller of two: the span of the region's own clamped corner
// images (the image of a rectangle on which w > 0 is the convex quadrilateral
// of its corner images, and the clamp is monotone), and the mean-value bound
// sup|dX/dx| (tw - 1) + sup|dX/dy| (th - 1).  For X = (a x + b y + c) / w with
// w = g x + h y + i, dX/dx = ((a h - g b) y + (a i - g c)) / w^2 and dX/dy =
// ((b g - h a) x + (b i - h c)) / w^2: affine numerators, largest in size at
// the region's corners, over the smallest w there.  The result equals the
// full scan's.
struct PerspBox {
    int bw, bh;  // -1: some corner has w <= 0
};

static inline double clamp_coord(double v, double hi)
{
    v = v != v ? -2.0 : v;
    return v < -2.0 ? -2.0 : (v > hi ? hi : v);
}

// Tap box of the output rectangle [x0, x1] x [y0, y1] from its corners.
static PerspBox corner_box(const ImageJob &j, double x0, double x1, double y0, double y1)
{
    const double hx = j.sw + 1.0, hy = j.sh + 1.0;
    double xmin = 1e300, xmax = -1e300, ymin = 1e300, ymax = -1e300;
    for (int q = 0; q < 4; q++) {
        const double cx = (q & 1) ? x1 : x0, cy = (q & 2) ? y1 : y0;
        const double w = j.proj[0] * cx + j.proj[1] * cy + j.proj[2];
        if (!(w > 0.0))
            return {-1, -1};
        const double X = clamp_coord((j.inv[0] * cx + j.inv[1] * cy + j.inv[2]) / w, hx);
        const double Y = clamp_coord((j.inv[3] * cx + j.inv[4] * cy + j.inv[5]) / w, hy);
        xmin = X < xmin ? X : xmin;
        xmax = X > xmax ? X : xmax;
        ymin = Y < ymin ? Y : ymin;
        ymax = Y > ymax ? Y : ymax;
    }
    return {(int)(std::floor(xmax) - std::floor(xmin)), (int)(std::floor(ymax) - std::floor(ymin))};
}

static TileGeom persp_geom(const ImageJob &j, int tw, int th)
{
    const int tx_n = (j.dw + tw - 1) / tw, ty_n = (j.dh + th - 1) / th;
    const int rtx = (tx_n + 15) / 16, rty = (ty_n + 15) / 16;  // tiles per region
    const double a = j.inv[0], b = j.inv[1], c = j.inv[2], d = j.inv[3], e = j.inv[4], f = j.inv[5];
    const double g = j.proj[0], h = j.proj[1], i = j.proj[2];
    const double hx = j.sw + 1.0, hy = j.sh + 1.0;
    struct Region {
        int tx0, tx1, ty0, ty1;  // tile range, half-open
        double ux, uy;           // bounds on the tiles' corner-image spans
    };
    Region regs[16 * 16];  // on the stack: the launch path allocates nothing
    int nreg = 0;
    for (int ry = 0; ry < ty_n; ry += rty) {
        for (int rx = 0; rx < tx_n; rx += rtx) {
            Region r{rx, std::min(rx + rtx, tx_n), ry, std::min(ry + rty, ty_n), 1e300, 1e300};
            const double X0 = (double)rx * tw, X1 = (double)(std::min(r.tx1 * tw, j.dw) - 1);
            const double Y0 = (double)ry * th, Y1 = (double)(std::min(r.ty1 * th, j.dh) - 1);
            double wmin = 1e300, xlo = 1e300, xhi = -1e300, ylo = 1e300, yhi = -1e300;
            bool pos = true;
            for (int q = 0; q < 4; q++) {
                const double cx = (q & 1) ? X1 : X0, cy = (q & 2) ? Y1 : Y0;
                const double w = g * cx + h * cy + i;
                pos = pos && w > 0.0;
                wmin = w < wmin ? w : wmin;
                if (pos) {
                    const double X = clamp_coord((a * cx + b * cy + c) / w, hx);
                    const double Y = clamp_coord((d * cx + e * cy + f) / w, hy);
                    xlo = X < xlo ? X : xlo;
                    xhi = X > xhi ? X : xhi;
                    ylo = Y < ylo ? Y : ylo;
                    yhi = Y > yhi ? Y : yhi;
                }
            }
            if (pos) {
                auto amax = [](double p, double q) { return std::fabs(p) > std::fabs(q) ? std::fabs(p) : std::fabs(q); };
                const double w2 = wmin * wmin;
                const double sxx = amax((a * h - g * b) * Y0 + (a * i - g * c), (a * h - g * b) * Y1 + (a * i - g * c));
                const double sxy = amax((b * g - h * a) * X0 + (b * i - h * c), (b * g - h * a) * X1 + (b * i - h * c));
                const double syx = amax((d * h - g * e) * Y0 + (d * i - g * f), (d * h - g * e) * Y1 + (d * i - g * f));
                const double syy = amax((e * g - h * d) * X0 + (e * i - h * f), (e * g - h * d) * X1 + (e * i - h * f));
                const double mx = (sxx * (tw - 1) + sxy * (th - 1)) / w2;
                const double my = (syx * (tw - 1) + syy * (th - 1)) / w2;
                // relative and absolute margins cover the rounding of the bound
                r.ux = std::min(mx, xhi - xlo) * (1.0 + 1e-9) + 1e-6;
                r.uy = std::min(my, yhi - ylo) * (1.0 + 1e-9) + 1e-6;
                r.ux = r.ux == r.ux ? r.ux : 1e300;  // w^2 underflow: no bound
                r.uy = r.uy == r.uy ? r.uy : 1e300;
            }
            regs[nreg++] = r;
        }
    }
    // regions with the largest bounds first, so the running maximum rises early
    std::sort(regs, regs + nreg, [](const Region &p, const Region &q) { return p.ux + p.uy > q.ux + q.uy; });
    int maxw = 0, maxh = 0;
    for (int ri = 0; ri < nreg; ri++) {
        const Region &r = regs[ri];
        // floor(p) - floor(q) <= ceil(p - q): a region whose bound cannot beat
        // both maxima has no tile that would change them
        if (maxw > 0 && std::ceil(r.ux) + 6.0 <= (double)maxw && std::ceil(r.uy) + 6.0 <= (double)maxh)
            continue;
        for (int ty = r.ty0; ty < r.ty1; ty++) {
            for (int tx = r.tx0; tx < r.tx1; tx++) {
                const int x0 = tx * tw, x1 = std::min(x0 + tw, j.dw) - 1;
                const int y0 = ty * th, y1 = std::min(y0 + th, j.dh) - 1;
                const PerspBox bx = corner_box(j, x0, x1, y0, y1);
                if (bx.bw < 0)
                    continue;
                const int bw = bx.bw + 6, bh = bx.bh + 6;
                if (tile_lds_bytes(TileGeom{bank_pitch(bw + KT_SPILL), bh}, tw, th) > KT_LDS_CAP)
                    continue;
                maxw = std::max(maxw, bw);
                maxh = std::max(maxh, bh);
            }
        }
    }
    TileGeom G;
    G.pitch = maxw > 0 ? bank_pitch(maxw + KT_SPILL) : 0;
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
        G.pitch = (int)std::fmin(std::ceil(ex) + 4.0, (double)j.sw + 6.0) + KT_SPILL;
        G.rows = (int)std::fmin(std::ceil(ey) + 4.0, (double)j.sh + 6.0);
        G.pitch = bank_pitch(G.pitch);
    } else {
        const double rx = (double)j.sw / (double)j.dw, ry = (double)j.sh / (double)j.dh;
        G.pitch = (int)std::fmin(std::ceil(rx * (tw - 1)) + 3.0, (double)j.sw + 4.0) + KT_SPILL;
        // rows_contig (ry <= 2): the floors of tap rows a span ry (th - 1)
        // apart differ by at most its ceiling, plus the second tap row
        G.rows = ry <= 2.0 ? (int)std::fmin(2.0 * th, std::ceil(ry * (th - 1)) + 3.0) : 2 * th;
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
    // box rows, the margin before row 0, then the resize tables
    return ((size_t)G.rows * G.pitch + KT_MARGIN) * 4 + (size_t)(2 * tw + 2 * th) * 4;
}

template <int OP, int C, bool F32, int PX, int TXT, int CPT, int RPT>
static hipError_t launch_cfg(const ImageJob &j, const Epilogue &e, hipStream_t s, int mode, bool gather,
                             bool &fits)
{
    using L = Layout<PX, TXT, CPT, RPT>;
    constexpr int TW = L::TW, TH = L::TH, MAXIT = 3;
    // a persistent workgroup holds its next tile's loads in registers while it
    // interpolates: one group per thread (the rest is staged at commit)
    constexpr int MAXIT_PERS = 1;
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
    if constexpr (C == 3 || C == 4) {  // other sources: one workgroup per tile
        if (mode == GRID_PERSISTENT) {
            auto kern = k_tiled<OP, C, F32, PX, TXT, CPT, RPT, MAXIT_PERS, true>;
            const int grid = persistent_grid(t.ntiles, blocks_per_cu(reinterpret_cast<const void *>(kern), lds));
            hipLaunchKernelGGL(kern, dim3(grid), dim3(KT_THREADS), lds, s, t, e, G);
            return hipGetLastError();
        }
    }
    auto kern = k_tiled<OP, C, F32, PX, TXT, CPT, RPT, MAXIT, false>;
    hipLaunchKernelGGL(kern, dim3(t.ntiles), dim3(KT_THREADS), lds, s, t, e, G);
    return hipGetLastError();
}

template <int OP, int C, bool F32>
static hipError_t launch_shape(const TileCfg &cfg, const ImageJob &j, const Epilogue &e, hipStream_t s, bool gather,
                               bool &fits)
{
#define KR_TRY(PX, TXT, CPT, RPT)                                                                        \
    if (cfg.px == PX && cfg.txt == TXT && cfg.cpt == CPT && cfg.rpt == RPT)                              \
        return launch_cfg<OP, C, F32, PX, TXT, CPT, RPT>(j, e, s, cfg.grid, gather, fits);
    if constexpr (C < 3 || C == KT_F32_SOURCE) {
        if constexpr (OP != OP_RESIZE) {
            KR_WARP_CFGS_NARROW(KR_TRY)
        } else {
            KR_RESIZE_CFGS_NARROW(KR_TRY)
        }
    } else if constexpr (OP != OP_RESIZE) {
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
// first choice.  gather: a resize whose taps are read from global memory
// (it shrinks x by more than 3).  narrow: a one- or two-channel source
// (4-pixel runs, one workgroup per tile).
static int default_cfgs(int op, bool f32, bool gather, bool narrow, TileCfg *out)
{
    int n = 0;
    const char *tile = std::getenv("KR_TILE");
    const char *grid = std::getenv("KR_GRID");
    int force = -1;
    if (grid)
        force = std::strcmp(grid, "full") == 0 ? GRID_FULL
                : std::strcmp(grid, "persistent") == 0 ? GRID_PERSISTENT : -1;
    int px = 0, txt = 0, cpt = 0, rpt = 0;
    if (tile && std::sscanf(tile, "%dx%dx%dx%d", &px, &txt, &cpt, &rpt) == 4)
        out[n++] = TileCfg{px, txt, cpt, rpt, force >= 0 ? force : GRID_PERSISTENT};
    auto add = [&](int a, int b, int c, int d, bool pers) {
        out[n++] = TileCfg{a, b, c, d, force >= 0 ? force : (pers ? GRID_PERSISTENT : GRID_FULL)};
    };
    if (narrow) {
        if (op != OP_RESIZE) {
            add(4, 16, 1, 2, false);
            add(4, 8, 1, 1, false);
        } else {
            add(4, gather ? 64 : 16, 1, 1, false);
        }
        return n;
    }
    // the autotuner's choices on MI355X for 4K sources (3840x2160x3 u8, every
    // source read from HBM): f32 warps run best on a persistent grid of 16-row
    // columns, u8 warps and resizes with one workgroup per tile
    if (op != OP_RESIZE) {
        if (f32) {
            add(1, 64, 1, 16, true);
            add(1, 64, 1, 8, false);
        } else {
            add(4, 16, 1, 4, false);
            add(4, 16, 1, 2, false);
        }
        add(1, 64, 1, 8, false);
    } else if (gather) {
        // nothing is staged: a thread's outputs are a chain of dependent tap
        // loads, so short chains (4 pixels of one row per thread) and many
        // small tiles win (the 256 mixed-size images of the batch workload,
        // 201 of them past 3x, resized one by one: 2.92 -> 1.42 ms)
        add(4, 64, 1, 1, false);
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
    n += default_cfgs(OP, F32, wants_gather(j, OP), C < 3 || C == KT_F32_SOURCE, cfgs + n);
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

bool tunable_source(int c, kr_dtype st) { return st == KR_U8 && (c == 3 || c == 4); }

bool tiled_image_supported(int c, kr_dtype st) { return st == KR_U8 && c >= 1 && c <= 4; }

bool tiled_f32_supported(int c, kr_dtype st) { return st == KR_F32 && c == 1; }

template <int OP>
static hipError_t launch_op(int c, bool f, const ImageJob &j, const Epilogue &e, hipStream_t s)
{
    switch (c) {
    case 1:
        return f ? launch_c<OP, 1, true>(j, e, s) : launch_c<OP, 1, false>(j, e, s);
    case 2:
        return f ? launch_c<OP, 2, true>(j, e, s) : launch_c<OP, 2, false>(j, e, s);
    case 3:
        return f ? launch_c<OP, 3, true>(j, e, s) : launch_c<OP, 3, false>(j, e, s);
    default:
        return f ? launch_c<OP, 4, true>(j, e, s) : launch_c<OP, 4, false>(j, e, s);
    }
}

hipError_t launch_tiled_f32(int op, const ImageJob &j, const Epilogue &e, hipStream_t s)
{
    if (op == OP_PERSP)
        return launch_c<OP_PERSP, KT_F32_SOURCE, true>(j, e, s);
    if (op == OP_WARP)
        return launch_c<OP_WARP, KT_F32_SOURCE, true>(j, e, s);
    return launch_c<OP_RESIZE, KT_F32_SOURCE, true>(j, e, s);
}

hipError_t launch_tiled(int op, int c, kr_dtype dt, const ImageJob &j, const Epilogue &e, hipStream_t s)
{
    const bool f = dt == KR_F32;
    if (op == OP_PERSP)
        return launch_op<OP_PERSP>(c, f, j, e, s);
    if (op == OP_WARP)
        return launch_op<OP_WARP>(c, f, j, e, s);
    return launch_op<OP_RESIZE>(c, f, j, e, s);
}

}  // namespace kr
