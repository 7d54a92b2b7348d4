// batch.hip -- many resizes / warps of uneven sizes in one launch per
// operation: the kernel walks a work-list of output tiles spanning every
// image.  Image i owns global tiles [first_tile_i, first_tile_i + ntiles_i);
// a tile finds its image by binary search over first_tile.  The per-tile work
// is exactly the single-image kernels' (tiled.h), so every image's output is
// bit-identical to its single-image call.
//
// Host side: validation, the tile list (prefix sums of per-image tile
// counts), the launch-wide LDS geometry, the C ABI entry points
// kr_resize_batch / kr_batch_plan_* (plans capture their launches in a HIP
// graph; they record no memset nodes).
#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <string>
#include <new>
#include <vector>

#include "batch_internal.h"
#include "kr_api_internal.h"
#include "tune.h"

namespace kr {

// PIPE: persistent grid (each workgroup walks its XCD's tile range,
// prefetching the next tile); else at most one tile per workgroup.
template <int OP, int C, bool F32, int PX, int TXT, int CPT, int RPT, int MAXIT, bool PIPE>
__global__ __launch_bounds__(KT_THREADS) void k_batch(const TiledJob *__restrict__ jobs, int njobs, TileBins bins,
                                                      Epilogue e, TileGeom G)
{
    extern __shared__ uint32_t lds[];
    TileSeq seq(blockIdx.x, gridDim.x, bins.start);
    // f32 outputs leave through non-temporal stores (no kernel of the launch
    // reads them back)
    run_tiles<OP, C, F32, Layout<PX, TXT, CPT, RPT, true>, MAXIT, PIPE>(G, e, lds, [&](TiledJob &t, int &tile) {
        int g;
        if (!seq.take(g))
            return false;
        int lo = 0, hi = njobs - 1;
        while (lo < hi) {
            const int mid = (lo + hi + 1) >> 1;
            if (jobs[mid].first_tile <= g)
                lo = mid;
            else
                hi = mid - 1;
        }
        t = jobs[lo];
        tile = g - t.first_tile;
        return true;
    });
}

template <int OP, int C, bool F32, int PX, int TXT, int CPT, int RPT>
static hipError_t launch_group_cfg(const BatchGroup &g, const Epilogue &e, hipStream_t s)
{
    int widest = 0;  // largest per-XCD tile range
    for (int k = 0; k < 8; k++)
        widest = std::max(widest, g.bins.start[k + 1] - g.bins.start[k]);
    if constexpr (C >= 3) {  // one- and two-channel sources: one workgroup per tile
        if (g.cfg.grid == GRID_PERSISTENT) {
            auto kern = k_batch<OP, C, F32, PX, TXT, CPT, RPT, 1, true>;
            const long resident = (long)blocks_per_cu(reinterpret_cast<const void *>(kern), g.lds) * device_cus();
            const int grid = (int)std::max(8L, std::min(8L * widest, resident & ~7L));
            hipLaunchKernelGGL(kern, dim3(grid), dim3(KT_THREADS), g.lds, s, g.jobs_dev, g.njobs, g.bins, e, g.G);
            return hipGetLastError();
        }
    }
    auto kern = k_batch<OP, C, F32, PX, TXT, CPT, RPT, 3, false>;
    hipLaunchKernelGGL(kern, dim3(8 * std::max(widest, 1)), dim3(KT_THREADS), g.lds, s, g.jobs_dev, g.njobs, g.bins,
                       e, g.G);
    return hipGetLastError();
}

template <int OP, int C, bool F32>
static hipError_t launch_group_c(const BatchGroup &g, const Epilogue &e, hipStream_t s)
{
#define KR_TRY(PX, TXT, CPT, RPT)                                                                        \
    if (g.cfg.px == PX && g.cfg.txt == TXT && g.cfg.cpt == CPT && g.cfg.rpt == RPT)                      \
        return launch_group_cfg<OP, C, F32, PX, TXT, CPT, RPT>(g, e, s);
    if constexpr (C < 3) {
        if constexpr (OP == OP_WARP) {
            KR_BATCH_WARP_CFGS_NARROW(KR_TRY)
        } else {
            KR_BATCH_RESIZE_CFGS_NARROW(KR_TRY)
        }
    } else if constexpr (OP == OP_WARP) {
        KR_BATCH_WARP_CFGS(KR_TRY)
    } else {
        KR_BATCH_RESIZE_CFGS(KR_TRY)
    }
#undef KR_TRY
    return hipErrorInvalidValue;
}

template <int OP>
static hipError_t launch_group_op(const BatchGroup &g, int c, bool f, const Epilogue &e, hipStream_t s)
{
    switch (c) {
    case 1:
        return f ? launch_group_c<OP, 1, true>(g, e, s) : launch_group_c<OP, 1, false>(g, e, s);
    case 2:
        return f ? launch_group_c<OP, 2, true>(g, e, s) : launch_group_c<OP, 2, false>(g, e, s);
    case 3:
        return f ? launch_group_c<OP, 3, true>(g, e, s) : launch_group_c<OP, 3, false>(g, e, s);
    default:
        return f ? launch_group_c<OP, 4, true>(g, e, s) : launch_group_c<OP, 4, false>(g, e, s);
    }
}

hipError_t launch_group(const BatchGroup &g, int c, kr_dtype dt, const Epilogue &e, hipStream_t s)
{
    if (g.njobs == 0)
        return hipSuccess;
    const bool f = dt == KR_F32;
    return g.op == OP_WARP ? launch_group_op<OP_WARP>(g, c, f, e, s) : launch_group_op<OP_RESIZE>(g, c, f, e, s);
}

// LDS per workgroup of a batch launch.  Every workgroup of the launch takes
// the same LDS size, the widest pitch times the most rows over its staged
// items, and that size sets the resident workgroups per CU (160 KB / size).
// The 64 warps of 1080p images: 0.37 ms per plan when only each item's own
// box had to fit 48 KB (the launch box came to 49 KB, three workgroups per
// CU); with the launch box held to the budget (fit_launch_box), 0.335 ms at
// 48 KB, 0.330 ms at 32 KB (five per CU), 0.361 ms at 28 KB (more tiles on
// the gather path).  The 256-image resize batch is the same at all of them.
constexpr size_t KB_LDS_BUDGET = 32 * 1024;

// Tile shape of a batch group when the batch class is not tuned: small
// tiles, so that batches of small outputs still produce many tiles
// (one- and two-channel sources: 4-pixel runs).
static TileCfg default_batch_cfg(int op, bool f32, int c)
{
    (void)op;
    return f32 && c >= 3 ? TileCfg{1, 64, 1, 4, GRID_FULL} : TileCfg{4, 16, 1, 1, GRID_FULL};
}

static int cfg_tw(const TileCfg &c) { return c.txt * c.px * c.cpt; }
static int cfg_th(const TileCfg &c) { return (KT_THREADS / c.txt) * c.rpt; }

// Estimated bytes an item moves: output bytes plus the source bytes its taps
// touch (about the output's pixels times the source area per output pixel,
// at most 4: beyond that the taps skip rows and columns); tiles that read
// their taps from global memory count half again.
static double item_cost(const ImageJob &j, int op, bool f32, int c, bool staged)
{
    const double px = (double)j.dh * (double)j.dw;
    const double ratio = op == OP_RESIZE ? (double)j.sh * (double)j.sw / px
                                         : std::fabs(j.inv[0] * j.inv[4] - j.inv[1] * j.inv[3]);
    const double bytes = px * c * ((f32 ? 4.0 : 1.0) + std::min(ratio, 4.0));
    return staged ? bytes : 1.5 * bytes;
}

// Keep the launch's box within the budget: while the widest pitch times the
// most rows over the staged items exceeds it, the staged item with the
// largest box among those that set the pitch or the rows moves to the gather
// path.
static void fit_launch_box(const std::vector<ImageJob> &imgs, int op, int tw, int th, size_t budget,
                           std::vector<bool> &stage)
{
    const int n = (int)imgs.size();
    std::vector<TileGeom> geo(n);
    for (int i = 0; i < n; i++)
        geo[i] = stage[i] ? tile_geom(imgs[i], op, tw, th) : TileGeom{0, 0};
    while (true) {
        TileGeom G{0, 0};
        for (int i = 0; i < n; i++)
            if (stage[i]) {
                G.pitch = std::max(G.pitch, geo[i].pitch);
                G.rows = std::max(G.rows, geo[i].rows);
            }
        if (tile_lds_bytes(G, tw, th) <= budget)
            return;
        int drop = -1;
        long best = -1;
        for (int i = 0; i < n; i++) {
            if (!stage[i] || (geo[i].pitch != G.pitch && geo[i].rows != G.rows))
                continue;
            const long area = (long)geo[i].pitch * geo[i].rows;
            if (area > best) {
                best = area;
                drop = i;
            }
        }
        if (drop < 0)
            return;
        stage[drop] = false;
    }
}

// One group: job table (tile prefix sums, items ordered bin by bin), per-XCD
// bins and the launch-wide LDS geometry, the largest box among the items
// that are staged (stage[i]); the others read their taps from global memory.
static void build_group(int op, const TileCfg &cfg, bool f32, int c, const std::vector<ImageJob> &imgs,
                        const std::vector<bool> &stage, BatchGroup &g, std::vector<TiledJob> &table)
{
    g.op = op;
    g.cfg = cfg;
    const int tw = cfg_tw(cfg), th = cfg_th(cfg);
    const int n = (int)imgs.size();
    // longest processing time first: items by cost, largest first, each into
    // the least loaded of the 8 bins
    std::vector<int> order(n);
    std::vector<double> cost(n);
    for (int i = 0; i < n; i++) {
        order[i] = i;
        cost[i] = item_cost(imgs[i], op, f32, c, stage[i]);
    }
    std::stable_sort(order.begin(), order.end(), [&](int a, int b) { return cost[a] > cost[b]; });
    double load[8] = {0, 0, 0, 0, 0, 0, 0, 0};
    std::vector<int> bin_of(n);
    for (int i : order) {
        int k = 0;
        for (int q = 1; q < 8; q++)
            k = load[q] < load[k] ? q : k;
        bin_of[i] = k;
        load[k] += cost[i];
    }
    double total = 0, top = 0;
    for (double l : load) {
        total += l;
        top = std::max(top, l);
    }
    // too few items to balance whole images (one large item, say): equal
    // tile counts per XCD over the list in submission order instead
    const bool by_item = n >= 8 && top <= 1.1 * total / 8.0;
    table.clear();
    g.G = TileGeom{0, 0};
    int first = 0;
    for (int k = 0; k < 8; k++) {
        g.bins.start[k] = first;
        for (int q = 0; q < n; q++) {
            const int i = by_item ? order[q] : q;
            if (by_item ? bin_of[i] != k : k != 0)
                continue;
            const ImageJob &j = imgs[i];
            TiledJob t = make_tiled_job(j, op, tw, th);
            t.first_tile = first;
            first += t.ntiles;
            table.push_back(t);
            if (!stage[i])
                continue;
            const TileGeom Gi = tile_geom(j, op, tw, th);
            g.G.pitch = std::max(g.G.pitch, Gi.pitch);
            g.G.rows = std::max(g.G.rows, Gi.rows);
        }
    }
    g.bins.start[8] = first;
    if (!by_item)
        for (int k = 0; k <= 8; k++)
            g.bins.start[k] = (int)((long)first * k / 8);
    g.njobs = (int)table.size();
    g.ntiles = first;
    g.lds = tile_lds_bytes(g.G, tw, th);
}

static bool fits(const ImageJob &j, int op, const TileCfg &c, size_t budget)
{
    return tile_lds_bytes(tile_geom(j, op, cfg_tw(c), cfg_th(c)), cfg_tw(c), cfg_th(c)) <= budget;
}

// One group per operation.  Resizes that shrink x by 2 or more share no taps
// between neighbouring outputs, while their boxes (over twice the tile width)
// would set the LDS size of every workgroup of the launch: such items read
// their taps directly, which keeps the group's LDS and so its occupancy at the
// size the milder items need.  Warps whose boxes exceed the batch LDS budget
// (strong shrinks) likewise take the global-gather path for their tiles, and
// so do the items that would widen the launch's box past the budget.
void build_batch(const std::vector<ImageJob> imgs[2], bool f32, int c, const TileCfg *const force[2], BatchBuild &b)
{
    b.groups.clear();
    b.tables.clear();
    for (int k = 0; k < 2; k++) {
        if (imgs[k].empty())
            continue;
        const int op = k == 0 ? OP_RESIZE : OP_WARP;
        TileCfg P, tuned;
        if (c < 3)  // untuned: the configurations compiled for them
            P = default_batch_cfg(op, f32, c);
        else if (force[k])
            P = *force[k];
        else if (tune_lookup(tune_key_batch(op, c, f32, imgs[k]), &tuned))
            P = tuned;
        else
            P = default_batch_cfg(op, f32, c);
        std::vector<bool> stage;
        for (const ImageJob &j : imgs[k])
            stage.push_back(op == OP_RESIZE ? !wants_gather(j, op) && (double)j.sw < 2.0 * (double)j.dw &&
                                                  fits(j, op, P, KB_LDS_BUDGET)
                                            : fits(j, op, P, KB_LDS_BUDGET));
        fit_launch_box(imgs[k], op, cfg_tw(P), cfg_th(P), KB_LDS_BUDGET, stage);
        b.groups.emplace_back();
        b.tables.emplace_back();
        build_group(op, P, f32, c, imgs[k], stage, b.groups.back(), b.tables.back());
    }
}

size_t BatchBuild::bytes() const
{
    size_t n = 0;
    for (const BatchGroup &g : groups)
        n += table_bytes(g.njobs);
    return n;
}

void BatchBuild::pack(uint8_t *host) const
{
    size_t off = 0;
    for (size_t i = 0; i < groups.size(); i++) {
        std::memcpy(host + off, tables[i].data(), tables[i].size() * sizeof(TiledJob));
        off += table_bytes(groups[i].njobs);
    }
}

void BatchBuild::bind(void *dev)
{
    size_t off = 0;
    for (BatchGroup &g : groups) {
        g.jobs_dev = reinterpret_cast<const TiledJob *>(static_cast<uint8_t *>(dev) + off);
        off += table_bytes(g.njobs);
    }
}

}  // namespace kr

using namespace kr;

// ------------------------------------------------------------------ validation
static kr_status check_items(const kr_batch_item *items, int n, int c, kr_dtype st, kr_dtype dt, kr_border border,
                             float bval, const kr_normalize *norm, std::vector<ImageJob> &rs,
                             std::vector<ImageJob> &ws)
{
    if (!items && n > 0)
        return fail(KR_ERR_INVALID_ARGUMENT, "items pointer is NULL");
    if (n < 0 || n > (1 << 20))
        return fail(KR_ERR_INVALID_ARGUMENT, "item count %d out of range", n);
    rs.clear();
    ws.clear();
    for (int i = 0; i < n; i++) {
        const kr_batch_item &it = items[i];
        kr_status s = check_common(it.src, it.src_h, it.src_w, c, st, it.dst, it.dst_h, it.dst_w, dt, border, bval,
                                   norm, it.src_pitch);
        if (s != KR_OK)
            return fail(s, "item %d: %s", i, kr_last_error());
        if (it.op != KR_OP_RESIZE && it.op != KR_OP_WARP)
            return fail(KR_ERR_INVALID_ARGUMENT, "item %d: unknown op %d", i, it.op);
        ImageJob j;
        std::memset(&j, 0, sizeof j);
        set_source(j, it.src, it.src_h, it.src_w, c, st, it.src_pitch);
        j.dst = it.dst; j.dh = it.dst_h; j.dw = it.dst_w;
        if (it.op == KR_OP_WARP) {
            if (it.flags & ~KR_WARP_INVERSE_MAP)
                return fail(KR_ERR_INVALID_ARGUMENT, "item %d: unknown warp flags 0x%x", i, it.flags);
            s = check_matrix(it.m, it.flags, j.inv);
            if (s != KR_OK)
                return fail(s, "item %d: %s", i, kr_last_error());
            ws.push_back(j);
        } else {
            rs.push_back(j);
        }
    }
    // destinations must not overlap each other or any source
    const size_t es_d = dt == KR_U8 ? 1 : 4;
    struct R { uintptr_t a, b; };
    std::vector<R> dsts, srcs;
    for (int i = 0; i < n; i++) {
        const uintptr_t d = reinterpret_cast<uintptr_t>(items[i].dst);
        dsts.push_back({d, d + (uintptr_t)items[i].dst_h * items[i].dst_w * c * es_d});
        const uintptr_t s0 = reinterpret_cast<uintptr_t>(items[i].src);
        srcs.push_back({s0, s0 + source_span(items[i].src_h, items[i].src_w, c, st, items[i].src_pitch)});
    }
    std::vector<R> sd = dsts;
    std::sort(sd.begin(), sd.end(), [](const R &x, const R &y) { return x.a < y.a; });
    for (size_t i = 1; i < sd.size(); i++)
        if (sd[i].a < sd[i - 1].b)
            return fail(KR_ERR_INVALID_ARGUMENT, "batch destinations overlap");
    std::vector<R> ss = srcs;
    std::sort(ss.begin(), ss.end(), [](const R &x, const R &y) { return x.a < y.a; });
    for (const R &d : sd) {
        // first source starting at or after d.b cannot overlap; check its predecessors
        auto it = std::lower_bound(ss.begin(), ss.end(), d.b, [](const R &x, uintptr_t v) { return x.a < v; });
        for (auto k = ss.begin(); k != it; ++k)
            if (k->b > d.a)
                return fail(KR_ERR_INVALID_ARGUMENT, "a batch destination overlaps a source");
    }
    return KR_OK;
}

// Device layout of a batch workspace: the job tables of the batch's groups,
// each 256-byte aligned (at most KB_MAX_GROUPS groups over n items).
size_t kr::table_bytes(int n) { return ((size_t)n * sizeof(TiledJob) + 255) & ~(size_t)255; }

// Validate a batch, write its work-list into the device buffer table (of
// table_bytes bytes) on stream and enqueue its launches.
static kr_status enqueue_batch(const kr_batch_item *items, int n, int c, kr_dtype src_t, kr_dtype dst_t,
                               kr_border border, float border_value, const kr_normalize *norm, int dst_layout,
                               void *table, size_t table_bytes, hipStream_t s)
{
    if (dst_layout != KR_LAYOUT_HWC && dst_layout != KR_LAYOUT_CHW)
        return fail(KR_ERR_INVALID_ARGUMENT, "unknown destination layout %d", dst_layout);
    std::vector<ImageJob> rs, ws;
    kr_status st = check_items(items, n, c, src_t, dst_t, border, border_value, norm, rs, ws);
    if (st != KR_OK)
        return st;
    if (n == 0)
        return KR_OK;
    if (!tiled_image_supported(c, src_t))
        return fail(KR_ERR_UNSUPPORTED, "batched launches need u8 sources");
    if (!table || reinterpret_cast<uintptr_t>(table) % 256 != 0)
        return fail(KR_ERR_INVALID_ARGUMENT, "workspace must be a 256-byte aligned device pointer");
    if (table_bytes < kr_resize_batch_workspace_size(n))
        return fail(KR_ERR_WORKSPACE_TOO_SMALL, "workspace of %zu bytes, %zu needed", table_bytes,
                    kr_resize_batch_workspace_size(n));
    Epilogue e = make_epilogue(c, border, border_value, norm);
    e.planar = dst_layout == KR_LAYOUT_CHW;
    const bool f32 = dst_t == KR_F32;
    const std::vector<ImageJob> imgs[2] = {rs, ws};
    const TileCfg *const none[2] = {nullptr, nullptr};
    BatchBuild bb;
    build_batch(imgs, f32, c, none, bb);
    std::vector<uint8_t> host(bb.bytes());
    bb.pack(host.data());
    // pageable source: the runtime stages it before the call returns
    hipError_t err = hipMemcpyAsync(table, host.data(), host.size(), hipMemcpyHostToDevice, s);
    if (err != hipSuccess)
        return fail(KR_ERR_HIP, "work-list upload failed: %s", hipGetErrorString(err));
    bb.bind(table);
    for (const BatchGroup &g : bb.groups) {
        err = launch_group(g, c, dst_t, e, s);
        if (err != hipSuccess)
            return fail(KR_ERR_HIP, "batch launch failed: %s", hipGetErrorString(err));
    }
    return KR_OK;
}

extern "C" {

size_t kr_resize_batch_workspace_size(int n) { return n > 0 ? table_bytes(n) + KB_MAX_GROUPS * 256 : 256; }

kr_status kr_resize_batch(const kr_batch_item *items, int n, int c, kr_dtype src_t, kr_dtype dst_t, kr_border border,
                          float border_value, const kr_normalize *norm, void *workspace, size_t workspace_bytes,
                          void *stream)
{
    return kr_resize_batch_ex(items, n, c, src_t, dst_t, border, border_value, norm, KR_LAYOUT_HWC, workspace,
                              workspace_bytes, stream);
}

kr_status kr_resize_batch_ex(const kr_batch_item *items, int n, int c, kr_dtype src_t, kr_dtype dst_t,
                             kr_border border, float border_value, const kr_normalize *norm, int dst_layout,
                             void *workspace, size_t workspace_bytes, void *stream)
{
    clear_error();
    return enqueue_batch(items, n, c, src_t, dst_t, border, border_value, norm, dst_layout, workspace,
                         workspace_bytes, (hipStream_t)stream);
}

}  // extern "C"

// ------------------------------------------------------------------ allocation-free form
// The batch entry point for callers that cannot allocate: its work-list goes
// to a device array of the library's own instead of a caller workspace.
// Each GPU holds its own copy of the array from the library's load until the
// process ends; host code reaches it only through the address
// hipGetSymbolAddress returns on that device (the array's name is a host-side
// stand-in, not a device address).
namespace {

constexpr size_t KB_SCRATCH_BYTES = size_t(1) << 20;
static_assert(KB_SCRATCH_BYTES == KR_NOALLOC_SCRATCH_BYTES, "kr.h states the scratch size");
static_assert(KR_NOALLOC_MAX_ITEMS * sizeof(TiledJob) + 255 + KB_MAX_GROUPS * 256 <= KB_SCRATCH_BYTES,
              "the largest allocation-free batch's work-list fits the scratch");

static __device__ __align__(256) uint8_t scratch[KB_SCRATCH_BYTES];

constexpr int KB_MAX_DEVICES = 64;
std::mutex g_scratch_mu;
void *g_scratch_ptr[KB_MAX_DEVICES];  // per device, set once with that device current

// The current device's address of scratch, looked up on the first call on
// that device.
hipError_t scratch_on_current_device(void **out)
{
    int dev = -1;
    hipError_t err = hipGetDevice(&dev);
    if (err != hipSuccess)
        return err;
    if (dev < 0 || dev >= KB_MAX_DEVICES)
        return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> g(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void *p = nullptr;
        err = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (err != hipSuccess)
            return err;
        if (!p)
            return hipErrorInvalidSymbol;
        g_scratch_ptr[dev] = p;
    }
    *out = g_scratch_ptr[dev];
    return hipSuccess;
}

}  // namespace

extern "C" kr_status kr_resize_batch_noalloc(const kr_batch_item *items, int n, int c, kr_dtype src_t,
                                             kr_dtype dst_t, kr_border border, float border_value,
                                             const kr_normalize *norm, int dst_layout, void *stream)
{
    clear_error();
    if (n < 0)
        return fail(KR_ERR_INVALID_ARGUMENT, "item count %d out of range", n);
    if (n > KR_NOALLOC_MAX_ITEMS)
        return fail(KR_ERR_WORKSPACE_TOO_SMALL,
                    "%d items: the allocation-free entry point takes at most %d (its work-list lives in a "
                    "%zu-byte device scratch)", n, KR_NOALLOC_MAX_ITEMS, KB_SCRATCH_BYTES);
    void *ws = nullptr;
    const hipError_t err = scratch_on_current_device(&ws);
    if (err != hipSuccess)
        return fail(KR_ERR_HIP, "device scratch lookup failed: %s", hipGetErrorString(err));
    return enqueue_batch(items, n, c, src_t, dst_t, border, border_value, norm, dst_layout, ws, KB_SCRATCH_BYTES,
                         (hipStream_t)stream);
}

// ------------------------------------------------------------------ plans
struct kr_batch_plan {
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    void *table = nullptr;      // device job tables
    hipEvent_t last = nullptr;  // recorded after each replay
    int ntiles = 0;
};

static void plan_free(kr_batch_plan *p)
{
    if (!p)
        return;
    if (p->exec)
        (void)hipGraphExecDestroy(p->exec);
    if (p->graph)
        (void)hipGraphDestroy(p->graph);
    if (p->table)
        (void)hipFree(p->table);
    if (p->last)
        (void)hipEventDestroy(p->last);
    delete p;
}

extern "C" {

kr_status kr_batch_plan_create(const kr_batch_item *items, int n, int c, kr_dtype src_t, kr_dtype dst_t,
                               kr_border border, float border_value, const kr_normalize *norm, kr_batch_plan **plan)
{
    return kr_batch_plan_create_ex(items, n, c, src_t, dst_t, border, border_value, norm, KR_LAYOUT_HWC, plan);
}

kr_status kr_batch_plan_create_ex(const kr_batch_item *items, int n, int c, kr_dtype src_t, kr_dtype dst_t,
                                  kr_border border, float border_value, const kr_normalize *norm, int dst_layout,
                                  kr_batch_plan **plan)
{
    clear_error();
    if (!plan)
        return fail(KR_ERR_INVALID_ARGUMENT, "plan pointer is NULL");
    *plan = nullptr;
    std::vector<ImageJob> rs, ws;
    kr_status st = check_items(items, n, c, src_t, dst_t, border, border_value, norm, rs, ws);
    if (st != KR_OK)
        return st;
    if (n == 0)
        return fail(KR_ERR_INVALID_ARGUMENT, "a plan needs at least one item");
    if (!tiled_image_supported(c, src_t))
        return fail(KR_ERR_UNSUPPORTED, "batched launches need u8 sources");
    if (dst_layout != KR_LAYOUT_HWC && dst_layout != KR_LAYOUT_CHW)
        return fail(KR_ERR_INVALID_ARGUMENT, "unknown destination layout %d", dst_layout);
    Epilogue e = make_epilogue(c, border, border_value, norm);
    e.planar = dst_layout == KR_LAYOUT_CHW;
    const bool f32 = dst_t == KR_F32;
    kr_batch_plan *p = new (std::nothrow) kr_batch_plan();
    if (!p)
        return fail(KR_ERR_INVALID_ARGUMENT, "out of host memory");
    const std::vector<ImageJob> imgs[2] = {rs, ws};
    const TileCfg *const none[2] = {nullptr, nullptr};
    BatchBuild bb;
    build_batch(imgs, f32, c, none, bb);
    std::vector<uint8_t> host(bb.bytes());
    bb.pack(host.data());
    hipError_t err = hipEventCreateWithFlags(&p->last, hipEventDisableTiming);
    if (err == hipSuccess)
        err = hipMalloc(&p->table, host.size());
    if (err != hipSuccess) {
        plan_free(p);
        return fail(KR_ERR_HIP, "plan allocation failed: %s", hipGetErrorString(err));
    }
    err = hipMemcpy(p->table, host.data(), host.size(), hipMemcpyHostToDevice);
    if (err != hipSuccess) {
        plan_free(p);
        return fail(KR_ERR_HIP, "plan upload failed: %s", hipGetErrorString(err));
    }
    bb.bind(p->table);
    for (const BatchGroup &g : bb.groups)
        p->ntiles += g.ntiles;
    hipStream_t cs = nullptr;
    err = hipStreamCreateWithFlags(&cs, hipStreamNonBlocking);
    if (err == hipSuccess)
        err = hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal);
    if (err == hipSuccess) {
        hipError_t lerr = hipSuccess;
        for (size_t k = 0; k < bb.groups.size() && lerr == hipSuccess; k++)
            lerr = launch_group(bb.groups[k], c, dst_t, e, cs);
        err = hipStreamEndCapture(cs, &p->graph);
        if (err == hipSuccess)
            err = lerr;
    }
    if (err == hipSuccess)
        err = hipGraphInstantiate(&p->exec, p->graph, nullptr, nullptr, 0);
    if (cs)
        (void)hipStreamDestroy(cs);
    if (err != hipSuccess) {
        plan_free(p);
        return fail(KR_ERR_HIP, "plan graph capture failed: %s", hipGetErrorString(err));
    }
    *plan = p;
    return KR_OK;
}

kr_status kr_batch_plan_launch(kr_batch_plan *plan, void *stream)
{
    clear_error();
    if (!plan || !plan->exec)
        return fail(KR_ERR_INVALID_ARGUMENT, "plan is NULL");
    // replays of one plan write the same outputs: each is ordered after the
    // previous one (on whichever stream that ran), so the event recorded
    // after the latest replay completes only after all of them
    hipError_t err = hipStreamWaitEvent((hipStream_t)stream, plan->last, 0);
    if (err == hipSuccess)
        err = hipGraphLaunch(plan->exec, (hipStream_t)stream);
    if (err == hipSuccess)
        err = hipEventRecord(plan->last, (hipStream_t)stream);
    if (err != hipSuccess)
        return fail(KR_ERR_HIP, "plan launch failed: %s", hipGetErrorString(err));
    return KR_OK;
}

void kr_batch_plan_destroy(kr_batch_plan *plan)
{
    if (!plan)
        return;
    // waits for this plan's own replays only (not the whole device)
    if (plan->last)
        (void)hipEventSynchronize(plan->last);
    plan_free(plan);
}

}  // extern "C"

// ------------------------------------------------------------------ autotuning
extern "C" kr_status kr_autotune_batch(const kr_batch_item *items, int n, int c, kr_dtype src_t, kr_dtype dst_t,
                                       kr_border border, float border_value, const kr_normalize *norm,
                                       void *workspace, size_t workspace_bytes, int reps, void *scrub,
                                       size_t scrub_bytes, void *stream, char *report, size_t report_len)
{
    clear_error();
    std::vector<ImageJob> imgs[2];
    kr_status st = check_items(items, n, c, src_t, dst_t, border, border_value, norm, imgs[0], imgs[1]);
    if (st != KR_OK)
        return st;
    if (!tunable_source(c, src_t))
        return fail(KR_ERR_UNSUPPORTED, "only batches of u8 sources with 3 or 4 channels have tunable configurations");
    if (!workspace || reinterpret_cast<uintptr_t>(workspace) % 256 != 0)
        return fail(KR_ERR_INVALID_ARGUMENT, "workspace must be a 256-byte aligned device pointer");
    if (workspace_bytes < kr_resize_batch_workspace_size(n))
        return fail(KR_ERR_WORKSPACE_TOO_SMALL, "workspace too small");
    if (reps < 1 || reps > 1000)
        return fail(KR_ERR_INVALID_ARGUMENT, "reps must be in [1, 1000]");
    st = check_scrub(scrub, scrub_bytes);
    if (st != KR_OK)
        return st;
    const Epilogue e = make_epilogue(c, border, border_value, norm);
    const bool f32 = dst_t == KR_F32;
    hipStream_t s = (hipStream_t)stream;
    std::string rep;
    kr_status result = KR_OK;
    for (int k = 0; k < 2 && result == KR_OK; k++) {
        if (imgs[k].empty())
            continue;
        const int op = k == 0 ? OP_RESIZE : OP_WARP;
        TileCfg best{};
        float best_ms = -1;
        for (const TileCfg &cfg : batch_candidates(op)) {
            std::vector<ImageJob> only[2];
            only[k] = imgs[k];
            const TileCfg *force[2] = {nullptr, nullptr};
            force[k] = &cfg;
            BatchBuild bb;
            build_batch(only, f32, c, force, bb);
            bool fits = true;
            for (const BatchGroup &g : bb.groups)
                fits = fits && g.lds <= KT_LDS_CAP;
            if (!fits)
                continue;
            std::vector<uint8_t> host(bb.bytes());
            bb.pack(host.data());
            // the host image must outlive the copy: time_launches synchronises the stream
            hipError_t err = hipMemcpyAsync(workspace, host.data(), host.size(), hipMemcpyHostToDevice, s);
            bb.bind(workspace);
            auto launch_all = [&]() {
                hipError_t e2 = hipSuccess;
                for (const BatchGroup &g : bb.groups)
                    if (e2 == hipSuccess)
                        e2 = launch_group(g, c, dst_t, e, s);
                return e2;
            };
            if (err == hipSuccess)
                err = launch_all();  // warm-up
            float ms = 0;
            if (err == hipSuccess)
                err = time_launches(launch_all, reps, scrub, scrub_bytes, s, ms);
            if (err != hipSuccess) {
                result = fail(KR_ERR_HIP, "autotune launch failed: %s", hipGetErrorString(err));
                break;
            }
            if (best_ms < 0 || ms < best_ms) {
                best_ms = ms;
                best = cfg;
            }
        }
        if (result == KR_OK && best_ms >= 0) {
            const TuneKey key = tune_key_batch(op, c, f32, imgs[k]);
            tune_store(key, best);
            char line[256];
            std::snprintf(line, sizeof line, "%s -> %s (%.1f us); ", tune_key_string(key).c_str(),
                          tune_cfg_string(best).c_str(), best_ms * 1000.0f);
            rep += line;
        }
    }
    if (result == KR_OK && report && report_len > 0)
        std::snprintf(report, report_len, "%s", rep.c_str());
    return result;
}
