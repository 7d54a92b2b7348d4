// tune.cpp -- the autotuning table: keys, lookup/store, text persistence.
#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <fstream>
#include <map>
#include <mutex>
#include <sstream>
#include <tuple>

#include "tune.h"

namespace kr {

namespace {

std::mutex g_mu;
std::map<std::tuple<int, int, int, int, int, int>, TileCfg> g_table;
bool g_loaded = false;

std::tuple<int, int, int, int, int, int> tup(const TuneKey &k)
{
    return std::make_tuple(k.op, k.c, k.f32, k.batch, k.sclass, k.zclass);
}

// Source pixels read per output pixel: resize = area ratio; warp = |det| of
// the inverse map.
double scale_of(int op, const ImageJob &j)
{
    if (op == OP_RESIZE)
        return ((double)j.sh * j.sw) / ((double)j.dh * j.dw);
    return std::fabs(j.inv[0] * j.inv[4] - j.inv[1] * j.inv[3]);
}

int sclass_of(double ratio)
{
    if (!(ratio > 0.0))
        return 0;
    return std::max(-8, std::min(8, (int)std::lround(2.0 * std::log2(ratio))));
}

int zclass_of(double px) { return std::max(0, std::min(15, (int)(std::log2(std::max(px, 1.0)) / 2.0))); }

bool known_cfg(const TuneKey &k, const TileCfg &c)
{
    if ((k.op != OP_RESIZE && k.op != OP_WARP && k.op != OP_PERSP) || (k.c != 3 && k.c != 4) ||
        (k.f32 != 0 && k.f32 != 1) || (k.op == OP_PERSP && k.batch != 0) ||
        (k.batch != 0 && k.batch != 1))
        return false;
    for (const TileCfg &x : k.batch ? batch_candidates(k.op) : image_candidates(k.op))
        if (x.px == c.px && x.txt == c.txt && x.cpt == c.cpt && x.rpt == c.rpt && x.grid == c.grid)
            return true;
    return false;
}

// Parse the text form (one entry per line, '#' comments).  The first entry
// line is the build key, "key <arch> <kernel-source hash>"; a table whose key
// differs from this library's (another GPU architecture, or kernels edited
// since it was measured) is stale: TABLE_STALE, nothing taken.  All or
// nothing otherwise: a malformed line or a configuration the library was not
// compiled with rejects the whole text (TABLE_BAD).
enum { TABLE_OK, TABLE_BAD, TABLE_STALE };

int parse_table(const std::string &text, std::vector<std::pair<TuneKey, TileCfg>> &out)
{
    std::istringstream in(text);
    std::string line;
    bool keyed = false;
    while (std::getline(in, line)) {
        const size_t first = line.find_first_not_of(" \t\r");
        if (first == std::string::npos || line[first] == '#')
            continue;
        if (!keyed) {
            char arch[32], sha[32];
            int used = 0;
            if (std::sscanf(line.c_str(), " key %31s %31s %n", arch, sha, &used) != 2 ||
                line.find_first_not_of(" \t\r", used) != std::string::npos)
                return TABLE_BAD;
            if (std::string(arch) + " " + sha != tune_build_key())
                return TABLE_STALE;
            keyed = true;
            continue;
        }
        TuneKey k;
        TileCfg c;
        int pers = 0, used = 0;
        if (std::sscanf(line.c_str(), "%d %d %d %d %d %d %d %d %d %d %d %n", &k.op, &k.c, &k.f32, &k.batch,
                        &k.sclass, &k.zclass, &c.px, &c.txt, &c.cpt, &c.rpt, &pers, &used) != 11 ||
            line.find_first_not_of(" \t\r", used) != std::string::npos || pers < GRID_FULL || pers > GRID_PERSISTENT)
            return TABLE_BAD;
        c.grid = pers;
        if (!known_cfg(k, c))
            return TABLE_BAD;
        out.push_back({k, c});
    }
    return keyed || out.empty() ? TABLE_OK : TABLE_BAD;
}

void load_env_locked()
{
    if (g_loaded)
        return;
    g_loaded = true;
    const char *path = std::getenv("KR_AUTOTUNE_CACHE");
    if (!path)
        return;
    std::ifstream f(path);
    if (!f)
        return;
    std::stringstream ss;
    ss << f.rdbuf();
    std::vector<std::pair<TuneKey, TileCfg>> v;
    const int r = parse_table(ss.str(), v);
    if (r != TABLE_OK) {
        std::fprintf(stderr, "libkr: ignoring %s tuning cache %s\n", r == TABLE_STALE ? "stale" : "malformed", path);
        return;
    }
    for (const auto &kv : v)
        g_table[tup(kv.first)] = kv.second;
}

}  // namespace

TuneKey tune_key_image(int op, int c, bool f32, const ImageJob &j)
{
    return TuneKey{op, c, f32 ? 1 : 0, 0, sclass_of(scale_of(op, j)), zclass_of((double)j.dh * j.dw)};
}

TuneKey tune_key_batch(int op, int c, bool f32, const std::vector<ImageJob> &imgs)
{
    std::vector<double> sc;
    double px = 0;
    for (const ImageJob &j : imgs) {
        sc.push_back(scale_of(op, j));
        px += (double)j.dh * j.dw;
    }
    double med = 1.0;
    if (!sc.empty()) {
        std::nth_element(sc.begin(), sc.begin() + sc.size() / 2, sc.end());
        med = sc[sc.size() / 2];
    }
    return TuneKey{op, c, f32 ? 1 : 0, 1, sclass_of(med), zclass_of(px)};
}

bool tune_lookup(const TuneKey &k, TileCfg *cfg)
{
    std::lock_guard<std::mutex> g(g_mu);
    load_env_locked();
    auto it = g_table.find(tup(k));
    if (it == g_table.end())
        return false;
    *cfg = it->second;
    return true;
}

void tune_store(const TuneKey &k, const TileCfg &cfg)
{
    std::lock_guard<std::mutex> g(g_mu);
    load_env_locked();
    g_table[tup(k)] = cfg;
}

void tune_clear()
{
    std::lock_guard<std::mutex> g(g_mu);
    g_table.clear();
    g_loaded = true;
}

std::string tune_key_string(const TuneKey &k)
{
    char b[128];
    std::snprintf(b, sizeof b, "%s c=%d %s %s scale=%d size=%d", k.op == OP_PERSP ? "perspective" : (k.op == OP_WARP ? "warp" : "resize"), k.c,
                  k.f32 ? "f32" : "u8", k.batch ? "batch" : "image", k.sclass, k.zclass);
    return b;
}

std::string tune_cfg_string(const TileCfg &c)
{
    char b[96];
    std::snprintf(b, sizeof b, "%dx%dx%dx%d %s", c.px, c.txt, c.cpt, c.rpt, c.grid == GRID_PERSISTENT ? "persistent" : "full");
    return b;
}

std::string tune_dump()
{
    std::lock_guard<std::mutex> g(g_mu);
    load_env_locked();
    std::ostringstream o;
    o << "# op c f32 batch sclass zclass px txt cpt rpt grid\n";
    o << "key " << tune_build_key() << '\n';
    for (const auto &kv : g_table) {
        const auto &k = kv.first;
        const TileCfg &c = kv.second;
        o << std::get<0>(k) << ' ' << std::get<1>(k) << ' ' << std::get<2>(k) << ' ' << std::get<3>(k) << ' '
          << std::get<4>(k) << ' ' << std::get<5>(k) << ' ' << c.px << ' ' << c.txt << ' ' << c.cpt << ' ' << c.rpt
          << ' ' << c.grid << '\n';
    }
    return o.str();
}

int tune_load_text(const std::string &text)
{
    std::vector<std::pair<TuneKey, TileCfg>> v;
    const int r = parse_table(text, v);
    if (r != TABLE_OK)
        return r == TABLE_STALE ? 2 : 1;
    std::lock_guard<std::mutex> g(g_mu);
    g_loaded = true;
    for (const auto &kv : v)
        g_table[tup(kv.first)] = kv.second;
    return 0;
}

// The build this library's tables belong to: the GPU architecture it was
// compiled for and the hash of its kernel sources (passed by the build).
const char *tune_build_key()
{
#ifndef KR_SOURCE_SHA
#define KR_SOURCE_SHA "unknown"
#endif
    return "gfx950 " KR_SOURCE_SHA;
}

hipError_t time_launches(const std::function<hipError_t()> &launch, int reps, void *scrub, size_t scrub_bytes,
                         hipStream_t s, float &ms)
{
    hipEvent_t a = nullptr, b = nullptr;
    hipError_t err = hipEventCreate(&a);
    if (err == hipSuccess)
        err = hipEventCreate(&b);
    const size_t half = scrub_bytes / 2 / 16 * 16;
    auto scrub_once = [&]() { return launch_copy(static_cast<uint8_t *>(scrub) + half, scrub, half, s); };
    // one timed run of `reps` iterations of body, in ms
    auto timed = [&](const std::function<hipError_t()> &body, float &t) {
        hipError_t e2 = hipEventRecord(a, s);
        for (int r = 0; r < reps && e2 == hipSuccess; r++)
            e2 = body();
        if (e2 == hipSuccess)
            e2 = hipEventRecord(b, s);
        if (e2 == hipSuccess)
            e2 = hipEventSynchronize(b);
        if (e2 == hipSuccess)
            e2 = hipEventElapsedTime(&t, a, b);
        return e2;
    };
    float t1 = 0, t2 = 0;
    if (err == hipSuccess) {
        if (!scrub) {
            err = timed(launch, t1);
            ms = t1 / (float)reps;
        } else {
            // (scrub, launch) pairs minus scrubs alone: the launch then pays for
            // reading its source from HBM and for the write-back of its output
            // (forced by the next scrub), as in a stream of distinct images
            err = timed([&]() {
                hipError_t e3 = scrub_once();
                return e3 == hipSuccess ? launch() : e3;
            }, t1);
            if (err == hipSuccess)
                err = timed(scrub_once, t2);
            ms = std::max(t1 - t2, 1e-6f) / (float)reps;
        }
    }
    if (a)
        (void)hipEventDestroy(a);
    if (b)
        (void)hipEventDestroy(b);
    return err;
}

std::vector<TileCfg> image_candidates(int op)
{
    std::vector<TileCfg> v;
#define KR_ADD(PX, TXT, CPT, RPT)                   \
    v.push_back(TileCfg{PX, TXT, CPT, RPT, GRID_PERSISTENT});  \
    v.push_back(TileCfg{PX, TXT, CPT, RPT, GRID_FULL});
    if (op != OP_RESIZE) {
        KR_WARP_CFGS(KR_ADD)
    } else {
        KR_RESIZE_CFGS(KR_ADD)
    }
#undef KR_ADD
    return v;
}

std::vector<TileCfg> batch_candidates(int op)
{
    std::vector<TileCfg> v;
#define KR_ADD(PX, TXT, CPT, RPT)                            \
    v.push_back(TileCfg{PX, TXT, CPT, RPT, GRID_FULL});     \
    v.push_back(TileCfg{PX, TXT, CPT, RPT, GRID_PERSISTENT});
    if (op == OP_WARP) {
        KR_BATCH_WARP_CFGS(KR_ADD)
    } else {
        KR_BATCH_RESIZE_CFGS(KR_ADD)
    }
#undef KR_ADD
    return v;
}

}  // namespace kr
