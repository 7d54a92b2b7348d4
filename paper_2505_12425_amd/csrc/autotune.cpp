// autotune.cpp -- the tuner's single-image entry point and the persistence of
// the tuned table (kr_autotune_*).
#include <cstdio>
#include <cstring>
#include <string>

#include "kr_api_internal.h"
#include "tiled_launch.h"
#include "tune.h"

using namespace kr;

namespace kr {

kr_status check_scrub(const void *scrub, size_t bytes)
{
    if (!scrub)
        return KR_OK;
    if (reinterpret_cast<uintptr_t>(scrub) % 16 != 0 || bytes < 32)
        return fail(KR_ERR_INVALID_ARGUMENT, "scrub must be 16-byte aligned and at least 32 bytes");
    return KR_OK;
}

}  // namespace kr

extern "C" {

kr_status kr_autotune_image(int op, const void *src, int src_h, int src_w, int c, kr_dtype src_t, void *dst,
                            int dst_h, int dst_w, kr_dtype dst_t, const double m[6], int flags, kr_border border,
                            float border_value, const kr_normalize *norm, int reps, void *scrub, size_t scrub_bytes,
                            void *stream, char *report, size_t report_len)
{
    clear_error();
    if (op != KR_OP_RESIZE && op != KR_OP_WARP)
        return fail(KR_ERR_INVALID_ARGUMENT, "unknown op %d", op);
    kr_status st = check_common(src, src_h, src_w, c, src_t, dst, dst_h, dst_w, dst_t, border, border_value, norm);
    if (st != KR_OK)
        return st;
    if (!tunable_source(c, src_t))
        return fail(KR_ERR_UNSUPPORTED, "only u8 sources with 3 or 4 channels have tunable configurations");
    if (reps < 1 || reps > 1000)
        return fail(KR_ERR_INVALID_ARGUMENT, "reps must be in [1, 1000]");
    st = check_scrub(scrub, scrub_bytes);
    if (st != KR_OK)
        return st;
    ImageJob j;
    std::memset(&j, 0, sizeof j);
    if (op == KR_OP_WARP) {
        if (flags & ~KR_WARP_INVERSE_MAP)
            return fail(KR_ERR_INVALID_ARGUMENT, "unknown warp flags 0x%x", flags);
        st = check_matrix(m, flags, j.inv);
        if (st != KR_OK)
            return st;
    }
    j.src = src; j.dst = dst; j.sh = src_h; j.sw = src_w; j.dh = dst_h; j.dw = dst_w;
    j.sp = src_w;  // contiguous source
    j.sk = 0;
    const Epilogue e = make_epilogue(c, border, border_value, norm);
    hipStream_t s = (hipStream_t)stream;
    TileCfg best{};
    float best_ms = -1;
    for (const TileCfg &cfg : image_candidates(op)) {
        bool fits = false;
        hipError_t err = launch_tiled_cfg(op, c, dst_t, cfg, j, e, s, fits);  // warm-up
        if (err == hipSuccess && !fits)
            continue;
        float ms = 0;
        if (err == hipSuccess)
            err = time_launches([&] { return launch_tiled_cfg(op, c, dst_t, cfg, j, e, s, fits); }, reps, scrub,
                                scrub_bytes, s, ms);
        if (err != hipSuccess)
            return fail(KR_ERR_HIP, "autotune launch failed: %s", hipGetErrorString(err));
        if (best_ms < 0 || ms < best_ms) {
            best_ms = ms;
            best = cfg;
        }
    }
    if (best_ms < 0)
        return KR_OK;  // no tiled configuration fits: launches keep the global-gather path
    const TuneKey key = tune_key_image(op, c, dst_t == KR_F32, j);
    tune_store(key, best);
    if (report && report_len > 0)
        std::snprintf(report, report_len, "%s -> %s (%.1f us)", tune_key_string(key).c_str(),
                      tune_cfg_string(best).c_str(), best_ms * 1000.0f);
    return KR_OK;
}

size_t kr_autotune_save(char *buf, size_t len)
{
    const std::string text = tune_dump();
    if (buf && len > 0)
        std::snprintf(buf, len, "%s", text.c_str());
    return text.size() + 1;
}

kr_status kr_autotune_load(const char *text)
{
    clear_error();
    if (!text)
        return fail(KR_ERR_INVALID_ARGUMENT, "text is NULL");
    const int r = tune_load_text(text);
    if (r == 1)
        return fail(KR_ERR_INVALID_ARGUMENT, "malformed tuning table line");
    if (r == 2)
        return fail(KR_ERR_UNSUPPORTED, "tuning table made for another build (this library: %s); ignored",
                    tune_build_key());
    return KR_OK;
}

const char *kr_build_key(void) { return tune_build_key(); }

void kr_autotune_clear(void) { tune_clear(); }

}  // extern "C"
