// dispatch.hip -- chooses the kernel for one image: the exact-2x downscale
// kernel where it applies, the LDS-tiled kernels for u8 sources and
// one-channel f32 sources, the per-pixel kernels for other f32 sources.
#include "kr_device.h"

namespace kr {

bool tiled_image_supported(int c, kr_dtype st);
bool tiled_f32_supported(int c, kr_dtype st);
hipError_t launch_tiled(int op, int c, kr_dtype dt, const ImageJob &j, const Epilogue &e, hipStream_t s);
hipError_t launch_tiled_f32(int op, const ImageJob &j, const Epilogue &e, hipStream_t s);

hipError_t launch_resize(int c, kr_dtype st, kr_dtype dt, const ImageJob &j, const Epilogue &e, hipStream_t s)
{
    if (is_half_scale(st, j))
        return launch_half(c, dt, j, e, s);
    if (tiled_image_supported(c, st))
        return launch_tiled(OP_RESIZE, c, dt, j, e, s);
    if (tiled_f32_supported(c, st))
        return launch_tiled_f32(OP_RESIZE, j, e, s);
    return launch_generic(OP_RESIZE, c, st, dt, j, e, s);
}

hipError_t launch_resize_gray(kr_dtype dt, const ImageJob &j, const Epilogue &e, hipStream_t s)
{
    if (is_half_scale(KR_U8, j))
        return launch_half(3, dt, j, e, s);
    return launch_tiled(OP_RESIZE, 3, dt, j, e, s);
}

hipError_t launch_warp(int c, kr_dtype st, kr_dtype dt, const ImageJob &j, const Epilogue &e, hipStream_t s)
{
    // pixel permutations (flips, quarter turns, transposes with whole offsets)
    // of u8 sources: the same bits without interpolation
    int m[6];
    if (st == KR_U8 && !e.planar && !e.gray && permutation_map(j, m))
        return launch_permute(c, dt, j, m, e, s);
    if (tiled_image_supported(c, st))
        return launch_tiled(OP_WARP, c, dt, j, e, s);
    if (tiled_f32_supported(c, st))
        return launch_tiled_f32(OP_WARP, j, e, s);
    return launch_generic(OP_WARP, c, st, dt, j, e, s);
}

hipError_t launch_persp(int c, kr_dtype st, kr_dtype dt, const ImageJob &j, const Epilogue &e, hipStream_t s)
{
    if (tiled_image_supported(c, st))
        return launch_tiled(OP_PERSP, c, dt, j, e, s);
    if (tiled_f32_supported(c, st))
        return launch_tiled_f32(OP_PERSP, j, e, s);
    return launch_generic(OP_PERSP, c, st, dt, j, e, s);
}

}  // namespace kr
