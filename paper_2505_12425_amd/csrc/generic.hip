// generic.hip -- one-thread-per-pixel bilinear resize / warp kernels.
//
// These evaluate the resampling definition directly: every tap is read from
// global memory with its own border test.  They cover every channel count,
// dtype pair and matrix, and serve as the fallback for the tiled kernels
// when a warp's inverse-mapped footprint does not fit in LDS.
//
// Coordinate rules (the paper prints none; these are the fixed readings):
//  * resize: half-pixel centres, source x = ((2 dx + 1) W_in - W_out) / (2 W_out)
//    held as an exact rational; floor and remainder are integers;
//  * warp: xs = fma(A, x, fma(B, y, C)), ys = fma(D, x, fma(E, y, F)) in
//    binary64, clamped to [-2, W + 1] x [-2, H + 1];
//  * u8 weights w1 = round-half-even(2048 frac), w0 = 2048 - w1; exact integer
//    accumulation; out = (acc + 2^21) >> 22.  f32: unquantised weights.
#include "kr_device.h"

namespace kr {

template <int C, typename S, typename D, int OP>
__global__ __launch_bounds__(256) void k_generic(ImageJob j, Epilogue e)
{
    const int x = blockIdx.x * 64 + (threadIdx.x & 63);
    const int y = blockIdx.y * 4 + (threadIdx.x >> 6);
    if (x >= j.dw || y >= j.dh)
        return;
    int x0, y0, wx1, wy1;
    float fx, fy;
    if (OP == OP_RESIZE) {
        resize_axis(x, j.sw, j.dw, x0, wx1, fx);
        resize_axis(y, j.sh, j.dh, y0, wy1, fy);
    } else {
        const double xs = __builtin_fma(j.inv[0], (double)x, __builtin_fma(j.inv[1], (double)y, j.inv[2]));
        const double ys = __builtin_fma(j.inv[3], (double)x, __builtin_fma(j.inv[4], (double)y, j.inv[5]));
        warp_axis(xs, j.sw, x0, wx1, fx);
        warp_axis(ys, j.sh, y0, wy1, fy);
    }
    const S *src = static_cast<const S *>(j.src);
    D *dst = static_cast<D *>(j.dst) + ((size_t)y * (size_t)j.dw + (size_t)x) * C;
    if constexpr (is_u8<D>::value) {
        const int wx[2] = {2048 - wx1, wx1};
        const int wy[2] = {2048 - wy1, wy1};
        int acc[C];
#pragma unroll
        for (int c = 0; c < C; c++)
            acc[c] = 0;
#pragma unroll
        for (int i = 0; i < 2; i++) {
#pragma unroll
            for (int k = 0; k < 2; k++) {
                const int w = wy[i] * wx[k];
                int p[C];
                tap_int<C>(src, j.sh, j.sw, x0 + k, y0 + i, e, p);
#pragma unroll
                for (int c = 0; c < C; c++)
                    acc[c] += w * p[c];
            }
        }
#pragma unroll
        for (int c = 0; c < C; c++)
            dst[c] = (uint8_t)((acc[c] + (1 << 21)) >> 22);
    } else {
        float p00[C], p01[C], p10[C], p11[C];
        tap_float<C>(src, j.sh, j.sw, x0, y0, e, p00);
        tap_float<C>(src, j.sh, j.sw, x0 + 1, y0, e, p01);
        tap_float<C>(src, j.sh, j.sw, x0, y0 + 1, e, p10);
        tap_float<C>(src, j.sh, j.sw, x0 + 1, y0 + 1, e, p11);
#pragma unroll
        for (int c = 0; c < C; c++) {
            const float top = (1.0f - fx) * p00[c] + fx * p01[c];
            const float bot = (1.0f - fx) * p10[c] + fx * p11[c];
            const float v = (1.0f - fy) * top + fy * bot;
            dst[c] = v * e.alpha[c] + e.beta[c];
        }
    }
}

template <int C, typename S, typename D>
static hipError_t launch_generic_t(int op, const ImageJob &j, const Epilogue &e, hipStream_t s)
{
    dim3 grid((j.dw + 63) / 64, (j.dh + 3) / 4);
    if (op == OP_RESIZE)
        hipLaunchKernelGGL((k_generic<C, S, D, OP_RESIZE>), grid, dim3(256), 0, s, j, e);
    else
        hipLaunchKernelGGL((k_generic<C, S, D, OP_WARP>), grid, dim3(256), 0, s, j, e);
    return hipGetLastError();
}

template <int C>
static hipError_t launch_generic_c(int op, kr_dtype st, kr_dtype dt, const ImageJob &j,
                                   const Epilogue &e, hipStream_t s)
{
    if (st == KR_U8 && dt == KR_U8)
        return launch_generic_t<C, uint8_t, uint8_t>(op, j, e, s);
    if (st == KR_U8 && dt == KR_F32)
        return launch_generic_t<C, uint8_t, float>(op, j, e, s);
    return launch_generic_t<C, float, float>(op, j, e, s);
}

hipError_t launch_generic(int op, int c, kr_dtype st, kr_dtype dt, const ImageJob &j,
                          const Epilogue &e, hipStream_t s)
{
    switch (c) {
    case 1: return launch_generic_c<1>(op, st, dt, j, e, s);
    case 2: return launch_generic_c<2>(op, st, dt, j, e, s);
    case 3: return launch_generic_c<3>(op, st, dt, j, e, s);
    default: return launch_generic_c<4>(op, st, dt, j, e, s);
    }
}

// ---------------------------------------------------------------- copy probe
// 16-byte vector copy: the bandwidth ceiling the resampling kernels are
// compared with.  Grid-stride over 16-byte chunks, byte tail by one thread.
__global__ __launch_bounds__(256) void k_copy(u32x4 *__restrict__ dst, const u32x4 *__restrict__ src,
                                              size_t n16, uint8_t *dst_b, const uint8_t *src_b,
                                              size_t bytes)
{
    const size_t stride = (size_t)gridDim.x * blockDim.x;
    for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n16; i += stride)
        __builtin_nontemporal_store(__builtin_nontemporal_load(src + i), dst + i);
    if (blockIdx.x == 0 && threadIdx.x == 0)
        for (size_t b = n16 * 16; b < bytes; b++)
            dst_b[b] = src_b[b];
}

hipError_t launch_copy(void *dst, const void *src, size_t bytes, hipStream_t s)
{
    const size_t n16 = bytes / 16;
    size_t blocks = (n16 + 255) / 256;
    if (blocks > 256 * 16)
        blocks = 256 * 16;
    if (blocks < 1)
        blocks = 1;
    hipLaunchKernelGGL(k_copy, dim3((unsigned)blocks), dim3(256), 0, s, (u32x4 *)dst, (const u32x4 *)src,
                       n16, (uint8_t *)dst, (const uint8_t *)src, bytes);
    return hipGetLastError();
}

}  // namespace kr
