// generic.hip -- one-thread-per-pixel bilinear resize / warp kernels.
//
// These evaluate the resampling definition directly: every tap is read from
// global memory with its own border test.  They serve f32 sources (every
// channel count and matrix); u8 sources run on the LDS-tiled kernels, whose
// global-gather path takes the tiles whose footprint does not fit in LDS.
//
// Coordinate rules (the paper prints none; these are the fixed readings):
//  * resize: half-pixel centres, source x = ((2 dx + 1) W_in - W_out) / (2 W_out)
//    held as an exact rational; floor and remainder are integers;
//  * warp: xs = fma(A, x, fma(B, y, C)), ys = fma(D, x, fma(E, y, F)) in
//    binary64, clamped to [-2, W + 1] x [-2, H + 1];
//  * perspective warp: the same two rows divided by w = fma(G, x, fma(H, y, I))
//    (binary64 quotients; not-a-number reads as -2), then clamped;
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
    generic_pixel<C, S, D, OP>(j, e, x, y);
}

template <int C, typename S, typename D>
static hipError_t launch_generic_t(int op, const ImageJob &j, const Epilogue &e, hipStream_t s)
{
    dim3 grid((j.dw + 63) / 64, (j.dh + 3) / 4);
    if (op == OP_RESIZE)
        hipLaunchKernelGGL((k_generic<C, S, D, OP_RESIZE>), grid, dim3(256), 0, s, j, e);
    else if (op == OP_PERSP)
        hipLaunchKernelGGL((k_generic<C, S, D, OP_PERSP>), grid, dim3(256), 0, s, j, e);
    else
        hipLaunchKernelGGL((k_generic<C, S, D, OP_WARP>), grid, dim3(256), 0, s, j, e);
    return hipGetLastError();
}

template <int C>
static hipError_t launch_generic_c(int op, kr_dtype st, kr_dtype dt, const ImageJob &j,
                                   const Epilogue &e, hipStream_t s)
{
    if (st != KR_F32 || dt != KR_F32)
        return hipErrorNotSupported;  // u8 sources: the tiled kernels
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
// compared with.  Grid-stride over groups of four 16-byte chunks per thread
// (four loads in flight before the stores), byte tail by one thread.
__global__ __launch_bounds__(256) void k_copy(u32x4 *__restrict__ dst, const u32x4 *__restrict__ src,
                                              size_t n16, uint8_t *dst_b, const uint8_t *src_b,
                                              size_t bytes)
{
    const size_t stride = (size_t)gridDim.x * 1024;
    for (size_t b = (size_t)blockIdx.x * 1024 + threadIdx.x; b < n16; b += stride) {
        u32x4 r[4];
#pragma unroll
        for (int k = 0; k < 4; k++)
            if (b + k * 256 < n16)
                r[k] = src[b + k * 256];
#pragma unroll
        for (int k = 0; k < 4; k++)
            if (b + k * 256 < n16)
                dst[b + k * 256] = r[k];
    }
    if (blockIdx.x == 0 && threadIdx.x == 0)
        for (size_t b = n16 * 16; b < bytes; b++)
            dst_b[b] = src_b[b];
}

hipError_t launch_copy(void *dst, const void *src, size_t bytes, hipStream_t s)
{
    const size_t n16 = bytes / 16;
    size_t blocks = (n16 + 1023) / 1024;
    if (blocks > 256 * 8)
        blocks = 256 * 8;
    if (blocks < 1)
        blocks = 1;
    hipLaunchKernelGGL(k_copy, dim3((unsigned)blocks), dim3(256), 0, s, (u32x4 *)dst, (const u32x4 *)src,
                       n16, (uint8_t *)dst, (const uint8_t *)src, bytes);
    return hipGetLastError();
}

// Traffic-mix probe (kr_hbm_stream): one output chunk per thread and step,
// grid-stride; output chunk i reads input chunks [i << shrink, (i + 1) <<
// shrink) or input chunk i >> grow.
__global__ __launch_bounds__(256) void k_stream(u32x4 *__restrict__ dst, const u32x4 *__restrict__ src, size_t n_out,
                                                int shrink, int grow)
{
    const size_t stride = (size_t)gridDim.x * 256;
    const int k = 1 << shrink;
    for (size_t i = (size_t)blockIdx.x * 256 + threadIdx.x; i < n_out; i += stride) {
        const size_t j = (i << shrink) >> grow;
        u32x4 v = src[j];
        for (int q = 1; q < k; q++)
            v ^= src[j + q];
        dst[i] = v;
    }
}

hipError_t launch_stream(void *dst, size_t n_out, const void *src, int shrink, int grow, hipStream_t s)
{
    // enough workgroups to fill the chip several times over, the rest by striding
    size_t blocks = (n_out + 255) / 256;
    if (blocks > 256 * 8)
        blocks = 256 * 8;
    hipLaunchKernelGGL(k_stream, dim3((unsigned)blocks), dim3(256), 0, s, (u32x4 *)dst, (const u32x4 *)src, n_out,
                       shrink, grow);
    return hipGetLastError();
}

}  // namespace kr
