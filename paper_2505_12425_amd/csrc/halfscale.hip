// halfscale.hip -- bilinear resize by exactly 2 in both axes (W_in = 2 W_out,
// H_in = 2 H_out), u8 sources.
//
// With half-pixel centres the source coordinate of output column d is
// ((2d + 1) 2 W_out - W_out) / (2 W_out) = 2d + 1/2: the taps are columns 2d
// and 2d + 1 with fraction 1/2, and the same holds for rows.  Every tap lies
// inside the image, so neither border rule applies.  The general definition
// then reduces exactly to:
//   u8:  w0 = w1 = 1024, acc = 2^20 (a + b + c + d), out = (a + b + c + d + 2) >> 2;
//   f32: the blend with 2-D weights 1/4 is exact, v = (a + b + c + d) / 4, then
//        the epilogue fma(v, alpha_c, beta_c) -- the same bits as the general
//        kernels.
// No tap is shared between outputs, so there is nothing to stage: each lane
// owns 4 consecutive output pixels of a row and reads the 8-pixel runs of its
// two source rows (8 C contiguous bytes each) with dword-aligned vector loads,
// realigned with alignbyte.  A wave reads 64 such runs back to back.  u8
// results leave as 4-pixel stores (contiguous across the wave); f32 results
// are transposed through LDS within the wave first, so that each store
// instruction writes 64 consecutive 16-byte chunks instead of chunks 3 or 4
// apart.  The fused gray form (an RGB source, the gray epilogue) stores the luma
// of each mean pixel through the tiled engine's gray stores, so its bits
// equal the tiled kernel's for the same resize.
#include "kr_device.h"
#include "tiled.h"

namespace kr {

namespace {

constexpr int HS_TX = 64, HS_TY = 4, HS_RPT = 2;

// 8 C bytes of a source row starting at byte b (b >= 0, inside the image) as
// 2 C dwords.  nbytes: bytes from src to the image's last byte.
template <int C>
__device__ __forceinline__ void load_run8(const uint8_t *__restrict__ src, size_t nbytes, size_t b,
                                          uint32_t (&w)[2 * C])
{
    constexpr int N = 2 * C + 1;  // dwords covering 8 C bytes from any byte offset
    const size_t f = b & ~(size_t)3;
    if (f + 4 * N <= nbytes) {
        struct __attribute__((packed, aligned(4))) Run { uint32_t d[N]; };
        const Run r = *reinterpret_cast<const Run *>(src + f);
        const uint32_t sh = (uint32_t)(b & 3);
#pragma unroll
        for (int i = 0; i < 2 * C; i++)
            w[i] = __builtin_amdgcn_alignbyte(r.d[i + 1], r.d[i], sh);
    } else {
        // the image's last bytes: byte by byte, and nothing past the end
#pragma unroll
        for (int i = 0; i < 2 * C; i++) {
            uint32_t v = 0;
#pragma unroll
            for (int k = 0; k < 4; k++)
                if (b + 4 * i + k < nbytes)
                    v |= (uint32_t)src[b + 4 * i + k] << (8 * k);
            w[i] = v;
        }
    }
}

template <int C>
__device__ __forceinline__ uint32_t byte_at(const uint32_t (&w)[2 * C], int i)
{
    return (w[i >> 2] >> (8 * (i & 3))) & 0xFFu;
}

template <int C, bool DST_F32>
__global__ __launch_bounds__(HS_TX * HS_TY) void k_half(ImageJob j, Epilogue e)
{
    // f32 output: a wave's 256 pixels (3 or 4 KB) go through LDS so that each
    // (non-temporal) store instruction writes 64 consecutive 16-byte chunks
    __shared__ f32x4 xpose[DST_F32 ? HS_TY * HS_TX * C : 1];
    const int x = (blockIdx.x * HS_TX + threadIdx.x) * 4;
    const int xw = blockIdx.x * HS_TX * 4;  // the wave's first output column
    if (x >= j.dw)
        return;
    const int n = min(4, j.dw - x);
    const uint8_t *src = static_cast<const uint8_t *>(j.src);
    const size_t nbytes = (size_t)src_end(j) * C;
    const bool aligned = store4_aligned<C, DST_F32>(j.dw);
#pragma unroll
    for (int rr = 0; rr < HS_RPT; rr++) {
        const int y = blockIdx.y * (HS_TY * HS_RPT) + threadIdx.y + rr * HS_TY;
        if (y >= j.dh)
            break;
        const size_t lin = (size_t)j.sk + (size_t)(2 * y) * j.sp + 2 * (size_t)x;
        uint32_t r0[2 * C], r1[2 * C];
        load_run8<C>(src, nbytes, lin * C, r0);
        load_run8<C>(src, nbytes, (lin + j.sp) * C, r1);
        uint32_t s[4][C];
#pragma unroll
        for (int k = 0; k < 4; k++)
#pragma unroll
            for (int c = 0; c < C; c++)
                s[k][c] = byte_at<C>(r0, 2 * k * C + c) + byte_at<C>(r0, (2 * k + 1) * C + c) +
                          byte_at<C>(r1, 2 * k * C + c) + byte_at<C>(r1, (2 * k + 1) * C + c);
        if constexpr (!DST_F32) {
            uint32_t P[4];
#pragma unroll
            for (int k = 0; k < 4; k++) {
                uint32_t p = 0;
#pragma unroll
                for (int c = 0; c < C; c++)
                    p |= ((s[k][c] + 2u) >> 2) << (8 * c);
                P[k] = p;
            }
            if constexpr (C == 3) {
                if (e.gray) {  // the fused gray form: luma of each mean pixel
                    store_gray_u8<4>(j, y, x, j.dw, P);
                    continue;
                }
            }
            store_u8_4<C>(static_cast<uint8_t *>(j.dst) + ((size_t)y * j.dw + x) * C, n, aligned, P);
        } else {
            float o[4][C];
#pragma unroll
            for (int k = 0; k < 4; k++)
#pragma unroll
                for (int c = 0; c < C; c++)
                    o[k][c] = __builtin_fmaf((float)s[k][c] * 0.25f, e.alpha[c], e.beta[c]);
            if constexpr (C == 3) {
                if (e.gray) {  // channel values unnormalised (alpha 1, beta 0); the gray gets galpha, gbeta
                    store_gray_f32<C, 4, true>(j, e, y, x, j.dw, o);
                    continue;
                }
            }
            float *row = static_cast<float *>(j.dst) + (size_t)y * j.dw * C;
            if (aligned && xw + 4 * HS_TX <= j.dw) {
                // whole wave inside the row (uniform per wave): lane l's 4 C
                // floats are chunks C l .. C l + C - 1 of the wave's run;
                // write them, read back chunks i * 64 + l, store those
                f32x4 *buf = xpose + threadIdx.y * HS_TX * C;
                const float *flat = &o[0][0];
#pragma unroll
                for (int i = 0; i < C; i++)
                    buf[C * threadIdx.x + i] = f32x4{flat[4 * i], flat[4 * i + 1], flat[4 * i + 2], flat[4 * i + 3]};
                __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
                __builtin_amdgcn_wave_barrier();
                __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
                f32x4 *out = reinterpret_cast<f32x4 *>(row + (size_t)xw * C);
#pragma unroll
                for (int i = 0; i < C; i++)
                    __builtin_nontemporal_store(buf[i * HS_TX + threadIdx.x], &out[i * HS_TX + threadIdx.x]);
                // the next row's writes must not overtake these reads
                __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
                __builtin_amdgcn_wave_barrier();
                __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
            } else {
                store_f32_4<C, true>(row + (size_t)x * C, n, aligned, o);
            }
        }
    }
}

template <int C>
hipError_t launch_c(kr_dtype dt, const ImageJob &j, const Epilogue &e, hipStream_t s)
{
    const dim3 block(HS_TX, HS_TY);
    const dim3 grid((j.dw + 4 * HS_TX - 1) / (4 * HS_TX), (j.dh + HS_TY * HS_RPT - 1) / (HS_TY * HS_RPT));
    if (dt == KR_F32)
        hipLaunchKernelGGL((k_half<C, true>), grid, block, 0, s, j, e);
    else
        hipLaunchKernelGGL((k_half<C, false>), grid, block, 0, s, j, e);
    return hipGetLastError();
}

}  // namespace

bool is_half_scale(kr_dtype st, const ImageJob &j)
{
    return st == KR_U8 && j.sw == 2 * j.dw && j.sh == 2 * j.dh;
}

hipError_t launch_half(int c, kr_dtype dt, const ImageJob &j, const Epilogue &e, hipStream_t s)
{
    switch (c) {
    case 1: return launch_c<1>(dt, j, e, s);
    case 2: return launch_c<2>(dt, j, e, s);
    case 3: return launch_c<3>(dt, j, e, s);
    default: return launch_c<4>(dt, j, e, s);
    }
}

}  // namespace kr
