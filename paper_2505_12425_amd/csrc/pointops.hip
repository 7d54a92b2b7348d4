// pointops.hip -- the paper's per-pixel benchmark operators (Sec. III):
// flip (horizontal and/or vertical; an exact permutation of pixels) and RGB
// to gray (ITU-R BT.601 luma; 14-bit fixed point for u8 output, binary32 for
// f32 output with the optional normalisation as epilogue).
//
// Launch shape as for the nearest-neighbour resize: 64 x 4 threads; u8
// outputs take 4 consecutive pixels per thread (one 12- or 4-byte store),
// f32 flips one pixel per thread (each store instruction of a wave is one
// contiguous run), f32 gray 4 pixels (16 bytes).  Outputs leave through
// non-temporal stores: no kernel of the call reads them back.
#include "kr_internal.h"
#include "tiled.h"

namespace kr {

namespace {

constexpr int PO_TX = 64, PO_TY = 4, PO_RPT = 2;

// Source and destination of one flip or gray launch.  Source pixel (x, y) is
// pixel number sk + y * sp + x from src (as in ImageJob); the destination is
// contiguous, w pixels per row.
struct PtJob {
    const void *src;
    void *dst;
    int h, w, sp, sk;
};

// Pixels lin .. lin + 3 of a u8 image with C channels (byte c = channel c),
// for lin a multiple of 4: one 4-, 8-, 12- or 16-byte aligned load.
template <int C>
__device__ __forceinline__ void load_run4(const uint8_t *__restrict__ src, size_t lin, uint32_t (&P)[4])
{
    const uint8_t *p = src + lin * C;
    if constexpr (C == 3) {
        struct __attribute__((packed, aligned(4))) W3 { uint32_t a, b, c; };
        const W3 d = *reinterpret_cast<const W3 *>(p);
        P[0] = d.a & 0xFFFFFFu;
        P[1] = __builtin_amdgcn_alignbyte(d.b, d.a, 3) & 0xFFFFFFu;
        P[2] = __builtin_amdgcn_alignbyte(d.c, d.b, 2) & 0xFFFFFFu;
        P[3] = d.c >> 8;
    } else if constexpr (C == 4) {
        const u32x4 d = *reinterpret_cast<const u32x4 *>(p);
        P[0] = d.x; P[1] = d.y; P[2] = d.z; P[3] = d.w;
    } else if constexpr (C == 2) {
        const u32x2 d = *reinterpret_cast<const u32x2 *>(p);
        P[0] = d.x & 0xFFFFu; P[1] = d.x >> 16; P[2] = d.y & 0xFFFFu; P[3] = d.y >> 16;
    } else {
        const uint32_t d = *reinterpret_cast<const uint32_t *>(p);
        P[0] = d & 0xFFu; P[1] = (d >> 8) & 0xFFu; P[2] = (d >> 16) & 0xFFu; P[3] = d >> 24;
    }
}

// ---------------------------------------------------------------- flip
template <int C>
__global__ __launch_bounds__(PO_TX * PO_TY) void k_flip_u8(PtJob j, int fx, int fy)
{
    const uint8_t *__restrict__ src = static_cast<const uint8_t *>(j.src);
    uint8_t *__restrict__ dst = static_cast<uint8_t *>(j.dst);
    const int h = j.h, w = j.w;
    const int x = (blockIdx.x * PO_TX + threadIdx.x) * 4;
    if (x >= w)
        return;
    const int n = min(4, w - x);
    const size_t nbytes = ((size_t)j.sk + (size_t)(h - 1) * j.sp + w) * C;
    const bool aligned = store4_aligned<C, false>(w);
    // 4-pixel source runs start on multiples of 4 pixels from src
    const bool runs = (w & 3) == 0 && ((j.sp | j.sk) & 3) == 0;
    int sx[4];
#pragma unroll
    for (int k = 0; k < 4; k++) {
        const int xx = min(x + k, w - 1);
        sx[k] = fx ? w - 1 - xx : xx;
    }
#pragma unroll
    for (int rr = 0; rr < PO_RPT; rr++) {
        const int y = blockIdx.y * (PO_TY * PO_RPT) + threadIdx.y + rr * PO_TY;
        if (y >= h)
            break;
        const size_t row = (size_t)j.sk + (size_t)(fy ? h - 1 - y : y) * j.sp;
        uint32_t P[4];
        if (n == 4 && runs) {
            // the four source pixels are one aligned run (reversed when fx)
            uint32_t R[4];
            load_run4<C>(src, row + (size_t)min(sx[0], sx[3]), R);
#pragma unroll
            for (int k = 0; k < 4; k++)
                P[k] = fx ? R[3 - k] : R[k];
        } else {
#pragma unroll
            for (int k = 0; k < 4; k++)
                P[k] = load_u8_px<C>(src, nbytes, row + sx[k]);
        }
        store_u8_4<C>(dst + ((size_t)y * w + x) * C, n, aligned, P);
    }
}

// f32: the samples' bits are moved unchanged (one pixel per thread).
template <int C>
__global__ __launch_bounds__(PO_TX * PO_TY) void k_flip_f32(PtJob j, int fx, int fy)
{
    const uint32_t *__restrict__ src = static_cast<const uint32_t *>(j.src);
    uint32_t *__restrict__ dst = static_cast<uint32_t *>(j.dst);
    const int h = j.h, w = j.w;
    const int x = blockIdx.x * PO_TX + threadIdx.x;
    if (x >= w)
        return;
    const int sx = fx ? w - 1 - x : x;
#pragma unroll
    for (int rr = 0; rr < 4 * PO_RPT; rr++) {
        const int y = blockIdx.y * (PO_TY * 4 * PO_RPT) + threadIdx.y + rr * PO_TY;
        if (y >= h)
            break;
        const uint32_t *s = src + ((size_t)j.sk + (size_t)(fy ? h - 1 - y : y) * j.sp + sx) * C;
        uint32_t *d = dst + ((size_t)y * w + x) * C;
        if constexpr (C == 3) {
            struct __attribute__((packed, aligned(4))) W3 { uint32_t a, b, c; };
            const W3 v = *reinterpret_cast<const W3 *>(s);
            __builtin_nontemporal_store(v.a, d);
            __builtin_nontemporal_store(v.b, d + 1);
            __builtin_nontemporal_store(v.c, d + 2);
        } else {
#pragma unroll
            for (int c = 0; c < C; c++)
                __builtin_nontemporal_store(s[c], d + c);
        }
    }
}

// ---------------------------------------------------------------- gray
__device__ __forceinline__ uint32_t gray_u8(uint32_t p)
{
    const uint32_t acc = 4899u * (p & 0xFFu) + 9617u * ((p >> 8) & 0xFFu) + 1868u * ((p >> 16) & 0xFFu);
    return (acc + 8192u) >> 14;
}

__device__ __forceinline__ float gray_f32(float r, float g, float b, const Epilogue &e)
{
    const float v = __builtin_fmaf(0.114f, b, __builtin_fmaf(0.587f, g, 0.299f * r));
    return __builtin_fmaf(v, e.alpha[0], e.beta[0]);
}

template <bool SRC_F32, bool DST_F32>
__global__ __launch_bounds__(PO_TX * PO_TY) void k_gray(PtJob j, Epilogue e)
{
    const void *__restrict__ src = j.src;
    void *__restrict__ dst = j.dst;
    const int h = j.h, w = j.w;
    const int x = (blockIdx.x * PO_TX + threadIdx.x) * 4;
    if (x >= w)
        return;
    const int n = min(4, w - x);
    const size_t nbytes = ((size_t)j.sk + (size_t)(h - 1) * j.sp + w) * 3 * (SRC_F32 ? 4 : 1);
    const bool runs = ((j.sp | j.sk) & 3) == 0;  // 4-pixel source runs start on multiples of 4
#pragma unroll
    for (int rr = 0; rr < PO_RPT; rr++) {
        const int y = blockIdx.y * (PO_TY * PO_RPT) + threadIdx.y + rr * PO_TY;
        if (y >= h)
            break;
        const size_t lin = (size_t)y * w + x;                      // destination pixel
        const size_t slin = (size_t)j.sk + (size_t)y * j.sp + x;   // source pixel
        float o[4];
        uint32_t g[4];
        if constexpr (!SRC_F32) {
            if (n == 4 && runs) {
                uint32_t P[4];
                load_run4<3>(static_cast<const uint8_t *>(src), slin, P);
#pragma unroll
                for (int k = 0; k < 4; k++) {
                    if constexpr (DST_F32)
                        o[k] = gray_f32((float)(P[k] & 0xFFu), (float)((P[k] >> 8) & 0xFFu),
                                        (float)((P[k] >> 16) & 0xFFu), e);
                    else
                        g[k] = gray_u8(P[k]);
                }
                goto store;
            }
        }
#pragma unroll
        for (int k = 0; k < 4; k++) {
            const size_t q = slin + (size_t)min(k, n - 1);
            if constexpr (SRC_F32) {
                const float *s = static_cast<const float *>(src) + q * 3;
                o[k] = gray_f32(s[0], s[1], s[2], e);
            } else {
                const uint32_t p = load_u8_px<3>(static_cast<const uint8_t *>(src), nbytes, q);
                if constexpr (DST_F32)
                    o[k] = gray_f32((float)(p & 0xFFu), (float)((p >> 8) & 0xFFu), (float)((p >> 16) & 0xFFu), e);
                else
                    g[k] = gray_u8(p);
            }
        }
    store:
        if constexpr (DST_F32) {
            float *d = static_cast<float *>(dst) + lin;
            if (n == 4 && (w & 3) == 0) {
                __builtin_nontemporal_store(f32x4{o[0], o[1], o[2], o[3]}, reinterpret_cast<f32x4 *>(d));
            } else {
                for (int k = 0; k < n; k++)
                    d[k] = o[k];
            }
        } else {
            uint8_t *d = static_cast<uint8_t *>(dst) + lin;
            if (n == 4 && (w & 3) == 0) {
                __builtin_nontemporal_store(g[0] | (g[1] << 8) | (g[2] << 16) | (g[3] << 24),
                                            reinterpret_cast<uint32_t *>(d));
            } else {
                for (int k = 0; k < n; k++)
                    d[k] = (uint8_t)g[k];
            }
        }
    }
}

}  // namespace

hipError_t launch_flip(int c, kr_dtype t, const ImageJob &ij, int fx, int fy, hipStream_t s)
{
    const PtJob j{ij.src, ij.dst, ij.sh, ij.sw, ij.sp, ij.sk};
    const int h = j.h, w = j.w;
    const dim3 block(PO_TX, PO_TY);
    if (t == KR_U8) {
        const dim3 grid((w + 4 * PO_TX - 1) / (4 * PO_TX), (h + PO_TY * PO_RPT - 1) / (PO_TY * PO_RPT));
        switch (c) {
        case 1: hipLaunchKernelGGL(k_flip_u8<1>, grid, block, 0, s, j, fx, fy); break;
        case 2: hipLaunchKernelGGL(k_flip_u8<2>, grid, block, 0, s, j, fx, fy); break;
        case 3: hipLaunchKernelGGL(k_flip_u8<3>, grid, block, 0, s, j, fx, fy); break;
        default: hipLaunchKernelGGL(k_flip_u8<4>, grid, block, 0, s, j, fx, fy); break;
        }
    } else {
        const dim3 grid((w + PO_TX - 1) / PO_TX, (h + 4 * PO_TY * PO_RPT - 1) / (4 * PO_TY * PO_RPT));
        switch (c) {
        case 1: hipLaunchKernelGGL(k_flip_f32<1>, grid, block, 0, s, j, fx, fy); break;
        case 2: hipLaunchKernelGGL(k_flip_f32<2>, grid, block, 0, s, j, fx, fy); break;
        case 3: hipLaunchKernelGGL(k_flip_f32<3>, grid, block, 0, s, j, fx, fy); break;
        default: hipLaunchKernelGGL(k_flip_f32<4>, grid, block, 0, s, j, fx, fy); break;
        }
    }
    return hipGetLastError();
}

hipError_t launch_gray(kr_dtype st, kr_dtype dt, const ImageJob &ij, const Epilogue &e, hipStream_t s)
{
    const PtJob j{ij.src, ij.dst, ij.sh, ij.sw, ij.sp, ij.sk};
    const dim3 block(PO_TX, PO_TY);
    const dim3 grid((j.w + 4 * PO_TX - 1) / (4 * PO_TX), (j.h + PO_TY * PO_RPT - 1) / (PO_TY * PO_RPT));
    if (st == KR_F32)
        hipLaunchKernelGGL((k_gray<true, true>), grid, block, 0, s, j, e);
    else if (dt == KR_F32)
        hipLaunchKernelGGL((k_gray<false, true>), grid, block, 0, s, j, e);
    else
        hipLaunchKernelGGL((k_gray<false, false>), grid, block, 0, s, j, e);
    return hipGetLastError();
}

}  // namespace kr
