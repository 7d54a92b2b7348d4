// tiled.h -- LDS-tiled bilinear resize, affine and perspective warp for u8
// sources with 1-4 interleaved channels (device code shared by the per-image
// and the batched kernels).
//
// One workgroup (4 waves) produces an output tile; each lane owns runs of PX
// consecutive pixels (the lane layout is a template parameter, see Layout).
//
//  1. The source box the tile's 2x2 taps can touch is found from its corners
//     (the inverse map is monotone along each output axis, so its extremes sit
//     at the corners; resize uses exact per-column/per-row integer tables).
//  2. The box rows are staged into LDS as one dword per pixel.  Staging walks
//     16-pixel groups aligned on the image's linear pixel index: a group is 48
//     (RGB) or 64 (RGBA) contiguous, 16-byte aligned bytes, read with dwordx4
//     loads that a wave issues as contiguous 1 KB requests.  RGB groups are
//     widened to one dword per pixel with byte-align ops.
//  3. Each pixel reads its four taps with two ds_read2_b32, interpolates with
//     v_perm (channel pairs) + v_dot2_u32_u16 (horizontal, 11-bit weights) +
//     u24 multiply-adds (vertical).  Stores: with 4-pixel runs a lane writes
//     12/16 contiguous bytes (u8) at once; with 1-pixel runs the 64 lanes of
//     a wave own 64 consecutive pixels, so each store instruction writes one
//     contiguous run (768 bytes of f32 RGB; RGB u8 packed across lane quads
//     with one DPP exchange and a byte permute, 192 bytes).
//
// Border rule per tap.  Tiles whose box lies inside the image take no border
// logic at all.  Other tiles stage clamped rows; REPLICATE additionally copies
// edge pixels into the out-of-image columns of the box; CONSTANT zeroes the
// weights of out-of-image taps and adds border * (missing weight).
#pragma once

#include "kr_device.h"

namespace kr {

typedef unsigned short u16x2 __attribute__((ext_vector_type(2)));

constexpr int KT_THREADS = 256;
// LDS box rows.  Staging writes whole 16-pixel groups aligned on the source's
// pixel numbering, so a row's writes reach up to KT_SPILL pixels before and
// after its box.  Row s of the box starts at dword s * pitch + KT_MARGIN; with
// pitch >= box width + KT_SPILL one row's spill ends before the next row's
// box begins and starts after the previous row's box ends (neighbouring
// spills may overlap: they hold pixels nobody reads).  KT_MARGIN dwords
// before row 0 take its left spill; the last row's right spill stays inside
// its own pitch.
constexpr int KT_MARGIN = 16;
constexpr int KT_SPILL = 15;

// Per-image parameters of the tiled kernels.
struct TiledJob {
    ImageJob j;
    double m2048[6];  // warp inverse map scaled by 2048 (exact), for the u8 path
    double rden_x;    // resize: 1 / (2 dst_w), rounded (exact quotients by correction)
    double rden_y;    // resize: 1 / (2 dst_h), rounded
    int op;           // OP_RESIZE or OP_WARP
    int rows_contig;  // resize: stage the tile's source rows once each (vertical ratio <= 2, every row
                      // of the span is a tap row); else two LDS rows per output row
    int tiles_x;      // output tiles per row
    int ntiles;       // output tiles in the image
    int first_tile;   // index of the image's first tile in a batch work-list
};

// ------------------------------------------------------------------ helpers
// round-half-even of a binary64 value |X| < 2^51 to int32: adding 1.5 * 2^52
// leaves the rounded integer in the low mantissa bits.
__device__ __forceinline__ int rne_i32(double X)
{
    const double r = X + 6755399441055744.0;
    return (int)(uint32_t)__builtin_bit_cast(uint64_t, r);
}

__device__ __forceinline__ uint32_t udot2(uint32_t a, uint32_t b)
{
    return __builtin_amdgcn_udot2(__builtin_bit_cast(u16x2, a), __builtin_bit_cast(u16x2, b), 0u, false);
}

__device__ __forceinline__ int clampi(int v, int lo, int hi) { return v < lo ? lo : (v > hi ? hi : v); }

// k / d for 0 <= k < 2^22, 1 <= d < 2^22: a float-reciprocal estimate (off by
// at most one) corrected with the exact remainder.
__device__ __forceinline__ int udiv_small(int k, int d)
{
    int q = (int)((float)k * __builtin_amdgcn_rcpf((float)d));
    const int r = k - q * d;
    q += r >= d ? 1 : 0;
    q -= r < 0 ? 1 : 0;
    return q;
}

// Blocks are handed to the 8 XCDs round-robin; give each XCD one contiguous
// run of tiles so that neighbouring tiles (which share source rows) meet in
// the same L2.
__device__ __forceinline__ int xcd_tile(int b, int n)
{
    const int k = b & 7, q = n >> 3, r = n & 7;
    return k * q + (k < r ? k : r) + (b >> 3);
}

// One source pixel of C <= 4 u8 channels as a dword (byte c = channel c),
// read byte by byte (used off the fast path).
template <int C>
__device__ __forceinline__ uint32_t load_px_bytes(const uint8_t *src, size_t lin)
{
    const uint8_t *p = src + lin * C;
    uint32_t v = 0;
#pragma unroll
    for (int c = 0; c < C; c++)
        v |= (uint32_t)p[c] << (8 * c);
    return v;
}

// Source pixel of C u8 channels at pixel index lin (byte c = channel c), in
// an image of nbytes bytes: RGBA one dword, RGB a dword-aligned 8-byte load
// (bytewise at the very end of the buffer), fewer channels bytewise.
template <int C>
__device__ __forceinline__ uint32_t load_u8_px(const uint8_t *__restrict__ src, size_t nbytes, size_t lin)
{
    if constexpr (C == 4) {
        return *reinterpret_cast<const uint32_t *>(src + lin * 4);
    } else if constexpr (C == 3) {
        const size_t b = lin * 3, f = b & ~(size_t)3;
        if (f + 8 <= nbytes) {
            struct __attribute__((packed, aligned(4))) D2 { uint32_t a, b; };
            const D2 d = *reinterpret_cast<const D2 *>(src + f);
            return __builtin_amdgcn_alignbyte(d.b, d.a, (uint32_t)(b & 3)) & 0xFFFFFFu;
        }
        return load_px_bytes<3>(src, lin);
    } else {
        return load_px_bytes<C>(src, lin);
    }
}


// ------------------------------------------------------------------ pixel math
// u8 interpolation of one pixel from its four tap dwords (byte c = channel c).
// wxp packs the horizontal weights w0 | w1 << 16 (w0 + w1 = 2048); wy0_4,
// wy1_4 are 4x the vertical weights.  Per channel and tap row, v_perm builds
// the u16 pair (left, right) and v_dot2 forms h = w0 l + w1 r (< 2^20) plus
// 1024; then v = wy0_4 h0 + wy1_4 h1 = 4 acc + 1024 (wy0_4 + wy1_4), which is
// 4 acc + 2^23 when the vertical weights sum to 2048.  Channel c's output is
// the top byte of v[c]: (4 acc + 2^23) >> 24 == (acc + 2^21) >> 22.
template <int C>
__device__ __forceinline__ void interp_u8(uint32_t t00, uint32_t t01, uint32_t t10, uint32_t t11, uint32_t wxp,
                                          uint32_t wy0_4, uint32_t wy1_4, uint32_t (&v)[C])
{
#pragma unroll
    for (int c = 0; c < C; c++) {
        const uint32_t sel = (uint32_t)c | 0x00000C00u | ((uint32_t)(4 + c) << 16) | 0x0C000000u;
        const uint32_t h0 = __builtin_amdgcn_udot2(__builtin_bit_cast(u16x2, __builtin_amdgcn_perm(t01, t00, sel)),
                                                   __builtin_bit_cast(u16x2, wxp), 1024u, false);
        const uint32_t h1 = __builtin_amdgcn_udot2(__builtin_bit_cast(u16x2, __builtin_amdgcn_perm(t11, t10, sel)),
                                                   __builtin_bit_cast(u16x2, wxp), 1024u, false);
        v[c] = __umul24(h1, wy1_4) + __umul24(h0, wy0_4);
    }
}

// CONSTANT border on an edge tile: zero the weights of out-of-image taps
// (tap (i, j) is inside iff row i and column j are) and return what must be
// added to v so that it equals 4 (acc + border * missing weight) + 2^23.
__device__ __forceinline__ uint32_t mask_weights(int x0, int y0, int W, int H, uint32_t &wx0, uint32_t &wx1,
                                                 uint32_t &wy0, uint32_t &wy1, uint32_t bval)
{
    wx0 = (unsigned)x0 < (unsigned)W ? wx0 : 0u;
    wx1 = (unsigned)(x0 + 1) < (unsigned)W ? wx1 : 0u;
    wy0 = (unsigned)y0 < (unsigned)H ? wy0 : 0u;
    wy1 = (unsigned)(y0 + 1) < (unsigned)H ? wy1 : 0u;
    const uint32_t missing = (1u << 22) - __umul24(wy0 + wy1, wx0 + wx1);
    return (1u << 23) - 4096u * (wy0 + wy1) + 4u * bval * missing;
}

// f32 interpolation with unquantised weights (blend4), plus the border's
// share when EXTRA (CONSTANT border with masked taps), then
// out = v * alpha + beta.  The operation order is fixed (explicit fma, no
// contraction), so every kernel path produces the same bits.  SF: the taps
// are binary32 pixels of a one-channel f32 source; with EXTRA a tap whose
// weight is zero counts as 0 (a masked tap's LDS word is not a pixel and may
// hold any bits, a NaN included).
template <int C, bool EXTRA, bool SF = false>
__device__ __forceinline__ void interp_f32(uint32_t t00, uint32_t t01, uint32_t t10, uint32_t t11, float wx0,
                                           float wx1, float wy0, float wy1, float extra, const Epilogue &e,
                                           float (&o)[C])
{
    const Weights2 w = weights2(wx0, wx1, wy0, wy1);
#pragma unroll
    for (int c = 0; c < C; c++) {
        float p00, p01, p10, p11;
        if constexpr (SF) {
            p00 = __builtin_bit_cast(float, t00);
            p01 = __builtin_bit_cast(float, t01);
            p10 = __builtin_bit_cast(float, t10);
            p11 = __builtin_bit_cast(float, t11);
            if constexpr (EXTRA) {
                p00 = wx0 != 0.0f && wy0 != 0.0f ? p00 : 0.0f;
                p01 = wx1 != 0.0f && wy0 != 0.0f ? p01 : 0.0f;
                p10 = wx0 != 0.0f && wy1 != 0.0f ? p10 : 0.0f;
                p11 = wx1 != 0.0f && wy1 != 0.0f ? p11 : 0.0f;
            }
        } else {
            p00 = (float)((t00 >> (8 * c)) & 0xFFu);
            p01 = (float)((t01 >> (8 * c)) & 0xFFu);
            p10 = (float)((t10 >> (8 * c)) & 0xFFu);
            p11 = (float)((t11 >> (8 * c)) & 0xFFu);
        }
        float v = blend4(p00, p01, p10, p11, w);
        if constexpr (EXTRA)
            v = v + extra;
        o[c] = __builtin_fmaf(v, e.alpha[c], e.beta[c]);
    }
}

// A wave-uniform value copied into vector registers once.  A vector
// instruction reads at most one scalar register, so an fma with two uniform
// operands (alpha and beta of the epilogue, a map coefficient and its offset)
// would otherwise copy one of them for every pixel; the empty asm pins the
// copy in a vector register, where the compiler cannot rematerialise it.
template <typename T>
__device__ __forceinline__ T in_vgpr(T v)
{
    asm("" : "+v"(v));
    return v;
}

// The epilogue with beta in vector registers, for the f32 paths.
template <int C, bool F32>
__device__ __forceinline__ Epilogue epilogue_in_vgpr(const Epilogue &e)
{
    Epilogue v = e;
    if constexpr (F32) {
#pragma unroll
        for (int c = 0; c < C; c++)
            v.beta[c] = in_vgpr(e.beta[c]);
    }
    return v;
}

// ------------------------------------------------------------------ stores
// Lane layout (see compute below): a lane owns PX consecutive pixels of a row.
// PX = 4: the lane stores 4 pixels at once (12/16 contiguous bytes for u8,
// 48/64 for f32).  PX = 1: the 64 lanes of a wave own 64 consecutive pixels of
// one row, so each store instruction writes one contiguous run (RGB u8 is
// packed across lane quads with a DPP exchange).
__device__ __forceinline__ int lane_id() { return (int)(threadIdx.x & 63); }

// floor(num / den) and the remainder, for |num| < 2^31 and 0 < den < 2^17,
// from a rounded reciprocal rden of den: num * rden is within 2^-20 of the
// exact quotient, so the floor is off by at most one and the exact integer
// remainder corrects it.
__device__ __forceinline__ int floor_div_r(int num, int den, double rden, int &rem)
{
    int q = (int)__builtin_floor((double)num * rden);
    int r = num - q * den;
    if (r < 0) {
        q -= 1;
        r += den;
    } else if (r >= den) {
        q += 1;
        r -= den;
    }
    rem = r;
    return q;
}

// Resize axis map (half-pixel centres, exact rational) with the reciprocal of
// den = 2 n_out: i0 = floor(((2 d + 1) n_in - n_out) / den); w1 =
// round-half-even(2048 r / den) by the exact integer rule; f = r / den (f32,
// correctly rounded).
__device__ __forceinline__ int resize_i0_r(int d, int n_in, int n_out, double rden)
{
    int r;
    return floor_div_r((2 * d + 1) * n_in - n_out, 2 * n_out, rden, r);
}

__device__ __forceinline__ void resize_axis_r(int d, int n_in, int n_out, double rden, int &i0, int &w1, float &f)
{
    const int den = 2 * n_out;
    int r, r2;
    i0 = floor_div_r((2 * d + 1) * n_in - n_out, den, rden, r);
    const int t = 4096 * r + den;  // < 2^28
    int q = floor_div_r(t, 2 * den, 0.5 * rden, r2);
    if (r2 == 0 && (q & 1))
        q -= 1;
    w1 = q;
    f = (float)r / (float)den;
}

// Pack per-channel results (top byte of v[c]) into one pixel dword, byte c =
// channel c.
template <int C>
__device__ __forceinline__ uint32_t pack_px(const uint32_t (&v)[C])
{
    if constexpr (C == 1)
        return v[0] >> 24;
    else if constexpr (C == 2)
        return __builtin_amdgcn_perm(v[1], v[0], 0x0C0C0703u);
    else if constexpr (C == 3)
        return __builtin_amdgcn_perm(v[2], __builtin_amdgcn_perm(v[1], v[0], 0x0C0C0703u), 0x0C070100u);
    else
        return __builtin_amdgcn_perm(v[3], v[2], 0x07030C0Cu) | __builtin_amdgcn_perm(v[1], v[0], 0x0C0C0703u);
}

// Whether 4-pixel chunks starting at multiple-of-4 columns of rows dw pixels
// wide are aligned for the vector stores below (RGB u8: 4 bytes; otherwise
// 16); the destination base is 16-byte aligned.
template <int C, bool F32>
__device__ __forceinline__ bool store4_aligned(int dw)
{
    // u8: 4 pixels are 4 (C = 1), 8, 12 (dword-aligned) or 16 bytes; f32: 16,
    // 32, 48 or 64 bytes, stored as 16-byte vectors
    const size_t row_bytes = (size_t)dw * C * (F32 ? 4 : 1);
    const size_t mask = F32 ? 15 : (C == 1 || C == 3 ? 3 : (C == 2 ? 7 : 15));
    return (row_bytes & mask) == 0;
}

// Four u8 pixels (pixel k = P[k], byte c = channel c); n valid pixels.
// RGB and RGBA runs leave through non-temporal stores (no kernel of the call
// reads them back; with outputs written back to HBM the 4K warp to u8 runs
// 5-8 % faster than with plain stores).
template <int C>
__device__ __forceinline__ void store_u8_4(uint8_t *p, int n, bool aligned, const uint32_t (&P)[4])
{
    if (n == 4 && aligned) {
        if constexpr (C == 3) {
            // R0 G0 B0 R1 | G1 B1 R2 G2 | B2 R3 G3 B3
            uint32_t *q = reinterpret_cast<uint32_t *>(p);
            __builtin_nontemporal_store(__builtin_amdgcn_perm(P[1], P[0], 0x04020100u), q);
            __builtin_nontemporal_store(__builtin_amdgcn_perm(P[2], P[1], 0x05040201u), q + 1);
            __builtin_nontemporal_store(__builtin_amdgcn_perm(P[3], P[2], 0x06050402u), q + 2);
        } else if constexpr (C == 4) {
            __builtin_nontemporal_store(u32x4{P[0], P[1], P[2], P[3]}, reinterpret_cast<u32x4 *>(p));
        } else if constexpr (C == 2) {
            __builtin_nontemporal_store(u32x2{__builtin_amdgcn_perm(P[1], P[0], 0x05040100u),
                                              __builtin_amdgcn_perm(P[3], P[2], 0x05040100u)},
                                        reinterpret_cast<u32x2 *>(p));
        } else {
            __builtin_nontemporal_store(
                __builtin_amdgcn_perm(__builtin_amdgcn_perm(P[3], P[2], 0x0C0C0400u),
                                      __builtin_amdgcn_perm(P[1], P[0], 0x0C0C0400u), 0x05040100u),
                reinterpret_cast<uint32_t *>(p));
        }
    } else {
        for (int k = 0; k < n; k++)
#pragma unroll
            for (int c = 0; c < C; c++)
                p[k * C + c] = (uint8_t)(P[k] >> (8 * c));
    }
}

// f32 vector store; NT: non-temporal (streaming) store, for outputs that no
// later kernel of the launch reads.
template <bool NT, typename V>
__device__ __forceinline__ void put(V *q, V v)
{
    if constexpr (NT)
        __builtin_nontemporal_store(v, q);
    else
        *q = v;
}

template <int C, bool NT = false>
__device__ __forceinline__ void store_f32_4(float *p, int n, bool aligned, const float (&o)[4][C])
{
    if (n == 4 && aligned) {
        f32x4 *q = reinterpret_cast<f32x4 *>(p);
        if constexpr (C == 3) {
            put<NT>(q + 0, f32x4{o[0][0], o[0][1], o[0][2], o[1][0]});
            put<NT>(q + 1, f32x4{o[1][1], o[1][2], o[2][0], o[2][1]});
            put<NT>(q + 2, f32x4{o[2][2], o[3][0], o[3][1], o[3][2]});
        } else if constexpr (C == 4) {
#pragma unroll
            for (int k = 0; k < 4; k++)
                put<NT>(q + k, f32x4{o[k][0], o[k][1], o[k][2], o[k][3]});
        } else if constexpr (C == 2) {
            put<NT>(q + 0, f32x4{o[0][0], o[0][1], o[1][0], o[1][1]});
            put<NT>(q + 1, f32x4{o[2][0], o[2][1], o[3][0], o[3][1]});
        } else {
            put<NT>(q, f32x4{o[0][0], o[1][0], o[2][0], o[3][0]});
        }
    } else {
        for (int k = 0; k < n; k++)
#pragma unroll
            for (int c = 0; c < C; c++)
                p[k * C + c] = o[k][c];
    }
}

// Byte selectors of the three dwords a quad of RGB pixels packs into: lane j
// of the quad takes bytes [j, j + 4) of {own 0, own 1, own 2, next 0, next 1,
// next 2}.
__device__ __forceinline__ uint32_t quad_selector(int j)
{
    return (uint32_t)(0x0000060504020100ull >> (8 * j));
}

// One u8 pixel per lane (PX = 1).  RGB: all lanes of the wave must call this
// together (the quad exchange reads the neighbouring lane); quads inside the
// row store three packed dwords, a ragged tail quad stores bytes.
template <int C>
__device__ __forceinline__ void store_u8_px(uint8_t *row, int x, int x_end, bool row_aligned, uint32_t P, uint32_t sel)
{
    if constexpr (C == 4) {
        if (x < x_end)
            __builtin_nontemporal_store(P, reinterpret_cast<uint32_t *>(row + 4 * (size_t)x));
    } else {
        const uint32_t Pn = (uint32_t)__builtin_amdgcn_update_dpp(0, (int)P, 0xF9, 0xF, 0xF, false);
        const int j = lane_id() & 3;
        const int xq = x - j;
        if (row_aligned && xq + 3 < x_end) {
            if (j < 3)
                __builtin_nontemporal_store(__builtin_amdgcn_perm(Pn, P, sel),
                                            reinterpret_cast<uint32_t *>(row + 3 * (size_t)xq + 4 * j));
        } else if (x < x_end) {
            uint8_t *q = row + 3 * (size_t)x;
            q[0] = (uint8_t)P;
            q[1] = (uint8_t)(P >> 8);
            q[2] = (uint8_t)(P >> 16);
        }
    }
}

template <int C, bool NT = false>
__device__ __forceinline__ void store_f32_px(float *row, int x, int x_end, const float (&o)[C])
{
    if (x >= x_end)
        return;
    // 32-bit byte offset (a row is far below 4 GiB): with a wave-uniform row
    // pointer the store takes it as scalar base plus vector offset
    float *q = reinterpret_cast<float *>(reinterpret_cast<char *>(row) + (uint32_t)x * (uint32_t)(4 * C));
    if constexpr (C == 3) {
        if constexpr (NT) {  // three adjacent dwords: one 12-byte store
            put<true>(q, o[0]);
            put<true>(q + 1, o[1]);
            put<true>(q + 2, o[2]);
        } else {
            struct __attribute__((packed, aligned(4))) F3 { float a, b, c; };
            *reinterpret_cast<F3 *>(q) = F3{o[0], o[1], o[2]};
        }
    } else {
        put<NT>(reinterpret_cast<f32x4 *>(q), f32x4{o[0], o[1], o[2], o[3]});
    }
}

// Store the PX pixels of one lane run starting at column x (u8).
template <int C, int PX>
__device__ __forceinline__ void store_run_u8(uint8_t *row, int x, int x_end, bool aligned, const uint32_t (&P)[PX],
                                             uint32_t sel)
{
    if constexpr (PX == 4)
        store_u8_4<C>(row + (size_t)x * C, min(4, x_end - x), aligned, P);
    else
        store_u8_px<C>(row, x, x_end, aligned, P[0], sel);
}

template <int C, int PX, bool NT = false>
__device__ __forceinline__ void store_run_f32(float *row, int x, int x_end, bool aligned, const float (&o)[PX][C])
{
    if constexpr (PX == 4) {
        if (x < x_end)
            store_f32_4<C, NT>(row + (size_t)x * C, min(4, x_end - x), aligned, o);
    } else {
        store_f32_px<C, NT>(row, x, x_end, o[0]);
    }
}

// BT.601 luma of an RGB pixel (byte c = channel c): u8 with 14-bit weights
// (summing to 2^14, so grey stays grey), rounded half up; f32 in binary32
// with the fma chain of the standalone RGB -> gray kernel, so that a fused
// gray equals resampling followed by that kernel, bit for bit.
__device__ __forceinline__ uint32_t luma_u8(uint32_t p)
{
    const uint32_t acc = 4899u * (p & 0xFFu) + 9617u * ((p >> 8) & 0xFFu) + 1868u * ((p >> 16) & 0xFFu);
    return (acc + 8192u) >> 14;
}

__device__ __forceinline__ float luma_f32(float r, float g, float b)
{
    return __builtin_fmaf(0.114f, b, __builtin_fmaf(0.587f, g, 0.299f * r));
}

// Gray output (one channel, row y of dw pixels): the lane's PX pixels from
// their RGB results.  4-pixel runs are one dword (u8) or one 16-byte vector
// (f32) when the row width is a multiple of 4.
template <int PX>
__device__ __forceinline__ void store_gray_u8(const ImageJob &j, int y, int x, int x_end, const uint32_t (&P)[PX])
{
    uint8_t *row = static_cast<uint8_t *>(j.dst) + (size_t)y * (size_t)j.dw;
    const int n = min(PX, x_end - x);
    if (n <= 0)
        return;
    if constexpr (PX == 4) {
        if (n == 4 && (j.dw & 3) == 0) {
            __builtin_nontemporal_store(
                luma_u8(P[0]) | (luma_u8(P[1]) << 8) | (luma_u8(P[2]) << 16) | (luma_u8(P[3]) << 24),
                reinterpret_cast<uint32_t *>(row + x));
            return;
        }
    }
    for (int k = 0; k < n; k++)
        row[x + k] = (uint8_t)luma_u8(P[k]);
}

template <int C, int PX, bool NT>
__device__ __forceinline__ void store_gray_f32(const ImageJob &j, const Epilogue &e, int y, int x, int x_end,
                                               const float (&o)[PX][C])
{
    float *row = static_cast<float *>(j.dst) + (size_t)y * (size_t)j.dw;
    const int n = min(PX, x_end - x);
    if (n <= 0)
        return;
    float g[PX];
#pragma unroll
    for (int k = 0; k < PX; k++)
        g[k] = __builtin_fmaf(luma_f32(o[k][0], o[k][1], o[k][2]), e.galpha, e.gbeta);
    if constexpr (PX == 4) {
        if (n == 4 && (j.dw & 3) == 0) {
            put<NT>(reinterpret_cast<f32x4 *>(row + x), f32x4{g[0], g[1], g[2], g[3]});
            return;
        }
    }
    for (int k = 0; k < n; k++)
        put<NT>(row + x + k, g[k]);
}

// Store one lane run of output row y, interleaved (HWC, through the runs
// above) or planar (CHW: channel c of pixel (x, y) at c * dh * dw + y * dw +
// x; a 4-pixel run is one dword (u8) or one 16-byte vector (f32) per plane
// when the row width is a multiple of 4), or as one gray channel.  The
// branches are uniform per launch.
template <int C, int PX>
__device__ __forceinline__ void store_row_u8(const ImageJob &j, const Epilogue &e, int y, int x, int x_end,
                                             bool aligned, const uint32_t (&P)[PX], uint32_t sel)
{
    const bool planar = e.planar;
    if constexpr (C == 3) {
        if (e.gray) {
            store_gray_u8<PX>(j, y, x, x_end, P);
            return;
        }
    }
    if (!planar) {
        store_run_u8<C, PX>(static_cast<uint8_t *>(j.dst) + (size_t)y * (size_t)j.dw * C, x, x_end, aligned, P, sel);
        return;
    }
    const size_t plane = (size_t)j.dh * (size_t)j.dw;
    uint8_t *row = static_cast<uint8_t *>(j.dst) + (size_t)y * (size_t)j.dw + x;
    const int n = min(PX, x_end - x);
    if (n <= 0)
        return;
#pragma unroll
    for (int c = 0; c < C; c++) {
        if constexpr (PX == 4) {
            if (n == 4 && (j.dw & 3) == 0) {
                const uint32_t lo = __builtin_amdgcn_perm(P[1], P[0], 0x0C0C0400u + 0x00000101u * c);
                const uint32_t hi = __builtin_amdgcn_perm(P[3], P[2], 0x0C0C0400u + 0x00000101u * c);
                __builtin_nontemporal_store(__builtin_amdgcn_perm(hi, lo, 0x05040100u),
                                            reinterpret_cast<uint32_t *>(row + c * plane));
                continue;
            }
        }
        for (int k = 0; k < n; k++)
            row[c * plane + k] = (uint8_t)(P[k] >> (8 * c));
    }
}

template <int C, int PX, bool NT = false>
__device__ __forceinline__ void store_row_f32(const ImageJob &j, const Epilogue &e, int y, int x, int x_end,
                                              bool aligned, const float (&o)[PX][C])
{
    const bool planar = e.planar;
    if constexpr (C == 3) {
        if (e.gray) {
            store_gray_f32<C, PX, NT>(j, e, y, x, x_end, o);
            return;
        }
    }
    if (!planar) {
        size_t off = (size_t)y * (size_t)j.dw * C;
        if constexpr (PX == 1)
            asm("" : "+s"(off));  // one row per wave: keep its offset scalar, lane offsets 32-bit
        store_run_f32<C, PX, NT>(static_cast<float *>(j.dst) + off, x, x_end, aligned, o);
        return;
    }
    const size_t plane = (size_t)j.dh * (size_t)j.dw;
    float *row = static_cast<float *>(j.dst) + (size_t)y * (size_t)j.dw + x;
    const int n = min(PX, x_end - x);
    if (n <= 0)
        return;
#pragma unroll
    for (int c = 0; c < C; c++) {
        if constexpr (PX == 4) {
            if (n == 4 && (j.dw & 3) == 0) {
                put<NT>(reinterpret_cast<f32x4 *>(row + c * plane), f32x4{o[0][c], o[1][c], o[2][c], o[3][c]});
                continue;
            }
        }
        for (int k = 0; k < n; k++)
            put<NT>(row + c * plane + k, o[k][c]);
    }
}

// ------------------------------------------------------------------ tile plan
// Launch-wide LDS geometry: every tile of a launch stages into rows x pitch dwords.
struct TileGeom {
    int pitch;  // LDS row pitch in dwords (>= box width + KT_SPILL)
    int rows;   // LDS rows (box rows for warps, 2 * tile height for resizes)
};

// Everything one tile needs, uniform across the workgroup.
struct Plan {
    int ox0, oy0, ox1, oy1;  // output pixels covered (inclusive)
    int bx0, bw;             // box columns [bx0, bx0 + bw)
    int by0, nslots;         // slot s = source row by0 + s (warps; resizes with rows_contig),
                             // else (resizes) two slots per output row
    int cx0, cx1, ng;        // in-image box columns; 16-pixel groups per slot (upper bound)
    bool inside;             // every tap of the tile lies inside the image
    bool direct;             // box exceeds the LDS budget: per-pixel evaluation
    bool blank;              // warps, CONSTANT border: every tap lies outside the image,
                             // so every output is the border value (nothing staged)
};

// u8 coordinate of one axis: the 2048-scaled binary64 coordinate X gives
// N = rne(X), x0 = N >> 11, w1 = N & 2047.  This equals floor and
// round-half-even of the unscaled coordinate: rne(2048 xs) = 2048 floor(xs) +
// rne(2048 frac); when rne(2048 frac) = 2048 the taps move right by one with
// weights (2048, 0), which gives the same exact sum.  Scaling by 2048 is exact,
// so fma(2048 A, x, fma(2048 B, y, 2048 C)) = 2048 fma(A, x, fma(B, y, C)).
__device__ __forceinline__ double clamp_scaled(double X, int n)
{
    const double lo = -4096.0, hi = 2048.0 * ((double)n + 1.0);
    return X < lo ? lo : (X > hi ? hi : X);
}

__device__ __forceinline__ double clamp_plain(double X, int n)
{
    const double hi = (double)n + 1.0;
    return X < -2.0 ? -2.0 : (X > hi ? hi : X);
}

// Perspective source coordinate on one axis: num / w in binary64 (correctly
// rounded); a quotient that is not a number reads as -2; clamped to
// [-2, n + 1] like the affine coordinates.
__device__ __forceinline__ double persp_coord(double num, double w, int n)
{
    double v = num / w;
    v = v != v ? -2.0 : v;
    const double hi = (double)n + 1.0;
    return v < -2.0 ? -2.0 : (v > hi ? hi : v);
}

template <int OP, int TW, int TH, bool F32>
__device__ __forceinline__ Plan make_plan(const TiledJob &t, int tile, const TileGeom &G, bool constant_border)
{
    const ImageJob &j = t.j;
    const int H = j.sh, W = j.sw;
    Plan p;
    const int ty = tile / t.tiles_x, tx = tile - ty * t.tiles_x;
    p.ox0 = tx * TW;
    p.oy0 = ty * TH;
    p.ox1 = min(p.ox0 + TW, j.dw) - 1;
    p.oy1 = min(p.oy0 + TH, j.dh) - 1;
    int x0min, x0max, y0min, y0max;
    bool persp_ok = true;
    // The four bounds come from four independent evaluations: lane q of the
    // wave computes the q-th one and every lane reads them back (readlane).
    const int q = lane_id() & 3;
    if constexpr (OP == OP_RESIZE) {
        const int d = q == 0 ? p.ox0 : (q == 1 ? p.ox1 : (q == 2 ? p.oy0 : p.oy1));
        const int v = q < 2 ? resize_i0_r(d, W, j.dw, t.rden_x) : resize_i0_r(d, H, j.dh, t.rden_y);
        x0min = __builtin_amdgcn_readlane(v, 0);
        x0max = __builtin_amdgcn_readlane(v, 1);
        y0min = __builtin_amdgcn_readlane(v, 2);
        y0max = __builtin_amdgcn_readlane(v, 3);
        p.inside = x0min >= 0 && x0max + 1 <= W - 1 && y0min >= 0 && y0max + 1 <= H - 1;
        if (t.rows_contig) {
            p.by0 = y0min;
            p.nslots = y0max + 2 - y0min;
        } else {
            p.by0 = 0;
            p.nslots = 2 * (p.oy1 - p.oy0 + 1);
        }
    } else if constexpr (OP == OP_PERSP) {
        // Tap box from the four corners (lane q takes corner q).  Where w > 0
        // at the corners it is positive over the whole tile, whose image is
        // then the convex quadrilateral of the corner images; the box gets
        // one extra pixel on each side for the rounding of the quotients.  A
        // tile reaching w <= 0 evaluates its pixels from global memory.
        const double cx = (double)((q & 1) ? p.ox1 : p.ox0), cy = (double)((q & 2) ? p.oy1 : p.oy0);
        const double w = __builtin_fma(j.proj[0], cx, __builtin_fma(j.proj[1], cy, j.proj[2]));
        const double X = persp_coord(__builtin_fma(j.inv[0], cx, __builtin_fma(j.inv[1], cy, j.inv[2])), w, W);
        const double Y = persp_coord(__builtin_fma(j.inv[3], cx, __builtin_fma(j.inv[4], cy, j.inv[5])), w, H);
        const int ix = (int)__builtin_floor(X), iy = (int)__builtin_floor(Y);
        const int pos = w > 0.0 ? 1 : 0;
        persp_ok = (__builtin_amdgcn_readlane(pos, 0) & __builtin_amdgcn_readlane(pos, 1) &
                    __builtin_amdgcn_readlane(pos, 2) & __builtin_amdgcn_readlane(pos, 3)) != 0;
        const int a0 = __builtin_amdgcn_readlane(ix, 0), a1 = __builtin_amdgcn_readlane(ix, 1);
        const int a2 = __builtin_amdgcn_readlane(ix, 2), a3 = __builtin_amdgcn_readlane(ix, 3);
        const int b0 = __builtin_amdgcn_readlane(iy, 0), b1 = __builtin_amdgcn_readlane(iy, 1);
        const int b2 = __builtin_amdgcn_readlane(iy, 2), b3 = __builtin_amdgcn_readlane(iy, 3);
        x0min = min(min(a0, a1), min(a2, a3)) - 1;
        x0max = max(max(a0, a1), max(a2, a3)) + 1;
        y0min = min(min(b0, b1), min(b2, b3)) - 1;
        y0max = max(max(b0, b1), max(b2, b3)) + 1;
        p.inside = persp_ok && x0min >= 0 && x0max + 1 <= W - 1 && y0min >= 0 && y0max + 1 <= H - 1;
        p.by0 = y0min;
        p.nslots = y0max + 2 - y0min;
    } else {
        // Tap box from the four corners (lane q takes corner q).  fma(A, x,
        // fma(B, y, C)) is monotone in x and in y separately, and so are the
        // clamp and the rounding, so the extremes over the tile sit at its
        // corners.  First unclamped, to find interior tiles (no clamp, no
        // border logic per pixel).
        const double *m = F32 ? j.inv : t.m2048;
        const double b = F32 ? 1.0e9 : 2.0e9;  // keeps the integer conversion in range
        const double cx = (double)((q & 1) ? p.ox1 : p.ox0), cy = (double)((q & 2) ? p.oy1 : p.oy0);
        const double X = __builtin_fma(m[0], cx, __builtin_fma(m[1], cy, m[2]));
        const double Y = __builtin_fma(m[3], cx, __builtin_fma(m[4], cy, m[5]));
        auto corner_bounds = [&](int ix, int iy) {
            const int a0 = __builtin_amdgcn_readlane(ix, 0), a1 = __builtin_amdgcn_readlane(ix, 1);
            const int a2 = __builtin_amdgcn_readlane(ix, 2), a3 = __builtin_amdgcn_readlane(ix, 3);
            const int b0 = __builtin_amdgcn_readlane(iy, 0), b1 = __builtin_amdgcn_readlane(iy, 1);
            const int b2 = __builtin_amdgcn_readlane(iy, 2), b3 = __builtin_amdgcn_readlane(iy, 3);
            x0min = min(min(a0, a1), min(a2, a3));
            x0max = max(max(a0, a1), max(a2, a3));
            y0min = min(min(b0, b1), min(b2, b3));
            y0max = max(max(b0, b1), max(b2, b3));
        };
        {
            const double Xb = X < -b ? -b : (X > b ? b : X);
            const double Yb = Y < -b ? -b : (Y > b ? b : Y);
            const int ix = F32 ? (int)__builtin_floor(Xb) : (rne_i32(Xb) >> 11);
            const int iy = F32 ? (int)__builtin_floor(Yb) : (rne_i32(Yb) >> 11);
            corner_bounds(ix, iy);
        }
        p.inside = x0min >= 0 && x0max + 1 <= W - 1 && y0min >= 0 && y0max + 1 <= H - 1;
        if (!p.inside) {
            int ix, iy;
            if (F32) {
                ix = (int)__builtin_floor(clamp_plain(X, W));
                iy = (int)__builtin_floor(clamp_plain(Y, H));
            } else {
                ix = rne_i32(clamp_scaled(X, W)) >> 11;
                iy = rne_i32(clamp_scaled(Y, H)) >> 11;
            }
            corner_bounds(ix, iy);
        }
        p.by0 = y0min;
        p.nslots = y0max + 2 - y0min;
    }
    p.bx0 = x0min;
    p.bw = x0max + 2 - x0min;
    p.direct = !persp_ok || p.bw + KT_SPILL > G.pitch || p.nslots > G.rows;
    // The bounds hold every pixel's top-left tap (x0, y0); its taps are x0,
    // x0 + 1 and y0, y0 + 1.  If all of them fall left of, right of, above or
    // below the image, every tap reads the border constant, whose weights sum
    // to one: the u8 result is the border value exactly, the f32 one is
    // 0 + b before the epilogue, as on the interpolating path.
    p.blank = OP != OP_RESIZE && constant_border && persp_ok &&
              (x0max + 1 < 0 || x0min > W - 1 || y0max + 1 < 0 || y0min > H - 1);
    if (p.blank)
        p.direct = false;
    p.cx0 = max(p.bx0, 0);
    p.cx1 = min(p.bx0 + p.bw - 1, W - 1);
    p.ng = (p.direct || p.blank || p.cx0 > p.cx1) ? 0 : ((p.cx1 - p.cx0) >> 4) + 2;
    return p;
}

// Source row held by LDS slot s (inside [0, H - 1]).
template <int OP>
__device__ __forceinline__ int slot_row(const TiledJob &t, const Plan &p, int s)
{
    const ImageJob &j = t.j;
    int y;
    if constexpr (OP == OP_RESIZE) {
        y = t.rows_contig ? p.by0 + s : resize_i0_r(p.oy0 + (s >> 1), j.sh, j.dh, t.rden_y) + (s & 1);
    } else {
        y = p.by0 + s;
    }
    return clampi(y, 0, j.sh - 1);
}

// ------------------------------------------------------------------ staging
// Box rows are staged as one dword per pixel.  Work item k covers one
// 16-pixel group (aligned on the image's linear pixel index) of one slot:
// 16 C contiguous, 16-byte aligned source bytes (48 for RGB, 64 for RGBA).
template <int C> struct GroupRegs { u32x4 q[C]; };

template <int C, int MAXIT> struct Prefetch {
    GroupRegs<C> g[MAXIT];
    int dst[MAXIT];  // LDS dword index of the group's first pixel, -1 = none
    int p0[MAXIT];   // linear index of the group's first pixel
};

// Work items of a tile's staging: each slot's groups in runs of four, so that
// four consecutive lanes read 192 (RGB) or 256 (RGBA) contiguous source
// bytes, and consecutive runs of lanes take consecutive slots (with a pitch of
// 17 (mod 32) their LDS writes start on different banks).
__device__ __forceinline__ int staging_items(const Plan &p) { return p.nslots * ((p.ng + 3) & ~3); }

// Locate work item k: its slot s, group index gi within the slot's row, LDS
// destination and first pixel; false if the slot's row has no such group.
template <int OP>
__device__ __forceinline__ bool group_of(const TiledJob &t, const Plan &p, const TileGeom &G, int k, int &dst, int &p0,
                                         int &s, int &gi)
{
    const int run = udiv_small(k >> 2, p.nslots);
    s = (k >> 2) - run * p.nslots;
    gi = 4 * run + (k & 3);
    const int rowbase = t.j.sk + slot_row<OP>(t, p, s) * t.j.sp;
    const int g = ((rowbase + p.cx0) >> 4) + gi;
    if (g > ((rowbase + p.cx1) >> 4))
        return false;
    p0 = g << 4;
    dst = s * G.pitch + KT_MARGIN + (p0 - rowbase - p.bx0);
    return true;
}

template <int C>
__device__ __forceinline__ void load_group(const uint8_t *__restrict__ src, int p0, GroupRegs<C> &r)
{
    const u32x4 *q = reinterpret_cast<const u32x4 *>(src + (size_t)p0 * C);
#pragma unroll
    for (int i = 0; i < C; i++)
        r.q[i] = q[i];
}

// Widen a loaded group to 16 pixel dwords in LDS (bytes past a pixel's C
// channels are unspecified: those of the next pixels, or zero).
template <int C>
__device__ __forceinline__ void write_group(uint32_t *d, const GroupRegs<C> &r)
{
    if constexpr (C == 1) {
        const uint32_t w[4] = {r.q[0].x, r.q[0].y, r.q[0].z, r.q[0].w};
#pragma unroll
        for (int t = 0; t < 4; t++) {
            d[4 * t + 0] = w[t];
            d[4 * t + 1] = w[t] >> 8;
            d[4 * t + 2] = w[t] >> 16;
            d[4 * t + 3] = w[t] >> 24;
        }
    } else if constexpr (C == 2) {
        const uint32_t w[8] = {r.q[0].x, r.q[0].y, r.q[0].z, r.q[0].w, r.q[1].x, r.q[1].y, r.q[1].z, r.q[1].w};
#pragma unroll
        for (int t = 0; t < 8; t++) {
            d[2 * t + 0] = w[t];
            d[2 * t + 1] = w[t] >> 16;
        }
    } else if constexpr (C == 3) {
        const uint32_t w[12] = {r.q[0].x, r.q[0].y, r.q[0].z, r.q[0].w, r.q[1].x, r.q[1].y,
                                r.q[1].z, r.q[1].w, r.q[2].x, r.q[2].y, r.q[2].z, r.q[2].w};
#pragma unroll
        for (int t = 0; t < 4; t++) {
            const uint32_t u0 = w[3 * t], u1 = w[3 * t + 1], u2 = w[3 * t + 2];
            d[4 * t + 0] = u0;
            d[4 * t + 1] = __builtin_amdgcn_alignbyte(u1, u0, 3);
            d[4 * t + 2] = __builtin_amdgcn_alignbyte(u2, u1, 2);
            d[4 * t + 3] = u2 >> 8;
        }
    } else {
#pragma unroll
        for (int t = 0; t < 4; t++) {
            d[4 * t + 0] = r.q[t].x;
            d[4 * t + 1] = r.q[t].y;
            d[4 * t + 2] = r.q[t].z;
            d[4 * t + 3] = r.q[t].w;
        }
    }
}

// A group that reaches before the image's first pixel or past its last one
// (views into larger buffers; the last group of any image): its pixels
// inside [lo, hi) one by one.
template <int C>
__device__ __noinline__ void write_tail_group(uint32_t *d, const uint8_t *src, int p0, int lo, int hi)
{
#pragma unroll 1
    for (int i = p0 < lo ? lo - p0 : 0; i < 16 && p0 + i < hi; i++)
        d[i] = load_px_bytes<C>(src, (size_t)(p0 + i));
}

// Issue the loads of this thread's first MAXIT work items of a tile.  The
// staging threads are numbered lt = 0 .. NLT - 1 (the whole workgroup).
template <int OP, int C, int MAXIT, int NLT = KT_THREADS>
__device__ __forceinline__ void prefetch(const TiledJob &t, const Plan &p, const TileGeom &G, Prefetch<C, MAXIT> &pf,
                                         int lt)
{
    const uint8_t *src = static_cast<const uint8_t *>(t.j.src);
    const int lo = t.j.sk, hi = src_end(t.j);
    const int total = staging_items(p);
#pragma unroll
    for (int it = 0; it < MAXIT; it++) {
        const int k = lt + it * NLT;
        pf.dst[it] = -1;
        int dst, p0, s, gi;
        if (k < total && group_of<OP>(t, p, G, k, dst, p0, s, gi)) {
            pf.dst[it] = dst;
            pf.p0[it] = p0;
            if (p0 >= lo && p0 + 16 <= hi)
                load_group<C>(src, p0, pf.g[it]);
        }
    }
}

// Write the prefetched groups to LDS, then stage any remaining work items
// directly (boxes larger than MAXIT groups per thread), MAXIT at a time.
// prefetch() by the whole workgroup at raised wave priority: while other
// workgroups of the CU interpolate, the waves issuing a tile's staging loads
// get the instruction slots first, so the loads leave early (4K warp to f32
// 31.6 -> 30.6 us; u8 outputs unchanged).
template <int OP, int C, int MAXIT>
__device__ __forceinline__ void prefetch_urgent(const TiledJob &t, const Plan &p, const TileGeom &G,
                                                Prefetch<C, MAXIT> &pf)
{
    __builtin_amdgcn_s_setprio(2);
    prefetch<OP, C, MAXIT>(t, p, G, pf, threadIdx.x);
    __builtin_amdgcn_s_setprio(0);
}

template <int OP, int C, int MAXIT, int NLT = KT_THREADS>
__device__ __forceinline__ void commit(const TiledJob &t, const Plan &p, const TileGeom &G,
                                       Prefetch<C, MAXIT> &pf, uint32_t *lds, int lt)
{
    const uint8_t *src = static_cast<const uint8_t *>(t.j.src);
    const int lo = t.j.sk, hi = src_end(t.j);
#pragma unroll
    for (int it = 0; it < MAXIT; it++) {
        if (pf.dst[it] >= 0) {
            if (pf.p0[it] >= lo && pf.p0[it] + 16 <= hi)
                write_group<C>(lds + pf.dst[it], pf.g[it]);
            else
                write_tail_group<C>(lds + pf.dst[it], src, pf.p0[it], lo, hi);
        }
    }
    const int total = staging_items(p);
    for (int k0 = lt + MAXIT * NLT; k0 < total; k0 += MAXIT * NLT) {
#pragma unroll
        for (int it = 0; it < MAXIT; it++) {
            const int k = k0 + it * NLT;
            pf.dst[it] = -1;
            int dst, p0, s, gi;
            if (k < total && group_of<OP>(t, p, G, k, dst, p0, s, gi)) {
                pf.dst[it] = dst;
                pf.p0[it] = p0;
                if (p0 >= lo && p0 + 16 <= hi)
                    load_group<C>(src, p0, pf.g[it]);
            }
        }
#pragma unroll
        for (int it = 0; it < MAXIT; it++) {
            if (pf.dst[it] >= 0) {
                if (pf.p0[it] >= lo && pf.p0[it] + 16 <= hi)
                    write_group<C>(lds + pf.dst[it], pf.g[it]);
                else
                    write_tail_group<C>(lds + pf.dst[it], src, pf.p0[it], lo, hi);
            }
        }
    }
}

// REPLICATE on a box that crosses the left/right image edge: the out-of-image
// columns of each slot take the slot row's edge pixel (read from global memory).
__device__ __forceinline__ bool needs_edge_fill(const TiledJob &t, const Plan &p, const Epilogue &e)
{
    return !p.direct && !p.inside && e.border == KR_BORDER_REPLICATE &&
           (p.bx0 < 0 || p.bx0 + p.bw - 1 > t.j.sw - 1);
}

template <int OP, int C, int NLT = KT_THREADS>
__device__ __forceinline__ void fill_edge_columns(const TiledJob &t, const Plan &p, const TileGeom &G, uint32_t *lds,
                                                  int lt)
{
    const uint8_t *src = static_cast<const uint8_t *>(t.j.src);
    const int W = t.j.sw;
    const int nl = p.bx0 < 0 ? -p.bx0 : 0;
    const int last = p.bx0 + p.bw - 1;
    const int nr = last > W - 1 ? last - (W - 1) : 0;
    const int per = nl + nr;
    for (int k = lt; k < p.nslots * per; k += NLT) {
        const int s = udiv_small(k, per);
        const int jj = k - s * per;
        const int col = jj < nl ? jj : p.bw - nr + (jj - nl);
        const int xc = clampi(p.bx0 + col, 0, W - 1);
        lds[s * G.pitch + KT_MARGIN + col] =
            load_px_bytes<C>(src, (size_t)t.j.sk + (size_t)slot_row<OP>(t, p, s) * t.j.sp + xc);
    }
}

// Resize tables after the box: per column (x0 - bx0 + margin, weights) and per
// output row (y0, weight).  F32: weights are the fraction's bit pattern.
template <int TW, int TH, bool F32, int NLT = KT_THREADS>
__device__ __forceinline__ void resize_tables(const TiledJob &t, const Plan &p, const TileGeom &G, uint32_t *lds,
                                              int lt)
{
    const ImageJob &j = t.j;
    uint32_t *tab = lds + G.rows * G.pitch + KT_MARGIN;
    for (int i = lt; i < TW + TH; i += NLT) {
        int i0, w1;
        float f;
        if (i < TW) {
            resize_axis_r(min(p.ox0 + i, p.ox1), j.sw, j.dw, t.rden_x, i0, w1, f);
            tab[i] = (uint32_t)(i0 - p.bx0 + KT_MARGIN);
            tab[TW + i] = F32 ? __builtin_bit_cast(uint32_t, f) : ((uint32_t)(2048 - w1) | ((uint32_t)w1 << 16));
        } else {
            resize_axis_r(min(p.oy0 + (i - TW), p.oy1), j.sh, j.dh, t.rden_y, i0, w1, f);
            tab[2 * TW + (i - TW)] = (uint32_t)i0;
            tab[2 * TW + TH + (i - TW)] = F32 ? __builtin_bit_cast(uint32_t, f) : (uint32_t)w1;
        }
    }
}

// ------------------------------------------------------------------ compute
// Lane layout: TXT lanes per tile row (64 / TXT rows per wave), each owning a
// run of PX consecutive pixels; CPT runs per lane, TXT * PX apart; RPT rows
// per lane, 256 / TXT apart.  Tile = (TXT * PX * CPT) x ((256 / TXT) * RPT).
// Pixels past the tile's right edge are computed as its last column (PX = 1
// keeps every lane in the quad exchange) and not stored.
template <int PX_, int TXT_, int CPT_, int RPT_, bool NT_ = false> struct Layout {
    static_assert(PX_ == 4 || (PX_ == 1 && TXT_ == 64), "one-pixel runs need whole-wave rows");
    static constexpr int PX = PX_, TXT = TXT_, CPT = CPT_, RPT = RPT_;
    static constexpr bool NT = NT_;  // f32 output through non-temporal stores
    static constexpr int SEG = TXT * PX;             // columns between a lane's runs
    static constexpr int TW = SEG * CPT;
    static constexpr int ROWS = KT_THREADS / TXT;    // tile rows per pass
    static constexpr int TH = ROWS * RPT;
    __device__ static int col0() { return PX * (int)(threadIdx.x % TXT); }
    __device__ static int row0() { return (int)(threadIdx.x / TXT); }
};

// Output row y of a lane.  With one-pixel runs a wave covers one row, so y is
// the same in every lane; reading it from the first lane lets the compiler
// keep it, and the row's address, in scalar registers.
template <class L>
__device__ __forceinline__ int wave_row(int y)
{
    if constexpr (L::PX == 1)
        return __builtin_amdgcn_readfirstlane(y);
    else
        return y;
}

template <int C, bool F32, class L>
__device__ __forceinline__ bool layout_aligned(int dw)
{
    if constexpr (L::PX == 4)
        return store4_aligned<C, F32>(dw);
    else
        return F32 || C == 4 || (((size_t)dw * C) & 3) == 0;
}

// PERSP: perspective warp (coordinates by persp_coord, always clamped; m is
// then the unscaled inverse map and the u8 path scales the quotients).
template <int C, bool F32, class L, bool CLAMP, bool MASK, bool PERSP, bool SF = false>
__device__ __forceinline__ void compute_warp_t(const TiledJob &t, const Plan &p, const TileGeom &G, const Epilogue &e,
                                               const uint32_t *lds)
{
    constexpr int PX = L::PX, CPT = L::CPT;
    const ImageJob &j = t.j;
    const int W = j.sw, H = j.sh;
    double m[6];
#pragma unroll
    for (int i = 0; i < 6; i++)
        m[i] = (F32 || PERSP) ? j.inv[i] : t.m2048[i];
    m[2] = in_vgpr(m[2]);
    m[5] = in_vgpr(m[5]);
    const Epilogue ev = epilogue_in_vgpr<C, F32>(e);
    const int pitch = G.pitch;
    const int base = p.by0 * pitch + p.bx0 - KT_MARGIN;
    const bool aligned = layout_aligned<C, F32, L>(j.dw);
    const uint32_t sel = quad_selector(lane_id() & 3);
    const int x_end = p.ox1 + 1;
    // u8 inside tiles: the round-half-even constant 1.5 * 2^52 less 2048
    // times the box origin (an even whole number, so ties still go to the
    // even neighbour, and the sum stays in [2^52, 2^53), where the spacing
    // is 1) leaves rne(X) - 2048 (bx0 - KT_MARGIN) in the low word: its high
    // bits are the LDS column, its low 11 bits the weight (a multiple of
    // 2048 moved), with no subtraction per pixel.
    const double rx = in_vgpr(6755399441055744.0 - 2048.0 * (double)(p.bx0 - KT_MARGIN));
    const double ry = in_vgpr(6755399441055744.0 - 2048.0 * (double)p.by0);
    double xd[CPT][PX];
#pragma unroll
    for (int c = 0; c < CPT; c++)
#pragma unroll
        for (int k = 0; k < PX; k++)
            xd[c][k] = (double)min(p.ox0 + c * L::SEG + L::col0() + k, p.ox1);
    for (int r = 0; r < L::RPT; r++) {
        const int y = wave_row<L>(p.oy0 + L::row0() + r * L::ROWS);
        if (y > p.oy1)
            break;
        const double rowX = __builtin_fma(m[1], (double)y, m[2]);
        const double rowY = __builtin_fma(m[4], (double)y, m[5]);
        const double rowW = PERSP ? __builtin_fma(j.proj[1], (double)y, j.proj[2]) : 0.0;
#pragma unroll
        for (int c = 0; c < CPT; c++) {
            const int xr = p.ox0 + c * L::SEG + L::col0();
            if constexpr (!F32) {
                uint32_t P[PX];
#pragma unroll
                for (int k = 0; k < PX; k++) {
                    double X, Y;
                    if constexpr (PERSP) {
                        const double wv = __builtin_fma(j.proj[0], xd[c][k], rowW);
                        X = 2048.0 * persp_coord(__builtin_fma(m[0], xd[c][k], rowX), wv, W);
                        Y = 2048.0 * persp_coord(__builtin_fma(m[3], xd[c][k], rowY), wv, H);
                    } else {
                        X = __builtin_fma(m[0], xd[c][k], rowX);
                        Y = __builtin_fma(m[3], xd[c][k], rowY);
                        if (CLAMP) {
                            X = clamp_scaled(X, W);
                            Y = clamp_scaled(Y, H);
                        }
                    }
                    uint32_t v[C];
                    uint32_t corr = 0;
                    if constexpr (!CLAMP && !PERSP) {
                        const uint32_t Nx = (uint32_t)__builtin_bit_cast(uint64_t, X + rx);
                        const uint32_t Ny = (uint32_t)__builtin_bit_cast(uint64_t, Y + ry);
                        const uint32_t a = __umul24(Ny >> 11, (uint32_t)pitch) + (Nx >> 11);
                        const uint32_t wy1_4 = (Ny << 2) & 8188u;
                        // (2048 - w) | w << 16 = 2048 + 65535 w
                        interp_u8<C>(lds[a], lds[a + 1], lds[a + pitch], lds[a + pitch + 1],
                                     __umul24(Nx & 2047u, 65535u) + 2048u, 8192u - wy1_4, wy1_4, v);
                    } else {
                        const int Nx = rne_i32(X), Ny = rne_i32(Y);
                        const int x0 = Nx >> 11, y0 = Ny >> 11;
                        uint32_t wx1 = (uint32_t)Nx & 2047u, wy1 = (uint32_t)Ny & 2047u;
                        uint32_t wx0 = 2048u - wx1, wy0 = 2048u - wy1;
                        if (MASK)
                            corr = mask_weights(x0, y0, W, H, wx0, wx1, wy0, wy1, (uint32_t)e.bval_i);
                        const int a = __mul24(y0, pitch) + x0 - base;
                        interp_u8<C>(lds[a], lds[a + 1], lds[a + pitch], lds[a + pitch + 1], wx0 | (wx1 << 16),
                                     wy0 << 2, wy1 << 2, v);
                    }
                    if (MASK) {
#pragma unroll
                        for (int q = 0; q < C; q++)
                            v[q] += corr;
                    }
                    P[k] = pack_px<C>(v);
                }
                store_row_u8<C, PX>(j, e, y, xr, x_end, aligned, P, sel);
            } else {
                float o[PX][C];
#pragma unroll
                for (int k = 0; k < PX; k++) {
                    double X, Y;
                    if constexpr (PERSP) {
                        const double wv = __builtin_fma(j.proj[0], xd[c][k], rowW);
                        X = persp_coord(__builtin_fma(m[0], xd[c][k], rowX), wv, W);
                        Y = persp_coord(__builtin_fma(m[3], xd[c][k], rowY), wv, H);
                    } else {
                        X = __builtin_fma(m[0], xd[c][k], rowX);
                        Y = __builtin_fma(m[3], xd[c][k], rowY);
                        if (CLAMP) {
                            X = clamp_plain(X, W);
                            Y = clamp_plain(Y, H);
                        }
                    }
                    int x0, y0;
                    float fx, fy;
                    if constexpr (!CLAMP && !PERSP) {
                        // inside tiles: X, Y >= 0 at every pixel (the tile's
                        // extremes sit at its corners), so truncation is the
                        // floor and fract(X) is X - floor(X), exactly
                        x0 = (int)X;
                        y0 = (int)Y;
                        fx = (float)__builtin_amdgcn_fract(X);
                        fy = (float)__builtin_amdgcn_fract(Y);
                    } else {
                        const double fxl = __builtin_floor(X), fyl = __builtin_floor(Y);
                        x0 = (int)fxl;
                        y0 = (int)fyl;
                        fx = (float)(X - fxl);
                        fy = (float)(Y - fyl);
                    }
                    float wx0 = 1.0f - fx, wx1 = fx, wy0 = 1.0f - fy, wy1 = fy, extra = 0.0f;
                    if (MASK) {
                        wx0 = (unsigned)x0 < (unsigned)W ? wx0 : 0.0f;
                        wx1 = (unsigned)(x0 + 1) < (unsigned)W ? wx1 : 0.0f;
                        wy0 = (unsigned)y0 < (unsigned)H ? wy0 : 0.0f;
                        wy1 = (unsigned)(y0 + 1) < (unsigned)H ? wy1 : 0.0f;
                        extra = e.bval_f * (1.0f - (wy0 + wy1) * (wx0 + wx1));
                    }
                    const int a = __mul24(y0, pitch) + x0 - base;
                    interp_f32<C, MASK, SF>(lds[a], lds[a + 1], lds[a + pitch], lds[a + pitch + 1], wx0, wx1, wy0,
                                            wy1, extra, ev, o[k]);
                }
                store_row_f32<C, PX, L::NT>(j, e, y, xr, x_end, aligned, o);
            }
        }
    }
}

template <int C, bool F32, class L, bool PERSP, bool SF = false>
__device__ __forceinline__ void compute_warp(const TiledJob &t, const Plan &p, const TileGeom &G, const Epilogue &e,
                                             const uint32_t *lds)
{
    if (p.inside)
        compute_warp_t<C, F32, L, false, false, PERSP, SF>(t, p, G, e, lds);
    else if (e.border == KR_BORDER_CONSTANT)
        compute_warp_t<C, F32, L, true, true, PERSP, SF>(t, p, G, e, lds);
    else
        compute_warp_t<C, F32, L, true, false, PERSP, SF>(t, p, G, e, lds);
}

template <int C, bool F32, class L, bool MASK, bool SF = false>
__device__ __forceinline__ void compute_resize_t(const TiledJob &t, const Plan &p, const TileGeom &G, const Epilogue &e,
                                                 const uint32_t *lds)
{
    constexpr int PX = L::PX, CPT = L::CPT, TW = L::TW, TH = L::TH;
    const ImageJob &j = t.j;
    const int H = j.sh, W = j.sw;
    const uint32_t *tab = lds + G.rows * G.pitch + KT_MARGIN;
    const int pitch = G.pitch;
    const bool aligned = layout_aligned<C, F32, L>(j.dw);
    const uint32_t sel = quad_selector(lane_id() & 3);
    const int x_end = p.ox1 + 1;
    int ca[CPT][PX];
    uint32_t cw[CPT][PX];
#pragma unroll
    for (int c = 0; c < CPT; c++)
#pragma unroll
        for (int k = 0; k < PX; k++) {
            const int cc = min(c * L::SEG + L::col0() + k, p.ox1 - p.ox0);
            ca[c][k] = (int)tab[cc];
            cw[c][k] = tab[TW + cc];
        }
    const Epilogue ev = epilogue_in_vgpr<C, F32>(e);
    for (int r = 0; r < L::RPT; r++) {
        const int rr = wave_row<L>(L::row0() + r * L::ROWS);
        const int y = p.oy0 + rr;
        if (y > p.oy1)
            break;
        const int y0 = (int)tab[2 * TW + rr];
        const uint32_t rw = tab[2 * TW + TH + rr];
        const int s0 = (t.rows_contig ? y0 - p.by0 : 2 * rr) * pitch;
        const bool vy0 = (unsigned)y0 < (unsigned)H, vy1 = (unsigned)(y0 + 1) < (unsigned)H;
#pragma unroll
        for (int c = 0; c < CPT; c++) {
            const int xr = p.ox0 + c * L::SEG + L::col0();
            if constexpr (!F32) {
                uint32_t P[PX];
#pragma unroll
                for (int k = 0; k < PX; k++) {
                    const int a = s0 + ca[c][k];
                    uint32_t wy1 = rw, wy0 = 2048u - rw;
                    uint32_t wx0 = cw[c][k] & 0xFFFFu, wx1 = cw[c][k] >> 16, corr = 0;
                    if (MASK)
                        corr = mask_weights(ca[c][k] - KT_MARGIN + p.bx0, y0, W, H, wx0, wx1, wy0, wy1,
                                            (uint32_t)e.bval_i);
                    uint32_t v[C];
                    interp_u8<C>(lds[a], lds[a + 1], lds[a + pitch], lds[a + pitch + 1],
                                 MASK ? (wx0 | (wx1 << 16)) : cw[c][k], wy0 << 2, wy1 << 2, v);
                    if (MASK) {
#pragma unroll
                        for (int q = 0; q < C; q++)
                            v[q] += corr;
                    }
                    P[k] = pack_px<C>(v);
                }
                store_row_u8<C, PX>(j, e, y, xr, x_end, aligned, P, sel);
            } else {
                const float fy = __builtin_bit_cast(float, rw);
                float o[PX][C];
#pragma unroll
                for (int k = 0; k < PX; k++) {
                    const int a = s0 + ca[c][k];
                    const float fx = __builtin_bit_cast(float, cw[c][k]);
                    float wx0 = 1.0f - fx, wx1 = fx, wy0 = 1.0f - fy, wy1 = fy, extra = 0.0f;
                    if (MASK) {
                        const int x0 = ca[c][k] - KT_MARGIN + p.bx0;
                        wx0 = (unsigned)x0 < (unsigned)W ? wx0 : 0.0f;
                        wx1 = (unsigned)(x0 + 1) < (unsigned)W ? wx1 : 0.0f;
                        wy0 = vy0 ? wy0 : 0.0f;
                        wy1 = vy1 ? wy1 : 0.0f;
                        extra = e.bval_f * (1.0f - (wy0 + wy1) * (wx0 + wx1));
                    }
                    interp_f32<C, MASK, SF>(lds[a], lds[a + 1], lds[a + pitch], lds[a + pitch + 1], wx0, wx1, wy0,
                                            wy1, extra, ev, o[k]);
                }
                store_row_f32<C, PX, L::NT>(j, e, y, xr, x_end, aligned, o);
            }
        }
    }
}

template <int C, bool F32, class L, bool SF = false>
__device__ __forceinline__ void compute_resize(const TiledJob &t, const Plan &p, const TileGeom &G, const Epilogue &e,
                                               const uint32_t *lds)
{
    if (!p.inside && e.border == KR_BORDER_CONSTANT)
        compute_resize_t<C, F32, L, true, SF>(t, p, G, e, lds);
    else
        compute_resize_t<C, F32, L, false, SF>(t, p, G, e, lds);
}

// ------------------------------------------------------------------ gather path
// Tiles whose box does not fit the LDS budget (and resizes with large
// down-sampling ratios, where neighbouring outputs share no taps) read their
// taps straight from global memory: per tap row, the two horizontal taps are
// 2 * C contiguous bytes, loaded as one dword-aligned 12-byte (RGB) or 8-byte
// (RGBA) read and realigned with byte-align ops (one and two channels: byte
// by byte).  Taps outside the image take the border rule per tap.

// The two horizontal taps at (x0, y) and (x0 + 1, y), both inside the image,
// as pixel dwords (byte c = channel c; RGB byte 3 unspecified).
template <int C>
__device__ __forceinline__ void load_tap_pair(const uint8_t *__restrict__ src, size_t nbytes, size_t lin, uint32_t &t0,
                                              uint32_t &t1)
{
    if constexpr (C == 4) {
        struct __attribute__((packed, aligned(4))) D2 { uint32_t a, b; };
        const D2 d = *reinterpret_cast<const D2 *>(src + lin * 4);
        t0 = d.a;
        t1 = d.b;
    } else if constexpr (C < 3) {
        (void)nbytes;
        t0 = load_px_bytes<C>(src, lin);
        t1 = load_px_bytes<C>(src, lin + 1);
    } else {
        const size_t b = lin * 3;
        const size_t f = b & ~(size_t)3;
        if (f + 12 <= nbytes) {
            struct __attribute__((packed, aligned(4))) D3 { uint32_t a, b, c; };
            const D3 d = *reinterpret_cast<const D3 *>(src + f);
            const uint32_t sh = (uint32_t)(b & 3);
            const uint32_t lo = __builtin_amdgcn_alignbyte(d.b, d.a, sh);
            const uint32_t hi = __builtin_amdgcn_alignbyte(d.c, d.b, sh);
            t0 = lo;
            t1 = __builtin_amdgcn_alignbyte(hi, lo, 3);
        } else {
            t0 = load_px_bytes<3>(src, lin);
            t1 = load_px_bytes<3>(src, lin + 1);
        }
    }
}

// The four taps of a pixel with top-left tap (x0, y0).  Returns false when a
// tap lies outside the image; the taps then hold the clamped (edge) pixels,
// which is the REPLICATE rule, and a CONSTANT border masks their weights.
template <int C>
__device__ __forceinline__ bool load_taps(const ImageJob &j, int x0, int y0, uint32_t &t00, uint32_t &t01,
                                          uint32_t &t10, uint32_t &t11)
{
    const uint8_t *src = static_cast<const uint8_t *>(j.src);
    const int W = j.sw, H = j.sh;
    const size_t sp = (size_t)j.sp, sk = (size_t)j.sk;
    const size_t nbytes = (size_t)src_end(j) * C;
    if ((unsigned)x0 < (unsigned)(W - 1) && (unsigned)y0 < (unsigned)(H - 1)) {
        const size_t lin = sk + (size_t)y0 * sp + x0;
        load_tap_pair<C>(src, nbytes, lin, t00, t01);
        load_tap_pair<C>(src, nbytes, lin + sp, t10, t11);
        return true;
    }
    const int xa = clampi(x0, 0, W - 1), xb = clampi(x0 + 1, 0, W - 1);
    const int ya = clampi(y0, 0, H - 1), yb = clampi(y0 + 1, 0, H - 1);
    t00 = load_px_bytes<C>(src, sk + (size_t)ya * sp + xa);
    t01 = load_px_bytes<C>(src, sk + (size_t)ya * sp + xb);
    t10 = load_px_bytes<C>(src, sk + (size_t)yb * sp + xa);
    t11 = load_px_bytes<C>(src, sk + (size_t)yb * sp + xb);
    return false;
}

// u8 result of one pixel from global taps.
template <int C>
__device__ __forceinline__ uint32_t gather_px_u8(const ImageJob &j, const Epilogue &e, int x0, int y0, uint32_t wx1,
                                                 uint32_t wy1)
{
    uint32_t t00, t01, t10, t11;
    const bool in = load_taps<C>(j, x0, y0, t00, t01, t10, t11);
    uint32_t wx0 = 2048u - wx1, wy0 = 2048u - wy1, corr = 0;
    if (!in && e.border == KR_BORDER_CONSTANT)
        corr = mask_weights(x0, y0, j.sw, j.sh, wx0, wx1, wy0, wy1, (uint32_t)e.bval_i);
    uint32_t v[C];
    interp_u8<C>(t00, t01, t10, t11, wx0 | (wx1 << 16), wy0 << 2, wy1 << 2, v);
#pragma unroll
    for (int q = 0; q < C; q++)
        v[q] += corr;
    return pack_px<C>(v);
}

// SF: one-channel f32 source (taps read as 4-byte pixels).
template <int C, bool SF = false>
__device__ __forceinline__ void gather_px_f32(const ImageJob &j, const Epilogue &e, int x0, int y0, float fx, float fy,
                                              float (&o)[C])
{
    uint32_t t00, t01, t10, t11;
    const bool in = load_taps<SF ? 4 : C>(j, x0, y0, t00, t01, t10, t11);
    float wx0 = 1.0f - fx, wx1 = fx, wy0 = 1.0f - fy, wy1 = fy, extra = 0.0f;
    if (!in && e.border == KR_BORDER_CONSTANT) {
        const int W = j.sw, H = j.sh;
        wx0 = (unsigned)x0 < (unsigned)W ? wx0 : 0.0f;
        wx1 = (unsigned)(x0 + 1) < (unsigned)W ? wx1 : 0.0f;
        wy0 = (unsigned)y0 < (unsigned)H ? wy0 : 0.0f;
        wy1 = (unsigned)(y0 + 1) < (unsigned)H ? wy1 : 0.0f;
        extra = e.bval_f * (1.0f - (wy0 + wy1) * (wx0 + wx1));
    }
    interp_f32<C, true, SF>(t00, t01, t10, t11, wx0, wx1, wy0, wy1, extra, e, o);
}

template <int OP, int C, bool F32, class L, bool SF = false>
__device__ __forceinline__ void compute_gather(const TiledJob &t, const Plan &p, const TileGeom &G, const Epilogue &e,
                                               const uint32_t *lds)
{
    constexpr int PX = L::PX, CPT = L::CPT, TW = L::TW, TH = L::TH;
    const ImageJob &j = t.j;
    const bool aligned = layout_aligned<C, F32, L>(j.dw);
    const uint32_t sel = quad_selector(lane_id() & 3);
    const int x_end = p.ox1 + 1;
    const uint32_t *tab = lds + G.rows * G.pitch + KT_MARGIN;
    double m[6];
#pragma unroll
    for (int i = 0; i < 6; i++)
        m[i] = (F32 || OP == OP_PERSP) ? j.inv[i] : t.m2048[i];
    for (int r = 0; r < L::RPT; r++) {
        const int rr = wave_row<L>(L::row0() + r * L::ROWS);
        const int y = p.oy0 + rr;
        if (y > p.oy1)
            break;
        double rowX = 0, rowY = 0, rowW = 0;
        int ry0 = 0;
        uint32_t rw = 0;
        if constexpr (OP != OP_RESIZE) {
            rowX = __builtin_fma(m[1], (double)y, m[2]);
            rowY = __builtin_fma(m[4], (double)y, m[5]);
            if constexpr (OP == OP_PERSP)
                rowW = __builtin_fma(j.proj[1], (double)y, j.proj[2]);
        } else {
            ry0 = (int)tab[2 * TW + rr];
            rw = tab[2 * TW + TH + rr];
        }
#pragma unroll
        for (int c = 0; c < CPT; c++) {
            const int xr = p.ox0 + c * L::SEG + L::col0();
            uint32_t P[PX];
            float o[PX][C];
#pragma unroll
            for (int k = 0; k < PX; k++) {
                const int cc = min(c * L::SEG + L::col0() + k, p.ox1 - p.ox0);
                int x0, y0;
                uint32_t wx1, wy1;
                float fx, fy;
                if constexpr (OP == OP_PERSP) {
                    const double xd = (double)(p.ox0 + cc);
                    const double wv = __builtin_fma(j.proj[0], xd, rowW);
                    const double X = persp_coord(__builtin_fma(m[0], xd, rowX), wv, j.sw);
                    const double Y = persp_coord(__builtin_fma(m[3], xd, rowY), wv, j.sh);
                    if constexpr (!F32) {
                        const int Nx = rne_i32(2048.0 * X), Ny = rne_i32(2048.0 * Y);
                        x0 = Nx >> 11; y0 = Ny >> 11;
                        wx1 = (uint32_t)Nx & 2047u; wy1 = (uint32_t)Ny & 2047u;
                        fx = fy = 0.0f;
                    } else {
                        const double fxl = __builtin_floor(X), fyl = __builtin_floor(Y);
                        x0 = (int)fxl; y0 = (int)fyl;
                        fx = (float)(X - fxl); fy = (float)(Y - fyl);
                        wx1 = wy1 = 0;
                    }
                } else if constexpr (OP == OP_WARP) {
                    const double xd = (double)(p.ox0 + cc);
                    double X = __builtin_fma(m[0], xd, rowX);
                    double Y = __builtin_fma(m[3], xd, rowY);
                    if constexpr (!F32) {
                        const int Nx = rne_i32(clamp_scaled(X, j.sw)), Ny = rne_i32(clamp_scaled(Y, j.sh));
                        x0 = Nx >> 11; y0 = Ny >> 11;
                        wx1 = (uint32_t)Nx & 2047u; wy1 = (uint32_t)Ny & 2047u;
                        fx = fy = 0.0f;
                    } else {
                        X = clamp_plain(X, j.sw);
                        Y = clamp_plain(Y, j.sh);
                        const double fxl = __builtin_floor(X), fyl = __builtin_floor(Y);
                        x0 = (int)fxl; y0 = (int)fyl;
                        fx = (float)(X - fxl); fy = (float)(Y - fyl);
                        wx1 = wy1 = 0;
                    }
                } else {
                    x0 = (int)tab[cc] - KT_MARGIN + p.bx0;
                    y0 = ry0;
                    const uint32_t cw = tab[TW + cc];
                    wx1 = cw >> 16; wy1 = rw;
                    fx = __builtin_bit_cast(float, cw);
                    fy = __builtin_bit_cast(float, rw);
                }
                if constexpr (!F32)
                    P[k] = gather_px_u8<C>(j, e, x0, y0, wx1, wy1);
                else
                    gather_px_f32<C, SF>(j, e, x0, y0, fx, fy, o[k]);
            }
            if constexpr (!F32)
                store_row_u8<C, PX>(j, e, y, xr, x_end, aligned, P, sel);
            else
                store_row_f32<C, PX, L::NT>(j, e, y, xr, x_end, aligned, o);
        }
    }
}

// A blank tile (see Plan::blank): every output pixel is the border value,
// u8: b in each channel; f32: fma(0 + b, alpha_c, beta_c), the bits the
// interpolating path produces when every weight is masked.
template <int C, bool F32, class L>
__device__ __forceinline__ void fill_blank(const TiledJob &t, const Plan &p, const Epilogue &e)
{
    constexpr int PX = L::PX, CPT = L::CPT;
    const ImageJob &j = t.j;
    const bool aligned = layout_aligned<C, F32, L>(j.dw);
    const uint32_t sel = quad_selector(lane_id() & 3);
    const int x_end = p.ox1 + 1;
    uint32_t P[PX];
    float o[PX][C];
    const uint32_t b = (uint32_t)e.bval_i;
    const uint32_t pix = C == 1 ? b : (C == 2 ? b * 0x101u : (C == 3 ? b * 0x10101u : b * 0x1010101u));
#pragma unroll
    for (int k = 0; k < PX; k++) {
        P[k] = pix;
#pragma unroll
        for (int c = 0; c < C; c++)
            o[k][c] = __builtin_fmaf(0.0f + e.bval_f, e.alpha[c], e.beta[c]);
    }
    for (int r = 0; r < L::RPT; r++) {
        const int y = wave_row<L>(p.oy0 + L::row0() + r * L::ROWS);
        if (y > p.oy1)
            break;
#pragma unroll
        for (int c = 0; c < CPT; c++) {
            const int xr = p.ox0 + c * L::SEG + L::col0();
            if constexpr (!F32)
                store_row_u8<C, PX>(j, e, y, xr, x_end, aligned, P, sel);
            else
                store_row_f32<C, PX, L::NT>(j, e, y, xr, x_end, aligned, o);
        }
    }
}

// ------------------------------------------------------------------ tile pipeline
// Stage -> (edge fill) -> issue the next tile's loads -> compute this tile.
// The next tile's global loads stay in flight in registers while this tile is
// interpolated from LDS.  PIPE = false: the workgroup owns exactly one tile
// (no registers stay reserved for a next tile during the interpolation).
// SF: a one-channel f32 source (C = 1, f32 output): its 4-byte pixels are
// staged as the 4-byte pixels of RGBA u8 are, one LDS word per pixel.
template <int OP, int C, bool F32, class L, int MAXIT, bool PIPE, bool SF = false, typename NextJob>
__device__ __forceinline__ void run_tiles(const TileGeom &G, const Epilogue &e, uint32_t *lds, NextJob next_job)
{
    static_assert(!SF || (C == 1 && F32), "f32 sources: one channel, f32 output");
    constexpr int SB = SF ? 4 : C;  // source bytes per pixel
    constexpr int TW = L::TW;
    constexpr int TH = L::TH;
    TiledJob t;
    int tile;
    if (!next_job(t, tile))
        return;
    const bool cb = e.border == KR_BORDER_CONSTANT;
    Plan p = make_plan<OP, TW, TH, F32>(t, tile, G, cb);
    if constexpr (!PIPE) {
        if (!p.direct) {
            Prefetch<SB, MAXIT> pf;
            prefetch_urgent<OP, SB, MAXIT>(t, p, G, pf);
            commit<OP, SB, MAXIT>(t, p, G, pf, lds, threadIdx.x);
        }
        if constexpr (OP == OP_RESIZE)
            resize_tables<TW, TH, F32>(t, p, G, lds, threadIdx.x);
        __syncthreads();
        if (needs_edge_fill(t, p, e)) {
            fill_edge_columns<OP, SB>(t, p, G, lds, threadIdx.x);
            __syncthreads();
        }
        if (p.blank)
            fill_blank<C, F32, L>(t, p, e);
        else if (p.direct)
            compute_gather<OP, C, F32, L, SF>(t, p, G, e, lds);
        else if constexpr (OP == OP_RESIZE)
            compute_resize<C, F32, L, SF>(t, p, G, e, lds);
        else
            compute_warp<C, F32, L, OP == OP_PERSP, SF>(t, p, G, e, lds);
        return;
    }
    Prefetch<SB, MAXIT> pf;
    prefetch_urgent<OP, SB, MAXIT>(t, p, G, pf);
    while (true) {
        if (!p.direct)
            commit<OP, SB, MAXIT>(t, p, G, pf, lds, threadIdx.x);
        if constexpr (OP == OP_RESIZE)
            resize_tables<TW, TH, F32>(t, p, G, lds, threadIdx.x);
        __syncthreads();
        if (needs_edge_fill(t, p, e)) {
            fill_edge_columns<OP, SB>(t, p, G, lds, threadIdx.x);
            __syncthreads();
        }
        TiledJob nt;
        int ntile;
        const bool more = next_job(nt, ntile);
        Plan np;
        if (more) {
            np = make_plan<OP, TW, TH, F32>(nt, ntile, G, cb);
            prefetch_urgent<OP, SB, MAXIT>(nt, np, G, pf);
        }
        if (p.blank)
            fill_blank<C, F32, L>(t, p, e);
        else if (p.direct)
            compute_gather<OP, C, F32, L, SF>(t, p, G, e, lds);
        else if constexpr (OP == OP_RESIZE)
            compute_resize<C, F32, L, SF>(t, p, G, e, lds);
        else
            compute_warp<C, F32, L, OP == OP_PERSP, SF>(t, p, G, e, lds);
        if (!more)
            break;
        __syncthreads();
        t = nt;
        p = np;
    }
}

// Static schedule of a persistent grid over n tiles, XCD-aware: blocks are
// dealt to the 8 XCDs round-robin, so XCD k (blocks b = k mod 8) owns the k-th
// contiguous eighth of the tiles and its blocks interleave over it, keeping
// neighbouring tiles (which share source rows) in one L2.  With one tile per
// block it is the bijection xcd_tile(); otherwise the grid is a multiple of 8.
struct TileSeq {
    int next, step, end;
    __device__ __forceinline__ TileSeq(int b, int grid, int n)
    {
        if (grid >= n) {
            next = xcd_tile(b, n);
            step = n;
            end = n;
        } else {
            const int k = b & 7, q = n >> 3, r = n & 7;
            const int start = k * q + (k < r ? k : r);
            next = start + (b >> 3);
            step = grid >> 3;
            end = start + q + (k < r ? 1 : 0);
        }
    }
    // Tile ranges given per XCD: XCD k (blocks b = k mod 8) owns tiles
    // [start[k], start[k + 1]) and its blocks interleave over them.  grid is
    // a multiple of 8; with grid / 8 >= the largest range each block takes at
    // most one tile.
    __device__ __forceinline__ TileSeq(int b, int grid, const int (&start)[9])
    {
        const int k = b & 7;
        next = start[k] + (b >> 3);
        step = grid >> 3;
        end = start[k + 1];
    }
    __device__ __forceinline__ bool take(int &tile)
    {
        if (next >= end)
            return false;
        tile = next;
        next += step;
        return true;
    }
};

// Per-XCD tile ranges of a batch launch (TileSeq above).
struct TileBins {
    int start[9];
};

}  // namespace kr
