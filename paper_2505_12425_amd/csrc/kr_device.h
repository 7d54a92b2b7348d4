// kr_device.h -- device helpers shared by libkr's kernels: coordinate maps,
// weights and border-aware taps.
#pragma once

#include "kr_internal.h"

namespace kr {

typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));
typedef unsigned int u32x3 __attribute__((ext_vector_type(3)));
typedef unsigned int u32x2 __attribute__((ext_vector_type(2)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

template <typename T> struct is_u8 { static constexpr bool value = false; };
template <> struct is_u8<uint8_t> { static constexpr bool value = true; };

// floor(a / b) for b > 0.
__device__ __forceinline__ int floor_div(int a, int b)
{
    int q = a / b;
    if (q * b != a && a < 0)
        q -= 1;
    return q;
}

// round-half-even(2048 r / den) for 0 <= r < den <= 65534, in integers:
// (4096 r + den) / (2 den) rounds half up; an exact quotient is a tie and
// moves to the even neighbour.
__device__ __forceinline__ int weight_from_ratio(int r, int den)
{
    const int t = 4096 * r + den;
    const int d2 = 2 * den;
    int q = t / d2;
    if (q * d2 == t && (q & 1))
        q -= 1;
    return q;
}

// Resize axis map with half-pixel centres: the source coordinate of output
// index d is ((2 d + 1) n_in - n_out) / (2 n_out), an exact rational.  i0 =
// its floor, w1 = round-half-even(2048 * fraction), f = fraction as f32.
//
// Evaluated with correctly rounded binary64 divisions, which give the exact
// integer results here.  When num / den is not an integer it lies at least
// 1/den > 2^-16 below the next one, while |num / den| < 2^30 keeps the
// rounding error under 2^-23: the floor is exact.  2048 r / den (< 2048) is
// rounded once from exact integers: an exact half stays exact, and any other
// value lies at least 1/(2 den) > 2^-17 from a half, far beyond the rounding
// error, so rint (ties to even) rounds as the exact rational would.  Sizes
// <= 32767 keep every product within int32.
__device__ __forceinline__ int resize_i0(int d, int n_in, int n_out)
{
    const int num = (2 * d + 1) * n_in - n_out;
    return (int)__builtin_floor((double)num / (double)(2 * n_out));
}

__device__ __forceinline__ void resize_axis(int d, int n_in, int n_out, int &i0, int &w1, float &f)
{
    const int num = (2 * d + 1) * n_in - n_out;
    const int den = 2 * n_out;
    const int q = (int)__builtin_floor((double)num / (double)den);
    const int r = num - q * den;
    i0 = q;
    w1 = (int)__builtin_rint((double)(2048 * r) / (double)den);
    f = (float)r / (float)den;
}

// Warp axis: clamp the binary64 source coordinate to [-2, n + 1], split into
// floor and fraction (exact), 11-bit weight by round-half-even.
__device__ __forceinline__ void warp_axis(double s, int n, int &i0, int &w1, float &f)
{
    s = __builtin_fmin(__builtin_fmax(s, -2.0), (double)n + 1.0);
    const double fl = __builtin_floor(s);
    const double fr = s - fl;
    i0 = (int)fl;
    w1 = (int)__builtin_rint(2048.0 * fr);
    f = (float)fr;
}

// f32 bilinear blend of four taps: the 2-D weights w_ij = wy_i * wx_j (one
// rounded product each, shared by the channels of a pixel), then
// v = w00 p00 + w01 p01 + w10 p10 + w11 p11 as one fixed chain of explicit
// fma, so that every kernel computes identical bits.  The caller adds the
// border's share under a CONSTANT border (adding +-0 to the non-negative sum
// of u8 taps changes nothing, so paths with and without that add agree) and
// applies the epilogue out = v * alpha + beta.
struct Weights2 {
    float w00, w01, w10, w11;
};

__device__ __forceinline__ Weights2 weights2(float wx0, float wx1, float wy0, float wy1)
{
    return Weights2{wy0 * wx0, wy0 * wx1, wy1 * wx0, wy1 * wx1};
}

__device__ __forceinline__ float blend4(float p00, float p01, float p10, float p11, const Weights2 &w)
{
    return __builtin_fmaf(w.w11, p11, __builtin_fmaf(w.w10, p10, __builtin_fmaf(w.w01, p01, w.w00 * p00)));
}

// One tap of C channels as floats with the border rule.
template <int C, typename S>
__device__ __forceinline__ void tap_float(const S *src, const ImageJob &j, int x, int y, const Epilogue &e, float (&p)[C])
{
    const int h = j.sh, w = j.sw;
    if ((unsigned)x >= (unsigned)w || (unsigned)y >= (unsigned)h) {
        if (e.border == KR_BORDER_CONSTANT) {
#pragma unroll
            for (int c = 0; c < C; c++)
                p[c] = e.bval_f;
            return;
        }
        x = x < 0 ? 0 : (x >= w ? w - 1 : x);
        y = y < 0 ? 0 : (y >= h ? h - 1 : y);
    }
    const S *q = src + ((size_t)j.sk + (size_t)y * (size_t)j.sp + (size_t)x) * C;
#pragma unroll
    for (int c = 0; c < C; c++)
        p[c] = (float)q[c];
}

// One output pixel (x, y) of an f32 source evaluated straight from the
// definition: every tap read from global memory with its own border test.
template <int C, typename S, typename D, int OP>
__device__ __forceinline__ void generic_pixel(const ImageJob &j, const Epilogue &e, int x, int y)
{
    int x0, y0, wx1, wy1;
    float fx, fy;
    if (OP == OP_RESIZE) {
        resize_axis(x, j.sw, j.dw, x0, wx1, fx);
        resize_axis(y, j.sh, j.dh, y0, wy1, fy);
    } else if (OP == OP_PERSP) {
        // binary64 quotients; warp_axis maps a quotient that is not a number
        // to -2 (fmax ignores it) and clamps infinities
        const double w = __builtin_fma(j.proj[0], (double)x, __builtin_fma(j.proj[1], (double)y, j.proj[2]));
        const double xs = __builtin_fma(j.inv[0], (double)x, __builtin_fma(j.inv[1], (double)y, j.inv[2])) / w;
        const double ys = __builtin_fma(j.inv[3], (double)x, __builtin_fma(j.inv[4], (double)y, j.inv[5])) / w;
        warp_axis(xs, j.sw, x0, wx1, fx);
        warp_axis(ys, j.sh, y0, wy1, fy);
    } else {
        const double xs = __builtin_fma(j.inv[0], (double)x, __builtin_fma(j.inv[1], (double)y, j.inv[2]));
        const double ys = __builtin_fma(j.inv[3], (double)x, __builtin_fma(j.inv[4], (double)y, j.inv[5]));
        warp_axis(xs, j.sw, x0, wx1, fx);
        warp_axis(ys, j.sh, y0, wy1, fy);
    }
    const S *src = static_cast<const S *>(j.src);
    D *dst = static_cast<D *>(j.dst) + ((size_t)y * (size_t)j.dw + (size_t)x) * C;
    static_assert(!is_u8<D>::value, "u8 outputs come from u8 sources, which the tiled kernels take");
    const Weights2 w = weights2(1.0f - fx, fx, 1.0f - fy, fy);
    float p00[C], p01[C], p10[C], p11[C];
    tap_float<C>(src, j, x0, y0, e, p00);
    tap_float<C>(src, j, x0 + 1, y0, e, p01);
    tap_float<C>(src, j, x0, y0 + 1, e, p10);
    tap_float<C>(src, j, x0 + 1, y0 + 1, e, p11);
#pragma unroll
    for (int c = 0; c < C; c++)
        dst[c] = __builtin_fmaf(blend4(p00[c], p01[c], p10[c], p11[c], w), e.alpha[c], e.beta[c]);
}

}  // namespace kr
