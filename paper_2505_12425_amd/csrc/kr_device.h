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
// index d is ((2 d + 1) n_in - n_out) / (2 n_out).  i0 = floor, w1 = 11-bit
// weight of the upper tap, f = fraction as f32.  Sizes <= 32767 keep every
// product within int32.
__device__ __forceinline__ void resize_axis(int d, int n_in, int n_out, int &i0, int &w1, float &f)
{
    const int num = (2 * d + 1) * n_in - n_out;
    const int den = 2 * n_out;
    const int q = floor_div(num, den);
    const int r = num - q * den;
    i0 = q;
    w1 = weight_from_ratio(r, den);
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

// One tap of C channels as integers (u8 source) with the border rule.
template <int C, typename S>
__device__ __forceinline__ void tap_int(const S *src, int h, int w, int x, int y, const Epilogue &e, int (&p)[C])
{
    if ((unsigned)x >= (unsigned)w || (unsigned)y >= (unsigned)h) {
        if (e.border == KR_BORDER_CONSTANT) {
#pragma unroll
            for (int c = 0; c < C; c++)
                p[c] = e.bval_i;
            return;
        }
        x = x < 0 ? 0 : (x >= w ? w - 1 : x);
        y = y < 0 ? 0 : (y >= h ? h - 1 : y);
    }
    const S *q = src + ((size_t)y * (size_t)w + (size_t)x) * C;
#pragma unroll
    for (int c = 0; c < C; c++)
        p[c] = (int)q[c];
}

// One tap of C channels as floats with the border rule.
template <int C, typename S>
__device__ __forceinline__ void tap_float(const S *src, int h, int w, int x, int y, const Epilogue &e, float (&p)[C])
{
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
    const S *q = src + ((size_t)y * (size_t)w + (size_t)x) * C;
#pragma unroll
    for (int c = 0; c < C; c++)
        p[c] = (float)q[c];
}

}  // namespace kr
