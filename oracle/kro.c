/*
 * kro.c -- reference oracle for bilinear / nearest resize and affine warp (TEST
 * INFRASTRUCTURE ONLY).
 *
 * This file is the plain, slow, obviously-correct CPU definition that the HIP
 * kernels are checked against.  Only the test suite, the smoke check and the
 * CPU-baseline leg of the benchmark may load it; the product library never
 * links or calls it, and it shares no code with the product.
 *
 * What it computes.  The paper (Sec. II-A, kornia-imgproc "geometric
 * transforms"; Sec. III, the benchmarked up- and down-sizing operators;
 * Sec. II-B.2, the interleaved Image<T, C> layout; Sec. II-B.4, caller-owned
 * output buffers) names the operators but prints no formula.  The definitions
 * below are the readings this project fixes for it:
 *
 *  - Images are HWC-contiguous, C interleaved channels, u8 or f32 samples.
 *  - Resize uses half-pixel centres: source x = (dx + 1/2) * W_in / W_out - 1/2,
 *    held as the exact rational num / den with num = (2 dx + 1) W_in - W_out,
 *    den = 2 W_out, so floor and fraction are exact integers.
 *  - Warp: the 2x3 matrix maps source to destination unless the caller says it
 *    is already the inverse.  Pixel j's centre is at coordinate j.  The inverse
 *    map is evaluated per destination pixel as xs = fma(A, x, fma(B, y, C)),
 *    ys = fma(D, x, fma(E, y, F)) in IEEE binary64 with correctly rounded fma,
 *    and clamped to [-2, W+1] x [-2, H+1] (beyond that every tap is a border
 *    tap either way).
 *  - Borders are handled per tap: a tap outside the image is the constant b
 *    (CONSTANT) or the nearest edge pixel (REPLICATE).  Weights always come
 *    from the unclamped coordinate.
 *  - u8 output: 11-bit per-axis weights w1 = round-half-even(2048 * frac),
 *    w0 = 2048 - w1; acc = sum wy_i * wx_j * p_ij exactly in integers;
 *    out = floor((acc + 2^21) / 2^22).
 *  - f32 output: the same taps with unquantised binary64 weights (1 - f, f),
 *    on the 0..255 scale; optionally normalised per channel as
 *    (v / 255 - mean_c) / std_c.  The oracle reports these values in binary64.
 *
 * Nearest-neighbour resize (kro_resize_nearest) takes the sample at
 * floor((d + 1/2) * n_in / n_out) per axis, an exact integer quotient.
 * Flip (kro_flip) mirrors the pixel order; RGB to gray (kro_rgb_to_gray)
 * uses BT.601 luma weights (14-bit fixed point for u8 output).  The
 * perspective warp (kro_warp_perspective) divides the homography's first two
 * rows by its third, in binary64, then proceeds as the affine warp.
 *
 * Parity status: every function here is pinned by the tests in
 * tests/test_oracle.py (closed forms, exact permutations, an exact-rational
 * brute force and library cross-checks); none is "parity unpinned".
 *
 * Build: gcc -O2 -std=c11 -ffp-contract=off -fopenmp -fPIC -shared kro.c -lm
 * (-ffp-contract=off so that no product/sum pair is silently fused.)
 */
#include <math.h>
#include <stdint.h>
#include <stddef.h>

enum { KRO_U8 = 0, KRO_F32 = 1 };        /* source sample types */
enum { KRO_OUT_U8 = 0, KRO_OUT_F64 = 1 }; /* oracle output types */
enum { KRO_CONSTANT = 0, KRO_REPLICATE = 1 };

/* floor(a / b) for b > 0 and any sign of a. */
static int64_t floor_div(int64_t a, int64_t b)
{
    int64_t q = a / b;
    if ((a % b) != 0 && a < 0)
        q -= 1;
    return q;
}

/* round-half-even(2048 * r / den) for 0 <= r < den, in exact integers.
 * 2048 r / den + 1/2 = (4096 r + den) / (2 den); its floor rounds half up,
 * and a tie (exact division) is moved down to the even neighbour. */
static int64_t weight_from_ratio(int64_t r, int64_t den)
{
    int64_t t = 4096 * r + den;
    int64_t q = t / (2 * den);
    if (t % (2 * den) == 0 && (q & 1))
        q -= 1;
    return q;
}

/* One source sample at integer position (x, y), channel ch, with the border
 * rule applied to this tap alone. */
static double tap(const void *src, int src_t, int h, int w, int c,
                  int64_t x, int64_t y, int ch, int border, double bval)
{
    if (x < 0 || x >= w || y < 0 || y >= h) {
        if (border == KRO_CONSTANT)
            return bval;
        if (x < 0) x = 0;
        if (x >= w) x = w - 1;
        if (y < 0) y = 0;
        if (y >= h) y = h - 1;
    }
    size_t idx = ((size_t)y * (size_t)w + (size_t)x) * (size_t)c + (size_t)ch;
    if (src_t == KRO_U8)
        return (double)((const uint8_t *)src)[idx];
    return (double)((const float *)src)[idx];
}

/* Integer tap for the u8 path (CONSTANT b is an integer in [0, 255]). */
static int64_t tap_u8(const uint8_t *src, int h, int w, int c,
                      int64_t x, int64_t y, int ch, int border, int64_t bval)
{
    if (x < 0 || x >= w || y < 0 || y >= h) {
        if (border == KRO_CONSTANT)
            return bval;
        if (x < 0) x = 0;
        if (x >= w) x = w - 1;
        if (y < 0) y = 0;
        if (y >= h) y = h - 1;
    }
    return src[((size_t)y * (size_t)w + (size_t)x) * (size_t)c + (size_t)ch];
}

/* Writes one output pixel, given the top-left tap (x0, y0) and the per-axis
 * weights: integer 11-bit weights for u8 output, binary64 fractions fx, fy
 * for f64 output. */
static void write_pixel(const void *src, int src_t, int sh, int sw, int c,
                        void *dst, int out_t, size_t didx,
                        int64_t x0, int64_t y0, int64_t wx1, int64_t wy1,
                        double fx, double fy, int border, double bval,
                        const double *mean, const double *stdv)
{
    for (int ch = 0; ch < c; ch++) {
        if (out_t == KRO_OUT_U8) {
            const uint8_t *s = (const uint8_t *)src;
            int64_t b = (int64_t)bval;
            int64_t wx0 = 2048 - wx1, wy0 = 2048 - wy1;
            int64_t acc = wy0 * wx0 * tap_u8(s, sh, sw, c, x0, y0, ch, border, b)
                        + wy0 * wx1 * tap_u8(s, sh, sw, c, x0 + 1, y0, ch, border, b)
                        + wy1 * wx0 * tap_u8(s, sh, sw, c, x0, y0 + 1, ch, border, b)
                        + wy1 * wx1 * tap_u8(s, sh, sw, c, x0 + 1, y0 + 1, ch, border, b);
            ((uint8_t *)dst)[didx + (size_t)ch] = (uint8_t)((acc + (1 << 21)) >> 22);
        } else {
            double v = (1.0 - fy) * (1.0 - fx) * tap(src, src_t, sh, sw, c, x0, y0, ch, border, bval)
                     + (1.0 - fy) * fx * tap(src, src_t, sh, sw, c, x0 + 1, y0, ch, border, bval)
                     + fy * (1.0 - fx) * tap(src, src_t, sh, sw, c, x0, y0 + 1, ch, border, bval)
                     + fy * fx * tap(src, src_t, sh, sw, c, x0 + 1, y0 + 1, ch, border, bval);
            if (mean && stdv)
                v = (v / 255.0 - mean[ch]) / stdv[ch];
            ((double *)dst)[didx + (size_t)ch] = v;
        }
    }
}

/* Bilinear resize with half-pixel centres.  Returns 0, or -1 on bad sizes. */
int kro_resize(const void *src, int sh, int sw, int c, int src_t,
               void *dst, int dh, int dw, int out_t,
               int border, double bval, const double *mean, const double *stdv,
               int nthreads)
{
    if (sh < 1 || sw < 1 || dh < 1 || dw < 1 || c < 1 || c > 4)
        return -1;
    if (nthreads < 1)
        nthreads = 1;
#pragma omp parallel for num_threads(nthreads) schedule(static)
    for (int dy = 0; dy < dh; dy++) {
        int64_t ny = (int64_t)(2 * dy + 1) * sh - dh, deny = 2 * (int64_t)dh;
        int64_t y0 = floor_div(ny, deny), ry = ny - y0 * deny;
        for (int dx = 0; dx < dw; dx++) {
            int64_t nx = (int64_t)(2 * dx + 1) * sw - dw, denx = 2 * (int64_t)dw;
            int64_t x0 = floor_div(nx, denx), rx = nx - x0 * denx;
            write_pixel(src, src_t, sh, sw, c, dst, out_t,
                        ((size_t)dy * (size_t)dw + (size_t)dx) * (size_t)c,
                        x0, y0, weight_from_ratio(rx, denx), weight_from_ratio(ry, deny),
                        (double)rx / (double)denx, (double)ry / (double)deny,
                        border, bval, mean, stdv);
        }
    }
    return 0;
}

/* Nearest-neighbour resize with half-pixel centres (the paper's other
 * benchmarked resize, Sec. III): output pixel dx takes source column
 * floor((dx + 1/2) * W_in / W_out) = floor((2 dx + 1) W_in / (2 W_out)), an
 * exact integer quotient of non-negative integers that never exceeds
 * W_in - 1; rows likewise.  u8 output (u8 sources only) copies the sample;
 * f64 output is the sample value, optionally normalised per channel as
 * (v / 255 - mean_c) / std_c.  Returns 0, or -1 on bad arguments. */
int kro_resize_nearest(const void *src, int sh, int sw, int c, int src_t,
                       void *dst, int dh, int dw, int out_t,
                       const double *mean, const double *stdv, int nthreads)
{
    if (sh < 1 || sw < 1 || dh < 1 || dw < 1 || c < 1 || c > 4)
        return -1;
    if (out_t == KRO_OUT_U8 && src_t != KRO_U8)
        return -1;
    if (nthreads < 1)
        nthreads = 1;
#pragma omp parallel for num_threads(nthreads) schedule(static)
    for (int dy = 0; dy < dh; dy++) {
        int64_t sy = ((int64_t)(2 * dy + 1) * sh) / (2 * (int64_t)dh);
        for (int dx = 0; dx < dw; dx++) {
            int64_t sx = ((int64_t)(2 * dx + 1) * sw) / (2 * (int64_t)dw);
            size_t sidx = ((size_t)sy * (size_t)sw + (size_t)sx) * (size_t)c;
            size_t didx = ((size_t)dy * (size_t)dw + (size_t)dx) * (size_t)c;
            for (int ch = 0; ch < c; ch++) {
                if (out_t == KRO_OUT_U8) {
                    ((uint8_t *)dst)[didx + (size_t)ch] = ((const uint8_t *)src)[sidx + (size_t)ch];
                } else {
                    double v = src_t == KRO_U8 ? (double)((const uint8_t *)src)[sidx + (size_t)ch]
                                               : (double)((const float *)src)[sidx + (size_t)ch];
                    if (mean && stdv)
                        v = (v / 255.0 - mean[ch]) / stdv[ch];
                    ((double *)dst)[didx + (size_t)ch] = v;
                }
            }
        }
    }
    return 0;
}

/* Flip (Sec. III "horizontal flip"): out(x, y) = in(flip_x ? W-1-x : x,
 * flip_y ? H-1-y : y), every channel, same sample type (1 byte or 4). */
int kro_flip(const void *src, int h, int w, int c, int src_t, void *dst, int flip_x, int flip_y)
{
    if (h < 1 || w < 1 || c < 1 || c > 4)
        return -1;
    const size_t es = src_t == KRO_U8 ? 1 : 4;
    for (int y = 0; y < h; y++) {
        int sy = flip_y ? h - 1 - y : y;
        for (int x = 0; x < w; x++) {
            int sx = flip_x ? w - 1 - x : x;
            const uint8_t *s = (const uint8_t *)src + ((size_t)sy * w + sx) * c * es;
            uint8_t *d = (uint8_t *)dst + ((size_t)y * w + x) * c * es;
            for (size_t b = 0; b < (size_t)c * es; b++)
                d[b] = s[b];
        }
    }
    return 0;
}

/* RGB to gray (Sec. III "RGB to grayscale"), ITU-R BT.601 luma weights.
 * u8 output (u8 sources): OpenCV-style 14-bit fixed point,
 * (4899 R + 9617 G + 1868 B + 2^13) >> 14 (weights sum to 2^14, so a grey
 * pixel keeps its value).  f64 output: 0.299 R + 0.587 G + 0.114 B on the
 * sample scale, optionally normalised as (v / 255 - mean) / std. */
int kro_rgb_to_gray(const void *src, int h, int w, int src_t, void *dst, int out_t,
                    const double *mean, const double *stdv, int nthreads)
{
    if (h < 1 || w < 1)
        return -1;
    if (out_t == KRO_OUT_U8 && src_t != KRO_U8)
        return -1;
    if (nthreads < 1)
        nthreads = 1;
#pragma omp parallel for num_threads(nthreads) schedule(static)
    for (int y = 0; y < h; y++) {
        for (int x = 0; x < w; x++) {
            size_t i = (size_t)y * w + x;
            double r, g, b;
            if (src_t == KRO_U8) {
                const uint8_t *p = (const uint8_t *)src + 3 * i;
                if (out_t == KRO_OUT_U8) {
                    int64_t acc = 4899 * (int64_t)p[0] + 9617 * (int64_t)p[1] + 1868 * (int64_t)p[2];
                    ((uint8_t *)dst)[i] = (uint8_t)((acc + (1 << 13)) >> 14);
                    continue;
                }
                r = p[0]; g = p[1]; b = p[2];
            } else {
                const float *p = (const float *)src + 3 * i;
                r = p[0]; g = p[1]; b = p[2];
            }
            double v = 0.299 * r + 0.587 * g + 0.114 * b;
            if (mean && stdv)
                v = (v / 255.0 - mean[0]) / stdv[0];
            ((double *)dst)[i] = v;
        }
    }
    return 0;
}

/* Inverse of the 2x3 affine map [[a, b, c], [d, e, f]] (rows of x' and y'),
 * by the fixed formula: det = a e - b d (two products, one difference);
 * A = e / det, B = -b / det, D = -d / det, E = a / det;
 * C = -(A c + B f), F = -(D c + E f).  Returns -1 if det is zero or not
 * finite. */
int kro_invert_affine(const double m[6], double inv[6])
{
    double p1 = m[0] * m[4];
    double p2 = m[1] * m[3];
    double det = p1 - p2;
    if (det == 0.0 || !isfinite(det))
        return -1;
    double A = m[4] / det, B = -m[1] / det, D = -m[3] / det, E = m[0] / det;
    double t1 = A * m[2], t2 = B * m[5];
    double C = -(t1 + t2);
    double t3 = D * m[2], t4 = E * m[5];
    double F = -(t3 + t4);
    inv[0] = A; inv[1] = B; inv[2] = C;
    inv[3] = D; inv[4] = E; inv[5] = F;
    return 0;
}

/* Bilinear affine warp.  m is source->destination unless inverse != 0, in
 * which case it already maps destination pixel centres to source coordinates.
 * Returns 0, or -1 on bad sizes or a singular matrix. */
int kro_warp(const void *src, int sh, int sw, int c, int src_t,
             void *dst, int dh, int dw, int out_t,
             const double m[6], int inverse,
             int border, double bval, const double *mean, const double *stdv,
             int nthreads)
{
    if (sh < 1 || sw < 1 || dh < 1 || dw < 1 || c < 1 || c > 4)
        return -1;
    double im[6];
    if (inverse) {
        for (int i = 0; i < 6; i++)
            im[i] = m[i];
    } else if (kro_invert_affine(m, im) != 0) {
        return -1;
    }
    if (nthreads < 1)
        nthreads = 1;
#pragma omp parallel for num_threads(nthreads) schedule(static)
    for (int y = 0; y < dh; y++) {
        for (int x = 0; x < dw; x++) {
            double xs = fma(im[0], (double)x, fma(im[1], (double)y, im[2]));
            double ys = fma(im[3], (double)x, fma(im[4], (double)y, im[5]));
            if (xs < -2.0) xs = -2.0;
            if (xs > (double)sw + 1.0) xs = (double)sw + 1.0;
            if (ys < -2.0) ys = -2.0;
            if (ys > (double)sh + 1.0) ys = (double)sh + 1.0;
            double fx0 = floor(xs), fy0 = floor(ys);
            double fx = xs - fx0, fy = ys - fy0;
            int64_t wx1 = (int64_t)nearbyint(2048.0 * fx);
            int64_t wy1 = (int64_t)nearbyint(2048.0 * fy);
            write_pixel(src, src_t, sh, sw, c, dst, out_t,
                        ((size_t)y * (size_t)dw + (size_t)x) * (size_t)c,
                        (int64_t)fx0, (int64_t)fy0, wx1, wy1, fx, fy,
                        border, bval, mean, stdv);
        }
    }
    return 0;
}

/* Inverse of a 3x3 homography m (row-major) by the adjugate: cofactors as
 * differences of two rounded products, det = (m00 c00 + m01 c01) + m02 c02,
 * inverse = cofactor matrix transposed, each entry divided by det.  Returns
 * -1 if det is zero or not finite. */
int kro_invert_homography(const double m[9], double inv[9])
{
    double c00 = m[4] * m[8] - m[5] * m[7];
    double c01 = m[5] * m[6] - m[3] * m[8];
    double c02 = m[3] * m[7] - m[4] * m[6];
    double det = (m[0] * c00 + m[1] * c01) + m[2] * c02;
    if (det == 0.0 || !isfinite(det))
        return -1;
    double c10 = m[2] * m[7] - m[1] * m[8];
    double c11 = m[0] * m[8] - m[2] * m[6];
    double c12 = m[1] * m[6] - m[0] * m[7];
    double c20 = m[1] * m[5] - m[2] * m[4];
    double c21 = m[2] * m[3] - m[0] * m[5];
    double c22 = m[0] * m[4] - m[1] * m[3];
    inv[0] = c00 / det; inv[1] = c10 / det; inv[2] = c20 / det;
    inv[3] = c01 / det; inv[4] = c11 / det; inv[5] = c21 / det;
    inv[6] = c02 / det; inv[7] = c12 / det; inv[8] = c22 / det;
    return 0;
}

/* Bilinear perspective warp (a homography; the "geometric transforms" of
 * Sec. II-A beyond the affine case).  m maps source to destination unless
 * inverse.  Destination pixel (x, y): w = fma(h20, x, fma(h21, y, h22)),
 * xs = fma(h00, x, fma(h01, y, h02)) / w, ys likewise (binary64, correctly
 * rounded); a coordinate that is not a number (w = 0 over 0) reads as -2;
 * then the clamp, taps, weights and borders of kro_warp. */
int kro_warp_perspective(const void *src, int sh, int sw, int c, int src_t,
                         void *dst, int dh, int dw, int out_t,
                         const double m[9], int inverse,
                         int border, double bval, const double *mean, const double *stdv,
                         int nthreads)
{
    if (sh < 1 || sw < 1 || dh < 1 || dw < 1 || c < 1 || c > 4)
        return -1;
    double im[9];
    if (inverse) {
        for (int i = 0; i < 9; i++)
            im[i] = m[i];
    } else if (kro_invert_homography(m, im) != 0) {
        return -1;
    }
    if (nthreads < 1)
        nthreads = 1;
#pragma omp parallel for num_threads(nthreads) schedule(static)
    for (int y = 0; y < dh; y++) {
        for (int x = 0; x < dw; x++) {
            double w = fma(im[6], (double)x, fma(im[7], (double)y, im[8]));
            double xs = fma(im[0], (double)x, fma(im[1], (double)y, im[2])) / w;
            double ys = fma(im[3], (double)x, fma(im[4], (double)y, im[5])) / w;
            if (xs != xs)
                xs = -2.0;
            if (ys != ys)
                ys = -2.0;
            if (xs < -2.0) xs = -2.0;
            if (xs > (double)sw + 1.0) xs = (double)sw + 1.0;
            if (ys < -2.0) ys = -2.0;
            if (ys > (double)sh + 1.0) ys = (double)sh + 1.0;
            double fx0 = floor(xs), fy0 = floor(ys);
            double fx = xs - fx0, fy = ys - fy0;
            int64_t wx1 = (int64_t)nearbyint(2048.0 * fx);
            int64_t wy1 = (int64_t)nearbyint(2048.0 * fy);
            write_pixel(src, src_t, sh, sw, c, dst, out_t,
                        ((size_t)y * (size_t)dw + (size_t)x) * (size_t)c,
                        (int64_t)fx0, (int64_t)fy0, wx1, wy1, fx, fy,
                        border, bval, mean, stdv);
        }
    }
    return 0;
}
