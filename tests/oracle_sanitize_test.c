/* oracle_sanitize_test.c -- runs every function of the oracle (oracle/kro.c)
 * under AddressSanitizer and UndefinedBehaviorSanitizer on small and
 * degenerate inputs: every operation, channel count, sample and output type
 * and border, 1x1 and one-row/one-column images, large up- and downscales,
 * maps that send every tap outside the image, huge coefficients and
 * homographies whose horizon crosses the output.  Each buffer is allocated at
 * exactly its size, so any read or write outside it is reported.  Prints
 * "OK" (the sanitizers abort on the first error). */
#include <math.h>
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

int kro_resize(const void *, int, int, int, int, void *, int, int, int, int, double, const double *, const double *, int);
int kro_resize_nearest(const void *, int, int, int, int, void *, int, int, int, const double *, const double *, int);
int kro_flip(const void *, int, int, int, int, void *, int, int);
int kro_rgb_to_gray(const void *, int, int, int, void *, int, const double *, const double *, int);
int kro_invert_affine(const double *, double *);
int kro_warp(const void *, int, int, int, int, void *, int, int, int, const double *, int, int, double,
             const double *, const double *, int);
int kro_invert_homography(const double *, double *);
int kro_warp_perspective(const void *, int, int, int, int, void *, int, int, int, const double *, int, int, double,
                         const double *, const double *, int);

static void *src_image(int h, int w, int c, int t, unsigned seed)
{
    const size_t n = (size_t)h * w * c;
    if (t == 0) {
        uint8_t *p = malloc(n);
        for (size_t i = 0; i < n; i++)
            p[i] = (uint8_t)((i * 2654435761u + seed) >> 7);
        return p;
    }
    float *p = malloc(n * sizeof(float));
    for (size_t i = 0; i < n; i++)
        p[i] = (float)((i * 2654435761u + seed) % 1000u) * 0.25f;
    return p;
}

static int fails = 0;
static void expect(int cond, const char *what, int line)
{
    if (!cond) {
        printf("FAIL line %d: %s\n", line, what);
        fails++;
    }
}
#define EXPECT(c) expect((c), #c, __LINE__)

int main(void)
{
    static const int sizes[][2] = {{1, 1}, {1, 7}, {7, 1}, {2, 2}, {5, 9}, {13, 4}, {31, 33}};
    const int ns = (int)(sizeof sizes / sizeof sizes[0]);
    const double mean[4] = {0.485, 0.456, 0.406, 0.5}, stdv[4] = {0.229, 0.224, 0.225, 0.25};
    for (int a = 0; a < ns; a++)
        for (int b = 0; b < ns; b++)
            for (int c = 1; c <= 4; c++)
                for (int st = 0; st < 2; st++) {
                    const int sh = sizes[a][0], sw = sizes[a][1], dh = sizes[b][0], dw = sizes[b][1];
                    void *src = src_image(sh, sw, c, st, (unsigned)(a * 31 + b));
                    uint8_t *d8 = malloc((size_t)dh * dw * c);
                    double *df = malloc((size_t)dh * dw * c * sizeof(double));
                    for (int border = 0; border < 2; border++) {
                        if (st == 0)
                            EXPECT(kro_resize(src, sh, sw, c, st, d8, dh, dw, 0, border, 7.0, NULL, NULL, 1) == 0);
                        EXPECT(kro_resize(src, sh, sw, c, st, df, dh, dw, 1, border, 7.0, mean, stdv, 1) == 0);
                        const double ms[][6] = {{1, 0, 0, 0, 1, 0},
                                                {0.3, -0.8, 2.5, 0.9, 0.4, -1.5},
                                                {1e-3, 0, 1e6, 0, 1e-3, -1e6},
                                                {1e6, 1e5, -3, -2e5, 1e6, 4},
                                                {-1, 0, sw - 1, 0, 1, 0}};
                        for (int k = 0; k < 5; k++) {
                            if (st == 0)
                                EXPECT(kro_warp(src, sh, sw, c, st, d8, dh, dw, 0, ms[k], k & 1, border, 3.0, NULL,
                                                NULL, 1) == 0);
                            EXPECT(kro_warp(src, sh, sw, c, st, df, dh, dw, 1, ms[k], k & 1, border, 3.0, mean, stdv,
                                            1) == 0);
                        }
                        const double hs[][9] = {{1, 0, 0, 0, 1, 0, 0, 0, 1},
                                                {0.9, 0.1, 1, -0.2, 1.1, 2, 0.01, -0.02, 1},
                                                {1, 0, 0, 0, 1, 0, 0.5, 0.5, -3},
                                                {0, 0, 0, 0, 0, 0, 0, 0, 1e-300}};
                        for (int k = 0; k < 4; k++) {
                            if (st == 0)
                                EXPECT(kro_warp_perspective(src, sh, sw, c, st, d8, dh, dw, 0, hs[k], k >= 2, border,
                                                            3.0, NULL, NULL, 1) == 0);
                            EXPECT(kro_warp_perspective(src, sh, sw, c, st, df, dh, dw, 1, hs[k], k >= 2, border,
                                                        3.0, mean, stdv, 1) == 0);
                        }
                    }
                    if (st == 0)
                        EXPECT(kro_resize_nearest(src, sh, sw, c, st, d8, dh, dw, 0, NULL, NULL, 1) == 0);
                    EXPECT(kro_resize_nearest(src, sh, sw, c, st, df, dh, dw, 1, mean, stdv, 1) == 0);
                    free(d8);
                    free(df);
                    void *fl = malloc((size_t)sh * sw * c * (st ? 4 : 1));
                    for (int fx = 0; fx < 2; fx++)
                        for (int fy = 0; fy < 2; fy++)
                            EXPECT(kro_flip(src, sh, sw, c, st, fl, fx, fy) == 0);
                    free(fl);
                    if (c == 3) {
                        uint8_t *g8 = malloc((size_t)sh * sw);
                        double *gf = malloc((size_t)sh * sw * sizeof(double));
                        if (st == 0)
                            EXPECT(kro_rgb_to_gray(src, sh, sw, st, g8, 0, NULL, NULL, 1) == 0);
                        EXPECT(kro_rgb_to_gray(src, sh, sw, st, gf, 1, mean, stdv, 1) == 0);
                        free(g8);
                        free(gf);
                    }
                    free(src);
                }
    /* bad sizes and singular maps are refused, not read */
    uint8_t px[3] = {1, 2, 3}, out[3];
    const double id[6] = {1, 0, 0, 0, 1, 0}, sing[6] = {1, 2, 0, 2, 4, 0}, nanm[6] = {NAN, 0, 0, 0, 1, 0};
    EXPECT(kro_resize(px, 0, 1, 3, 0, out, 1, 1, 0, 0, 0.0, NULL, NULL, 1) == -1);
    EXPECT(kro_resize(px, 1, 1, 5, 0, out, 1, 1, 0, 0, 0.0, NULL, NULL, 1) == -1);
    EXPECT(kro_warp(px, 1, 1, 3, 0, out, 1, 1, 0, sing, 0, 0, 0.0, NULL, NULL, 1) == -1);
    EXPECT(kro_warp(px, 1, 1, 3, 0, out, 1, 1, 0, nanm, 0, 0, 0.0, NULL, NULL, 1) == -1);
    EXPECT(kro_warp(px, 1, 1, 3, 0, out, 1, 1, 0, id, 0, 0, 0.0, NULL, NULL, 1) == 0);
    double inv[9];
    EXPECT(kro_invert_affine(sing, inv) == -1);
    const double hsing[9] = {1, 2, 3, 2, 4, 6, 0, 0, 1};
    EXPECT(kro_invert_homography(hsing, inv) == -1);
    if (!fails)
        printf("OK\n");
    return fails != 0;
}
