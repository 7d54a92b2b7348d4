// api_sanitize_test.cpp -- the C ABI's host-side validation (api.cpp) under
// AddressSanitizer and UndefinedBehaviorSanitizer on the CPU.  api.cpp is
// compiled with the host compiler against the HIP headers; the kernel
// launchers are replaced by stubs that record the image job they were given,
// so valid calls can be checked for what they would have launched (view
// offsets, pitches) without a GPU.  Prints "OK" or the first failure.
#include <cmath>
#include <cstdint>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <limits>

#include "kr_api_internal.h"

namespace kr {
static ImageJob g_job;
static int g_calls = 0;
static hipError_t record(const ImageJob &j)
{
    g_job = j;
    g_calls++;
    return hipSuccess;
}
hipError_t launch_resize(int, kr_dtype, kr_dtype, const ImageJob &j, const Epilogue &, hipStream_t) { return record(j); }
hipError_t launch_warp(int, kr_dtype, kr_dtype, const ImageJob &j, const Epilogue &, hipStream_t) { return record(j); }
hipError_t launch_persp(int, kr_dtype, kr_dtype, const ImageJob &j, const Epilogue &, hipStream_t) { return record(j); }
hipError_t launch_nearest(int, kr_dtype, kr_dtype, const ImageJob &j, const Epilogue &, hipStream_t) { return record(j); }
hipError_t launch_flip(int, kr_dtype, const ImageJob &j, int, int, hipStream_t) { return record(j); }
hipError_t launch_gray(kr_dtype, kr_dtype, const ImageJob &j, const Epilogue &, hipStream_t) { return record(j); }
hipError_t launch_tiled(int, int, kr_dtype, const ImageJob &j, const Epilogue &, hipStream_t) { return record(j); }
hipError_t launch_resize_gray(kr_dtype, const ImageJob &j, const Epilogue &, hipStream_t) { return record(j); }
hipError_t launch_copy(void *, const void *, size_t, hipStream_t) { g_calls++; return hipSuccess; }
hipError_t launch_stream(void *, size_t, const void *, int, int, hipStream_t) { g_calls++; return hipSuccess; }
}  // namespace kr

const char *hipGetErrorString(hipError_t) { return "stub"; }

static int g_fail = 0;
#define EXPECT(cond)                                                                  \
    do {                                                                              \
        if (!(cond)) {                                                                \
            std::printf("FAIL line %d: %s (%s)\n", __LINE__, #cond, kr_last_error()); \
            g_fail = 1;                                                               \
        }                                                                             \
    } while (0)

static void *P(uintptr_t a) { return reinterpret_cast<void *>(a); }

int main()
{
    const uintptr_t S = 0x100000000ull, D = 0x900000000ull;  // 16-byte aligned, never dereferenced
    const double id[6] = {1, 0, 0, 0, 1, 0};
    const double h9[9] = {1, 0, 0, 0, 1, 0, 0, 0, 1};
    const int dims[] = {0, 1, 2, 32767, 32768, -1, std::numeric_limits<int>::max(), std::numeric_limits<int>::min()};
    // every size combination: accepted exactly when inside [1, 32767]
    for (int h : dims)
        for (int w : dims) {
            const bool ok = h >= 1 && w >= 1 && h <= 32767 && w <= 32767;
            const kr_status r = kr_resize_bilinear(P(S), h, w, 3, KR_U8, P(D + (1ull << 36)), 8, 8, KR_U8,
                                                   KR_BORDER_REPLICATE, 0.0f, nullptr, nullptr);
            EXPECT((r == KR_OK) == ok);
            const kr_status q = kr_warp_affine(P(S), 8, 8, 4, KR_F32, P(D), h, w, KR_F32, id, 0, KR_BORDER_CONSTANT,
                                               0.0f, nullptr, nullptr);
            EXPECT((q == KR_OK) == ok);
        }
    // channel counts, dtype pairs, borders, border values
    for (int c = -1; c <= 6; c++)
        EXPECT((kr_flip(P(S), 4, 4, c, KR_U8, P(D), 1, 0, nullptr) == KR_OK) == (c >= 1 && c <= 4));
    for (int st = -1; st <= 2; st++)
        for (int dt = -1; dt <= 2; dt++) {
            const bool ok = (st == 0 && dt == 0) || (st == 0 && dt == 1) || (st == 1 && dt == 1);
            EXPECT((kr_resize_bilinear(P(S), 4, 4, 3, (kr_dtype)st, P(D), 4, 4, (kr_dtype)dt, KR_BORDER_REPLICATE,
                                       0.0f, nullptr, nullptr) == KR_OK) == ok);
        }
    const float bvals[] = {0.0f, 255.0f, 256.0f, -1.0f, 0.5f, NAN, INFINITY};
    for (float b : bvals) {
        const bool ok8 = std::isfinite(b) && b >= 0.0f && b <= 255.0f && b == std::floor(b);
        EXPECT((kr_warp_affine(P(S), 4, 4, 3, KR_U8, P(D), 4, 4, KR_U8, id, 0, KR_BORDER_CONSTANT, b, nullptr,
                               nullptr) == KR_OK) == ok8);
        EXPECT((kr_warp_affine(P(S), 4, 4, 3, KR_F32, P(D), 4, 4, KR_F32, id, 0, KR_BORDER_CONSTANT, b, nullptr,
                               nullptr) == KR_OK) == std::isfinite(b));
    }
    // matrices: non-finite, singular, huge
    const double bad[][6] = {{NAN, 0, 0, 0, 1, 0}, {1, 0, INFINITY, 0, 1, 0}, {1, 2, 0, 2, 4, 0},
                             {1e-300, 0, 0, 0, 1e-300, 0}, {1e300, 0, 0, 0, 1e300, 0}};
    for (const auto &m : bad)
        EXPECT(kr_warp_affine(P(S), 4, 4, 3, KR_U8, P(D), 4, 4, KR_U8, m, 0, KR_BORDER_CONSTANT, 0.0f, nullptr,
                              nullptr) != KR_OK);
    double inv[6];
    EXPECT(kr_invert_affine(bad[2], inv) == KR_ERR_SINGULAR_MATRIX);
    double inv9[9];
    EXPECT(kr_invert_homography(h9, inv9) == KR_OK);
    // normalisation
    kr_normalize n;
    for (int i = 0; i < 4; i++) {
        n.mean[i] = 0.5f;
        n.std[i] = 0.25f;
    }
    EXPECT(kr_resize_bilinear(P(S), 4, 4, 4, KR_U8, P(D), 4, 4, KR_F32, KR_BORDER_REPLICATE, 0, &n, nullptr) == KR_OK);
    EXPECT(kr_resize_bilinear(P(S), 4, 4, 4, KR_U8, P(D), 4, 4, KR_U8, KR_BORDER_REPLICATE, 0, &n, nullptr) != KR_OK);
    n.std[3] = 0.0f;
    EXPECT(kr_resize_bilinear(P(S), 4, 4, 4, KR_U8, P(D), 4, 4, KR_F32, KR_BORDER_REPLICATE, 0, &n, nullptr) != KR_OK);
    EXPECT(kr_resize_bilinear(P(S), 4, 4, 3, KR_U8, P(D), 4, 4, KR_F32, KR_BORDER_REPLICATE, 0, &n, nullptr) == KR_OK);
    // overlap: touching is fine, one byte of overlap is not
    const size_t src_bytes = 4 * 4 * 3;
    EXPECT(kr_resize_bilinear(P(S), 4, 4, 3, KR_U8, P(S + 48), 4, 4, KR_U8, KR_BORDER_REPLICATE, 0, nullptr,
                              nullptr) == KR_OK);
    EXPECT(kr_resize_bilinear(P(S + 16), 4, 4, 3, KR_U8, P(S), 4, 4, KR_U8, KR_BORDER_REPLICATE, 0, nullptr,
                              nullptr) != KR_OK);
    (void)src_bytes;
    // ranges that would wrap around the address space are rejected
    const uintptr_t top = ~(uintptr_t)15;
    EXPECT(kr_resize_bilinear(P(top), 4, 4, 3, KR_U8, P(D), 4, 4, KR_U8, KR_BORDER_REPLICATE, 0, nullptr,
                              nullptr) != KR_OK);
    EXPECT(kr_resize_bilinear(P(S), 4, 4, 3, KR_U8, P(top), 4, 4, KR_U8, KR_BORDER_REPLICATE, 0, nullptr,
                              nullptr) != KR_OK);
    EXPECT(kr_hbm_copy(P(D), P(S), ~(size_t)0 - 15, nullptr) != KR_OK);
    EXPECT(kr_hbm_stream(P(D), 16, P(top), 32, nullptr) != KR_OK);
    // views: every first-pixel offset within 16 bytes, for each pixel size
    for (int c = 1; c <= 4; c++)
        for (int f = 0; f < 2; f++) {
            const size_t px = (size_t)c * (f ? 4 : 1);
            for (size_t off = 0; off < 64; off++) {
                const uintptr_t a = S + off;
                int k = -1;
                for (int t = 0; t < 16; t++)
                    if (((a - (uintptr_t)t * px) & 15) == 0) {
                        k = t;
                        break;
                    }
                const int calls = kr::g_calls;
                const kr_status r = kr_resize_bilinear_view(P(a), 5, 7, 9 * px, c, f ? KR_F32 : KR_U8, P(D), 3, 3,
                                                            f ? KR_F32 : KR_U8, KR_BORDER_REPLICATE, 0, nullptr,
                                                            nullptr);
                EXPECT((r == KR_OK) == (k >= 0));
                if (r == KR_OK) {
                    EXPECT(kr::g_calls == calls + 1);
                    EXPECT(kr::g_job.sk == k && kr::g_job.sp == 9 && kr::g_job.sw == 7 && kr::g_job.sh == 5);
                    EXPECT(reinterpret_cast<uintptr_t>(kr::g_job.src) == a - (uintptr_t)k * px);
                    EXPECT(reinterpret_cast<uintptr_t>(kr::g_job.src) % 16 == 0);
                }
            }
        }
    // pitches: not whole pixels, shorter than a row, beyond the 2^31-pixel span
    EXPECT(kr_flip_view(P(S), 4, 4, 13, 3, KR_U8, P(D), 1, 0, nullptr) != KR_OK);
    EXPECT(kr_flip_view(P(S), 4, 4, 9, 3, KR_U8, P(D), 1, 0, nullptr) != KR_OK);
    EXPECT(kr_flip_view(P(S), 4, 4, 12, 3, KR_U8, P(D), 1, 0, nullptr) == KR_OK);
    EXPECT(kr_flip_view(P(S), 32767, 4, (size_t)3 << 20, 3, KR_U8, P(D), 1, 0, nullptr) != KR_OK);
    EXPECT(kr_flip_view(P(S), 2, 4, ~(size_t)0 - 2, 3, KR_U8, P(D), 1, 0, nullptr) != KR_OK);
    EXPECT(kr_rgb_to_gray_view(P(S), 32767, 32767, (size_t)32767 * 12, KR_F32, P(D + (1ull << 40)), KR_F32, nullptr,
                               nullptr) == KR_OK);  // a 12.9 GB view: within the 2^31-pixel span
    EXPECT(kr_rgb_to_gray_view(P(S), 32767, 32767, (size_t)65540 * 12, KR_F32, P(D + (1ull << 40)), KR_F32, nullptr,
                               nullptr) != KR_OK);  // over 2^31 - 32 pixels
    EXPECT(kr_rgb_to_gray_view(P(S), 1000, 1000, 3000, KR_U8, P(D), KR_U8, nullptr, nullptr) == KR_OK);
    EXPECT(kr_warp_perspective_view(P(S + 2), 7, 7, 28, 4, KR_U8, P(D), 7, 7, KR_U8, h9, 0, KR_BORDER_CONSTANT, 0,
                                    nullptr, nullptr) != KR_OK);  // 2 bytes in: not a whole number of RGBA pixels
    EXPECT(kr_warp_perspective_view(P(S + 2), 7, 7, 21, 3, KR_U8, P(D), 7, 7, KR_U8, h9, 0, KR_BORDER_CONSTANT, 0,
                                    nullptr, nullptr) == KR_OK);  // RGB: 6 pixels past the boundary
    EXPECT(kr_resize_nearest_view(P(S + 12), 7, 7, 36, 3, KR_U8, P(D), 7, 7, KR_U8, nullptr, nullptr) == KR_OK);
    // fused gray: RGB u8 in, one channel out; dst sized for one channel
    EXPECT(kr_resize_bilinear_gray(P(S), 8, 8, 0, P(S + 192), 8, 8, KR_U8, KR_BORDER_REPLICATE, 0, nullptr,
                                   nullptr) == KR_OK);  // adjacent, not overlapping
    EXPECT(kr_resize_bilinear_gray(P(S), 8, 8, 0, P(S + 176), 8, 8, KR_U8, KR_BORDER_REPLICATE, 0, nullptr,
                                   nullptr) != KR_OK);
    EXPECT(kr_warp_affine_gray(P(S), 8, 8, 0, P(D), 8, 8, KR_F32, id, 0, KR_BORDER_CONSTANT, 0.5f, nullptr,
                               nullptr) != KR_OK);  // the border value is a u8 sample
    EXPECT(kr_warp_affine_gray(P(S), 8, 8, 0, P(D), 8, 8, KR_F32, id, 2, KR_BORDER_CONSTANT, 0, nullptr,
                               nullptr) != KR_OK);  // unknown flag
    EXPECT(kr_warp_affine_gray(P(S), 8, 8, 0, P(D), 8, 8, KR_U8, id, 0, KR_BORDER_CONSTANT, 0, &n, nullptr) != KR_OK);
    EXPECT(kr_resize_bilinear_gray(P(S), 8, 8, 0, P(D), 8, 8, (kr_dtype)2, KR_BORDER_CONSTANT, 0, nullptr,
                                   nullptr) == KR_ERR_UNSUPPORTED);
    EXPECT(kr_resize_bilinear_gray(P(S + 3), 8, 8, 30, P(D), 8, 8, KR_U8, KR_BORDER_CONSTANT, 0, nullptr,
                                   nullptr) == KR_OK);  // an RGB view
    // the probes
    EXPECT(kr_hbm_stream(P(D), 16, P(S), 16ull << 9, nullptr) != KR_OK);
    EXPECT(kr_hbm_stream(P(D), 16, P(S), 16ull << 8, nullptr) == KR_OK);
    EXPECT(kr_hbm_stream(P(D), 48, P(S), 16, nullptr) != KR_OK);
    EXPECT(kr_hbm_copy(P(D), P(S), 0, nullptr) == KR_OK);
    EXPECT(kr_status_string((kr_status)99) != nullptr && kr_status_string(KR_OK) != nullptr);
    if (!g_fail)
        std::printf("OK\n");
    return g_fail;
}
