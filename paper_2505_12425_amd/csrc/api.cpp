// api.cpp -- libkr's C ABI for single images: argument validation, the
// inverse affine map, epilogue setup and dispatch to the kernels.
//
// Compiled with -ffp-contract=off: kr_invert_affine's formula must round each
// product and sum on its own, exactly as written.
#include <cmath>
#include <cstdint>
#include <cstdio>
#include <cstring>
#include <string>

#include "kr_api_internal.h"

namespace kr {

static thread_local std::string g_last_error;

kr_status fail(kr_status s, const char *fmt, ...)
{
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    g_last_error = buf;
    return s;
}

void clear_error() { g_last_error.clear(); }

static size_t elem_size(kr_dtype t) { return t == KR_U8 ? 1 : 4; }

kr_status check_image(const char *what, const void *p, int h, int w, int c)
{
    if (!p)
        return fail(KR_ERR_INVALID_ARGUMENT, "%s pointer is NULL", what);
    if (reinterpret_cast<uintptr_t>(p) % 16 != 0)
        return fail(KR_ERR_INVALID_ARGUMENT, "%s pointer is not 16-byte aligned", what);
    if (h < 1 || w < 1 || h > KR_MAX_DIM || w > KR_MAX_DIM)
        return fail(KR_ERR_INVALID_ARGUMENT, "%s size %dx%d outside [1, %d]", what, h, w, KR_MAX_DIM);
    (void)c;
    return KR_OK;
}

int view_shift(const void *src, size_t px_bytes)
{
    const uintptr_t a = reinterpret_cast<uintptr_t>(src);
    for (int k = 0; k < 16; k++)
        if (((a - (uintptr_t)k * px_bytes) & 15) == 0)
            return k;
    return -1;
}

kr_status check_source(const void *src, int h, int w, int c, kr_dtype st, size_t pitch)
{
    if (pitch == 0)
        return check_image("src", src, h, w, c);
    if (!src)
        return fail(KR_ERR_INVALID_ARGUMENT, "src pointer is NULL");
    if (h < 1 || w < 1 || h > KR_MAX_DIM || w > KR_MAX_DIM)
        return fail(KR_ERR_INVALID_ARGUMENT, "src size %dx%d outside [1, %d]", h, w, KR_MAX_DIM);
    const size_t px = (size_t)c * elem_size(st);
    if (view_shift(src, px) < 0)
        return fail(KR_ERR_INVALID_ARGUMENT, "src view does not start a whole number of pixels past a 16-byte boundary");
    if (pitch < (size_t)w * px || pitch % px != 0)
        return fail(KR_ERR_INVALID_ARGUMENT, "src pitch %zu is not a whole number of pixels >= the row's %zu bytes",
                    pitch, (size_t)w * px);
    // (bounded first so that the span below cannot wrap)
    if (pitch / px > (size_t)INT32_MAX || 15 + (size_t)(h - 1) * (pitch / px) + (size_t)w > (size_t)INT32_MAX - 16)
        return fail(KR_ERR_INVALID_ARGUMENT, "src view spans more than 2^31 - 32 pixels");
    return KR_OK;
}

void set_source(ImageJob &j, const void *src, int h, int w, int c, kr_dtype st, size_t pitch)
{
    j.sh = h;
    j.sw = w;
    if (pitch == 0) {
        j.src = src;
        j.sp = w;
        j.sk = 0;
        return;
    }
    const size_t px = (size_t)c * elem_size(st);
    j.sk = view_shift(src, px);
    j.sp = (int)(pitch / px);
    j.src = static_cast<const uint8_t *>(src) - (size_t)j.sk * px;
}

size_t source_span(int h, int w, int c, kr_dtype st, size_t pitch)
{
    const size_t row = (size_t)w * (size_t)c * elem_size(st);
    return (size_t)(h - 1) * (pitch ? pitch : row) + row;
}

kr_status check_common(const void *src, int sh, int sw, int c, kr_dtype st, void *dst, int dh, int dw,
                       kr_dtype dt, kr_border border, float bval, const kr_normalize *norm, size_t src_pitch)
{
    if (c < 1 || c > 4)
        return fail(KR_ERR_UNSUPPORTED, "channel count %d not in [1, 4]", c);
    if (!((st == KR_U8 && dt == KR_U8) || (st == KR_U8 && dt == KR_F32) || (st == KR_F32 && dt == KR_F32)))
        return fail(KR_ERR_UNSUPPORTED, "dtype pair (%d -> %d) not supported", (int)st, (int)dt);
    if (border != KR_BORDER_CONSTANT && border != KR_BORDER_REPLICATE)
        return fail(KR_ERR_UNSUPPORTED, "border mode %d not supported", (int)border);
    kr_status s = check_source(src, sh, sw, c, st, src_pitch);
    if (s != KR_OK)
        return s;
    s = check_image("dst", dst, dh, dw, c);
    if (s != KR_OK)
        return s;
    if (!std::isfinite(bval))
        return fail(KR_ERR_INVALID_ARGUMENT, "border value is not finite");
    if (st == KR_U8 && (bval < 0.0f || bval > 255.0f || bval != std::floor(bval)))
        return fail(KR_ERR_INVALID_ARGUMENT, "u8 border value %g is not an integer in [0, 255]", (double)bval);
    if (norm) {
        if (dt != KR_F32)
            return fail(KR_ERR_INVALID_ARGUMENT, "normalisation needs an f32 destination");
        for (int i = 0; i < c; i++)
            if (!std::isfinite(norm->mean[i]) || !std::isfinite(norm->std[i]) || norm->std[i] == 0.0f)
                return fail(KR_ERR_INVALID_ARGUMENT, "normalisation channel %d has a bad mean/std", i);
    }
    const uintptr_t s0 = reinterpret_cast<uintptr_t>(src);
    const uintptr_t s1 = range_end(src, source_span(sh, sw, c, st, src_pitch));
    const uintptr_t d0 = reinterpret_cast<uintptr_t>(dst);
    const uintptr_t d1 = range_end(dst, (size_t)dh * (size_t)dw * (size_t)c * elem_size(dt));
    if (!s1 || !d1)
        return fail(KR_ERR_INVALID_ARGUMENT, "src or dst range wraps past the end of the address space");
    if (s0 < d1 && d0 < s1)
        return fail(KR_ERR_INVALID_ARGUMENT, "src and dst overlap");
    return KR_OK;
}

Epilogue make_epilogue(int c, kr_border border, float bval, const kr_normalize *norm)
{
    Epilogue e;
    std::memset(&e, 0, sizeof e);
    for (int i = 0; i < 4; i++) {
        e.alpha[i] = 1.0f;
        e.beta[i] = 0.0f;
    }
    if (norm) {
        for (int i = 0; i < c; i++) {
            const double sd = (double)norm->std[i];
            e.alpha[i] = (float)(1.0 / (255.0 * sd));
            e.beta[i] = (float)(-(double)norm->mean[i] / sd);
        }
    }
    e.bval_f = bval;
    e.bval_i = (int)bval;
    e.border = (int)border;
    return e;
}

// The fused gray forms: RGB u8 source (a view when src_pitch != 0), one
// channel out (u8 or f32); the u8 rules for the border value; norm (f32 only)
// normalises the gray with mean[0], std[0].
static kr_status check_gray(const void *src, int sh, int sw, size_t src_pitch, void *dst, int dh, int dw,
                            kr_dtype dt, kr_border border, float bval, const kr_normalize *norm)
{
    if (dt != KR_U8 && dt != KR_F32)
        return fail(KR_ERR_UNSUPPORTED, "dtype pair (0 -> %d) not supported", (int)dt);
    if (border != KR_BORDER_CONSTANT && border != KR_BORDER_REPLICATE)
        return fail(KR_ERR_UNSUPPORTED, "border mode %d not supported", (int)border);
    kr_status s = check_source(src, sh, sw, 3, KR_U8, src_pitch);
    if (s == KR_OK)
        s = check_image("dst", dst, dh, dw, 1);
    if (s != KR_OK)
        return s;
    if (!std::isfinite(bval) || bval < 0.0f || bval > 255.0f || bval != std::floor(bval))
        return fail(KR_ERR_INVALID_ARGUMENT, "u8 border value %g is not an integer in [0, 255]", (double)bval);
    if (norm) {
        if (dt != KR_F32)
            return fail(KR_ERR_INVALID_ARGUMENT, "normalisation needs an f32 destination");
        if (!std::isfinite(norm->mean[0]) || !std::isfinite(norm->std[0]) || norm->std[0] == 0.0f)
            return fail(KR_ERR_INVALID_ARGUMENT, "normalisation has a bad mean/std");
    }
    const uintptr_t s0 = reinterpret_cast<uintptr_t>(src), d0 = reinterpret_cast<uintptr_t>(dst);
    const uintptr_t s1 = range_end(src, source_span(sh, sw, 3, KR_U8, src_pitch));
    const uintptr_t d1 = range_end(dst, (size_t)dh * (size_t)dw * elem_size(dt));
    if (!s1 || !d1)
        return fail(KR_ERR_INVALID_ARGUMENT, "src or dst range wraps past the end of the address space");
    if (s0 < d1 && d0 < s1)
        return fail(KR_ERR_INVALID_ARGUMENT, "src and dst overlap");
    return KR_OK;
}

// Channels unnormalised (the gray combines the 0..255 values), the gray then
// normalised with mean[0], std[0] like the standalone RGB -> gray operator.
static Epilogue make_gray_epilogue(kr_border border, float bval, const kr_normalize *norm)
{
    Epilogue e = make_epilogue(3, border, bval, nullptr);
    e.gray = 1;
    e.galpha = 1.0f;
    e.gbeta = 0.0f;
    if (norm) {
        const double sd = (double)norm->std[0];
        e.galpha = (float)(1.0 / (255.0 * sd));
        e.gbeta = (float)(-(double)norm->mean[0] / sd);
    }
    return e;
}

kr_status check_matrix(const double m[6], int flags, double inv[6])
{
    if (!m)
        return fail(KR_ERR_INVALID_ARGUMENT, "matrix pointer is NULL");
    for (int i = 0; i < 6; i++)
        if (!std::isfinite(m[i]))
            return fail(KR_ERR_SINGULAR_MATRIX, "matrix entry %d is not finite", i);
    if (flags & KR_WARP_INVERSE_MAP) {
        for (int i = 0; i < 6; i++)
            inv[i] = m[i];
        return KR_OK;
    }
    return invert_affine_impl(m, inv);
}

kr_status invert_affine_impl(const double m[6], double inv[6])
{
    const double a = m[0], b = m[1], c = m[2], d = m[3], e = m[4], f = m[5];
    double mx = std::fabs(a);
    mx = std::fmax(mx, std::fabs(b));
    mx = std::fmax(mx, std::fabs(d));
    mx = std::fmax(mx, std::fabs(e));
    const double p1 = a * e;
    const double p2 = b * d;
    const double det = p1 - p2;
    if (!std::isfinite(det) || std::fabs(det) <= 1e-12 * mx * mx || det == 0.0)
        return fail(KR_ERR_SINGULAR_MATRIX, "affine matrix is singular (det = %g)", det);
    const double A = e / det, B = -b / det, D = -d / det, E = a / det;
    const double t1 = A * c, t2 = B * f;
    const double C = -(t1 + t2);
    const double t3 = D * c, t4 = E * f;
    const double F = -(t3 + t4);
    if (!std::isfinite(A) || !std::isfinite(B) || !std::isfinite(C) || !std::isfinite(D) ||
        !std::isfinite(E) || !std::isfinite(F))
        return fail(KR_ERR_SINGULAR_MATRIX, "inverse of the affine matrix is not finite");
    inv[0] = A; inv[1] = B; inv[2] = C;
    inv[3] = D; inv[4] = E; inv[5] = F;
    return KR_OK;
}

}  // namespace kr

using namespace kr;

extern "C" {

kr_status kr_resize_bilinear_view(const void *src, int src_h, int src_w, size_t src_pitch, int c, kr_dtype src_t,
                                  void *dst, int dst_h, int dst_w, kr_dtype dst_t, kr_border border,
                                  float border_value, const kr_normalize *norm, void *stream)
{
    clear_error();
    kr_status s = check_common(src, src_h, src_w, c, src_t, dst, dst_h, dst_w, dst_t, border, border_value, norm,
                               src_pitch);
    if (s != KR_OK)
        return s;
    ImageJob j;
    std::memset(&j, 0, sizeof j);
    set_source(j, src, src_h, src_w, c, src_t, src_pitch);
    j.dst = dst; j.dh = dst_h; j.dw = dst_w;
    const Epilogue e = make_epilogue(c, border, border_value, norm);
    const hipError_t err = launch_resize(c, src_t, dst_t, j, e, (hipStream_t)stream);
    if (err != hipSuccess)
        return fail(KR_ERR_HIP, "resize launch failed: %s", hipGetErrorString(err));
    return KR_OK;
}

kr_status kr_resize_bilinear(const void *src, int src_h, int src_w, int c, kr_dtype src_t, void *dst,
                             int dst_h, int dst_w, kr_dtype dst_t, kr_border border, float border_value,
                             const kr_normalize *norm, void *stream)
{
    return kr_resize_bilinear_view(src, src_h, src_w, 0, c, src_t, dst, dst_h, dst_w, dst_t, border, border_value,
                                   norm, stream);
}

kr_status kr_warp_affine_view(const void *src, int src_h, int src_w, size_t src_pitch, int c, kr_dtype src_t,
                              void *dst, int dst_h, int dst_w, kr_dtype dst_t, const double m[6], int flags,
                              kr_border border, float border_value, const kr_normalize *norm, void *stream)
{
    clear_error();
    kr_status s = check_common(src, src_h, src_w, c, src_t, dst, dst_h, dst_w, dst_t, border, border_value, norm,
                               src_pitch);
    if (s != KR_OK)
        return s;
    if (flags & ~KR_WARP_INVERSE_MAP)
        return fail(KR_ERR_INVALID_ARGUMENT, "unknown warp flags 0x%x", flags);
    ImageJob j;
    std::memset(&j, 0, sizeof j);
    s = check_matrix(m, flags, j.inv);
    if (s != KR_OK)
        return s;
    set_source(j, src, src_h, src_w, c, src_t, src_pitch);
    j.dst = dst; j.dh = dst_h; j.dw = dst_w;
    const Epilogue e = make_epilogue(c, border, border_value, norm);
    const hipError_t err = launch_warp(c, src_t, dst_t, j, e, (hipStream_t)stream);
    if (err != hipSuccess)
        return fail(KR_ERR_HIP, "warp launch failed: %s", hipGetErrorString(err));
    return KR_OK;
}

kr_status kr_warp_affine(const void *src, int src_h, int src_w, int c, kr_dtype src_t, void *dst,
                         int dst_h, int dst_w, kr_dtype dst_t, const double m[6], int flags,
                         kr_border border, float border_value, const kr_normalize *norm, void *stream)
{
    return kr_warp_affine_view(src, src_h, src_w, 0, c, src_t, dst, dst_h, dst_w, dst_t, m, flags, border,
                               border_value, norm, stream);
}

kr_status kr_resize_bilinear_gray(const void *src, int src_h, int src_w, size_t src_pitch, void *dst, int dst_h,
                                  int dst_w, kr_dtype dst_t, kr_border border, float border_value,
                                  const kr_normalize *norm, void *stream)
{
    clear_error();
    const kr_status s = check_gray(src, src_h, src_w, src_pitch, dst, dst_h, dst_w, dst_t, border, border_value,
                                   norm);
    if (s != KR_OK)
        return s;
    ImageJob j;
    std::memset(&j, 0, sizeof j);
    set_source(j, src, src_h, src_w, 3, KR_U8, src_pitch);
    j.dst = dst; j.dh = dst_h; j.dw = dst_w;
    const hipError_t err = launch_resize_gray(dst_t, j, make_gray_epilogue(border, border_value, norm),
                                              (hipStream_t)stream);
    if (err != hipSuccess)
        return fail(KR_ERR_HIP, "resize launch failed: %s", hipGetErrorString(err));
    return KR_OK;
}

kr_status kr_warp_affine_gray(const void *src, int src_h, int src_w, size_t src_pitch, void *dst, int dst_h,
                              int dst_w, kr_dtype dst_t, const double m[6], int flags, kr_border border,
                              float border_value, const kr_normalize *norm, void *stream)
{
    clear_error();
    kr_status s = check_gray(src, src_h, src_w, src_pitch, dst, dst_h, dst_w, dst_t, border, border_value, norm);
    if (s != KR_OK)
        return s;
    if (flags & ~KR_WARP_INVERSE_MAP)
        return fail(KR_ERR_INVALID_ARGUMENT, "unknown warp flags 0x%x", flags);
    ImageJob j;
    std::memset(&j, 0, sizeof j);
    s = check_matrix(m, flags, j.inv);
    if (s != KR_OK)
        return s;
    set_source(j, src, src_h, src_w, 3, KR_U8, src_pitch);
    j.dst = dst; j.dh = dst_h; j.dw = dst_w;
    const hipError_t err = launch_tiled(OP_WARP, 3, dst_t, j, make_gray_epilogue(border, border_value, norm),
                                        (hipStream_t)stream);
    if (err != hipSuccess)
        return fail(KR_ERR_HIP, "warp launch failed: %s", hipGetErrorString(err));
    return KR_OK;
}

kr_status kr_resize_nearest_view(const void *src, int src_h, int src_w, size_t src_pitch, int c, kr_dtype src_t,
                                 void *dst, int dst_h, int dst_w, kr_dtype dst_t, const kr_normalize *norm,
                                 void *stream)
{
    clear_error();
    kr_status s = check_common(src, src_h, src_w, c, src_t, dst, dst_h, dst_w, dst_t, KR_BORDER_REPLICATE, 0.0f,
                               norm, src_pitch);
    if (s != KR_OK)
        return s;
    ImageJob j;
    std::memset(&j, 0, sizeof j);
    set_source(j, src, src_h, src_w, c, src_t, src_pitch);
    j.dst = dst; j.dh = dst_h; j.dw = dst_w;
    const Epilogue e = make_epilogue(c, KR_BORDER_REPLICATE, 0.0f, norm);
    const hipError_t err = launch_nearest(c, src_t, dst_t, j, e, (hipStream_t)stream);
    if (err != hipSuccess)
        return fail(KR_ERR_HIP, "nearest resize launch failed: %s", hipGetErrorString(err));
    return KR_OK;
}

kr_status kr_resize_nearest(const void *src, int src_h, int src_w, int c, kr_dtype src_t, void *dst, int dst_h,
                            int dst_w, kr_dtype dst_t, const kr_normalize *norm, void *stream)
{
    return kr_resize_nearest_view(src, src_h, src_w, 0, c, src_t, dst, dst_h, dst_w, dst_t, norm, stream);
}

kr_status kr_flip_view(const void *src, int h, int w, size_t src_pitch, int c, kr_dtype t, void *dst, int flip_x,
                       int flip_y, void *stream)
{
    clear_error();
    kr_status s = check_common(src, h, w, c, t, dst, h, w, t, KR_BORDER_REPLICATE, 0.0f, nullptr, src_pitch);
    if (s != KR_OK)
        return s;
    if ((flip_x != 0 && flip_x != 1) || (flip_y != 0 && flip_y != 1))
        return fail(KR_ERR_INVALID_ARGUMENT, "flip flags must be 0 or 1");
    ImageJob j;
    std::memset(&j, 0, sizeof j);
    set_source(j, src, h, w, c, t, src_pitch);
    j.dst = dst; j.dh = h; j.dw = w;
    const hipError_t err = launch_flip(c, t, j, flip_x, flip_y, (hipStream_t)stream);
    if (err != hipSuccess)
        return fail(KR_ERR_HIP, "flip launch failed: %s", hipGetErrorString(err));
    return KR_OK;
}

kr_status kr_flip(const void *src, int h, int w, int c, kr_dtype t, void *dst, int flip_x, int flip_y, void *stream)
{
    return kr_flip_view(src, h, w, 0, c, t, dst, flip_x, flip_y, stream);
}

kr_status kr_rgb_to_gray_view(const void *src, int h, int w, size_t src_pitch, kr_dtype src_t, void *dst,
                              kr_dtype dst_t, const kr_normalize *norm, void *stream)
{
    clear_error();
    if (!((src_t == KR_U8 && dst_t == KR_U8) || (src_t == KR_U8 && dst_t == KR_F32) ||
          (src_t == KR_F32 && dst_t == KR_F32)))
        return fail(KR_ERR_UNSUPPORTED, "dtype pair (%d -> %d) not supported", (int)src_t, (int)dst_t);
    kr_status s = check_source(src, h, w, 3, src_t, src_pitch);
    if (s == KR_OK)
        s = check_image("dst", dst, h, w, 1);
    if (s != KR_OK)
        return s;
    if (norm) {
        if (dst_t != KR_F32)
            return fail(KR_ERR_INVALID_ARGUMENT, "normalisation needs an f32 destination");
        if (!std::isfinite(norm->mean[0]) || !std::isfinite(norm->std[0]) || norm->std[0] == 0.0f)
            return fail(KR_ERR_INVALID_ARGUMENT, "normalisation has a bad mean/std");
    }
    const uintptr_t s0 = reinterpret_cast<uintptr_t>(src), d0 = reinterpret_cast<uintptr_t>(dst);
    const uintptr_t s1 = range_end(src, source_span(h, w, 3, src_t, src_pitch));
    const uintptr_t d1 = range_end(dst, (size_t)h * (size_t)w * elem_size(dst_t));
    if (!s1 || !d1)
        return fail(KR_ERR_INVALID_ARGUMENT, "src or dst range wraps past the end of the address space");
    if (s0 < d1 && d0 < s1)
        return fail(KR_ERR_INVALID_ARGUMENT, "src and dst overlap");
    ImageJob j;
    std::memset(&j, 0, sizeof j);
    set_source(j, src, h, w, 3, src_t, src_pitch);
    j.dst = dst; j.dh = h; j.dw = w;
    const Epilogue e = make_epilogue(1, KR_BORDER_REPLICATE, 0.0f, norm);
    const hipError_t err = launch_gray(src_t, dst_t, j, e, (hipStream_t)stream);
    if (err != hipSuccess)
        return fail(KR_ERR_HIP, "gray launch failed: %s", hipGetErrorString(err));
    return KR_OK;
}

kr_status kr_rgb_to_gray(const void *src, int h, int w, kr_dtype src_t, void *dst, kr_dtype dst_t,
                         const kr_normalize *norm, void *stream)
{
    return kr_rgb_to_gray_view(src, h, w, 0, src_t, dst, dst_t, norm, stream);
}

// Inverse of a 3x3 homography by the adjugate (fixed evaluation order:
// cofactors as differences of two rounded products, det = (m00 c00 +
// m01 c01) + m02 c02, entries divided by det).  Singular: det zero, not
// finite, or |det| <= 1e-12 max|m_ij|^3.
static kr_status invert_homography_impl(const double m[9], double inv[9])
{
    const double c00 = m[4] * m[8] - m[5] * m[7];
    const double c01 = m[5] * m[6] - m[3] * m[8];
    const double c02 = m[3] * m[7] - m[4] * m[6];
    const double det = (m[0] * c00 + m[1] * c01) + m[2] * c02;
    double mx = 0.0;
    for (int i = 0; i < 9; i++)
        mx = std::fmax(mx, std::fabs(m[i]));
    if (det == 0.0 || !std::isfinite(det) || std::fabs(det) <= 1e-12 * mx * mx * mx)
        return fail(KR_ERR_SINGULAR_MATRIX, "homography is singular (det %g)", det);
    const double c10 = m[2] * m[7] - m[1] * m[8];
    const double c11 = m[0] * m[8] - m[2] * m[6];
    const double c12 = m[1] * m[6] - m[0] * m[7];
    const double c20 = m[1] * m[5] - m[2] * m[4];
    const double c21 = m[2] * m[3] - m[0] * m[5];
    const double c22 = m[0] * m[4] - m[1] * m[3];
    inv[0] = c00 / det; inv[1] = c10 / det; inv[2] = c20 / det;
    inv[3] = c01 / det; inv[4] = c11 / det; inv[5] = c21 / det;
    inv[6] = c02 / det; inv[7] = c12 / det; inv[8] = c22 / det;
    return KR_OK;
}

kr_status kr_invert_homography(const double m[9], double inv[9])
{
    clear_error();
    if (!m || !inv)
        return fail(KR_ERR_INVALID_ARGUMENT, "NULL matrix pointer");
    for (int i = 0; i < 9; i++)
        if (!std::isfinite(m[i]))
            return fail(KR_ERR_SINGULAR_MATRIX, "matrix entry %d is not finite", i);
    return invert_homography_impl(m, inv);
}

kr_status kr_warp_perspective_view(const void *src, int src_h, int src_w, size_t src_pitch, int c, kr_dtype src_t,
                                   void *dst, int dst_h, int dst_w, kr_dtype dst_t, const double m[9], int flags,
                                   kr_border border, float border_value, const kr_normalize *norm, void *stream)
{
    clear_error();
    kr_status s = check_common(src, src_h, src_w, c, src_t, dst, dst_h, dst_w, dst_t, border, border_value, norm,
                               src_pitch);
    if (s != KR_OK)
        return s;
    if (flags & ~KR_WARP_INVERSE_MAP)
        return fail(KR_ERR_INVALID_ARGUMENT, "unknown warp flags 0x%x", flags);
    if (!m)
        return fail(KR_ERR_INVALID_ARGUMENT, "matrix pointer is NULL");
    double inv[9];
    for (int i = 0; i < 9; i++)
        if (!std::isfinite(m[i]))
            return fail(KR_ERR_SINGULAR_MATRIX, "matrix entry %d is not finite", i);
    if (flags & KR_WARP_INVERSE_MAP) {
        for (int i = 0; i < 9; i++)
            inv[i] = m[i];
    } else {
        s = invert_homography_impl(m, inv);
        if (s != KR_OK)
            return s;
    }
    ImageJob j;
    std::memset(&j, 0, sizeof j);
    set_source(j, src, src_h, src_w, c, src_t, src_pitch);
    j.dst = dst; j.dh = dst_h; j.dw = dst_w;
    for (int i = 0; i < 6; i++)
        j.inv[i] = inv[i];
    for (int i = 0; i < 3; i++)
        j.proj[i] = inv[6 + i];
    const Epilogue e = make_epilogue(c, border, border_value, norm);
    const hipError_t err = launch_persp(c, src_t, dst_t, j, e, (hipStream_t)stream);
    if (err != hipSuccess)
        return fail(KR_ERR_HIP, "perspective warp launch failed: %s", hipGetErrorString(err));
    return KR_OK;
}

kr_status kr_warp_perspective(const void *src, int src_h, int src_w, int c, kr_dtype src_t, void *dst, int dst_h,
                              int dst_w, kr_dtype dst_t, const double m[9], int flags, kr_border border,
                              float border_value, const kr_normalize *norm, void *stream)
{
    return kr_warp_perspective_view(src, src_h, src_w, 0, c, src_t, dst, dst_h, dst_w, dst_t, m, flags, border,
                                    border_value, norm, stream);
}

kr_status kr_invert_affine(const double m[6], double inv[6])
{
    clear_error();
    if (!m || !inv)
        return fail(KR_ERR_INVALID_ARGUMENT, "NULL matrix pointer");
    for (int i = 0; i < 6; i++)
        if (!std::isfinite(m[i]))
            return fail(KR_ERR_SINGULAR_MATRIX, "matrix entry %d is not finite", i);
    return invert_affine_impl(m, inv);
}

const char *kr_status_string(kr_status s)
{
    switch (s) {
    case KR_OK: return "ok";
    case KR_ERR_INVALID_ARGUMENT: return "invalid argument";
    case KR_ERR_UNSUPPORTED: return "unsupported";
    case KR_ERR_SINGULAR_MATRIX: return "singular matrix";
    case KR_ERR_WORKSPACE_TOO_SMALL: return "workspace too small";
    case KR_ERR_OUT_OF_BUDGET: return "out of budget";
    case KR_ERR_HIP: return "HIP error";
    }
    return "unknown status";
}

const char *kr_last_error(void) { return g_last_error.c_str(); }

kr_status kr_hbm_copy(void *dst, const void *src, size_t bytes, void *stream)
{
    clear_error();
    if (!dst || !src)
        return fail(KR_ERR_INVALID_ARGUMENT, "NULL pointer");
    if (reinterpret_cast<uintptr_t>(dst) % 16 || reinterpret_cast<uintptr_t>(src) % 16)
        return fail(KR_ERR_INVALID_ARGUMENT, "copy pointers must be 16-byte aligned");
    const uintptr_t s0 = reinterpret_cast<uintptr_t>(src), d0 = reinterpret_cast<uintptr_t>(dst);
    const uintptr_t s1 = range_end(src, bytes), d1 = range_end(dst, bytes);
    if (!s1 || !d1)
        return fail(KR_ERR_INVALID_ARGUMENT, "copy range wraps past the end of the address space");
    if (s0 < d1 && d0 < s1)
        return fail(KR_ERR_INVALID_ARGUMENT, "copy ranges overlap");
    if (bytes == 0)
        return KR_OK;
    const hipError_t err = launch_copy(dst, src, bytes, (hipStream_t)stream);
    if (err != hipSuccess)
        return fail(KR_ERR_HIP, "copy launch failed: %s", hipGetErrorString(err));
    return KR_OK;
}

kr_status kr_hbm_stream(void *dst, size_t dst_bytes, const void *src, size_t src_bytes, void *stream)
{
    clear_error();
    if (!dst || !src)
        return fail(KR_ERR_INVALID_ARGUMENT, "NULL pointer");
    if (reinterpret_cast<uintptr_t>(dst) % 16 || reinterpret_cast<uintptr_t>(src) % 16)
        return fail(KR_ERR_INVALID_ARGUMENT, "stream pointers must be 16-byte aligned");
    if (dst_bytes == 0 || src_bytes == 0 || dst_bytes % 16 || src_bytes % 16)
        return fail(KR_ERR_INVALID_ARGUMENT, "sizes must be positive multiples of 16");
    const size_t big = dst_bytes > src_bytes ? dst_bytes : src_bytes;
    const size_t small = dst_bytes > src_bytes ? src_bytes : dst_bytes;
    if (big % small)
        return fail(KR_ERR_INVALID_ARGUMENT, "size ratio is not a power of two");
    const size_t ratio = big / small;
    if (ratio & (ratio - 1))
        return fail(KR_ERR_INVALID_ARGUMENT, "size ratio is not a power of two");
    int lg = 0;
    while (((size_t)1 << lg) < ratio)
        lg++;
    if (src_bytes > dst_bytes && lg > 8)
        return fail(KR_ERR_INVALID_ARGUMENT, "at most 256 input chunks per output chunk");
    const uintptr_t s0 = reinterpret_cast<uintptr_t>(src), d0 = reinterpret_cast<uintptr_t>(dst);
    const uintptr_t s1 = range_end(src, src_bytes), d1 = range_end(dst, dst_bytes);
    if (!s1 || !d1)
        return fail(KR_ERR_INVALID_ARGUMENT, "stream range wraps past the end of the address space");
    if (s0 < d1 && d0 < s1)
        return fail(KR_ERR_INVALID_ARGUMENT, "stream ranges overlap");
    const hipError_t err = launch_stream(dst, dst_bytes / 16, src, src_bytes > dst_bytes ? lg : 0,
                                         dst_bytes > src_bytes ? lg : 0, (hipStream_t)stream);
    if (err != hipSuccess)
        return fail(KR_ERR_HIP, "stream launch failed: %s", hipGetErrorString(err));
    return KR_OK;
}

}  // extern "C"
