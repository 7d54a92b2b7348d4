// kr_api_internal.h -- host-side helpers shared by libkr's ABI translation
// units (validation, error state, parameter setup).
#pragma once

#include <cstdarg>

#include "kr_internal.h"

namespace kr {

constexpr int KR_MAX_DIM = 32767;

kr_status fail(kr_status s, const char *fmt, ...);
void clear_error();
kr_status check_image(const char *what, const void *p, int h, int w, int c);
// src_pitch: bytes between source rows, 0 for a contiguous source.
kr_status check_common(const void *src, int sh, int sw, int c, kr_dtype st, void *dst, int dh, int dw,
                       kr_dtype dt, kr_border border, float bval, const kr_normalize *norm, size_t src_pitch = 0);
// A source given as a view into a larger buffer (pitch bytes between rows; 0
// = contiguous): pitch a whole number of pixels and at least one row, first
// pixel a whole number of pixels past a 16-byte boundary.
kr_status check_source(const void *src, int h, int w, int c, kr_dtype st, size_t pitch);
// Fill j.src, sh, sw, sp, sk for a source that passed check_source.
void set_source(ImageJob &j, const void *src, int h, int w, int c, kr_dtype st, size_t pitch);
// Bytes from a source's first byte to its last one, plus one.
size_t source_span(int h, int w, int c, kr_dtype st, size_t pitch);
// One past the last byte of [p, p + n), or 0 if the range wraps past the top
// of the address space (no such buffer exists: the caller rejects it).
inline uintptr_t range_end(const void *p, size_t n)
{
    const uintptr_t a = reinterpret_cast<uintptr_t>(p), e = a + n;
    return e < a ? 0 : e;
}
Epilogue make_epilogue(int c, kr_border border, float bval, const kr_normalize *norm);
kr_status check_matrix(const double m[6], int flags, double inv[6]);
kr_status invert_affine_impl(const double m[6], double inv[6]);
// Tuner scrub buffer: NULL, or 16-byte aligned and >= 32 bytes.
kr_status check_scrub(const void *scrub, size_t bytes);

}  // namespace kr
