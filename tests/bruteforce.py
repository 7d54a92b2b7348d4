"""Exact-rational brute force of the resampling definitions (test-only).

Written independently of the C oracle: every coordinate, weight and blend is
carried in ``fractions.Fraction``; a binary64 fma is emulated as the correctly
rounded conversion of the exact a*x + t (``float(Fraction)`` rounds to
nearest-even).  Python float arithmetic is IEEE binary64 without contraction,
so the fixed inverse-map formula is reproduced operation by operation.  Meant
for inputs up to about 64x64.
"""
from __future__ import annotations

import math
from fractions import Fraction

import numpy as np


def fma(a: float, x: float, t: float) -> float:
    return float(Fraction(a) * Fraction(x) + Fraction(t))


def rne(q: Fraction) -> int:
    """Round a rational to the nearest integer, ties to even (Python's round)."""
    return round(q)


def invert_affine(m):
    a, b, c, d, e, f = [float(v) for v in np.asarray(m, np.float64).reshape(6)]
    det = a * e - b * d
    A, B, D, E = e / det, -b / det, -d / det, a / det
    C = -(A * c + B * f)
    F = -(D * c + E * f)
    return (A, B, C, D, E, F)


def _tap(src, x, y, ch, border, bval):
    h, w = src.shape[0], src.shape[1]
    if 0 <= x < w and 0 <= y < h:
        return Fraction(src[y, x, ch].item())
    if border == 0:
        return Fraction(bval)
    return Fraction(src[min(max(y, 0), h - 1), min(max(x, 0), w - 1), ch].item())


def _blend(src, x0, y0, fx: Fraction, fy: Fraction, out, border, bval, mean, std):
    c = src.shape[2]
    res = []
    for ch in range(c):
        taps = [[_tap(src, x0 + j, y0 + i, ch, border, bval) for j in (0, 1)] for i in (0, 1)]
        if out == "u8":
            wx1 = rne(2048 * fx)
            wy1 = rne(2048 * fy)
            wx = (2048 - wx1, wx1)
            wy = (2048 - wy1, wy1)
            acc = sum(wy[i] * wx[j] * taps[i][j] for i in (0, 1) for j in (0, 1))
            res.append(math.floor((acc + 2 ** 21) / Fraction(2 ** 22)))
        else:
            wx = (1 - fx, fx)
            wy = (1 - fy, fy)
            v = sum(wy[i] * wx[j] * taps[i][j] for i in (0, 1) for j in (0, 1))
            if mean is not None:
                v = (v / 255 - Fraction(mean[ch])) / Fraction(std[ch])
            res.append(float(v))
    return res


def resize(src: np.ndarray, dh: int, dw: int, out="u8", border=1, bval=0, mean=None, std=None):
    """Half-pixel-centre bilinear resize: source x = (dx + 1/2) W/dw - 1/2 exactly."""
    h, w, c = src.shape
    dst = np.zeros((dh, dw, c), np.uint8 if out == "u8" else np.float64)
    for dy in range(dh):
        ys = (Fraction(2 * dy + 1, 2)) * Fraction(h, dh) - Fraction(1, 2)
        y0 = math.floor(ys)
        for dx in range(dw):
            xs = (Fraction(2 * dx + 1, 2)) * Fraction(w, dw) - Fraction(1, 2)
            x0 = math.floor(xs)
            dst[dy, dx, :] = _blend(src, x0, y0, xs - x0, ys - y0, out, border, bval, mean, std)
    return dst


def warp(src: np.ndarray, m, dh: int, dw: int, out="u8", inverse=False, border=0, bval=0,
         mean=None, std=None):
    """Affine warp: per destination pixel centre (x, y), xs = fma(A, x, fma(B, y, C)),
    ys = fma(D, x, fma(E, y, F)) in binary64, clamped to [-2, W+1] x [-2, H+1]."""
    h, w, c = src.shape
    A, B, C, D, E, F = ([float(v) for v in np.asarray(m, np.float64).reshape(6)] if inverse
                        else invert_affine(m))
    dst = np.zeros((dh, dw, c), np.uint8 if out == "u8" else np.float64)
    for y in range(dh):
        for x in range(dw):
            xs = fma(A, float(x), fma(B, float(y), C))
            ys = fma(D, float(x), fma(E, float(y), F))
            xs = min(max(xs, -2.0), w + 1.0)
            ys = min(max(ys, -2.0), h + 1.0)
            fxs, fys = Fraction(xs), Fraction(ys)
            x0, y0 = math.floor(fxs), math.floor(fys)
            dst[y, x, :] = _blend(src, x0, y0, fxs - x0, fys - y0, out, border, bval, mean, std)
    return dst


def resize_nearest(src: np.ndarray, dh: int, dw: int, out="u8", mean=None, std=None):
    """Nearest neighbour with half-pixel centres, from the definition: the
    sample whose cell contains the output centre, source coordinate
    (d + 1/2) * n_in / n_out as an exact Fraction, then its floor."""
    h, w, c = src.shape
    res = np.zeros((dh, dw, c), np.uint8 if out == "u8" else np.float64)
    for dy in range(dh):
        sy = math.floor((Fraction(dy) + Fraction(1, 2)) * Fraction(h, dh))
        for dx in range(dw):
            sx = math.floor((Fraction(dx) + Fraction(1, 2)) * Fraction(w, dw))
            for ch in range(c):
                v = src[sy, sx, ch]
                if out == "u8":
                    res[dy, dx, ch] = v
                else:
                    v = float(v)
                    res[dy, dx, ch] = (v / 255.0 - mean[ch]) / std[ch] if mean is not None else v
    return res


def invert_homography(m):
    """Adjugate inverse of a 3x3 homography in binary64, each cofactor a
    difference of two rounded products, det = (m00 c00 + m01 c01) + m02 c02,
    each inverse entry the cofactor divided by det."""
    a = [float(v) for v in np.asarray(m, np.float64).reshape(9)]
    c00 = a[4] * a[8] - a[5] * a[7]
    c01 = a[5] * a[6] - a[3] * a[8]
    c02 = a[3] * a[7] - a[4] * a[6]
    det = (a[0] * c00 + a[1] * c01) + a[2] * c02
    c10 = a[2] * a[7] - a[1] * a[8]
    c11 = a[0] * a[8] - a[2] * a[6]
    c12 = a[1] * a[6] - a[0] * a[7]
    c20 = a[1] * a[5] - a[2] * a[4]
    c21 = a[2] * a[3] - a[0] * a[5]
    c22 = a[0] * a[4] - a[1] * a[3]
    return [c00 / det, c10 / det, c20 / det, c01 / det, c11 / det, c21 / det, c02 / det, c12 / det, c22 / det]


def warp_perspective(src: np.ndarray, m, dh: int, dw: int, out="u8", inverse=False, border=0, bval=0,
                     mean=None, std=None):
    """Homography warp: w = fma(G, x, fma(H, y, I)); xs = fma(A, x, fma(B, y, C)) / w,
    ys likewise, each quotient the binary64 rounding of the exact ratio; a
    not-a-number coordinate reads as -2; then the affine warp's clamp and taps."""
    h, w, c = src.shape
    inv = [float(v) for v in np.asarray(m, np.float64).reshape(9)] if inverse else invert_homography(m)
    dst = np.zeros((dh, dw, c), np.uint8 if out == "u8" else np.float64)
    for y in range(dh):
        for x in range(dw):
            den = fma(inv[6], float(x), fma(inv[7], float(y), inv[8]))
            num = [fma(inv[0], float(x), fma(inv[1], float(y), inv[2])),
                   fma(inv[3], float(x), fma(inv[4], float(y), inv[5]))]
            q = []
            for v in num:
                if den == 0.0:
                    r = math.copysign(math.inf, v) * math.copysign(1.0, den) if v != 0.0 else -2.0
                else:
                    r = float(Fraction(v) / Fraction(den))
                q.append(r)
            xs = min(max(q[0], -2.0), w + 1.0)
            ys = min(max(q[1], -2.0), h + 1.0)
            fxs, fys = Fraction(xs), Fraction(ys)
            x0, y0 = math.floor(fxs), math.floor(fys)
            dst[y, x, :] = _blend(src, x0, y0, fxs - x0, fys - y0, out, border, bval, mean, std)
    return dst
