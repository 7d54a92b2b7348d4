"""Reference oracle for bilinear / nearest resize and affine warp -- TEST INFRASTRUCTURE.

Only ``tests/``, ``__graft_entry__.smoke()`` and the CPU-baseline leg of
``bench.py`` may import this package.  The product library never loads it and
the two share no code.

The arithmetic lives in ``kro.c`` (plain C, binary64 / exact integers); this
module only compiles it with gcc and marshals numpy arrays.  The definitions
(half-pixel centres, exact-rational resize coordinates, the binary64 fma chain
for the warp's inverse map, per-tap borders, 11-bit u8 weights) are stated in
the header of ``kro.c``.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "kro.c")
_LIB_PATH = os.path.join(_HERE, "libkro.so")
_lib = None

CONSTANT = 0
REPLICATE = 1


def build() -> str:
    """Compile kro.c into oracle/libkro.so (always recompiles)."""
    tmp = _LIB_PATH + ".tmp"
    cmd = ["gcc", "-O2", "-std=c11", "-ffp-contract=off", "-fopenmp", "-fPIC",
           "-shared", _SRC, "-o", tmp, "-lm"]
    subprocess.run(cmd, check=True)
    os.replace(tmp, _LIB_PATH)
    return _LIB_PATH


def _load():
    global _lib
    if _lib is not None:
        return _lib
    override = os.environ.get("KRO_LIB")  # a mutated build, for the pin-strength test
    if override:
        lib = ctypes.CDLL(override)
    else:
        if not os.path.exists(_LIB_PATH) or os.path.getmtime(_LIB_PATH) < os.path.getmtime(_SRC):
            build()
        lib = ctypes.CDLL(_LIB_PATH)
    vp, i, d = ctypes.c_void_p, ctypes.c_int, ctypes.c_double
    dp = ctypes.POINTER(ctypes.c_double)
    lib.kro_resize.argtypes = [vp, i, i, i, i, vp, i, i, i, i, d, dp, dp, i]
    lib.kro_resize.restype = i
    lib.kro_warp.argtypes = [vp, i, i, i, i, vp, i, i, i, dp, i, i, d, dp, dp, i]
    lib.kro_warp.restype = i
    lib.kro_resize_nearest.argtypes = [vp, i, i, i, i, vp, i, i, i, dp, dp, i]
    lib.kro_resize_nearest.restype = i
    lib.kro_flip.argtypes = [vp, i, i, i, i, vp, i, i]
    lib.kro_flip.restype = i
    lib.kro_rgb_to_gray.argtypes = [vp, i, i, i, vp, i, dp, dp, i]
    lib.kro_rgb_to_gray.restype = i
    lib.kro_invert_homography.argtypes = [dp, dp]
    lib.kro_invert_homography.restype = i
    lib.kro_warp_perspective.argtypes = [vp, i, i, i, i, vp, i, i, i, dp, i, i, d, dp, dp, i]
    lib.kro_warp_perspective.restype = i
    lib.kro_invert_affine.argtypes = [dp, dp]
    lib.kro_invert_affine.restype = i
    _lib = lib
    return lib


def _src_args(src: np.ndarray):
    if src.ndim == 2:
        src = src[:, :, None]
    if src.ndim != 3:
        raise ValueError("src must be HxW or HxWxC")
    src = np.ascontiguousarray(src)
    if src.dtype == np.uint8:
        st = 0
    elif src.dtype == np.float32:
        st = 1
    else:
        raise TypeError("src dtype must be uint8 or float32")
    return src, st


def _norm_args(mean, std, c):
    if mean is None:
        return None, None, None
    m = (ctypes.c_double * 4)(*[float(v) for v in list(mean)[:c]] + [0.0] * (4 - c))
    s = (ctypes.c_double * 4)(*[float(v) for v in list(std)[:c]] + [1.0] * (4 - c))
    return m, s, (m, s)


def resize(src: np.ndarray, dh: int, dw: int, out: str = "u8", border: int = REPLICATE,
           bval: float = 0.0, mean=None, std=None, threads: int = 1) -> np.ndarray:
    """Oracle bilinear resize.  ``out`` is "u8" (fixed-point path) or "f64"
    (the f32 path's values, reported in binary64)."""
    lib = _load()
    src, st = _src_args(src)
    h, w, c = src.shape
    if out == "u8":
        dst = np.zeros((dh, dw, c), np.uint8)
        ot = 0
    else:
        dst = np.zeros((dh, dw, c), np.float64)
        ot = 1
    m, s, _keep = _norm_args(mean, std, c)
    rc = lib.kro_resize(src.ctypes.data, h, w, c, st, dst.ctypes.data, dh, dw, ot,
                        border, float(bval), m, s, threads)
    if rc != 0:
        raise ValueError("kro_resize rejected its arguments")
    return dst


def resize_nearest(src: np.ndarray, dh: int, dw: int, out: str = "u8", mean=None, std=None,
                   threads: int = 1) -> np.ndarray:
    """Oracle nearest-neighbour resize (half-pixel centres).  ``out`` is "u8"
    (u8 sources: the copied samples) or "f64" (the f32 path's values)."""
    lib = _load()
    src, st = _src_args(src)
    h, w, c = src.shape
    if out == "u8":
        dst = np.zeros((dh, dw, c), np.uint8)
        ot = 0
    else:
        dst = np.zeros((dh, dw, c), np.float64)
        ot = 1
    m, s, _keep = _norm_args(mean, std, c)
    rc = lib.kro_resize_nearest(src.ctypes.data, h, w, c, st, dst.ctypes.data, dh, dw, ot, m, s, threads)
    if rc != 0:
        raise ValueError("kro_resize_nearest rejected its arguments")
    return dst


def flip(src: np.ndarray, flip_x: bool = True, flip_y: bool = False) -> np.ndarray:
    """Oracle flip: mirrors columns (flip_x) and/or rows (flip_y); same dtype."""
    lib = _load()
    src, st = _src_args(src)
    h, w, c = src.shape
    dst = np.zeros_like(src)
    if lib.kro_flip(src.ctypes.data, h, w, c, st, dst.ctypes.data, int(flip_x), int(flip_y)) != 0:
        raise ValueError("kro_flip rejected its arguments")
    return dst


def rgb_to_gray(src: np.ndarray, out: str = "u8", mean=None, std=None, threads: int = 1) -> np.ndarray:
    """Oracle RGB -> gray (BT.601): HxWx3 -> HxWx1, "u8" (14-bit fixed point)
    or "f64"."""
    lib = _load()
    src, st = _src_args(src)
    h, w, c = src.shape
    if c != 3:
        raise ValueError("rgb_to_gray needs 3 channels")
    dst = np.zeros((h, w, 1), np.uint8 if out == "u8" else np.float64)
    m, s, _keep = _norm_args(mean, std, 1)
    if lib.kro_rgb_to_gray(src.ctypes.data, h, w, st, dst.ctypes.data, 0 if out == "u8" else 1, m, s, threads) != 0:
        raise ValueError("kro_rgb_to_gray rejected its arguments")
    return dst


def warp(src: np.ndarray, m6, dh: int, dw: int, out: str = "u8", inverse: bool = False,
         border: int = CONSTANT, bval: float = 0.0, mean=None, std=None,
         threads: int = 1) -> np.ndarray:
    """Oracle bilinear affine warp.  ``m6`` is the row-major 2x3 matrix,
    source->destination unless ``inverse``."""
    lib = _load()
    src, st = _src_args(src)
    h, w, c = src.shape
    if out == "u8":
        dst = np.zeros((dh, dw, c), np.uint8)
        ot = 0
    else:
        dst = np.zeros((dh, dw, c), np.float64)
        ot = 1
    mm = (ctypes.c_double * 6)(*[float(v) for v in np.asarray(m6, np.float64).reshape(6)])
    nm, ns, _keep = _norm_args(mean, std, c)
    rc = lib.kro_warp(src.ctypes.data, h, w, c, st, dst.ctypes.data, dh, dw, ot, mm,
                      1 if inverse else 0, border, float(bval), nm, ns, threads)
    if rc != 0:
        raise ValueError("kro_warp rejected its arguments")
    return dst


def resize_gray(src: np.ndarray, dh: int, dw: int, out: str = "u8", border: int = REPLICATE,
                bval: float = 0.0, mean=None, std=None, threads: int = 1) -> np.ndarray:
    """Bilinear resize of an RGB image to one BT.601 gray channel, the
    resize followed by the RGB -> gray operator (paper Sec. III benchmarks
    both; the camera-stream listing of Sec. IV-B converts a captured frame
    to gray).  Reading: the fused form computes exactly that composition.
    u8: each channel interpolated and rounded to u8 (11-bit weights), then
    the 14-bit gray weights and their own rounding; f64: the unnormalised
    channel values, the gray combination, then (v / 255 - mean) / std with
    mean[0], std[0].  HxWx3 -> dh x dw x 1."""
    if out == "u8":
        return rgb_to_gray(resize(src, dh, dw, "u8", border, bval, threads=threads), "u8", threads=threads)
    return _gray_f64(resize(src, dh, dw, "f64", border, bval, threads=threads), mean, std)


def warp_gray(src: np.ndarray, m6, dh: int, dw: int, out: str = "u8", inverse: bool = False,
              border: int = CONSTANT, bval: float = 0.0, mean=None, std=None, threads: int = 1) -> np.ndarray:
    """Affine warp of an RGB image to one BT.601 gray channel: the warp
    followed by the RGB -> gray operator, with the same reading as
    resize_gray (u8: per-channel rounding, then the gray rounding)."""
    if out == "u8":
        return rgb_to_gray(warp(src, m6, dh, dw, "u8", inverse, border, bval, threads=threads), "u8",
                           threads=threads)
    return _gray_f64(warp(src, m6, dh, dw, "f64", inverse, border, bval, threads=threads), mean, std)


def _gray_f64(v: np.ndarray, mean, std) -> np.ndarray:
    """BT.601 luma of binary64 RGB values, in the order kro_rgb_to_gray uses
    (0.299 R + 0.587 G + 0.114 B), then the optional normalisation."""
    g = 0.299 * v[..., 0] + 0.587 * v[..., 1] + 0.114 * v[..., 2]
    if mean is not None:
        g = (g / 255.0 - float(list(mean)[0])) / float(list(std)[0])
    return g[..., None]


def invert_affine(m6) -> np.ndarray:
    """Inverse of a 2x3 affine map by the fixed formula in kro.c."""
    lib = _load()
    mm = (ctypes.c_double * 6)(*[float(v) for v in np.asarray(m6, np.float64).reshape(6)])
    out = (ctypes.c_double * 6)()
    if lib.kro_invert_affine(mm, out) != 0:
        raise ValueError("singular affine matrix")
    return np.array(list(out), np.float64)


def invert_homography(m9):
    """The oracle's inverse of a 3x3 homography (adjugate formula)."""
    lib = _load()
    a = (ctypes.c_double * 9)(*[float(v) for v in np.asarray(m9, np.float64).reshape(9)])
    out = (ctypes.c_double * 9)()
    if lib.kro_invert_homography(a, out) != 0:
        raise ValueError("singular homography")
    return np.array(list(out))


def warp_perspective(src: np.ndarray, m9, dh: int, dw: int, out: str = "u8", inverse: bool = False,
                     border: int = CONSTANT, bval: float = 0.0, mean=None, std=None, threads: int = 1) -> np.ndarray:
    """Oracle bilinear perspective warp.  ``m9`` is the row-major 3x3 homography,
    source->destination unless ``inverse``."""
    lib = _load()
    src, st = _src_args(src)
    h, w, c = src.shape
    if out == "u8":
        dst = np.zeros((dh, dw, c), np.uint8)
        ot = 0
    else:
        dst = np.zeros((dh, dw, c), np.float64)
        ot = 1
    mm = (ctypes.c_double * 9)(*[float(v) for v in np.asarray(m9, np.float64).reshape(9)])
    m, s, _keep = _norm_args(mean, std, c)
    rc = lib.kro_warp_perspective(src.ctypes.data, h, w, c, st, dst.ctypes.data, dh, dw, ot, mm, int(inverse),
                                  border, float(bval), m, s, threads)
    if rc != 0:
        raise ValueError("kro_warp_perspective rejected its arguments")
    return dst
