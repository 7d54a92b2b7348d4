"""Thin ctypes binding over libkr.so (include/kr.h).

Argument marshalling only: every step of resampling runs in the library's HIP
kernels.  torch tensors supply device memory and streams.  The library is
loaded on first use; if it has not been built this raises ``KrError`` -- there
is no fallback path.
"""
from __future__ import annotations

import ctypes
import os

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libkr.so")

# kr_status
OK = 0
ERR_INVALID_ARGUMENT = 1
ERR_UNSUPPORTED = 2
ERR_SINGULAR_MATRIX = 3
ERR_WORKSPACE_TOO_SMALL = 4
ERR_OUT_OF_BUDGET = 5
ERR_HIP = 6
# kr_dtype
U8 = 0
F32 = 1
# kr_border
CONSTANT = 0
REPLICATE = 1
# flags / ops
WARP_INVERSE_MAP = 1
OP_RESIZE = 0
OP_WARP = 1
LAYOUT_HWC = 0
LAYOUT_CHW = 1
NOALLOC_MAX_ITEMS = 4096  # kr.h KR_NOALLOC_MAX_ITEMS


class KrError(RuntimeError):
    def __init__(self, status: int, message: str):
        super().__init__(f"kr status {status}: {message}")
        self.status = status


class Normalize(ctypes.Structure):
    _fields_ = [("mean", ctypes.c_float * 4), ("std", ctypes.c_float * 4)]


class BatchItem(ctypes.Structure):
    _fields_ = [("op", ctypes.c_int), ("src", ctypes.c_void_p), ("src_h", ctypes.c_int),
                ("src_w", ctypes.c_int), ("dst", ctypes.c_void_p), ("dst_h", ctypes.c_int),
                ("dst_w", ctypes.c_int), ("m", ctypes.c_double * 6), ("flags", ctypes.c_int),
                ("src_pitch", ctypes.c_size_t)]


_lib = None


def lib():
    """The loaded libkr.so with argument types declared."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise KrError(-1, f"{LIB_PATH} is not built; run `python -m paper_2505_12425_amd.build`")
    L = ctypes.CDLL(LIB_PATH)
    vp, i, f, d = ctypes.c_void_p, ctypes.c_int, ctypes.c_float, ctypes.c_double
    npp = ctypes.POINTER(Normalize)
    dp = ctypes.POINTER(ctypes.c_double)
    L.kr_resize_bilinear.argtypes = [vp, i, i, i, i, vp, i, i, i, i, f, npp, vp]
    L.kr_resize_bilinear.restype = i
    L.kr_warp_affine.argtypes = [vp, i, i, i, i, vp, i, i, i, dp, i, i, f, npp, vp]
    L.kr_warp_affine.restype = i
    L.kr_resize_nearest.argtypes = [vp, i, i, i, i, vp, i, i, i, npp, vp]
    L.kr_resize_nearest.restype = i
    L.kr_warp_perspective.argtypes = [vp, i, i, i, i, vp, i, i, i, dp, i, i, f, npp, vp]
    L.kr_warp_perspective.restype = i
    L.kr_resize_bilinear_gray.argtypes = [vp, i, i, ctypes.c_size_t, vp, i, i, i, i, f, npp, vp]
    L.kr_resize_bilinear_gray.restype = i
    L.kr_warp_affine_gray.argtypes = [vp, i, i, ctypes.c_size_t, vp, i, i, i, dp, i, i, f, npp, vp]
    L.kr_warp_affine_gray.restype = i
    sz_ = ctypes.c_size_t
    L.kr_resize_bilinear_view.argtypes = [vp, i, i, sz_, i, i, vp, i, i, i, i, f, npp, vp]
    L.kr_resize_bilinear_view.restype = i
    L.kr_warp_affine_view.argtypes = [vp, i, i, sz_, i, i, vp, i, i, i, dp, i, i, f, npp, vp]
    L.kr_warp_affine_view.restype = i
    L.kr_warp_perspective_view.argtypes = [vp, i, i, sz_, i, i, vp, i, i, i, dp, i, i, f, npp, vp]
    L.kr_warp_perspective_view.restype = i
    L.kr_resize_nearest_view.argtypes = [vp, i, i, sz_, i, i, vp, i, i, i, npp, vp]
    L.kr_resize_nearest_view.restype = i
    L.kr_flip_view.argtypes = [vp, i, i, sz_, i, i, vp, i, i, vp]
    L.kr_flip_view.restype = i
    L.kr_rgb_to_gray_view.argtypes = [vp, i, i, sz_, i, vp, i, npp, vp]
    L.kr_rgb_to_gray_view.restype = i
    L.kr_invert_homography.argtypes = [dp, dp]
    L.kr_invert_homography.restype = i
    L.kr_flip.argtypes = [vp, i, i, i, i, vp, i, i, vp]
    L.kr_flip.restype = i
    L.kr_rgb_to_gray.argtypes = [vp, i, i, i, vp, i, npp, vp]
    L.kr_rgb_to_gray.restype = i
    L.kr_invert_affine.argtypes = [dp, dp]
    L.kr_invert_affine.restype = i
    L.kr_status_string.argtypes = [i]
    L.kr_status_string.restype = ctypes.c_char_p
    L.kr_last_error.argtypes = []
    L.kr_last_error.restype = ctypes.c_char_p
    L.kr_hbm_copy.argtypes = [vp, vp, ctypes.c_size_t, vp]
    L.kr_hbm_copy.restype = i
    L.kr_hbm_stream.argtypes = [vp, ctypes.c_size_t, vp, ctypes.c_size_t, vp]
    L.kr_hbm_stream.restype = i
    if hasattr(L, "kr_resize_batch"):
        bip = ctypes.POINTER(BatchItem)
        L.kr_resize_batch_workspace_size.argtypes = [i]
        L.kr_resize_batch_workspace_size.restype = ctypes.c_size_t
        L.kr_resize_batch.argtypes = [bip, i, i, i, i, i, f, npp, vp, ctypes.c_size_t, vp]
        L.kr_resize_batch.restype = i
        L.kr_batch_plan_create.argtypes = [bip, i, i, i, i, i, f, npp, ctypes.POINTER(vp)]
        L.kr_batch_plan_create.restype = i
        L.kr_resize_batch_ex.argtypes = [bip, i, i, i, i, i, f, npp, i, vp, ctypes.c_size_t, vp]
        L.kr_resize_batch_ex.restype = i
        L.kr_resize_batch_noalloc.argtypes = [bip, i, i, i, i, i, f, npp, i, vp]
        L.kr_resize_batch_noalloc.restype = i
        L.kr_batch_plan_create_ex.argtypes = [bip, i, i, i, i, i, f, npp, i, ctypes.POINTER(vp)]
        L.kr_batch_plan_create_ex.restype = i
        L.kr_batch_plan_launch.argtypes = [vp, vp]
        L.kr_batch_plan_launch.restype = i
        L.kr_batch_plan_destroy.argtypes = [vp]
        L.kr_batch_plan_destroy.restype = None
    if hasattr(L, "kr_autotune_image"):
        cp, sz = ctypes.c_char_p, ctypes.c_size_t
        L.kr_autotune_image.argtypes = [i, vp, i, i, i, i, vp, i, i, i, dp, i, i, f, npp, i, vp, sz, vp, cp, sz]
        L.kr_autotune_image.restype = i
        L.kr_autotune_batch.argtypes = [ctypes.POINTER(BatchItem), i, i, i, i, i, f, npp, vp, sz, i, vp, sz, vp,
                                        cp, sz]
        L.kr_autotune_batch.restype = i
        L.kr_autotune_save.argtypes = [cp, sz]
        L.kr_autotune_save.restype = sz
        L.kr_autotune_load.argtypes = [cp]
        L.kr_autotune_load.restype = i
        L.kr_autotune_clear.argtypes = []
        L.kr_autotune_clear.restype = None
        L.kr_build_key.argtypes = []
        L.kr_build_key.restype = cp
    _lib = L
    return L


def last_error() -> str:
    return lib().kr_last_error().decode()


def check(status: int) -> None:
    if status != OK:
        raise KrError(status, last_error())


def _normalize(mean, std, c: int):
    if mean is None:
        return None
    n = Normalize()
    for k in range(c):
        n.mean[k] = float(mean[k])
        n.std[k] = float(std[k])
    for k in range(c, 4):
        n.std[k] = 1.0
    return ctypes.pointer(n)


def _m6(m):
    vals = [float(v) for v in (m.reshape(-1).tolist() if hasattr(m, "reshape") else m)]
    if len(vals) != 6:
        raise ValueError("affine matrix needs 6 entries (row-major 2x3)")
    return (ctypes.c_double * 6)(*vals)


def _image(t):
    """(pointer, H, W, C, kr_dtype) of a contiguous HWC (or HW) device tensor."""
    import torch
    if not t.is_cuda:
        raise ValueError("tensor must live on the GPU")
    if not t.is_contiguous():
        raise ValueError("tensor must be contiguous HWC")
    if t.dtype == torch.uint8:
        dt = U8
    elif t.dtype == torch.float32:
        dt = F32
    else:
        raise TypeError(f"unsupported dtype {t.dtype}")
    if t.dim() == 2:
        h, w, c = t.shape[0], t.shape[1], 1
    elif t.dim() == 3:
        h, w, c = t.shape
    else:
        raise ValueError("tensor must be HxW or HxWxC")
    return t.data_ptr(), int(h), int(w), int(c), dt


def _dtype(t) -> int:
    import torch
    if t.dtype == torch.uint8:
        return U8
    if t.dtype == torch.float32:
        return F32
    raise TypeError(f"unsupported dtype {t.dtype}")


def _source(t):
    """(pointer, H, W, pitch bytes, C, kr_dtype) of an HWC (or HW) device tensor
    that may be a view: pixels and channels packed (channel stride 1, pixel
    stride C), rows any whole number of pixels apart.  pitch is 0 for a
    contiguous tensor that starts on a 16-byte boundary (the plain entry
    points); anything else goes through the view entry points."""
    if t.is_contiguous() and t.data_ptr() % 16 == 0:
        ptr, h, w, c, dt = _image(t)
        return ptr, h, w, 0, c, dt
    if not t.is_cuda:
        raise ValueError("tensor must live on the GPU")
    if t.dim() not in (2, 3):
        raise ValueError("tensor must be HxW or HxWxC")
    c = 1 if t.dim() == 2 else int(t.shape[2])
    if t.stride(-1) != 1 or (t.dim() == 3 and t.stride(1) != c):
        raise ValueError("source view must have packed pixels (channel stride 1, pixel stride C)")
    return (t.data_ptr(), int(t.shape[0]), int(t.shape[1]), int(t.stride(0)) * t.element_size(), c, _dtype(t))


def _stream(stream):
    if stream is not None:
        return stream.cuda_stream if hasattr(stream, "cuda_stream") else stream
    import torch
    return torch.cuda.current_stream().cuda_stream


def resize(src, dst, border: int = REPLICATE, border_value: float = 0.0, mean=None, std=None,
           stream=None) -> None:
    """kr_resize_bilinear on torch tensors: src HWC u8/f32 -> dst HWC (its size is the target)."""
    sp, sh, sw, pitch, c, st = _source(src)
    dp_, dh, dw, dc, dt = _image(dst)
    if dc != c:
        raise ValueError("src and dst channel counts differ")
    args = (dp_, dh, dw, dt, border, float(border_value), _normalize(mean, std, c), _stream(stream))
    if pitch:
        check(lib().kr_resize_bilinear_view(sp, sh, sw, pitch, c, st, *args))
    else:
        check(lib().kr_resize_bilinear(sp, sh, sw, c, st, *args))


def resize_nearest(src, dst, mean=None, std=None, stream=None) -> None:
    """kr_resize_nearest on torch tensors: src HWC -> dst HWC (its size is the target)."""
    sp, sh, sw, pitch, c, st = _source(src)
    dp_, dh, dw, dc, dt = _image(dst)
    if dc != c:
        raise ValueError("src and dst channel counts differ")
    args = (dp_, dh, dw, dt, _normalize(mean, std, c), _stream(stream))
    if pitch:
        check(lib().kr_resize_nearest_view(sp, sh, sw, pitch, c, st, *args))
    else:
        check(lib().kr_resize_nearest(sp, sh, sw, c, st, *args))


def flip(src, dst, flip_x: bool = True, flip_y: bool = False, stream=None) -> None:
    """kr_flip on torch tensors of the same shape and dtype (src may be a view)."""
    sp, h, w, pitch, c, st = _source(src)
    dp_, dh, dw, dc, dt = _image(dst)
    if (dh, dw, dc, dt) != (h, w, c, st):
        raise ValueError("flip needs src and dst of the same shape and dtype")
    if pitch:
        check(lib().kr_flip_view(sp, h, w, pitch, c, st, dp_, int(flip_x), int(flip_y), _stream(stream)))
    else:
        check(lib().kr_flip(sp, h, w, c, st, dp_, int(flip_x), int(flip_y), _stream(stream)))


def rgb_to_gray(src, dst, mean=None, std=None, stream=None) -> None:
    """kr_rgb_to_gray: src HxWx3 (may be a view) -> dst HxW(x1)."""
    sp, h, w, pitch, c, st = _source(src)
    dp_, dh, dw, dc, dt = _image(dst)
    if c != 3 or dc != 1 or (dh, dw) != (h, w):
        raise ValueError("rgb_to_gray needs HxWx3 -> HxWx1")
    if pitch:
        check(lib().kr_rgb_to_gray_view(sp, h, w, pitch, st, dp_, dt, _normalize(mean, std, 1), _stream(stream)))
    else:
        check(lib().kr_rgb_to_gray(sp, h, w, st, dp_, dt, _normalize(mean, std, 1), _stream(stream)))


def warp_affine(src, dst, m, inverse: bool = False, border: int = CONSTANT, border_value: float = 0.0,
                mean=None, std=None, stream=None) -> None:
    """kr_warp_affine on torch tensors; m is the row-major 2x3 map (source->destination
    unless inverse)."""
    sp, sh, sw, pitch, c, st = _source(src)
    dp_, dh, dw, dc, dt = _image(dst)
    if dc != c:
        raise ValueError("src and dst channel counts differ")
    args = (dp_, dh, dw, dt, _m6(m), WARP_INVERSE_MAP if inverse else 0, border, float(border_value),
            _normalize(mean, std, c), _stream(stream))
    if pitch:
        check(lib().kr_warp_affine_view(sp, sh, sw, pitch, c, st, *args))
    else:
        check(lib().kr_warp_affine(sp, sh, sw, c, st, *args))


def resize_gray(src, dst, border: int = REPLICATE, border_value: float = 0.0, mean=None, std=None,
                stream=None) -> None:
    """kr_resize_bilinear_gray: RGB u8 source (contiguous or a view) -> one
    gray channel (HxWx1 u8 or f32) in one pass."""
    sp, sh, sw, pitch, c, st = _source(src)
    dp_, dh, dw, dc, dt = _image(dst)
    if c != 3 or st != U8 or dc != 1:
        raise ValueError("resize_gray takes an RGB u8 source and a one-channel destination")
    check(lib().kr_resize_bilinear_gray(sp, sh, sw, pitch, dp_, dh, dw, dt, border, float(border_value),
                                        _normalize(mean, std, 1), _stream(stream)))


def warp_affine_gray(src, dst, m, inverse: bool = False, border: int = CONSTANT, border_value: float = 0.0,
                     mean=None, std=None, stream=None) -> None:
    """kr_warp_affine_gray: RGB u8 source -> one gray channel, in one pass."""
    sp, sh, sw, pitch, c, st = _source(src)
    dp_, dh, dw, dc, dt = _image(dst)
    if c != 3 or st != U8 or dc != 1:
        raise ValueError("warp_affine_gray takes an RGB u8 source and a one-channel destination")
    check(lib().kr_warp_affine_gray(sp, sh, sw, pitch, dp_, dh, dw, dt, _m6(m), WARP_INVERSE_MAP if inverse else 0,
                                    border, float(border_value), _normalize(mean, std, 1), _stream(stream)))


def _m9(m):
    vals = [float(v) for v in (m.reshape(-1).tolist() if hasattr(m, "reshape") else m)]
    if len(vals) != 9:
        raise ValueError("homography must have 9 entries")
    return (ctypes.c_double * 9)(*vals)


def warp_perspective(src, dst, m, inverse: bool = False, border: int = CONSTANT, border_value: float = 0.0,
                     mean=None, std=None, stream=None) -> None:
    """kr_warp_perspective on torch tensors; m is the row-major 3x3 homography
    (source->destination unless inverse)."""
    sp, sh, sw, pitch, c, st = _source(src)
    dp_, dh, dw, dc, dt = _image(dst)
    if dc != c:
        raise ValueError("src and dst channel counts differ")
    args = (dp_, dh, dw, dt, _m9(m), WARP_INVERSE_MAP if inverse else 0, border, float(border_value),
            _normalize(mean, std, c), _stream(stream))
    if pitch:
        check(lib().kr_warp_perspective_view(sp, sh, sw, pitch, c, st, *args))
    else:
        check(lib().kr_warp_perspective(sp, sh, sw, c, st, *args))


def invert_homography(m):
    """kr_invert_homography: the library's inverse of a 3x3 homography."""
    out = (ctypes.c_double * 9)()
    check(lib().kr_invert_homography(_m9(m), out))
    return list(out)


def invert_affine(m):
    """kr_invert_affine: the library's inverse of a 2x3 map (host computation)."""
    out = (ctypes.c_double * 6)()
    check(lib().kr_invert_affine(_m6(m), out))
    return list(out)


def hbm_copy(dst, src, nbytes: int | None = None, stream=None) -> None:
    """kr_hbm_copy between two device tensors (the bandwidth ceiling probe)."""
    n = src.numel() * src.element_size() if nbytes is None else int(nbytes)
    check(lib().kr_hbm_copy(dst.data_ptr(), src.data_ptr(), n, _stream(stream)))


def hbm_stream(dst, src, dst_bytes: int | None = None, src_bytes: int | None = None, stream=None) -> None:
    """kr_hbm_stream: read src_bytes of src and write dst_bytes of dst (the
    traffic-mix bandwidth probe); sizes default to the tensors' byte sizes."""
    nd = dst.numel() * dst.element_size() if dst_bytes is None else int(dst_bytes)
    ns = src.numel() * src.element_size() if src_bytes is None else int(src_bytes)
    check(lib().kr_hbm_stream(dst.data_ptr(), nd, src.data_ptr(), ns, _stream(stream)))


# ---------------------------------------------------------------- batches
def _image_chw(t):
    """(pointer, H, W, C, kr_dtype) of a contiguous CHW device tensor."""
    if t.dim() != 3:
        raise ValueError("planar tensor must be CxHxW")
    ptr, c, h, w, dt = _image(t)  # dims read as (C, H, W)
    return ptr, h, w, c, dt


def _batch_items(specs, layout: int = LAYOUT_HWC):
    """ctypes array of BatchItem from specs: dicts with keys op ("resize" or
    "warp"), src, dst (tensors; src may be a view with packed pixels, dst CxHxW
    for the planar layout), and for warps m (2x3) and optional inverse."""
    n = len(specs)
    arr = (BatchItem * max(n, 1))()
    c = st = dt = None
    for i, sp in enumerate(specs):
        sp_ = dict(sp)
        sptr, sh, sw, pitch, sc, s_t = _source(sp_["src"])
        dptr, dh, dw, dc, d_t = _image_chw(sp_["dst"]) if layout == LAYOUT_CHW else _image(sp_["dst"])
        if sc != dc or (c is not None and (sc != c or s_t != st or d_t != dt)):
            raise ValueError("batch items must share channel count and dtypes")
        c, st, dt = sc, s_t, d_t
        it = arr[i]
        it.op = OP_WARP if sp_.get("op", "resize") == "warp" else OP_RESIZE
        it.src, it.src_h, it.src_w, it.src_pitch = sptr, sh, sw, pitch
        it.dst, it.dst_h, it.dst_w = dptr, dh, dw
        if it.op == OP_WARP:
            vals = [float(v) for v in (sp_["m"].reshape(-1).tolist() if hasattr(sp_["m"], "reshape") else sp_["m"])]
            for k in range(6):
                it.m[k] = vals[k]
            it.flags = WARP_INVERSE_MAP if sp_.get("inverse", False) else 0
        else:
            for k in range(6):
                it.m[k] = 0.0
            it.flags = 0
    return arr, n, c, st, dt


def batch_workspace_size(n: int) -> int:
    return int(lib().kr_resize_batch_workspace_size(n))


def resize_batch(specs, border: int = REPLICATE, border_value: float = 0.0, mean=None, std=None, workspace=None,
                 stream=None, layout: int = LAYOUT_HWC) -> None:
    """kr_resize_batch: every item of `specs` in one launch per operation.
    `workspace` is a device tensor of at least batch_workspace_size(n) bytes
    (allocated here if None)."""
    import torch
    arr, n, c, st, dt = _batch_items(specs, layout)
    if n == 0:
        return
    need = batch_workspace_size(n)
    if workspace is None:
        workspace = torch.empty(need, dtype=torch.uint8, device="cuda")
    check(lib().kr_resize_batch_ex(arr, n, c, st, dt, border, float(border_value), _normalize(mean, std, c),
                                   int(layout), workspace.data_ptr(), workspace.numel() * workspace.element_size(),
                                   _stream(stream)))


def prepare_batch(specs, border: int = REPLICATE, border_value: float = 0.0, mean=None, std=None, workspace=None,
                  stream=None, layout: int = LAYOUT_HWC):
    """resize_batch with the arguments marshalled once: returns a function
    that calls kr_resize_batch_ex on the same items each time (the library
    validates and builds the work-list on every call, as resize_batch does)."""
    import torch
    arr, n, c, st, dt = _batch_items(specs, layout)
    if n == 0:
        return lambda: None
    need = batch_workspace_size(n)
    if workspace is None:
        workspace = torch.empty(need, dtype=torch.uint8, device="cuda")
    norm = _normalize(mean, std, c)
    args = (arr, n, c, st, dt, border, float(border_value), norm, int(layout), workspace.data_ptr(),
            workspace.numel() * workspace.element_size(), _stream(stream))
    fn = lib().kr_resize_batch_ex

    def call():
        check(fn(*args))
    call.keep = (arr, norm, workspace)  # the marshalled arguments live as long as the function
    return call


def resize_batch_noalloc(specs, border: int = REPLICATE, border_value: float = 0.0, mean=None, std=None,
                         stream=None, layout: int = LAYOUT_HWC) -> None:
    """kr_resize_batch_noalloc: resize_batch with the work-list in the
    library's own device scratch (nothing is allocated; at most
    NOALLOC_MAX_ITEMS items; calls on one GPU must be ordered)."""
    arr, n, c, st, dt = _batch_items(specs, layout)
    if n == 0:
        return
    check(lib().kr_resize_batch_noalloc(arr, n, c, st, dt, border, float(border_value), _normalize(mean, std, c),
                                        int(layout), _stream(stream)))


# ---------------------------------------------------------------- autotuning
def _scrub(scrub):
    if scrub is None:
        return None, 0
    return scrub.data_ptr(), scrub.numel() * scrub.element_size()


def autotune_image(op: str, src, dst, m=None, inverse: bool = False, border: int = REPLICATE,
                   border_value: float = 0.0, mean=None, std=None, reps: int = 20, scrub=None, stream=None) -> str:
    """kr_autotune_image: time every tile configuration on this image and record
    the fastest for its class; dst receives the (correct) output.  scrub: None
    or a device tensor (> 256 MB) overwritten before each timed launch so the
    source comes from HBM.  Returns the one-line report."""
    sp, sh, sw, c, st = _image(src)
    dp_, dh, dw, dc, dt = _image(dst)
    if dc != c:
        raise ValueError("src and dst channel counts differ")
    rep = ctypes.create_string_buffer(512)
    is_warp = op == "warp"
    check(lib().kr_autotune_image(OP_WARP if is_warp else OP_RESIZE, sp, sh, sw, c, st, dp_, dh, dw, dt,
                                  _m6(m) if is_warp else None, WARP_INVERSE_MAP if inverse else 0, border,
                                  float(border_value), _normalize(mean, std, c), int(reps), *_scrub(scrub),
                                  _stream(stream), rep, len(rep)))
    return rep.value.decode()


def autotune_batch(specs, border: int = REPLICATE, border_value: float = 0.0, mean=None, std=None,
                   workspace=None, reps: int = 10, scrub=None, stream=None) -> str:
    """kr_autotune_batch: tune the batch's resize and warp launches (outputs are
    written, correctly, as by resize_batch).  Returns the report."""
    import torch
    arr, n, c, st, dt = _batch_items(specs)
    if n == 0:
        return ""
    if workspace is None:
        workspace = torch.empty(batch_workspace_size(n), dtype=torch.uint8, device="cuda")
    rep = ctypes.create_string_buffer(1024)
    check(lib().kr_autotune_batch(arr, n, c, st, dt, border, float(border_value), _normalize(mean, std, c),
                                  workspace.data_ptr(), workspace.numel() * workspace.element_size(), int(reps),
                                  *_scrub(scrub), _stream(stream), rep, len(rep)))
    return rep.value.decode()


def autotune_save() -> str:
    """The tuned table as text (kr_autotune_save)."""
    need = int(lib().kr_autotune_save(None, 0))
    buf = ctypes.create_string_buffer(need)
    lib().kr_autotune_save(buf, need)
    return buf.value.decode()


def autotune_load(text: str) -> None:
    check(lib().kr_autotune_load(text.encode()))


def autotune_clear() -> None:
    lib().kr_autotune_clear()


def build_key() -> str:
    """"<arch> <kernel-source hash>" of the loaded library (kr_build_key)."""
    return lib().kr_build_key().decode()


class BatchPlan:
    """kr_batch_plan_*: a validated work-list captured in a HIP graph; launch()
    replays it.  The tensors named by the specs must outlive the plan."""

    def __init__(self, specs, border: int = REPLICATE, border_value: float = 0.0, mean=None, std=None,
                 layout: int = LAYOUT_HWC):
        arr, n, c, st, dt = _batch_items(specs, layout)
        self._keep = [sp["src"] for sp in specs] + [sp["dst"] for sp in specs]
        h = ctypes.c_void_p()
        check(lib().kr_batch_plan_create_ex(arr, n, c, st, dt, border, float(border_value),
                                            _normalize(mean, std, c), int(layout), ctypes.byref(h)))
        self._h = h

    def launch(self, stream=None) -> None:
        check(lib().kr_batch_plan_launch(self._h, _stream(stream)))

    def close(self) -> None:
        if getattr(self, "_h", None):
            lib().kr_batch_plan_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


# ---------------------------------------------------------------- request server
class ServerConfig(ctypes.Structure):
    _fields_ = [("budget_bytes", ctypes.c_size_t), ("slots", ctypes.c_int), ("max_batch", ctypes.c_int)]


class Request(ctypes.Structure):
    _fields_ = [("op", ctypes.c_int), ("src", ctypes.c_void_p), ("src_h", ctypes.c_int), ("src_w", ctypes.c_int),
                ("dst_h", ctypes.c_int), ("dst_w", ctypes.c_int), ("m", ctypes.c_double * 6), ("flags", ctypes.c_int)]


class Completion(ctypes.Structure):
    _fields_ = [("id", ctypes.c_uint64), ("dst", ctypes.c_void_p), ("dst_bytes", ctypes.c_size_t),
                ("t_done", ctypes.c_double)]


def _server_lib():
    L = lib()
    if not getattr(L, "_server_decl", False):
        vp, i, f, d = ctypes.c_void_p, ctypes.c_int, ctypes.c_float, ctypes.c_double
        L.kr_server_create.argtypes = [ctypes.POINTER(ServerConfig), i, i, i, i, f, ctypes.POINTER(Normalize),
                                       ctypes.POINTER(vp)]
        L.kr_server_create.restype = i
        L.kr_server_now.argtypes = [vp]
        L.kr_server_now.restype = d
        L.kr_server_submit.argtypes = [vp, ctypes.POINTER(Request), ctypes.POINTER(ctypes.c_uint64)]
        L.kr_server_submit.restype = i
        L.kr_server_poll.argtypes = [vp, ctypes.POINTER(Completion), i, ctypes.POINTER(i)]
        L.kr_server_poll.restype = i
        L.kr_server_release.argtypes = [vp, ctypes.c_uint64]
        L.kr_server_release.restype = i
        L.kr_server_stats.argtypes = [vp, ctypes.POINTER(ctypes.c_size_t), ctypes.POINTER(ctypes.c_size_t),
                                      ctypes.POINTER(i)]
        L.kr_server_stats.restype = i
        L.kr_server_run_trace.argtypes = [vp, ctypes.POINTER(Request), ctypes.POINTER(d), i, ctypes.POINTER(d)]
        L.kr_server_run_trace.restype = i
        L.kr_server_destroy.argtypes = [vp]
        L.kr_server_destroy.restype = None
        L._server_decl = True
    return L


def make_request(op: str, src, dst_h: int, dst_w: int, m=None, inverse: bool = False) -> Request:
    """A kr_request for a resident source tensor (or (ptr, h, w) tuple)."""
    r = Request()
    if isinstance(src, tuple):
        r.src, r.src_h, r.src_w = src
    else:
        sp, sh, sw, _, _ = _image(src)
        r.src, r.src_h, r.src_w = sp, sh, sw
    r.op = OP_WARP if op == "warp" else OP_RESIZE
    r.dst_h, r.dst_w = dst_h, dst_w
    if r.op == OP_WARP:
        vals = [float(v) for v in (m.reshape(-1).tolist() if hasattr(m, "reshape") else m)]
        for k in range(6):
            r.m[k] = vals[k]
        r.flags = WARP_INVERSE_MAP if inverse else 0
    return r


class Server:
    """kr_server_*: continuous batching of resize/warp requests with outputs in
    a device arena of `budget_bytes`."""

    def __init__(self, budget_bytes: int, slots: int = 4, max_batch: int = 64, c: int = 3, out: str = "u8",
                 border: int = REPLICATE, border_value: float = 0.0, mean=None, std=None):
        L = _server_lib()
        cfg = ServerConfig(budget_bytes, slots, max_batch)
        h = ctypes.c_void_p()
        self.c, self.out = c, out
        check(L.kr_server_create(ctypes.byref(cfg), c, U8, U8 if out == "u8" else F32, border, float(border_value),
                                 _normalize(mean, std, c), ctypes.byref(h)))
        self._h = h

    def now(self) -> float:
        return _server_lib().kr_server_now(self._h)

    def submit(self, req: Request) -> int:
        rid = ctypes.c_uint64()
        check(_server_lib().kr_server_submit(self._h, ctypes.byref(req), ctypes.byref(rid)))
        return rid.value

    def poll(self, max_out: int = 256):
        buf = (Completion * max_out)()
        n = ctypes.c_int()
        check(_server_lib().kr_server_poll(self._h, buf, max_out, ctypes.byref(n)))
        return [(buf[k].id, buf[k].dst, buf[k].dst_bytes, buf[k].t_done) for k in range(n.value)]

    def release(self, rid: int) -> None:
        check(_server_lib().kr_server_release(self._h, rid))

    def stats(self):
        used, queued, busy = ctypes.c_size_t(), ctypes.c_size_t(), ctypes.c_int()
        check(_server_lib().kr_server_stats(self._h, ctypes.byref(used), ctypes.byref(queued), ctypes.byref(busy)))
        return used.value, queued.value, busy.value

    def run_trace(self, reqs, arrivals):
        n = len(reqs)
        arr = (Request * max(n, 1))(*reqs)
        t = (ctypes.c_double * max(n, 1))(*[float(a) for a in arrivals])
        lat = (ctypes.c_double * max(n, 1))()
        check(_server_lib().kr_server_run_trace(self._h, arr, t, n, lat))
        return [lat[k] for k in range(n)]

    def close(self) -> None:
        if getattr(self, "_h", None):
            _server_lib().kr_server_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
