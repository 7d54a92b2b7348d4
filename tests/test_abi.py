"""C-ABI checks that need no GPU: the library loads, exports every function
include/kr.h declares, and rejects bad arguments synchronously (validation runs
before any HIP call).  kr_invert_affine is host code and is compared bit for
bit with the oracle's independent implementation of the same formula."""
from __future__ import annotations

import ctypes
import math
import os
import re

import numpy as np
import pytest

import oracle
from paper_2505_12425_amd import kr
from paper_2505_12425_amd import workloads as wl

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "kr.h")

A = 0x7F0000000000  # a 16-byte aligned address; validation never dereferences it
B = 0x7F0100000000


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(kr_[a-z0-9_]+)\s*\(", text)))


def test_library_exports_every_declared_function():
    L = kr.lib()
    names = declared_functions()
    assert "kr_resize_bilinear" in names and "kr_warp_affine" in names and "kr_resize_batch" in names
    missing = [n for n in names if not hasattr(L, n)]
    assert not missing, f"declared in kr.h but not exported: {missing}"


def resize(**kw):
    a = dict(src=A, sh=480, sw=640, c=3, st=kr.U8, dst=B, dh=240, dw=320, dt=kr.U8,
             border=kr.REPLICATE, bval=0.0, norm=None, stream=None)
    a.update(kw)
    return kr.lib().kr_resize_bilinear(a["src"], a["sh"], a["sw"], a["c"], a["st"], a["dst"], a["dh"],
                                       a["dw"], a["dt"], a["border"], a["bval"], a["norm"], a["stream"])


def warp(m=(1, 0, 0, 0, 1, 0), flags=0, **kw):
    a = dict(src=A, sh=480, sw=640, c=3, st=kr.U8, dst=B, dh=480, dw=640, dt=kr.U8,
             border=kr.CONSTANT, bval=0.0, norm=None, stream=None)
    a.update(kw)
    mm = (ctypes.c_double * 6)(*[float(v) for v in m])
    return kr.lib().kr_warp_affine(a["src"], a["sh"], a["sw"], a["c"], a["st"], a["dst"], a["dh"],
                                   a["dw"], a["dt"], mm, flags, a["border"], a["bval"], a["norm"],
                                   a["stream"])


def norm_ptr(std=(0.229, 0.224, 0.225)):
    return kr._normalize((0.485, 0.456, 0.406), std, 3)


@pytest.mark.parametrize("kw,status", [
    (dict(src=0), kr.ERR_INVALID_ARGUMENT),
    (dict(dst=0), kr.ERR_INVALID_ARGUMENT),
    (dict(src=A + 4), kr.ERR_INVALID_ARGUMENT),
    (dict(dst=B + 8), kr.ERR_INVALID_ARGUMENT),
    (dict(sh=0), kr.ERR_INVALID_ARGUMENT),
    (dict(dw=0), kr.ERR_INVALID_ARGUMENT),
    (dict(sw=-3), kr.ERR_INVALID_ARGUMENT),
    (dict(dh=32768), kr.ERR_INVALID_ARGUMENT),
    (dict(c=0), kr.ERR_UNSUPPORTED),
    (dict(c=5), kr.ERR_UNSUPPORTED),
    (dict(st=kr.F32, dt=kr.U8), kr.ERR_UNSUPPORTED),
    (dict(st=7), kr.ERR_UNSUPPORTED),
    (dict(border=2), kr.ERR_UNSUPPORTED),
    (dict(bval=256.0), kr.ERR_INVALID_ARGUMENT),
    (dict(bval=-1.0), kr.ERR_INVALID_ARGUMENT),
    (dict(bval=1.5), kr.ERR_INVALID_ARGUMENT),
    (dict(bval=float("nan"), st=kr.F32, dt=kr.F32), kr.ERR_INVALID_ARGUMENT),
    (dict(dst=A + 16 * 1000), kr.ERR_INVALID_ARGUMENT),  # overlaps src
])
def test_resize_rejects(kw, status):
    assert resize(**kw) == status
    assert kr.last_error() != ""


def test_normalize_needs_f32_dst_and_nonzero_std():
    assert resize(norm=norm_ptr()) == kr.ERR_INVALID_ARGUMENT
    assert resize(dt=kr.F32, norm=norm_ptr(std=(0.2, 0.0, 0.2))) == kr.ERR_INVALID_ARGUMENT


@pytest.mark.parametrize("m,flags,status", [
    ((1, 2, 0, 2, 4, 0), 0, kr.ERR_SINGULAR_MATRIX),
    ((0, 0, 0, 0, 0, 0), 0, kr.ERR_SINGULAR_MATRIX),
    ((1, 0, float("nan"), 0, 1, 0), 0, kr.ERR_SINGULAR_MATRIX),
    ((float("inf"), 0, 0, 0, 1, 0), kr.WARP_INVERSE_MAP, kr.ERR_SINGULAR_MATRIX),
    ((1, 0, 0, 0, 1, 0), 4, kr.ERR_INVALID_ARGUMENT),
])
def test_warp_rejects(m, flags, status):
    assert warp(m, flags) == status


def test_warp_validates_images_too():
    assert warp(src=A + 1) == kr.ERR_INVALID_ARGUMENT
    assert warp(c=9) == kr.ERR_UNSUPPORTED


def test_status_strings():
    for s in range(7):
        assert kr.lib().kr_status_string(s).decode()
    assert kr.lib().kr_status_string(99).decode() == "unknown status"


def test_invert_affine_matches_oracle_bitwise():
    rng = np.random.default_rng(3)
    for i in range(500):
        if i % 2:
            m = wl.affine_compose(2160, 3840, rng.uniform(-45, 45), rng.uniform(0.5, 1.5),
                                  rng.uniform(-0.2, 0.2), rng.uniform(-400, 400), rng.uniform(-400, 400))
        else:
            m = rng.normal(size=(2, 3)) * 10.0 ** rng.integers(-3, 4)
        got = kr.invert_affine(m.reshape(6))
        exp = oracle.invert_affine(m.reshape(6))
        assert got == list(exp), (m, got, exp)


def test_invert_affine_rejects_singular():
    with pytest.raises(kr.KrError) as e:
        kr.invert_affine([2, 4, 1, 1, 2, 3])
    assert e.value.status == kr.ERR_SINGULAR_MATRIX
    # tiny but well-conditioned is fine (the rule is relative)
    inv = kr.invert_affine([1e-9, 0, 0, 0, 1e-9, 0])
    assert math.isclose(inv[0], 1e9)


def test_copy_probe_validation():
    L = kr.lib()
    assert L.kr_hbm_copy(0, A, 16, None) == kr.ERR_INVALID_ARGUMENT
    assert L.kr_hbm_copy(B, A + 3, 16, None) == kr.ERR_INVALID_ARGUMENT
    assert L.kr_hbm_copy(A + 16, A, 64, None) == kr.ERR_INVALID_ARGUMENT
    assert L.kr_hbm_copy(B, A, 0, None) == kr.OK  # nothing to do, nothing enqueued


def test_stream_probe_validation():
    """kr_hbm_stream rejects, before any launch, what its header rules out."""
    L = kr.lib()
    bad = kr.ERR_INVALID_ARGUMENT
    assert L.kr_hbm_stream(0, 64, A, 16, None) == bad             # NULL
    assert L.kr_hbm_stream(B, 64, A + 8, 16, None) == bad         # misaligned
    assert L.kr_hbm_stream(B, 0, A, 16, None) == bad              # empty
    assert L.kr_hbm_stream(B, 64, A, 24, None) == bad             # not a multiple of 16
    assert L.kr_hbm_stream(B, 48, A, 16, None) == bad             # ratio 3
    assert "power of two" in L.kr_last_error().decode()
    assert L.kr_hbm_stream(B, 16, A, 16 << 9, None) == bad        # 512 input chunks per output chunk
    assert L.kr_hbm_stream(A + 16, 64, A, 64, None) == bad        # overlap
    assert "overlap" in L.kr_last_error().decode()


def batch_items(n=2, op=0, dst_stride=4096):
    arr = (kr.BatchItem * n)()
    for i in range(n):
        arr[i].op = op
        arr[i].src, arr[i].src_h, arr[i].src_w = A, 100, 100
        arr[i].dst, arr[i].dst_h, arr[i].dst_w = B + i * dst_stride, 10, 10
    return arr


def test_batch_validation():
    L = kr.lib()
    ws = A + 0x10000000
    assert L.kr_resize_batch(batch_items(dst_stride=0), 2, 3, 0, 0, 1, 0.0, None, ws, 1 << 20, None) \
        == kr.ERR_INVALID_ARGUMENT  # overlapping destinations
    assert L.kr_resize_batch(batch_items(), 2, 3, 0, 0, 1, 0.0, None, ws, 16, None) == kr.ERR_WORKSPACE_TOO_SMALL
    assert L.kr_resize_batch(batch_items(), 2, 3, 0, 0, 1, 0.0, None, ws + 8, 1 << 20, None) \
        == kr.ERR_INVALID_ARGUMENT  # misaligned workspace
    assert L.kr_resize_batch(batch_items(op=7), 2, 3, 0, 0, 1, 0.0, None, ws, 1 << 20, None) \
        == kr.ERR_INVALID_ARGUMENT
    assert L.kr_resize_batch(batch_items(), 2, 5, 0, 0, 1, 0.0, None, ws, 1 << 20, None) == kr.ERR_UNSUPPORTED
    assert L.kr_resize_batch(batch_items(), 2, 3, 1, 1, 1, 0.0, None, ws, 1 << 20, None) == kr.ERR_UNSUPPORTED
    assert L.kr_resize_batch(None, 0, 3, 0, 0, 1, 0.0, None, None, 0, None) == kr.OK
    arr = batch_items(op=1)
    for k, v in enumerate([1, 2, 0, 2, 4, 0]):  # singular warp matrix
        arr[0].m[k] = v
    assert L.kr_resize_batch(arr, 2, 3, 0, 0, 0, 0.0, None, ws, 1 << 20, None) == kr.ERR_SINGULAR_MATRIX
    # a destination inside a source
    arr = batch_items()
    arr[1].dst = A + 64
    assert L.kr_resize_batch(arr, 2, 3, 0, 0, 1, 0.0, None, ws, 1 << 20, None) == kr.ERR_INVALID_ARGUMENT
    import ctypes
    h = ctypes.c_void_p()
    assert L.kr_batch_plan_create(batch_items(op=7), 2, 3, 0, 0, 1, 0.0, None, ctypes.byref(h)) \
        == kr.ERR_INVALID_ARGUMENT
    assert h.value is None
    assert L.kr_batch_plan_launch(None, None) == kr.ERR_INVALID_ARGUMENT
    L.kr_batch_plan_destroy(None)


def test_server_config_validation():
    L = kr._server_lib()
    h = ctypes.c_void_p()
    bad = [kr.ServerConfig(0, 1, 1), kr.ServerConfig(1 << 20, 0, 1), kr.ServerConfig(1 << 20, 17, 1),
           kr.ServerConfig(1 << 20, 1, 0), kr.ServerConfig(1 << 20, 1, 5000)]
    for cfg in bad:
        assert L.kr_server_create(ctypes.byref(cfg), 3, kr.U8, kr.U8, kr.REPLICATE, 0.0, None, ctypes.byref(h)) \
            == kr.ERR_INVALID_ARGUMENT
    ok = kr.ServerConfig(1 << 20, 2, 8)
    assert L.kr_server_create(ctypes.byref(ok), 5, kr.U8, kr.U8, kr.REPLICATE, 0.0, None, ctypes.byref(h)) \
        == kr.ERR_UNSUPPORTED
    assert L.kr_server_create(ctypes.byref(ok), 3, kr.F32, kr.F32, kr.REPLICATE, 0.0, None, ctypes.byref(h)) \
        == kr.ERR_UNSUPPORTED
    assert L.kr_server_create(ctypes.byref(ok), 3, kr.U8, kr.U8, kr.REPLICATE, 300.0, None, ctypes.byref(h)) \
        == kr.ERR_INVALID_ARGUMENT
    assert L.kr_server_create(None, 3, kr.U8, kr.U8, kr.REPLICATE, 0.0, None, ctypes.byref(h)) \
        == kr.ERR_INVALID_ARGUMENT
    assert h.value is None
    L.kr_server_destroy(None)


def test_autotune_table_roundtrip_and_validation():
    kr.autotune_clear()
    key = "key " + kr.build_key()
    header = "# op c f32 batch sclass zclass px txt cpt rpt grid\n" + key + "\n"
    assert kr.autotune_save() == header
    good = ("# comment\n" + key + "\n"
            "2 3 0 0 1 11 4 16 1 2 0\n"
            "1 3 0 0 0 11 4 16 1 4 1\n"
            "0 4 1 0 -4 10 1 64 2 4 0\n"
            "1 3 1 1 2 13 4 8 1 1 0\n"
            "1 3 1 0 1 11 1 64 1 8 1\n")
    kr.autotune_load(good)
    lines = [ln for ln in kr.autotune_save().splitlines() if not ln.startswith("#")]
    assert sorted(lines) == sorted(ln for ln in good.splitlines() if not ln.startswith("#"))
    before = kr.autotune_save()
    for bad in ["1 3 0 0 0 11 4 16 1 4\n",           # short line
                "1 3 0 0 0 11 4 16 1 4 1 9\n",       # trailing field
                "1 3 0 0 0 11 4 12 1 4 1\n",         # no such configuration
                "1 3 0 1 0 11 4 16 1 4 1\n",         # batches have no persistent grids
                "1 3 0 0 0 11 4 16 1 4 2\n",         # no such grid mode
                "3 3 0 0 0 11 4 16 1 4 1\n",         # unknown op
                "2 3 0 1 0 11 4 16 1 2 0\n",         # perspective warps have no batched form
                "1 2 0 0 0 11 4 16 1 4 1\n",         # channel count without configurations
                "0 3 0 0 0 11 1 64 2 4 0\nbogus\n"]:  # one bad line rejects the whole text
        with pytest.raises(kr.KrError) as e:
            kr.autotune_load(key + "\n" + bad)
        assert e.value.status == kr.ERR_INVALID_ARGUMENT
        assert kr.autotune_save() == before
    # no build key: rejected as malformed
    with pytest.raises(kr.KrError) as e:
        kr.autotune_load("1 3 0 0 0 11 4 16 1 4 1\n")
    assert e.value.status == kr.ERR_INVALID_ARGUMENT
    # a table measured on another build (kernel sources or architecture) is stale: ignored
    arch, sha = kr.build_key().split()
    for stale in [f"key {arch} {'0' * 16}", f"key gfx942 {sha}"]:
        with pytest.raises(kr.KrError) as e:
            kr.autotune_load(stale + "\n1 3 0 0 0 11 4 16 1 4 1\n")
        assert e.value.status == kr.ERR_UNSUPPORTED
        assert kr.autotune_save() == before
    # truncated save: NUL-terminated prefix, full length reported
    buf = ctypes.create_string_buffer(10)
    need = kr.lib().kr_autotune_save(buf, 10)
    assert need == len(before) + 1 and buf.value.decode() == before[:9]
    kr.autotune_clear()
    assert kr.autotune_save() == header


def test_build_key_names_arch_and_kernel_sources():
    from paper_2505_12425_amd.build import source_sha
    assert kr.build_key() == "gfx950 " + source_sha()


def test_stale_tuning_cache_file_is_ignored(tmp_path):
    """A KR_AUTOTUNE_CACHE file from another build is reported and ignored
    (checked in a fresh process: the file is read on first use)."""
    import subprocess
    import sys
    f = tmp_path / "stale.txt"
    f.write_text("key gfx950 " + "f" * 16 + "\n1 3 0 0 0 11 4 16 1 4 1\n")
    code = ("import sys; sys.path.insert(0, %r); from paper_2505_12425_amd import kr; "
            "print(repr(kr.autotune_save()))" % ROOT)
    r = subprocess.run([sys.executable, "-c", code], env={**os.environ, "KR_AUTOTUNE_CACHE": str(f)},
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 0, r.stderr
    assert "stale tuning cache" in r.stderr
    assert "1 3 0 0 0 11 4 16 1 4 1" not in r.stdout


def test_autotune_validation():
    L = kr.lib()
    rep = ctypes.create_string_buffer(64)
    m = (ctypes.c_double * 6)(1, 0, 0, 0, 1, 0)
    args = lambda **kw: [kw.get("op", 0), A, 480, 640, kw.get("c", 3), kw.get("st", kr.U8), B, 240, 320,
                         kr.U8, m, kw.get("flags", 0), kr.REPLICATE, 0.0, None, kw.get("reps", 5),
                         kw.get("scrub", None), kw.get("scrub_bytes", 0), None, rep, 64]
    assert L.kr_autotune_image(*args(op=5)) == kr.ERR_INVALID_ARGUMENT
    assert L.kr_autotune_image(*args(reps=0)) == kr.ERR_INVALID_ARGUMENT
    assert L.kr_autotune_image(*args(reps=1001)) == kr.ERR_INVALID_ARGUMENT
    assert L.kr_autotune_image(*args(c=1)) == kr.ERR_UNSUPPORTED
    assert L.kr_autotune_image(*args(op=1, flags=4)) == kr.ERR_INVALID_ARGUMENT
    assert L.kr_autotune_image(*args(scrub=A + 8, scrub_bytes=1 << 20)) == kr.ERR_INVALID_ARGUMENT
    assert L.kr_autotune_image(*args(scrub=A, scrub_bytes=16)) == kr.ERR_INVALID_ARGUMENT
    sing = (ctypes.c_double * 6)(1, 2, 0, 2, 4, 0)
    a = args(op=1)
    a[10] = sing
    assert L.kr_autotune_image(*a) == kr.ERR_SINGULAR_MATRIX
    ws = A + 0x10000000
    assert L.kr_autotune_batch(batch_items(dst_stride=0), 2, 3, 0, 0, 1, 0.0, None, ws, 1 << 20, 5, None, 0,
                               None, rep, 64) == kr.ERR_INVALID_ARGUMENT
    assert L.kr_autotune_batch(batch_items(), 2, 3, 0, 0, 1, 0.0, None, ws, 16, 5, None, 0, None, rep, 64) \
        == kr.ERR_WORKSPACE_TOO_SMALL
    assert L.kr_autotune_batch(batch_items(), 2, 3, 0, 0, 1, 0.0, None, ws, 1 << 20, 0, None, 0, None, rep, 64) \
        == kr.ERR_INVALID_ARGUMENT
    assert L.kr_autotune_batch(batch_items(), 2, 3, 0, 0, 1, 0.0, None, ws, 1 << 20, 5, A + 4, 1 << 20, None,
                               rep, 64) == kr.ERR_INVALID_ARGUMENT
    assert L.kr_autotune_load(None) == kr.ERR_INVALID_ARGUMENT


def test_nearest_validation():
    L = kr.lib()
    f = L.kr_resize_nearest
    assert f(None, 480, 640, 3, kr.U8, B, 240, 320, kr.U8, None, None) == kr.ERR_INVALID_ARGUMENT
    assert f(A, 0, 640, 3, kr.U8, B, 240, 320, kr.U8, None, None) == kr.ERR_INVALID_ARGUMENT
    assert f(A, 480, 640, 3, kr.U8, B, 240, 40000, kr.U8, None, None) == kr.ERR_INVALID_ARGUMENT
    assert f(A, 480, 640, 5, kr.U8, B, 240, 320, kr.U8, None, None) == kr.ERR_UNSUPPORTED
    assert f(A, 480, 640, 3, kr.F32, B, 240, 320, kr.U8, None, None) == kr.ERR_UNSUPPORTED
    assert f(A, 480, 640, 3, kr.U8, B, 240, 320, kr.U8, norm_ptr(), None) == kr.ERR_INVALID_ARGUMENT
    assert f(A, 480, 640, 3, kr.U8, A + 64, 240, 320, kr.U8, None, None) == kr.ERR_INVALID_ARGUMENT  # overlap
    assert f(A + 4, 480, 640, 3, kr.U8, B, 240, 320, kr.U8, None, None) == kr.ERR_INVALID_ARGUMENT  # misaligned


def test_flip_and_gray_validation():
    L = kr.lib()
    assert L.kr_flip(A, 10, 10, 3, kr.U8, B, 2, 0, None) == kr.ERR_INVALID_ARGUMENT
    assert L.kr_flip(A, 10, 10, 5, kr.U8, B, 1, 0, None) == kr.ERR_UNSUPPORTED
    assert L.kr_flip(A, 10, 10, 3, kr.U8, A + 16, 1, 0, None) == kr.ERR_INVALID_ARGUMENT  # overlap
    assert L.kr_flip(None, 10, 10, 3, kr.U8, B, 1, 0, None) == kr.ERR_INVALID_ARGUMENT
    g = L.kr_rgb_to_gray
    assert g(A, 10, 10, kr.F32, B, kr.U8, None, None) == kr.ERR_UNSUPPORTED
    assert g(A, 10, 10, kr.U8, B, kr.U8, norm_ptr(), None) == kr.ERR_INVALID_ARGUMENT
    assert g(A, 0, 10, kr.U8, B, kr.U8, None, None) == kr.ERR_INVALID_ARGUMENT
    assert g(A, 10, 10, kr.U8, A + 288, kr.U8, None, None) == kr.ERR_INVALID_ARGUMENT  # dst inside src (300 B)


def test_batch_layout_validation():
    L = kr.lib()
    ws = A + 0x10000000
    assert L.kr_resize_batch_ex(batch_items(), 2, 3, 0, 0, 1, 0.0, None, 2, ws, 1 << 20, None) \
        == kr.ERR_INVALID_ARGUMENT
    h = ctypes.c_void_p()
    assert L.kr_batch_plan_create_ex(batch_items(), 2, 3, 0, 0, 1, 0.0, None, -1, ctypes.byref(h)) \
        == kr.ERR_INVALID_ARGUMENT
    assert h.value is None


def test_invert_homography_matches_oracle_bitwise():
    rng = np.random.default_rng(17)
    for _ in range(50):
        m = wl.random_homography(int(rng.integers(10, 3000)), int(rng.integers(10, 3000)), rng, 0.3)
        assert kr.invert_homography(m) == list(oracle.invert_homography(m))
    with pytest.raises(kr.KrError) as e:
        kr.invert_homography([1, 2, 3, 2, 4, 6, 0, 0, 1])
    assert e.value.status == kr.ERR_SINGULAR_MATRIX
    with pytest.raises(kr.KrError):
        kr.invert_homography([1, 0, 0, 0, 1, 0, 0, 0, math.nan])


def test_perspective_validation():
    L = kr.lib()
    m = (ctypes.c_double * 9)(1, 0, 0, 0, 1, 0, 0, 0, 1)
    f = L.kr_warp_perspective
    assert f(A, 480, 640, 3, kr.U8, B, 480, 640, kr.U8, m, 4, 0, 0.0, None, None) == kr.ERR_INVALID_ARGUMENT
    assert f(A, 480, 640, 3, kr.U8, B, 480, 640, kr.U8, None, 0, 0, 0.0, None, None) == kr.ERR_INVALID_ARGUMENT
    sing = (ctypes.c_double * 9)(1, 2, 3, 2, 4, 6, 0, 0, 1)
    assert f(A, 480, 640, 3, kr.U8, B, 480, 640, kr.U8, sing, 0, 0, 0.0, None, None) == kr.ERR_SINGULAR_MATRIX
    nan = (ctypes.c_double * 9)(1, 0, 0, 0, 1, 0, 0, 0, math.nan)
    assert f(A, 480, 640, 3, kr.U8, B, 480, 640, kr.U8, nan, 1, 0, 0.0, None, None) == kr.ERR_SINGULAR_MATRIX
    assert f(A, 480, 640, 3, kr.U8, B, 480, 640, kr.U8, m, 0, 0, 300.0, None, None) == kr.ERR_INVALID_ARGUMENT


# ---------------------------------------------------------------- source views
def view_call(fn, pitch, src=A + 3 * 7, c=3, st=kr.U8, sh=100, sw=200, dst=B, **kw):
    """Call one of the *_view entry points with defaults that pass validation."""
    L = kr.lib()
    n = kw.pop("norm", None)
    dt = st  # (U8, U8) or (F32, F32)
    if fn == "resize":
        return L.kr_resize_bilinear_view(src, sh, sw, pitch, c, st, dst, 50, 100, dt, kr.REPLICATE, 0.0, n, None)
    if fn == "nearest":
        return L.kr_resize_nearest_view(src, sh, sw, pitch, c, st, dst, 50, 100, dt, n, None)
    if fn == "warp":
        mm = (ctypes.c_double * 6)(1, 0, 0, 0, 1, 0)
        return L.kr_warp_affine_view(src, sh, sw, pitch, c, st, dst, 50, 100, dt, mm, 0, kr.CONSTANT, 0.0, n, None)
    mm = (ctypes.c_double * 9)(1, 0, 0, 0, 1, 0, 0, 0, 1)
    return L.kr_warp_perspective_view(src, sh, sw, pitch, c, st, dst, 50, 100, dt, mm, 0, kr.CONSTANT, 0.0, n,
                                      None)


@pytest.mark.parametrize("fn", ["resize", "nearest", "warp", "persp"])
def test_view_validation(fn):
    # validation fails before anything touches the (fake) pointers; a valid
    # call on a CPU-only host would reach the HIP launch, so only rejections
    # are exercised here
    inval = kr.ERR_INVALID_ARGUMENT
    assert view_call(fn, 599) == inval                    # pitch below one row (600 bytes)
    assert view_call(fn, 601) == inval                    # pitch not a whole number of pixels
    assert view_call(fn, 3 * 1000, src=0) == inval        # NULL
    assert view_call(fn, 3 * 1000, sh=0) == inval         # empty
    # RGBA u8: the first pixel must be a whole number of 4-byte pixels past a
    # 16-byte boundary
    assert view_call(fn, 4 * 1000, src=A + 2, c=4) == inval
    # f32 RGB: 12-byte pixels; an address 2 bytes off the element grid fails
    assert view_call(fn, 12 * 1000, src=A + 2, st=kr.F32) == inval
    # a view spanning more than 2^31 pixels, and pitches whose span would wrap
    assert view_call(fn, 3 * 80000, sh=30000, sw=30000) == inval
    assert view_call(fn, 3 * (1 << 62), sh=5) == inval
    assert view_call(fn, 3 * ((1 << 31) + 1), sh=2) == inval
    # the view's span reaches the destination
    assert view_call(fn, 3 * 1000, dst=A + 16 * 18000) == inval  # inside rows 95..96 of the span
    assert "overlap" in kr.last_error()


def test_view_shift_rule():
    """Which view starts are accepted follows the 16-byte-boundary rule for
    each pixel size (checked through the error the pitch test leaves)."""
    L = kr.lib()

    def ok(addr, c, st):
        # an invalid pitch (below one row) fails after the start test: the
        # message says which test failed
        s = L.kr_resize_bilinear_view(addr, 10, 10, 1, c, st, B, 5, 5, kr.U8 if st == kr.U8 else kr.F32,
                                      kr.REPLICATE, 0.0, None, None)
        assert s == kr.ERR_INVALID_ARGUMENT
        return "16-byte" not in kr.last_error()

    for off in range(16):
        assert ok(A + off, 3, kr.U8)                # 3-byte pixels reach every byte address
        assert ok(A + off, 1, kr.U8)
        assert ok(A + off, 2, kr.U8) == (off % 2 == 0)
        assert ok(A + off, 4, kr.U8) == (off % 4 == 0)
        assert ok(A + off, 3, kr.F32) == (off % 4 == 0)
        assert ok(A + off, 4, kr.F32) == (off == 0)


def test_batch_item_layout_matches_header():
    # the ctypes mirror of kr_batch_item ends with the source pitch
    names = [f[0] for f in kr.BatchItem._fields_]
    assert names[-1] == "src_pitch"
    assert ctypes.sizeof(kr.BatchItem) % 8 == 0
