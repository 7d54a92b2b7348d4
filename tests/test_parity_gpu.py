"""GPU parity: libkr (through the C ABI) against the oracle, element by element.

u8 output must be bit-exact; f32 output within 1e-3 absolute on the 0..255
scale (normalised output: within 1e-3 / (255 std_c)).  Inputs are seeded and
synthetic (paper_2505_12425_amd.workloads).  Sizes span several tiles with
ragged tails; the 4K cases run at full size in the launch configuration the
benchmark times, and the oracle computes them in full.
"""
from __future__ import annotations

import numpy as np
import pytest

import oracle
from paper_2505_12425_amd import workloads as wl
from tests.gpu_util import assert_f32_close, assert_u8_equal, dev, gpu_resize, gpu_warp, say

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

from paper_2505_12425_amd import kr  # noqa: E402

CONST, REPL = 0, 1
MEAN, STD = wl.IMAGENET_MEAN, wl.IMAGENET_STD
TH = 8


def check_resize(img, dh, dw, border=REPL, bval=0, what=""):
    h, w, c = img.shape
    say(f"resize {what} {h}x{w}x{c} -> {dh}x{dw} border={border}")
    if img.dtype == np.uint8:
        assert_u8_equal(gpu_resize(img, dh, dw, "u8", border, bval),
                        oracle.resize(img, dh, dw, "u8", border, bval, threads=TH), f"resize u8 {what}")
    assert_f32_close(gpu_resize(img, dh, dw, "f32", border, bval),
                     oracle.resize(img, dh, dw, "f64", border, bval, threads=TH), f"resize f32 {what}")
    if c == 3:
        assert_f32_close(gpu_resize(img, dh, dw, "f32", border, bval, MEAN, STD),
                         oracle.resize(img, dh, dw, "f64", border, bval, MEAN, STD, threads=TH),
                         f"resize norm {what}", std=STD)


def check_warp(img, m, dh, dw, border=CONST, bval=0, inverse=False, what=""):
    h, w, c = img.shape
    say(f"warp {what} {h}x{w}x{c} -> {dh}x{dw} border={border} m={np.round(np.asarray(m).reshape(6), 4)}")
    if img.dtype == np.uint8:
        assert_u8_equal(gpu_warp(img, m, dh, dw, "u8", inverse, border, bval),
                        oracle.warp(img, m, dh, dw, "u8", inverse, border, bval, threads=TH), f"warp u8 {what}")
    assert_f32_close(gpu_warp(img, m, dh, dw, "f32", inverse, border, bval),
                     oracle.warp(img, m, dh, dw, "f64", inverse, border, bval, threads=TH), f"warp f32 {what}")
    if c == 3:
        assert_f32_close(gpu_warp(img, m, dh, dw, "f32", inverse, border, bval, MEAN, STD),
                         oracle.warp(img, m, dh, dw, "f64", inverse, border, bval, MEAN, STD, threads=TH),
                         f"warp norm {what}", std=STD)


# ------------------------------------------------------------------ 640x480 -> 320x240
def test_small_rgb_resize_half():
    img = wl.uniform_u8(480, 640, 3, seed=0)
    check_resize(img, 240, 320, what="640x480->320x240")


# ------------------------------------------------------------------ 4K
@pytest.fixture(scope="module")
def img4k():
    return wl.mixed_u8(2160, 3840, 3, seed=0)


def test_4k_resize_to_1080p(img4k):
    check_resize(img4k, 1080, 1920, what="4K mixed")
    check_resize(wl.gradient_u8(2160, 3840, 3), 1080, 1920, what="4K gradient")


@pytest.mark.parametrize("seed", [0, 1, 2, 3, 4])
def test_4k_warp(img4k, seed):
    m = wl.random_affine_4k(2160, 3840, seed)
    check_warp(img4k, m, 2160, 3840, CONST, 0, what=f"4K seed {seed}")


# ------------------------------------------------------------------ shapes and ratios
RESIZE_SHAPES = [
    # (h, w, dh, dw): ragged tails, strong up/down ratios, thin images
    (300, 517, 151, 259), (97, 131, 389, 262), (1000, 37, 63, 600), (64, 64, 4, 4),
    (16, 16, 512, 512), (31, 1, 7, 45), (1, 29, 17, 3), (1, 1, 9, 9), (2, 3, 1, 1),
    (1080, 1920, 224, 224), (2160, 240, 224, 224), (241, 2159, 224, 224),
]


@pytest.mark.parametrize("shape", RESIZE_SHAPES, ids=[f"{a}x{b}-{c}x{d}" for a, b, c, d in RESIZE_SHAPES])
@pytest.mark.parametrize("c", [3, 1])
def test_resize_shapes(shape, c):
    h, w, dh, dw = shape
    img = wl.uniform_u8(h, w, c, seed=h * 7 + w)
    check_resize(img, dh, dw, REPL, what=f"shape c={c}")


@pytest.mark.parametrize("c", [2, 4])
@pytest.mark.parametrize("border,bval", [(CONST, 17), (REPL, 0)])
def test_resize_channels_borders(c, border, bval):
    img = wl.uniform_u8(123, 77, c, seed=c)
    check_resize(img, 250, 160, border, bval, what=f"c={c}")


def test_resize_f32_source():
    img = wl.uniform_f32(211, 333, 3, seed=5)
    check_resize(img, 100, 500, REPL, what="f32 src")
    check_resize(img, 100, 500, CONST, -7.25, what="f32 src const")


WARPS = [
    # (h, w, dh, dw, theta, scale, shear, tx, ty)
    (300, 400, 300, 400, 17.0, 1.0, 0.0, 5.5, -3.25),
    (480, 640, 512, 512, -40.0, 0.6, 0.15, 20.0, 10.0),
    (257, 193, 300, 200, 90.0, 1.3, -0.2, 0.0, 0.0),
    (1080, 1920, 1080, 1920, 44.0, 0.5, 0.2, -150.0, 90.0),
    (100, 100, 333, 333, 10.0, 3.0, 0.0, 100.0, 100.0),
    (64, 48, 70, 90, 0.0, 0.1, 0.0, 0.0, 0.0),
]


@pytest.mark.parametrize("k", range(len(WARPS)))
@pytest.mark.parametrize("border,bval", [(CONST, 0), (CONST, 200), (REPL, 0)])
def test_warp_shapes(k, border, bval):
    h, w, dh, dw, th, s, sh, tx, ty = WARPS[k]
    img = wl.uniform_u8(h, w, 3, seed=k)
    m = wl.affine_compose(h, w, th, s, sh, tx, ty)
    check_warp(img, m, dh, dw, border, bval, what=f"case {k}")


@pytest.mark.parametrize("c", [1, 2, 4])
def test_warp_channels(c):
    img = wl.uniform_u8(150, 211, c, seed=40 + c)
    m = wl.affine_compose(150, 211, 25.0, 1.1, 0.1, 3.0, -4.0)
    check_warp(img, m, 160, 200, CONST, 9, what=f"c={c}")


def test_warp_f32_source():
    img = wl.uniform_f32(120, 170, 3, seed=50)
    m = wl.affine_compose(120, 170, -33.0, 0.9, 0.05, 1.0, 2.0)
    check_warp(img, m, 130, 160, CONST, 3.5, what="f32 src")
    check_warp(img, m, 130, 160, REPL, 0.0, what="f32 src repl")


# ------------------------------------------------------------------ exact cases
def test_identity_flip_rotation_exact():
    img = wl.uniform_u8(301, 301, 3, seed=60)
    n = 301
    say("identity / flip / rot90")
    assert_u8_equal(gpu_warp(img, [1, 0, 0, 0, 1, 0], n, n), img, "identity warp")
    assert_u8_equal(gpu_resize(img, n, n), img, "identity resize")
    assert_u8_equal(gpu_warp(img, [-1, 0, n - 1, 0, 1, 0], n, n), img[:, ::-1], "flip")
    assert_u8_equal(gpu_warp(img, [0, -1, n - 1, 1, 0, 0], n, n), np.rot90(img, k=-1), "rot90")


def test_inverse_map_flag():
    img = wl.uniform_u8(200, 260, 3, seed=61)
    check_warp(img, [0.8, 0.3, -5.6, -0.25, 1.1, 7.9], 222, 190, REPL, 0, inverse=True, what="inverse")


def test_all_border_warp():
    img = wl.uniform_u8(50, 50, 3, seed=62)
    say("all-border warp")
    got = gpu_warp(img, [1, 0, 1e6, 0, 1, -1e6], 40, 70, "u8", border=CONST, bval=42)
    assert (got == 42).all()


@pytest.mark.parametrize("c", [1, 2, 3, 4])
def test_exact_half_scale(c):
    """Resizes by exactly 2 in both axes take the 2x2-mean kernel: sizes with
    ragged 4-pixel groups, the smallest cases, both borders, and the last
    bytes of the buffer (the byte-wise tail)."""
    for h, w in ((2, 2), (2, 8), (4, 6), (34, 98), (62, 202), (480, 640), (301 * 2, 3 * 2)):
        img = wl.uniform_u8(h, w, c, seed=h * w + c)
        for border in (REPL, CONST):
            check_resize(img, h // 2, w // 2, border, 9, what=f"half c={c}")


@pytest.mark.parametrize("c", [1, 2, 3, 4])
def test_exact_half_scale_views(c):
    """The 2x2-mean kernel on crops of a larger buffer (odd pixel offsets, the
    parent's first and last bytes), u8 and normalised f32 outputs, including
    rows wider than one wave's 256 outputs (the f32 LDS transpose)."""
    par = wl.uniform_u8(300, 1100, c, seed=123 + c)
    dev_par = dev(par)
    mean, std = (MEAN + (0.5,))[:c], (STD + (0.25,))[:c]
    for (y, x, h, w) in ((1, 3, 100, 202), (0, 0, 298, 1098), (13, 7, 2, 2), (298, 1090, 2, 10), (5, 1, 40, 1024),
                         (3, 9, 6, 1040)):
        view = dev_par[y:y + h, x:x + w]
        host = np.ascontiguousarray(par[y:y + h, x:x + w])
        for out in ("u8", "f32"):
            say(f"half view c={c} {y},{x},{h}x{w} {out}")
            d = torch.empty((h // 2, w // 2, c), dtype=torch.uint8 if out == "u8" else torch.float32, device="cuda")
            if out == "u8":
                kr.resize(view, d, border=REPL)
            else:
                kr.resize(view, d, border=REPL, mean=mean, std=std)
            torch.cuda.synchronize()
            if out == "u8":
                assert_u8_equal(d.cpu().numpy(), oracle.resize(host, h // 2, w // 2, "u8", REPL, threads=TH), "half view")
            else:
                assert_f32_close(d.cpu().numpy(), oracle.resize(host, h // 2, w // 2, "f64", REPL, 0, mean, std,
                                                                threads=TH), "half view norm", std=std)


def test_blank_tiles_match_oracle():
    """Zoomed-out and shifted warps whose output is mostly border: tiles with
    every tap outside the source take the constant fill, their neighbours
    interpolate; both must equal the oracle (u8 bit-exact, f32 and
    normalised f32 within tolerance), with a non-zero border value, for RGB
    and RGBA."""
    for c in (3, 4):
        img = wl.uniform_u8(300, 410, c, seed=65 + c)
        for k, (th, sc, tx, ty) in enumerate([(17.0, 0.3, 0.0, 0.0), (-38.0, 0.45, 260.0, -90.0),
                                              (0.0, 1.0, 700.0, 0.0), (90.0, 0.2, -30.0, 40.0)]):
            m = wl.affine_compose(300, 410, th, sc, 0.0, tx, ty)
            check_warp(img, m, 333, 517, CONST, 37, what=f"blank tiles c={c} case {k}")


def test_huge_coefficients():
    img = wl.uniform_u8(64, 64, 3, seed=63)
    inv = [1.0e14 + 1.0 / 64, 0.0, -5.0e14 + 3.3, 0.0, 1.0, 0.25]
    check_warp(img, inv, 64, 64, CONST, 9, inverse=True, what="huge coefficients")


def test_max_width():
    img = wl.uniform_u8(2, 32767, 3, seed=64)
    check_resize(img, 3, 32767, what="max width identity-x")
    check_resize(img, 1, 1000, what="max width down")


def test_repeat_runs_bitwise():
    img = wl.mixed_u8(1080, 1920, 3, seed=70)
    m = wl.random_affine_4k(1080, 1920, 3)
    say("determinism x3")
    a = [gpu_warp(img, m, 1080, 1920) for _ in range(3)]
    b = [gpu_resize(img, 517, 911) for _ in range(3)]
    assert all(np.array_equal(a[0], x) for x in a[1:])
    assert all(np.array_equal(b[0], x) for x in b[1:])


def test_stored_oracle_digests():
    """GPU u8 outputs hash to the digests stored from the oracle."""
    import json
    import os
    from tests.golden import make_golden as mg
    stored = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "oracle_digests.json")))
    small = wl.uniform_u8(480, 640, 3, seed=0)
    big = wl.mixed_u8(2160, 3840, 3, seed=0)
    m = wl.random_affine_4k(2160, 3840, 0)
    got = {
        "small_resize_u8": gpu_resize(small, 240, 320, "u8", border=REPL),
        "4k_resize_u8": gpu_resize(big, 1080, 1920, "u8", border=REPL),
        "4k_warp_u8": gpu_warp(big, m, 2160, 3840, "u8", border=CONST),
    }
    for name, a in got.items():
        say(f"digest {name}")
        assert mg.digest(a) == stored[name]["sha256"], name
