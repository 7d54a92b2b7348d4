"""Pins of the C oracle against facts that do not come from the oracle itself.

Each pin is chosen so that a plausible slip in kro.c fails at least one of
them: a swapped weight (w0/w1), a dropped tap, a wrong sign in the half-pixel
offset, transposed x/y, a wrong rounding constant or tie rule, a wrong
inverse-matrix term or fma order, a border applied to the whole pixel instead
of per tap.

* closed forms: identity, constant images, exact 2x / 4x downsampling box
  means, 2x upsampling 9-3-3-1 weights, exact permutations (flip, 90 degree
  rotation), integer translations;
* an exact-rational brute force (tests/bruteforce.py) over whole 8x8..19x13
  images for every op x output type x border;
* library special cases: torch float64 ``interpolate`` (bilinear,
  align_corners=False) for the f32 resize and ``grid_sample`` for the f32 warp;
* algebraic invariants: linearity of the f32 path, M * M^-1 = I, the integer
  tie-to-even weight form against round(2048 r / den) in binary64.
"""
from __future__ import annotations

import math

import numpy as np
import pytest

import oracle
from paper_2505_12425_amd import workloads as wl
from tests import bruteforce as bf

CONST, REPL = oracle.CONSTANT, oracle.REPLICATE


# ---------------------------------------------------------------- identity
@pytest.mark.parametrize("c", [1, 3, 4])
def test_identity_resize_exact(c):
    img = wl.uniform_u8(17, 23, c, seed=1)
    assert np.array_equal(oracle.resize(img, 17, 23, "u8"), img)
    assert np.array_equal(oracle.resize(img, 17, 23, "f64"), img.astype(np.float64))
    imgf = wl.uniform_f32(9, 12, c, seed=2)
    assert np.array_equal(oracle.resize(imgf, 9, 12, "f64"), imgf.astype(np.float64))


@pytest.mark.parametrize("border", [CONST, REPL])
def test_identity_warp_exact(border):
    img = wl.uniform_u8(31, 29, 3, seed=3)
    eye = [1, 0, 0, 0, 1, 0]
    assert np.array_equal(oracle.warp(img, eye, 31, 29, "u8", border=border, bval=77), img)
    assert np.array_equal(oracle.warp(img, eye, 31, 29, "f64", border=border, bval=77),
                          img.astype(np.float64))


# ---------------------------------------------------------------- constants
@pytest.mark.parametrize("shape", [(40, 30, 17, 55), (7, 9, 64, 3), (1, 1, 5, 8)])
def test_constant_stays_constant(shape):
    h, w, dh, dw = shape
    img = np.full((h, w, 3), 173, np.uint8)
    assert (oracle.resize(img, dh, dw, "u8") == 173).all()
    assert np.allclose(oracle.resize(img, dh, dw, "f64"), 173.0, atol=1e-12)
    m = wl.affine_compose(h, w, 23.0, 1.1, 0.1, 2.5, -1.5)
    assert (oracle.warp(img, m, dh, dw, "u8", border=REPL) == 173).all()
    # CONSTANT border with the same value as the image is also constant
    assert (oracle.warp(img, m, dh, dw, "u8", border=CONST, bval=173) == 173).all()


# ---------------------------------------------------------------- box means
def test_exact_2x_down_is_box_mean():
    img = wl.uniform_u8(480, 640, 3, seed=0)
    got = oracle.resize(img, 240, 320, "u8")
    a = img.astype(np.int64)
    s = a[0::2, 0::2] + a[0::2, 1::2] + a[1::2, 0::2] + a[1::2, 1::2]
    assert np.array_equal(got, ((s + 2) >> 2).astype(np.uint8))
    gotf = oracle.resize(img, 240, 320, "f64")
    assert np.allclose(gotf, s / 4.0, atol=1e-12, rtol=0)


def test_exact_4x_down_is_centre_box_mean():
    img = wl.uniform_u8(64, 96, 3, seed=5)
    got = oracle.resize(img, 16, 24, "u8").astype(np.int64)
    a = img.astype(np.int64)
    s = a[1::4, 1::4] + a[1::4, 2::4] + a[2::4, 1::4] + a[2::4, 2::4]
    assert np.array_equal(got, (s + 2) >> 2)


def test_exact_2x_up_weights():
    img = wl.uniform_u8(20, 24, 3, seed=6)
    got = oracle.resize(img, 40, 48, "u8").astype(np.int64)
    a = img.astype(np.int64)
    # output (2i+1, 2j+1) sits at source (i + 1/4, j + 1/4): weights 3/4, 1/4
    i, j = np.meshgrid(np.arange(19), np.arange(23), indexing="ij")
    p = a[i, j]; q = a[i, j + 1]; r = a[i + 1, j]; s = a[i + 1, j + 1]
    exp = (9 * p + 3 * q + 3 * r + s + 8) >> 4
    assert np.array_equal(got[2 * i + 1, 2 * j + 1], exp)
    # output (2i+2, 2j+2) sits at source (i + 3/4, j + 3/4)
    exp2 = (p + 3 * q + 3 * r + 9 * s + 8) >> 4
    assert np.array_equal(got[2 * i + 2, 2 * j + 2], exp2)
    # the first output row/column replicate the edge (source -1/4 -> taps -1, 0)
    assert np.array_equal(got[0, 0], a[0, 0])


# ---------------------------------------------------------------- permutations
def test_flip_and_rot90_are_exact_permutations():
    n = 21
    img = wl.uniform_u8(n, n, 3, seed=7)
    flip = [-1, 0, n - 1, 0, 1, 0]
    assert np.array_equal(oracle.warp(img, flip, n, n, "u8"), img[:, ::-1])
    # forward map (x, y) -> (n-1-y, x): a 90 degree rotation
    rot = [0, -1, n - 1, 1, 0, 0]
    got = oracle.warp(img, rot, n, n, "u8")
    assert np.array_equal(got, np.rot90(img, k=-1))
    gotf = oracle.warp(img, rot, n, n, "f64")
    assert np.array_equal(gotf, np.rot90(img, k=-1).astype(np.float64))


@pytest.mark.parametrize("t", [(3, -2), (-5, 4), (0, 7)])
def test_integer_translation_is_exact_shift(t):
    tx, ty = t
    img = wl.uniform_u8(16, 19, 3, seed=8)
    got = oracle.warp(img, [1, 0, tx, 0, 1, ty], 16, 19, "u8", border=CONST, bval=0)
    exp = np.zeros_like(img)
    ys, xs = np.mgrid[0:16, 0:19]
    sx, sy = xs - tx, ys - ty
    ok = (sx >= 0) & (sx < 19) & (sy >= 0) & (sy < 16)
    exp[ys[ok], xs[ok]] = img[sy[ok], sx[ok]]
    assert np.array_equal(got, exp)


def test_warp_scale2_equals_resize_2x_down():
    img = wl.uniform_u8(36, 50, 3, seed=9)
    inv = [2.0, 0.0, 0.5, 0.0, 2.0, 0.5]
    a = oracle.warp(img, inv, 18, 25, "u8", inverse=True, border=CONST)
    b = oracle.resize(img, 18, 25, "u8")
    assert np.array_equal(a, b)


# ---------------------------------------------------------------- brute force
BF_CASES = [
    # (src h, w, dst h, dw)
    (8, 8, 8, 8), (8, 8, 5, 3), (8, 8, 13, 11), (8, 8, 3, 16), (13, 19, 7, 9), (5, 7, 19, 13),
]


@pytest.mark.parametrize("case", BF_CASES)
@pytest.mark.parametrize("border", [CONST, REPL])
def test_resize_matches_bruteforce(case, border):
    h, w, dh, dw = case
    img = wl.uniform_u8(h, w, 3, seed=h * 100 + w)
    bval = 201
    exp = bf.resize(img, dh, dw, "u8", border, bval)
    assert np.array_equal(oracle.resize(img, dh, dw, "u8", border, bval), exp)
    expf = bf.resize(img, dh, dw, "f64", border, bval)
    assert np.allclose(oracle.resize(img, dh, dw, "f64", border, bval), expf, atol=1e-9, rtol=0)
    mean, std = wl.IMAGENET_MEAN, wl.IMAGENET_STD
    expn = bf.resize(img, dh, dw, "f64", border, bval, mean, std)
    got = oracle.resize(img, dh, dw, "f64", border, bval, mean, std)
    assert np.allclose(got, expn, atol=1e-9, rtol=0)


WARP_MATS = [
    wl.affine_compose(8, 8, 30.0, 1.0, 0.0, 0.0, 0.0),
    wl.affine_compose(8, 8, -17.0, 0.7, 0.15, 1.3, -0.4),
    wl.affine_compose(8, 8, 44.0, 1.4, -0.2, -2.0, 1.0),
    wl.affine_compose(13, 19, 5.0, 2.3, 0.0, 0.25, 0.75),
]


@pytest.mark.parametrize("mi", range(len(WARP_MATS)))
@pytest.mark.parametrize("border", [CONST, REPL])
def test_warp_matches_bruteforce(mi, border):
    m = WARP_MATS[mi]
    h, w = (13, 19) if mi == 3 else (8, 8)
    img = wl.uniform_u8(h, w, 3, seed=mi)
    for dh, dw in [(h, w), (11, 6)]:
        exp = bf.warp(img, m, dh, dw, "u8", border=border, bval=33)
        got = oracle.warp(img, m, dh, dw, "u8", border=border, bval=33)
        assert np.array_equal(got, exp)
        expf = bf.warp(img, m, dh, dw, "f64", border=border, bval=33)
        gotf = oracle.warp(img, m, dh, dw, "f64", border=border, bval=33)
        assert np.allclose(gotf, expf, atol=1e-9, rtol=0)


def test_warp_f32_source_matches_bruteforce():
    img = wl.uniform_f32(9, 7, 3, seed=11)
    m = wl.affine_compose(9, 7, 12.0, 0.9, 0.05, 0.3, 0.2)
    exp = bf.warp(img, m, 9, 7, "f64", border=CONST, bval=-3.5)
    got = oracle.warp(img, m, 9, 7, "f64", border=CONST, bval=-3.5)
    assert np.allclose(got, exp, atol=1e-9, rtol=0)
    exp = bf.resize(img, 4, 13, "f64", border=REPL)
    got = oracle.resize(img, 4, 13, "f64", border=REPL)
    assert np.allclose(got, exp, atol=1e-9, rtol=0)


def test_inverse_map_flag_matches_bruteforce():
    img = wl.uniform_u8(8, 8, 3, seed=12)
    inv = [0.8, 0.3, -0.6, -0.25, 1.1, 0.9]
    exp = bf.warp(img, inv, 8, 8, "u8", inverse=True, border=REPL)
    assert np.array_equal(oracle.warp(img, inv, 8, 8, "u8", inverse=True, border=REPL), exp)


# ---------------------------------------------------------------- torch cross-checks
torch = pytest.importorskip("torch")


@pytest.mark.parametrize("shape", [(31, 47, 9, 100), (64, 64, 32, 32), (17, 5, 40, 23), (100, 80, 7, 9)])
def test_f32_resize_matches_torch_interpolate(shape):
    h, w, dh, dw = shape
    img = wl.uniform_u8(h, w, 3, seed=h + w)
    t = torch.from_numpy(img.astype(np.float64)).permute(2, 0, 1)[None]
    ref = torch.nn.functional.interpolate(t, size=(dh, dw), mode="bilinear",
                                          align_corners=False, antialias=False)
    ref = ref[0].permute(1, 2, 0).numpy()
    got = oracle.resize(img, dh, dw, "f64", border=REPL)
    assert np.allclose(got, ref, atol=1e-9, rtol=0)


@pytest.mark.parametrize("border,pad", [(CONST, "zeros"), (REPL, "border")])
def test_f32_warp_matches_torch_grid_sample(border, pad):
    h, w, dh, dw = 23, 31, 19, 27
    img = wl.uniform_u8(h, w, 3, seed=21)
    m = wl.affine_compose(h, w, 33.0, 1.2, 0.1, 3.3, -2.2)
    inv = bf.invert_affine(m)
    ys, xs = np.mgrid[0:dh, 0:dw].astype(np.float64)
    sx = inv[0] * xs + inv[1] * ys + inv[2]
    sy = inv[3] * xs + inv[4] * ys + inv[5]
    grid = np.stack([(2 * sx + 1) / w - 1, (2 * sy + 1) / h - 1], axis=-1)
    t = torch.from_numpy(img.astype(np.float64)).permute(2, 0, 1)[None]
    ref = torch.nn.functional.grid_sample(t, torch.from_numpy(grid)[None], mode="bilinear",
                                          padding_mode=pad, align_corners=False)
    ref = ref[0].permute(1, 2, 0).numpy()
    got = oracle.warp(img, m, dh, dw, "f64", border=border)
    assert np.allclose(got, ref, atol=1e-9, rtol=0)


# ---------------------------------------------------------------- invariants
def test_f32_resize_is_linear():
    a = wl.uniform_f32(33, 27, 3, seed=30)
    ra = oracle.resize(a, 50, 11, "f64")
    rb = oracle.resize((0.5 * a + 7.0).astype(np.float32), 50, 11, "f64")
    assert np.allclose(rb, 0.5 * ra + 7.0, atol=1e-4)


def test_normalize_is_affine_in_f32_output():
    img = wl.uniform_u8(48, 64, 3, seed=31)
    mean, std = wl.IMAGENET_MEAN, wl.IMAGENET_STD
    v = oracle.resize(img, 20, 30, "f64")
    n = oracle.resize(img, 20, 30, "f64", mean=mean, std=std)
    exp = (v / 255.0 - np.array(mean)) / np.array(std)
    assert np.allclose(n, exp, atol=1e-12)


@pytest.mark.parametrize("m", [
    [1, 0, 0, 0, 1, 0], [0, -1, 20, 1, 0, 0], [-1, 0, 31, 0, 1, 0], [1, 0, 5, 0, 1, -7],
])
def test_invert_affine_exact_for_permutations(m):
    inv = oracle.invert_affine(m)
    mm = np.array(m, np.float64).reshape(2, 3)
    full = np.vstack([mm, [0, 0, 1]])
    exp = np.linalg.inv(full)[:2].reshape(6)
    assert np.array_equal(inv, exp)


def test_invert_affine_roundtrip_and_formula():
    rng = np.random.default_rng(40)
    for _ in range(200):
        m = wl.affine_compose(1080, 1920, rng.uniform(-45, 45), rng.uniform(0.5, 1.5),
                              rng.uniform(-0.2, 0.2), rng.uniform(-100, 100), rng.uniform(-100, 100))
        inv = oracle.invert_affine(m)
        full = np.vstack([m, [0, 0, 1]])
        ifull = np.vstack([inv.reshape(2, 3), [0, 0, 1]])
        assert np.allclose(full @ ifull, np.eye(3), atol=1e-12)
        # bit-identical to the same formula written out in Python binary64
        assert tuple(inv) == bf.invert_affine(m.reshape(6))


def test_integer_weight_form_equals_binary64_rounding():
    # the oracle's exact integer tie-to-even weight equals round-half-even of the
    # binary64 quotient 2048 r / den (non-tie distances from k + 1/2 are >= 1/(2 den)).
    rng = np.random.default_rng(41)
    ties = 0
    for _ in range(3000):
        den = 2 * int(rng.integers(1, 40000))
        r = int(rng.integers(0, den))
        q = 2048.0 * r / den
        exp = int(np.rint(q))
        t = 4096 * r + den
        k = t // (2 * den)
        if t % (2 * den) == 0:
            ties += 1
            if k & 1:
                k -= 1
        assert k == exp
    # a 4 -> 8 resize has fractions 3/4 and 1/4 (weights 1536 and 512)
    img = np.array([[[0], [255], [0], [255]]], np.uint8)
    got = oracle.resize(img, 1, 8, "u8")[0, :, 0].astype(np.int64)
    # source x = (dx + 1/2)/2 - 1/2 -> -1/4, 1/4, 3/4, 5/4, ...
    exp = [0, 64, 191, 191, 64, 64, 191, 255]
    assert list(got) == exp


def test_degenerate_one_pixel_source():
    img = np.array([[[10, 200, 7]]], np.uint8)
    assert (oracle.resize(img, 5, 9, "u8") == img).all()
    # a warp of a 1x1 source with CONSTANT 0: the centre pixel keeps the value,
    # half-pixel offsets blend with the border
    got = oracle.warp(img, [1, 0, 0, 0, 1, 0], 1, 1, "u8", border=CONST)
    assert np.array_equal(got, img)
    got = oracle.warp(img, [1, 0, 0.5, 0, 1, 0], 1, 2, "u8", border=CONST)
    # destination x=0 -> source -0.5: taps -1 (border) and 0, weights 1/2 each
    assert list(got[0, 0]) == [(10 * 1024 * 2048 + 2 ** 21) >> 22, (200 * 2 ** 21 + 2 ** 21) >> 22,
                               (7 * 2 ** 21 + 2 ** 21) >> 22]


def test_all_border_warp():
    img = wl.uniform_u8(10, 10, 3, seed=50)
    got = oracle.warp(img, [1, 0, 1000, 0, 1, 1000], 6, 7, "u8", border=CONST, bval=42)
    assert (got == 42).all()
    gotf = oracle.warp(img, [1, 0, -1e9, 0, 1, 3e9], 6, 7, "f64", border=CONST, bval=42)
    assert (gotf == 42.0).all()


# ---------------------------------------------------------------- rounding-rule pins
def test_resize_weight_ties_go_to_even():
    # 6 -> 4096 along one axis: den = 8192 and every r = 2 (mod 4), so every
    # 2048 r / den = r / 4 is an exact half and the tie rule decides each weight.
    row = wl.uniform_u8(1, 6, 3, seed=60)
    got = oracle.resize(row, 1, 4096, "u8")
    assert np.array_equal(got, bf.resize(row, 1, 4096, "u8"))
    col = wl.uniform_u8(6, 1, 3, seed=61)
    got = oracle.resize(col, 4096, 1, "u8")
    assert np.array_equal(got, bf.resize(col, 4096, 1, "u8"))
    # the case really consists of ties
    assert all((4096 * (((2 * dx + 1) * 6 - 4096) % 8192) + 8192) % 16384 == 0 for dx in range(4096))


def test_warp_weight_ties_go_to_even():
    # inverse map xs = x (1 + 2^-12): frac = x / 4096, a tie for every odd x
    img = wl.uniform_u8(32, 40, 3, seed=62)
    a = 1.0 + 2.0 ** -12
    inv = [a, 0.0, 0.0, 0.0, a, 0.0]
    got = oracle.warp(img, inv, 32, 40, "u8", inverse=True, border=REPL)
    assert np.array_equal(got, bf.warp(img, inv, 32, 40, "u8", inverse=True, border=REPL))


@pytest.mark.parametrize("axis", [0, 1])
def test_warp_uses_fused_multiply_add(axis):
    # a huge coefficient makes the unfused product's rounding error visible in
    # the weights: 5 * (1e14 + 1/64) is not a multiple of ulp(5e14) = 1/16, so
    # the fused result keeps 5/64 where the unfused one rounds it to 4/64.
    # Only x = 5 (or y = 5) lands inside the image.
    img = wl.uniform_u8(8, 8, 3, seed=63)
    big = 1.0e14 + 1.0 / 64
    c = -5.0e14 + 3.3
    if axis == 0:
        inv = [big, 0.0, c, 0.0, 1.0, 0.25]
    else:
        inv = [1.0, 0.0, 0.25, 0.0, big, c]
    got = oracle.warp(img, inv, 8, 8, "u8", inverse=True, border=CONST, bval=9)
    exp = bf.warp(img, inv, 8, 8, "u8", inverse=True, border=CONST, bval=9)
    assert np.array_equal(got, exp)
    # the unfused evaluation would land elsewhere: check the case is sensitive
    fused = bf.fma(big, 5.0, c)
    unfused = big * 5.0 + c
    assert round(2048 * (fused % 1.0)) != round(2048 * (unfused % 1.0))


# ---------------------------------------------------------------- nearest neighbour
def test_nearest_identity_is_a_copy():
    img = wl.uniform_u8(23, 31, 3, seed=5)
    assert np.array_equal(oracle.resize_nearest(img, 23, 31), img)
    imgf = wl.uniform_f32(9, 12, 2, seed=6)
    assert np.array_equal(oracle.resize_nearest(imgf, 9, 12, "f64"), imgf.astype(np.float64))


@pytest.mark.parametrize("k", [2, 3, 5])
def test_nearest_integer_upscale_replicates(k):
    img = wl.uniform_u8(7, 9, 3, seed=k)
    exp = np.repeat(np.repeat(img, k, axis=0), k, axis=1)
    assert np.array_equal(oracle.resize_nearest(img, 7 * k, 9 * k), exp)


def test_nearest_exact_downscale_takes_cell_centres():
    img = wl.uniform_u8(24, 36, 3, seed=9)
    # 2x: the centre of output cell d lies on the edge between source 2d and
    # 2d + 1; half-pixel rounding takes 2d + 1.  3x: the middle sample 3d + 1.
    assert np.array_equal(oracle.resize_nearest(img, 12, 18), img[1::2, 1::2])
    assert np.array_equal(oracle.resize_nearest(img, 8, 12), img[1::3, 1::3])


@pytest.mark.parametrize("shape", [(8, 8, 5, 3), (6, 10, 13, 7), (11, 4, 3, 9), (1, 1, 4, 6), (9, 13, 1, 1)])
def test_nearest_matches_bruteforce(shape):
    h, w, dh, dw = shape
    img = wl.uniform_u8(h, w, 3, seed=h * w)
    assert np.array_equal(oracle.resize_nearest(img, dh, dw), bf.resize_nearest(img, dh, dw))
    mean, std = wl.IMAGENET_MEAN, wl.IMAGENET_STD
    got = oracle.resize_nearest(img, dh, dw, "f64", mean, std)
    assert np.allclose(got, bf.resize_nearest(img, dh, dw, "f64", mean, std), rtol=0, atol=1e-12)


@pytest.mark.parametrize("shape", [(40, 60, 17, 23), (17, 23, 40, 60), (480, 640, 240, 320), (33, 35, 100, 7)])
def test_nearest_matches_torch_nearest_exact(shape):
    h, w, dh, dw = shape
    img = wl.uniform_u8(h, w, 3, seed=h + 3 * w)
    t = torch.from_numpy(img.astype(np.float64)).permute(2, 0, 1)[None]
    ref = torch.nn.functional.interpolate(t, size=(dh, dw), mode="nearest-exact")[0].permute(1, 2, 0).numpy()
    assert np.array_equal(oracle.resize_nearest(img, dh, dw, "f64"), ref)
    assert np.array_equal(oracle.resize_nearest(img, dh, dw), ref.astype(np.uint8))


# ---------------------------------------------------------------- flip, RGB -> gray
@pytest.mark.parametrize("c", [1, 3, 4])
def test_flip_matches_numpy(c):
    img = wl.uniform_u8(13, 17, c, seed=c)
    assert np.array_equal(oracle.flip(img, True, False), img[:, ::-1])
    assert np.array_equal(oracle.flip(img, False, True), img[::-1])
    assert np.array_equal(oracle.flip(img, True, True), img[::-1, ::-1])
    assert np.array_equal(oracle.flip(img, False, False), img)
    f = wl.uniform_f32(9, 6, c, seed=c)
    assert np.array_equal(oracle.flip(f, True, False), f[:, ::-1])


def test_flip_equals_mirror_warp():
    img = wl.uniform_u8(19, 23, 3, seed=2)
    m = np.array([[-1.0, 0.0, 22.0], [0.0, 1.0, 0.0]])
    assert np.array_equal(oracle.flip(img, True, False), oracle.warp(img, m, 19, 23, "u8"))


def test_gray_u8_closed_forms():
    v = np.arange(256, dtype=np.uint8)
    grey = np.stack([v, v, v], axis=-1)[None]
    assert np.array_equal(oracle.rgb_to_gray(grey)[0, :, 0], v)  # weights sum to 2^14
    prim = np.array([[[255, 0, 0], [0, 255, 0], [0, 0, 255], [255, 255, 0]]], np.uint8)
    exp = [(4899 * 255 + 8192) >> 14, (9617 * 255 + 8192) >> 14, (1868 * 255 + 8192) >> 14,
           ((4899 + 9617) * 255 + 8192) >> 14]
    assert oracle.rgb_to_gray(prim)[0, :, 0].tolist() == exp == [76, 150, 29, 226]


def test_gray_matches_integer_and_float_definitions():
    img = wl.uniform_u8(31, 47, 3, seed=4)
    p = img.astype(np.int64)
    exp = (4899 * p[..., 0] + 9617 * p[..., 1] + 1868 * p[..., 2] + 8192) >> 14
    assert np.array_equal(oracle.rgb_to_gray(img)[..., 0], exp.astype(np.uint8))
    f = oracle.rgb_to_gray(img, "f64")[..., 0]
    q = img.astype(np.float64)
    assert np.allclose(f, q @ np.array([0.299, 0.587, 0.114]), rtol=0, atol=1e-12)
    fn = oracle.rgb_to_gray(img, "f64", [0.45], [0.25])[..., 0]
    assert np.allclose(fn, (f / 255.0 - 0.45) / 0.25, rtol=0, atol=1e-12)
    src = wl.uniform_f32(5, 8, 3, seed=1)
    g = oracle.rgb_to_gray(src, "f64")[..., 0]
    assert np.allclose(g, src.astype(np.float64) @ np.array([0.299, 0.587, 0.114]), rtol=0, atol=1e-9)


def test_gray_u8_within_bound_of_exact_bt601_over_all_inputs():
    """Every one of the 2^24 RGB triples, against the exact BT.601 luma
    0.299 R + 0.587 G + 0.114 B (an independent bound, not the integer
    formula restated): the 14-bit weights are each within 0.5/16384 of the
    exact ones, so the result is within 0.5 + 255 * 1.5 / 16384 < 0.524 of
    the exact value.  A swapped, truncated or dropped weight breaks the
    bound by far (swapping R and B is off by up to 47)."""
    v = np.arange(1 << 24, dtype=np.uint32)
    img = np.stack([(v >> 16) & 255, (v >> 8) & 255, v & 255], axis=-1).astype(np.uint8).reshape(4096, 4096, 3)
    g = oracle.rgb_to_gray(img, threads=8)[..., 0].astype(np.float64)
    q = img.astype(np.float64)
    exact = 0.299 * q[..., 0] + 0.587 * q[..., 1] + 0.114 * q[..., 2]
    err = np.abs(g - exact)
    assert err.max() < 0.524
    # and the rounding is to nearest: the bound is attained only near halves
    assert np.all((err <= 0.5) | (np.abs(exact - np.floor(exact) - 0.5) < 0.024))


# ---------------------------------------------------------------- fused RGB -> gray
GRAY_W = np.array([0.299, 0.587, 0.114])


@pytest.mark.parametrize("shape", [(31, 47, 17, 23), (20, 30, 45, 61), (64, 64, 32, 32)])
def test_resize_gray_on_grey_images_is_the_one_channel_resize(shape):
    """R = G = B: every channel resizes alike and gray(v, v, v) = v, so the
    fused result is the one-channel resize, bit for bit (an independent
    path through the oracle)."""
    h, w, dh, dw = shape
    g = wl.uniform_u8(h, w, 1, seed=h + w)
    rgb = np.repeat(g, 3, axis=-1)
    assert np.array_equal(oracle.resize_gray(rgb, dh, dw), oracle.resize(g, dh, dw))
    m = wl.affine_compose(h, w, 17.0, 0.9, 0.1, 2.5, -1.5)
    assert np.array_equal(oracle.warp_gray(rgb, m, dh, dw, bval=77.0),
                          oracle.warp(g, m, dh, dw, bval=77.0))


@pytest.mark.parametrize("border,bval", [(oracle.REPLICATE, 0.0), (oracle.CONSTANT, 40.0)])
def test_gray_commutes_with_resampling_f64(border, bval):
    """Both maps are linear (and the gray weights sum to one, so a constant
    border stays itself): gray after resampling equals resampling the gray
    image (here held as f32, so within its rounding: 255 * 2^-24 < 3e-5)."""
    img = wl.uniform_u8(29, 37, 3, seed=7)
    gray = (img.astype(np.float64) @ GRAY_W)[..., None].astype(np.float32)
    got = oracle.resize_gray(img, 41, 19, "f64", border, bval)
    assert np.allclose(got, oracle.resize(gray, 41, 19, "f64", border, bval), rtol=0, atol=3e-5)
    m = wl.affine_compose(29, 37, -23.0, 1.2, -0.1, 3.0, 4.0)
    got = oracle.warp_gray(img, m, 33, 35, "f64", border=border, bval=bval)
    assert np.allclose(got, oracle.warp(gray, m, 33, 35, "f64", border=border, bval=bval), rtol=0, atol=3e-5)
    n = oracle.warp_gray(img, m, 33, 35, "f64", border=border, bval=bval, mean=[0.45], std=[0.25])
    assert np.allclose(n, (got / 255.0 - 0.45) / 0.25, rtol=0, atol=1e-12)


def test_gray_u8_within_two_roundings_of_exact():
    """u8: each channel is within 1/2 of its exact interpolated value, and the
    14-bit gray is within 0.524 of the exact BT.601 combination of its
    inputs (the all-inputs bound above): within 1.03 of the exact gray of
    the exact interpolation.  A swapped or dropped channel is far off."""
    img = wl.uniform_u8(40, 56, 3, seed=3)
    exact = oracle.resize(img, 29, 31, "f64") @ GRAY_W
    assert np.abs(oracle.resize_gray(img, 29, 31)[..., 0] - exact).max() < 1.03
    m = wl.affine_compose(40, 56, 31.0, 1.1, 0.0, -2.0, 5.0)
    exact = oracle.warp(img, m, 40, 56, "f64") @ GRAY_W
    assert np.abs(oracle.warp_gray(img, m, 40, 56)[..., 0] - exact).max() < 1.03


# ---------------------------------------------------------------- perspective warp
def test_homography_inverse():
    assert np.array_equal(oracle.invert_homography([2, 0, 0, 0, 4, 0, 0, 0, 1]), [0.5, 0, 0, 0, 0.25, 0, 0, 0, 1])
    rng = np.random.default_rng(3)
    for _ in range(20):
        m = np.eye(3) + rng.uniform(-0.3, 0.3, (3, 3))
        inv = oracle.invert_homography(m).reshape(3, 3)
        assert np.allclose(m @ inv, np.eye(3), atol=1e-12)
        assert list(inv.reshape(9)) == bf.invert_homography(m)
    with pytest.raises(ValueError):
        oracle.invert_homography([1, 2, 3, 2, 4, 6, 0, 0, 1])


def test_perspective_identity_and_affine_special_cases():
    img = wl.uniform_u8(21, 27, 3, seed=8)
    assert np.array_equal(oracle.warp_perspective(img, np.eye(3), 21, 27, "u8"), img)
    inv6 = [0.93, 0.2, 1.7, -0.15, 1.04, -2.3]
    inv9 = inv6 + [0.0, 0.0, 1.0]
    for out in ("u8", "f64"):
        a = oracle.warp(img, inv6, 19, 25, out, inverse=True, border=CONST, bval=11)
        p = oracle.warp_perspective(img, inv9, 19, 25, out, inverse=True, border=CONST, bval=11)
        assert np.array_equal(a, p), out
    # a uniform third row divides exactly: [[1,0,0],[0,1,0],[0,0,2]] == affine scale 1/2
    half = oracle.warp(img, [0.5, 0, 0, 0, 0.5, 0], 30, 40, "u8", inverse=True, border=REPL)
    assert np.array_equal(oracle.warp_perspective(img, [1, 0, 0, 0, 1, 0, 0, 0, 2], 30, 40, "u8", inverse=True,
                                                  border=REPL), half)


@pytest.mark.parametrize("k", range(3))
def test_perspective_matches_bruteforce(k):
    img = wl.uniform_u8(10 + k, 12, 3, seed=20 + k)
    mats = [[1.05, 0.1, -0.5, -0.08, 0.97, 0.4, 0.01, -0.02, 1.0],
            [0.9, -0.2, 2.0, 0.15, 1.1, -1.0, -0.03, 0.015, 1.02],
            [1.0, 0.0, 0.0, 0.0, 1.0, 0.0, 0.12, 0.09, -0.6]]  # crosses the horizon
    m = mats[k]
    for border in (CONST, REPL):
        exp = bf.warp_perspective(img, m, 9, 13, "u8", border=border, bval=40)
        assert np.array_equal(oracle.warp_perspective(img, m, 9, 13, "u8", border=border, bval=40), exp)
        expf = bf.warp_perspective(img, m, 9, 13, "f64", border=border, bval=40)
        assert np.allclose(oracle.warp_perspective(img, m, 9, 13, "f64", border=border, bval=40), expf,
                           rtol=0, atol=1e-9)
