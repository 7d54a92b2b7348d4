"""GPU parity of the fused resample + RGB -> gray forms (kr_resize_bilinear_gray,
kr_warp_affine_gray) and of the pixel-permutation path of kr_warp_affine
against the oracle: u8 bit-exact, f32 within 1e-3 on the 0..255 scale
(normalised: |d| * 255 * std <= 1e-3).  Also: the fused forms equal the two
GPU operators run one after the other, bit for bit, and permutation warps
equal the interpolating kernels (the batch engine), bit for bit."""
from __future__ import annotations

import numpy as np
import pytest

import oracle
from paper_2505_12425_amd import workloads as wl
from tests.gpu_util import assert_f32_close, assert_u8_equal, dev, say

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

from paper_2505_12425_amd import kr  # noqa: E402

TH = 16
MEAN, STD = [0.449], [0.226]


def _gray_out(h, w, out):
    return torch.empty((h, w, 1), dtype=torch.uint8 if out == "u8" else torch.float32, device="cuda")


RESIZES = [(480, 640, 240, 320), (2160, 3840, 1080, 1920), (2160, 3840, 1440, 2560), (97, 131, 301, 277),
           (1, 1, 5, 7), (40, 3000, 41, 17), (333, 257, 333, 257), (74, 106, 37, 53)]


@pytest.mark.parametrize("shape", RESIZES, ids=[f"{a}x{b}-{c}x{d}" for a, b, c, d in RESIZES])
@pytest.mark.parametrize("out", ["u8", "f32", "norm"])
def test_resize_gray_matches_oracle(shape, out):
    h, w, dh, dw = shape
    img = wl.mixed_u8(h, w, 3, seed=h * 7 + w) if h * w > 100000 else wl.uniform_u8(h, w, 3, seed=h + w)
    border = kr.REPLICATE if dh % 2 else kr.CONSTANT
    bval = 0.0 if border == kr.REPLICATE else 60.0
    say(f"resize_gray {shape} {out}")
    d = _gray_out(dh, dw, "u8" if out == "u8" else "f32")
    mean, std = (MEAN, STD) if out == "norm" else (None, None)
    kr.resize_gray(dev(img), d, border=border, border_value=bval, mean=mean, std=std)
    torch.cuda.synchronize()
    got = d.cpu().numpy()
    if out == "u8":
        assert_u8_equal(got, oracle.resize_gray(img, dh, dw, "u8", border, bval, threads=TH), "resize_gray u8")
    else:
        exp = oracle.resize_gray(img, dh, dw, "f64", border, bval, mean, std, threads=TH)
        assert_f32_close(got, exp, f"resize_gray {out}", std=std)


WARPS = [(480, 640, 480, 640, 23.0, 1.1, 0.1), (2160, 3840, 2160, 3840, -17.0, 0.9, 0.0),
         (130, 170, 90, 250, 140.0, 0.6, -0.2), (31, 9, 64, 64, 45.0, 2.5, 0.0)]


@pytest.mark.parametrize("case", WARPS, ids=[f"{c[0]}x{c[1]}-{c[4]}" for c in WARPS])
@pytest.mark.parametrize("out", ["u8", "f32", "norm"])
def test_warp_gray_matches_oracle(case, out):
    h, w, dh, dw, rot, sc, sh = case
    img = wl.mixed_u8(h, w, 3, seed=5) if h * w > 100000 else wl.uniform_u8(h, w, 3, seed=h + w)
    m = wl.affine_compose(h, w, rot, sc, sh, (dw - w) / 2.0, (dh - h) / 2.0)
    for border, bval in ((kr.CONSTANT, 0.0), (kr.CONSTANT, 200.0), (kr.REPLICATE, 0.0)):
        say(f"warp_gray {case} {out} border={border} {bval}")
        d = _gray_out(dh, dw, "u8" if out == "u8" else "f32")
        mean, std = (MEAN, STD) if out == "norm" else (None, None)
        kr.warp_affine_gray(dev(img), d, m, border=border, border_value=bval, mean=mean, std=std)
        torch.cuda.synchronize()
        got = d.cpu().numpy()
        if out == "u8":
            assert_u8_equal(got, oracle.warp_gray(img, m, dh, dw, "u8", border=border, bval=bval, threads=TH),
                            "warp_gray u8")
        else:
            exp = oracle.warp_gray(img, m, dh, dw, "f64", border=border, bval=bval, mean=mean, std=std, threads=TH)
            assert_f32_close(got, exp, f"warp_gray {out}", std=std)


@pytest.mark.parametrize("out", ["u8", "f32", "norm"])
def test_fused_gray_equals_the_two_operators(out):
    """One pass equals resample, then kr_rgb_to_gray on the GPU, bit for bit."""
    img = wl.mixed_u8(1000, 1400, 3, seed=9)
    s = dev(img)
    dt = torch.uint8 if out == "u8" else torch.float32
    mean, std = (MEAN, STD) if out == "norm" else (None, None)
    m = wl.affine_compose(1000, 1400, 33.0, 1.15, 0.05, -20.0, 14.0)
    for op in ("resize", "resize2x", "warp"):
        dh, dw = {"resize": (613, 777), "resize2x": (500, 700), "warp": (1000, 1400)}[op]
        rgb = torch.empty((dh, dw, 3), dtype=dt, device="cuda")
        two = _gray_out(dh, dw, "u8" if out == "u8" else "f32")
        one = _gray_out(dh, dw, "u8" if out == "u8" else "f32")
        if op.startswith("resize"):  # resize2x: the exact-2x kernel on both sides
            kr.resize(s, rgb)
            kr.resize_gray(s, one, mean=mean, std=std)
        else:
            kr.warp_affine(s, rgb, m, border_value=7.0)
            kr.warp_affine_gray(s, one, m, border_value=7.0, mean=mean, std=std)
        kr.rgb_to_gray(rgb, two, mean=mean, std=std)
        torch.cuda.synchronize()
        assert np.array_equal(one.cpu().numpy(), two.cpu().numpy()), f"{op} {out}"


def test_gray_views_equal_contiguous_copies():
    img = wl.uniform_u8(300, 500, 3, seed=12)
    big = dev(img)
    view = big[17:281, 5:433]
    copy = view.contiguous()
    for fn, args in ((kr.resize_gray, ()), (kr.warp_affine_gray, (wl.affine_compose(264, 428, 12.0, 1.0, 0.0,
                                                                                      3.0, 1.0),))):
        for dh, dw in ((200, 300), (132, 214)):  # (132, 214): an exact 2x resize of the view
            if fn is kr.warp_affine_gray and dh != 200:
                continue
            for out in ("u8", "f32"):
                a, b = _gray_out(dh, dw, out), _gray_out(dh, dw, out)
                fn(view, a, *args)
                fn(copy, b, *args)
                torch.cuda.synchronize()
                assert np.array_equal(a.cpu().numpy(), b.cpu().numpy()), (fn.__name__, dh, dw, out)


def test_gray_validation():
    s = dev(wl.uniform_u8(8, 8, 3, seed=1))
    with pytest.raises(kr.KrError):
        kr.resize_gray(s, _gray_out(4, 4, "u8"), border_value=300.0)
    with pytest.raises(kr.KrError):
        kr.resize_gray(s, _gray_out(4, 4, "u8"), mean=MEAN, std=STD)  # normalisation needs f32
    with pytest.raises(ValueError):
        kr.resize_gray(dev(wl.uniform_u8(8, 8, 4, seed=1)), _gray_out(4, 4, "u8"))


# ---------------------------------------------------------------- permutations
def _perm_maps(h, w):
    """Forward maps that permute pixels: flips, quarter turns, transposes,
    whole-number shifts (some sending part of the output outside the
    source), as (name, 2x3 map, output size)."""
    return [
        ("flip_x", np.array([[-1.0, 0, w - 1], [0, 1, 0]]), (h, w)),
        ("flip_y", np.array([[1.0, 0, 0], [0, -1, h - 1]]), (h, w)),
        ("rot180", np.array([[-1.0, 0, w - 1], [0, -1, h - 1]]), (h, w)),
        ("rot90", np.array([[0.0, 1, 0], [-1, 0, w - 1]]), (w, h)),
        ("rot270", np.array([[0.0, -1, h - 1], [1, 0, 0]]), (w, h)),
        ("transpose", np.array([[0.0, 1, 0], [1, 0, 0]]), (w, h)),
        ("shift", np.array([[1.0, 0, 37], [0, 1, -21]]), (h, w)),
        ("rot90_shift", np.array([[0.0, 1, -50], [-1, 0, w + 9]]), (w + 30, h + 11)),
    ]


@pytest.mark.parametrize("shape", [(2160, 3840), (257, 333), (1, 7), (64, 64), (65, 130)])
@pytest.mark.parametrize("c", [1, 2, 3, 4])
def test_permutation_warps_match_oracle(shape, c):
    h, w = shape
    img = wl.mixed_u8(h, w, c, seed=c) if h * w > 100000 else wl.uniform_u8(h, w, c, seed=h + c)
    s = dev(img)
    for name, m, (dh, dw) in _perm_maps(h, w):
        if h * w > 100000 and name not in ("rot90", "flip_x", "shift"):
            continue
        for border, bval in ((kr.CONSTANT, 9.0), (kr.REPLICATE, 0.0)):
            say(f"permute {shape} c={c} {name} border={border}")
            d = torch.empty((dh, dw, c), dtype=torch.uint8, device="cuda")
            kr.warp_affine(s, d, m, border=border, border_value=bval)
            torch.cuda.synchronize()
            assert_u8_equal(d.cpu().numpy(), oracle.warp(img, m, dh, dw, "u8", border=border, bval=bval,
                                                         threads=TH), f"{name} u8")
            if h * w <= 100000:
                f = torch.empty((dh, dw, c), dtype=torch.float32, device="cuda")
                kr.warp_affine(s, f, m, border=border, border_value=bval, mean=[0.4] * c, std=[0.3] * c)
                torch.cuda.synchronize()
                exp = oracle.warp(img, m, dh, dw, "f64", border=border, bval=bval, mean=[0.4] * c, std=[0.3] * c,
                                  threads=TH)
                assert_f32_close(f.cpu().numpy(), exp, f"{name} f32", std=[0.3] * c)


@pytest.mark.parametrize("out", ["u8", "f32"])
def test_permutation_path_equals_interpolating_engine(out):
    """The batch engine always interpolates; a permutation map through it
    and through kr_warp_affine (the permutation kernel) agree bit for bit."""
    h, w = 300, 420
    img = wl.uniform_u8(h, w, 3, seed=77)
    s = dev(img)
    dt = torch.uint8 if out == "u8" else torch.float32
    for name, m, (dh, dw) in _perm_maps(h, w):
        a = torch.empty((dh, dw, 3), dtype=dt, device="cuda")
        b = torch.empty((dh, dw, 3), dtype=dt, device="cuda")
        kr.warp_affine(s, a, m, border=kr.CONSTANT, border_value=3.0)
        kr.resize_batch([{"op": "warp", "src": s, "dst": b, "m": m}], border=kr.CONSTANT, border_value=3.0)
        torch.cuda.synchronize()
        assert np.array_equal(a.cpu().numpy(), b.cpu().numpy()), name


def test_permutation_of_a_view():
    img = wl.uniform_u8(200, 300, 3, seed=4)
    big = dev(img)
    view = big[11:190, 7:263]
    h, w = view.shape[:2]
    m = np.array([[0.0, 1, 0], [-1, 0, w - 1]])
    d = torch.empty((w, h, 3), dtype=torch.uint8, device="cuda")
    kr.warp_affine(view, d, m)
    torch.cuda.synchronize()
    assert_u8_equal(d.cpu().numpy(), oracle.warp(np.ascontiguousarray(img[11:190, 7:263]), m, w, h, "u8"), "view")
