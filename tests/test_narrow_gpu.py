"""GPU parity of one- and two-channel u8 sources and one-channel f32 sources,
which run on the LDS-tiled kernels (one workgroup per tile, runs of 4 pixels
per lane): warps over the shapes of the RGB parity cases (rotations, shrinks,
zooms, tiles that are all border), resizes that stage boxes or gather their
taps from global memory, perspective warps, views into larger buffers,
normalised outputs, batches and 4K warps, each against the oracle (u8
bit-exact, f32 within 1e-3 absolute on the 0..255 scale)."""
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
from tests.test_parity_gpu import WARPS, check_resize, check_warp  # noqa: E402

CONST, REPL = 0, 1
TH = 8


@pytest.mark.parametrize("c", [1, 2])
@pytest.mark.parametrize("k", range(len(WARPS)))
@pytest.mark.parametrize("border,bval", [(CONST, 200), (REPL, 0)])
def test_narrow_warp_shapes(c, k, border, bval):
    h, w, dh, dw, th, s, sh, tx, ty = WARPS[k]
    img = wl.uniform_u8(h, w, c, seed=100 + 10 * k + c)
    m = wl.affine_compose(h, w, th, s, sh, tx, ty)
    check_warp(img, m, dh, dw, border, bval, what=f"narrow c={c} case {k}")


@pytest.mark.parametrize("c", [1, 2])
@pytest.mark.parametrize("shape", [(123, 77, 250, 160), (1080, 1920, 700, 1000), (300, 410, 47, 1201),
                                   (2160, 240, 224, 224), (31, 1, 7, 45), (5, 900, 900, 5)])
@pytest.mark.parametrize("border,bval", [(CONST, 17), (REPL, 0)])
def test_narrow_resize_shapes(c, shape, border, bval):
    h, w, dh, dw = shape
    img = wl.uniform_u8(h, w, c, seed=h + w + c)
    check_resize(img, dh, dw, border, bval, what=f"narrow c={c}")


@pytest.mark.parametrize("c", [1, 2])
def test_narrow_normalised(c):
    img = wl.mixed_u8(333, 517, c, seed=7 + c)
    mean, std = (0.45, 0.5)[:c], (0.226, 0.25)[:c]
    m = wl.affine_compose(333, 517, -21.0, 0.8, 0.05, 9.0, -4.0)
    say(f"narrow normalised c={c}")
    d = torch.empty((300, 480, c), dtype=torch.float32, device="cuda")
    kr.warp_affine(dev(img), d, m, border=CONST, border_value=5.0, mean=mean, std=std)
    torch.cuda.synchronize()
    assert_f32_close(d.cpu().numpy(), oracle.warp(img, m, 300, 480, "f64", False, CONST, 5.0, mean, std, threads=TH),
                     "narrow warp norm", std=std)
    d = torch.empty((211, 390, c), dtype=torch.float32, device="cuda")
    kr.resize(dev(img), d, border=REPL, mean=mean, std=std)
    torch.cuda.synchronize()
    assert_f32_close(d.cpu().numpy(), oracle.resize(img, 211, 390, "f64", REPL, 0, mean, std, threads=TH),
                     "narrow resize norm", std=std)


@pytest.mark.parametrize("c", [1, 2])
def test_narrow_views(c):
    """Crops of a larger buffer (odd offsets, the parent's first and last
    pixels): the staged groups start before and end after the view, and the
    last pixels of the view are read byte by byte."""
    par = wl.uniform_u8(260, 700, c, seed=31 + c)
    dev_par = dev(par)
    m = wl.affine_compose(100, 200, 12.0, 1.05, 0.0, 2.0, 1.0)
    for (y, x, h, w) in ((1, 3, 100, 200), (0, 0, 260, 700), (160, 500, 100, 200), (7, 13, 33, 41)):
        view = dev_par[y:y + h, x:x + w]
        host = np.ascontiguousarray(par[y:y + h, x:x + w])
        for out in ("u8", "f32"):
            say(f"narrow view c={c} {y},{x},{h}x{w} {out}")
            dt = torch.uint8 if out == "u8" else torch.float32
            dw_ = torch.empty((90, 170, c), dtype=dt, device="cuda")
            kr.warp_affine(view, dw_, m, border=REPL)
            dr = torch.empty((57, 311, c), dtype=dt, device="cuda")
            kr.resize(view, dr, border=CONST, border_value=3.0)
            torch.cuda.synchronize()
            ew = oracle.warp(host, m, 90, 170, "u8" if out == "u8" else "f64", False, REPL, 0, threads=TH)
            er = oracle.resize(host, 57, 311, "u8" if out == "u8" else "f64", CONST, 3.0, threads=TH)
            if out == "u8":
                assert_u8_equal(dw_.cpu().numpy(), ew, "narrow view warp")
                assert_u8_equal(dr.cpu().numpy(), er, "narrow view resize")
            else:
                assert_f32_close(dw_.cpu().numpy(), ew, "narrow view warp f32")
                assert_f32_close(dr.cpu().numpy(), er, "narrow view resize f32")


@pytest.mark.parametrize("c", [1, 2])
def test_narrow_perspective(c):
    img = wl.uniform_u8(240, 320, c, seed=70 + c)
    m9 = np.array([[0.9, 0.08, 12.0], [-0.05, 1.1, 4.0], [2e-4, -1e-4, 1.0]])
    for border, bval in ((CONST, 99), (REPL, 0)):
        for out in ("u8", "f32"):
            say(f"narrow perspective c={c} border={border} {out}")
            d = torch.empty((250, 300, c), dtype=torch.uint8 if out == "u8" else torch.float32, device="cuda")
            kr.warp_perspective(dev(img), d, m9, border=border, border_value=float(bval))
            torch.cuda.synchronize()
            exp = oracle.warp_perspective(img, m9, 250, 300, "u8" if out == "u8" else "f64", False, border, bval,
                                          threads=TH)
            if out == "u8":
                assert_u8_equal(d.cpu().numpy(), exp, "narrow perspective")
            else:
                assert_f32_close(d.cpu().numpy(), exp, "narrow perspective f32")


@pytest.mark.parametrize("c,out", [(1, "u8"), (2, "u8"), (1, "f32"), (2, "f32")])
def test_narrow_batch_equals_single_calls(c, out):
    """A mixed batch (resizes, exact halvings, warps, constant border) equals
    the single-image calls on the same items bit for bit, and the oracle."""
    rng = np.random.default_rng(500 + c)
    dt = torch.uint8 if out == "u8" else torch.float32
    specs, refs = [], []
    for i in range(12):
        h, w = int(rng.integers(30, 600)), int(rng.integers(30, 600))
        im = wl.uniform_u8(h, w, c, seed=600 + 13 * i + c)
        if i % 3 == 0:
            dh, dw = int(rng.integers(16, 500)), int(rng.integers(16, 500))
            m = wl.affine_compose(h, w, rng.uniform(-45, 45), rng.uniform(0.4, 1.8), rng.uniform(-0.2, 0.2),
                                  (dw - w) / 2.0, (dh - h) / 2.0)
            specs.append({"op": "warp", "src": dev(im), "m": m, "dst": torch.empty((dh, dw, c), dtype=dt, device="cuda")})
            refs.append(oracle.warp(im, m, dh, dw, out if out == "u8" else "f64", False, CONST, 40, threads=TH))
        else:
            dh, dw = (h // 2, w // 2) if i % 3 == 1 else (int(rng.integers(8, 700)), int(rng.integers(8, 700)))
            dh, dw = max(dh, 1), max(dw, 1)
            specs.append({"op": "resize", "src": dev(im), "dst": torch.empty((dh, dw, c), dtype=dt, device="cuda")})
            refs.append(oracle.resize(im, dh, dw, out if out == "u8" else "f64", CONST, 40, threads=TH))
    say(f"narrow batch c={c} out={out}")
    kr.resize_batch(specs, border=CONST, border_value=40.0)
    torch.cuda.synchronize()
    for i, (sp, ref) in enumerate(zip(specs, refs)):
        d = torch.empty_like(sp["dst"])
        if sp["op"] == "warp":
            kr.warp_affine(sp["src"], d, sp["m"], border=CONST, border_value=40.0)
        else:
            kr.resize(sp["src"], d, border=CONST, border_value=40.0)
        torch.cuda.synchronize()
        got = sp["dst"].cpu().numpy()
        assert np.array_equal(got.view(np.uint8), d.cpu().numpy().view(np.uint8)), f"item {i}: batch != single"
        if out == "u8":
            assert_u8_equal(got, ref, f"narrow batch item {i}")
        else:
            assert_f32_close(got, ref, f"narrow batch item {i}")


# ------------------------------------------------------------------ one-channel f32 sources
@pytest.mark.parametrize("k", range(len(WARPS)))
@pytest.mark.parametrize("border,bval", [(CONST, -3.5), (REPL, 0)])
def test_f32_gray_source_warps(k, border, bval):
    """One-channel f32 sources (depth-map-like values) stage their 4-byte
    pixels in LDS; edge tiles with a constant border must ignore the LDS
    words of masked taps."""
    h, w, dh, dw, th, s, sh, tx, ty = WARPS[k]
    img = wl.uniform_f32(h, w, 1, seed=200 + k)
    m = wl.affine_compose(h, w, th, s, sh, tx, ty)
    check_warp(img, m, dh, dw, border, bval, what=f"f32 gray case {k}")


@pytest.mark.parametrize("shape", [(123, 77, 250, 160), (1080, 1920, 700, 1000), (300, 410, 47, 1201),
                                   (2160, 240, 224, 224), (31, 1, 7, 45), (64, 48, 32, 24)])
@pytest.mark.parametrize("border,bval", [(CONST, 7.25), (REPL, 0)])
def test_f32_gray_source_resizes(shape, border, bval):
    h, w, dh, dw = shape
    img = wl.uniform_f32(h, w, 1, seed=h + 3 * w)
    check_resize(img, dh, dw, border, bval, what="f32 gray")


def test_f32_gray_source_perspective_views_norm():
    img = wl.uniform_f32(240, 320, 1, seed=77)
    m9 = np.array([[0.9, 0.08, 12.0], [-0.05, 1.1, 4.0], [2e-4, -1e-4, 1.0]])
    for border, bval in ((CONST, 99.0), (REPL, 0.0)):
        say(f"f32 gray perspective border={border}")
        d = torch.empty((250, 300, 1), dtype=torch.float32, device="cuda")
        kr.warp_perspective(dev(img), d, m9, border=border, border_value=bval)
        torch.cuda.synchronize()
        assert_f32_close(d.cpu().numpy(), oracle.warp_perspective(img, m9, 250, 300, "f64", False, border, bval,
                                                                   threads=TH), "f32 gray perspective")
    par = wl.uniform_f32(260, 700, 1, seed=78)
    dev_par = dev(par)
    m = wl.affine_compose(100, 200, 12.0, 1.05, 0.0, 2.0, 1.0)
    for (y, x, h, w) in ((1, 3, 100, 200), (0, 0, 260, 700), (160, 500, 100, 200), (7, 13, 33, 41)):
        say(f"f32 gray view {y},{x},{h}x{w}")
        view = dev_par[y:y + h, x:x + w]
        host = np.ascontiguousarray(par[y:y + h, x:x + w])
        d = torch.empty((90, 170, 1), dtype=torch.float32, device="cuda")
        kr.warp_affine(view, d, m, border=CONST, border_value=1.5, mean=(0.3,), std=(0.2,))
        torch.cuda.synchronize()
        assert_f32_close(d.cpu().numpy(), oracle.warp(host, m, 90, 170, "f64", False, CONST, 1.5, (0.3,), (0.2,),
                                                      threads=TH), "f32 gray view norm", std=(0.2,))


def test_narrow_4k_warp():
    img = wl.mixed_u8(2160, 3840, 1, seed=0)
    check_warp(img, wl.random_affine_4k(2160, 3840, 0), 2160, 3840, CONST, 0, what="4K gray seed 0")
    check_warp(wl.uniform_f32(2160, 3840, 1, seed=1), wl.random_affine_4k(2160, 3840, 3), 2160, 3840, CONST, 2.0,
               what="4K f32 gray seed 3")
