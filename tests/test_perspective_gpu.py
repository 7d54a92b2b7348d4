"""GPU parity of the bilinear perspective warp (kr_warp_perspective) against
the oracle, element by element: u8 bit-exact, f32 within 1e-3 on the 0..255
scale.  Covers the LDS-tiled path (u8 sources), the per-pixel path (f32
sources), tiles whose corners reach
w <= 0 (horizon crossings: quotients of either sign, infinities and 0/0),
both borders, the inverse flag, and the affine special case."""
from __future__ import annotations

import numpy as np
import pytest

import oracle
from paper_2505_12425_amd import workloads as wl
from tests.gpu_util import assert_f32_close, assert_u8_equal, dev, empty, say

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

from paper_2505_12425_amd import kr  # noqa: E402

TH = 16
CONST, REPL = 0, 1


def gpu_persp(img, m, dh, dw, out="u8", inverse=False, border=CONST, bval=0.0, mean=None, std=None):
    d = empty(dh, dw, img.shape[2], out)
    kr.warp_perspective(dev(img), d, m, inverse=inverse, border=border, border_value=bval, mean=mean, std=std)
    torch.cuda.synchronize()
    return d.cpu().numpy()


def check(img, m, dh, dw, what, inverse=False, border=CONST, bval=0.0):
    say(f"perspective {what}: {img.shape} -> {dh}x{dw}")
    if img.dtype == np.uint8:
        assert_u8_equal(gpu_persp(img, m, dh, dw, "u8", inverse, border, bval),
                        oracle.warp_perspective(img, m, dh, dw, "u8", inverse, border, bval, threads=TH), what)
    assert_f32_close(gpu_persp(img, m, dh, dw, "f32", inverse, border, bval),
                     oracle.warp_perspective(img, m, dh, dw, "f64", inverse, border, bval, threads=TH), what)


@pytest.mark.parametrize("seed", [0, 1])
def test_4k_tilt(seed):
    img = wl.mixed_u8(2160, 3840, 3, seed=seed)
    m = wl.random_homography(2160, 3840, np.random.default_rng(seed), 0.12)
    check(img, m, 2160, 3840, f"4K seed {seed}")


@pytest.mark.parametrize("c", [1, 2, 3, 4])
@pytest.mark.parametrize("border,bval", [(CONST, 0), (CONST, 77), (REPL, 0)])
def test_shapes_channels_borders(c, border, bval):
    rng = np.random.default_rng(10 * c + border)
    for h, w, dh, dw in ((333, 457, 300, 500), (64, 64, 131, 67), (17, 900, 40, 200)):
        img = wl.uniform_u8(h, w, c, seed=h + w + c)
        check(img, wl.random_homography(h, w, rng, 0.25), dh, dw, f"c={c} b={border}", border=border, bval=bval)


def test_horizon_crossing():
    img = wl.uniform_u8(300, 400, 3, seed=5)
    # inverse maps whose denominator changes sign inside the output
    for inv in ([1.0, 0.0, 0.0, 0.0, 1.0, 0.0, 0.004, 0.003, -1.0],
                [0.9, 0.1, 5.0, -0.1, 1.1, -3.0, -0.002, 0.0025, 0.2],
                [1.0, 0.0, 0.0, 0.0, 1.0, 0.0, 0.0, 0.005, -1.0]):  # w = 0 on row 200
        check(img, inv, 320, 420, "horizon", inverse=True, border=CONST, bval=3)
        check(img, inv, 320, 420, "horizon", inverse=True, border=REPL)


def test_f32_source_and_inverse_flag():
    img = wl.uniform_f32(150, 210, 3, seed=9)
    rng = np.random.default_rng(9)
    m = wl.random_homography(150, 210, rng, 0.2)
    inv = oracle.invert_homography(m)
    got = gpu_persp(img, inv, 160, 200, "f32", inverse=True)
    assert_f32_close(got, oracle.warp_perspective(img, inv, 160, 200, "f64", inverse=True, threads=TH), "f32 src")
    u8 = wl.uniform_u8(150, 210, 3, seed=9)
    assert np.array_equal(gpu_persp(u8, inv, 160, 200, "u8", inverse=True), gpu_persp(u8, m, 160, 200, "u8"))


def test_affine_special_case_equals_affine_warp():
    img = wl.uniform_u8(500, 700, 3, seed=2)
    inv6 = [0.93, 0.2, 1.7, -0.15, 1.04, -2.3]
    s = dev(img)
    for out in ("u8", "f32"):
        a = empty(480, 640, 3, out)
        kr.warp_affine(s, a, inv6, inverse=True, border=REPL)
        p = empty(480, 640, 3, out)
        kr.warp_perspective(s, p, inv6 + [0.0, 0.0, 1.0], inverse=True, border=REPL)
        torch.cuda.synchronize()
        assert np.array_equal(a.cpu().numpy(), p.cpu().numpy()), out


def test_mostly_border_output():
    """The source lands in a small quadrilateral of a large output: most tiles
    have every tap outside (constant fill), the rest interpolate."""
    for c in (3, 4):
        img = wl.uniform_u8(240, 320, c, seed=90 + c)
        m = np.array([[0.3, 0.05, 140.0], [0.02, 0.35, 90.0], [2e-4, 1e-4, 1.0]])
        check(img, m, 600, 800, f"mostly border c={c}", border=CONST, bval=77)
