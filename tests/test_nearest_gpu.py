"""GPU parity of the nearest-neighbour resize (kr_resize_nearest) against the
oracle, element by element: u8 bit-exact, f32 within 1e-3 on the 0..255 scale
(normalised: |d| * 255 * std_c <= 1e-3)."""
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


def gpu_nearest(img, dh, dw, out="u8", mean=None, std=None):
    d = empty(dh, dw, img.shape[2], out)
    kr.resize_nearest(dev(img), d, mean=mean, std=std)
    torch.cuda.synchronize()
    return d.cpu().numpy()


def check(img, dh, dw, what, mean=None, std=None):
    say(f"nearest {what}: {img.shape} -> {dh}x{dw}")
    if img.dtype == np.uint8:
        assert_u8_equal(gpu_nearest(img, dh, dw), oracle.resize_nearest(img, dh, dw, threads=TH), what)
    got = gpu_nearest(img, dh, dw, "f32", mean, std)
    assert_f32_close(got, oracle.resize_nearest(img, dh, dw, "f64", mean, std, threads=TH), what, std=std)


def test_small_rgb_half():
    check(wl.uniform_u8(480, 640, 3, seed=0), 240, 320, "640x480 -> 320x240")


def test_4k_down_and_up():
    img = wl.mixed_u8(2160, 3840, 3, seed=0)
    check(img, 1080, 1920, "4K -> 1080p")
    small = wl.mixed_u8(1080, 1920, 3, seed=1)
    check(small, 2160, 3840, "1080p -> 4K")


SHAPES = [(50, 70, 48, 64), (64, 64, 128, 128), (17, 23, 40, 61), (40, 61, 17, 23), (100, 100, 33, 77), (1, 1, 7, 9), (1, 50, 3, 17),
          (31, 1, 5, 3), (333, 257, 333, 257), (64, 64, 1, 1), (9, 1000, 13, 255), (1, 32767, 2, 5)]


@pytest.mark.parametrize("shape", SHAPES, ids=[f"{a}x{b}-{c}x{d}" for a, b, c, d in SHAPES])
@pytest.mark.parametrize("c", [1, 2, 3, 4])
def test_shapes_channels(shape, c):
    h, w, dh, dw = shape
    check(wl.uniform_u8(h, w, c, seed=h + w + c), dh, dw, f"c={c}")


def test_normalised_and_f32_source():
    img = wl.uniform_u8(123, 457, 3, seed=7)
    check(img, 224, 224, "normalised", wl.IMAGENET_MEAN, wl.IMAGENET_STD)
    imgf = wl.uniform_f32(77, 91, 3, seed=8)
    got = gpu_nearest(imgf, 50, 130, "f32")
    assert np.array_equal(got, oracle.resize_nearest(imgf, 50, 130, "f64").astype(np.float32))


def test_max_width_output():
    img = wl.uniform_u8(3, 1000, 3, seed=9)
    check(img, 2, 32767, "max width")
