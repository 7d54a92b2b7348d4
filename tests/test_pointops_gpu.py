"""GPU parity of flip (kr_flip) and RGB -> gray (kr_rgb_to_gray) against the
oracle: u8 bit-exact, f32 flips bit-exact (a permutation), f32 gray within
1e-3 on the 0..255 scale (normalised: |d| * 255 * std <= 1e-3)."""
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

SHAPES = [(480, 640), (2160, 3840), (1, 1), (7, 13), (33, 1), (1, 1023), (257, 333), (3, 32767)]


@pytest.mark.parametrize("shape", SHAPES, ids=[f"{a}x{b}" for a, b in SHAPES])
@pytest.mark.parametrize("c", [1, 2, 3, 4])
def test_flip_u8(shape, c):
    h, w = shape
    img = wl.uniform_u8(h, w, c, seed=h + w + c)
    s = dev(img)
    for fx, fy in ((1, 0), (0, 1), (1, 1), (0, 0)):
        say(f"flip u8 {h}x{w}x{c} fx={fx} fy={fy}")
        d = torch.empty_like(s)
        kr.flip(s, d, fx, fy)
        torch.cuda.synchronize()
        assert_u8_equal(d.cpu().numpy(), oracle.flip(img, fx, fy), f"flip {fx}{fy}")


@pytest.mark.parametrize("c", [1, 3, 4])
def test_flip_f32_bitwise(c):
    img = wl.uniform_f32(257, 333, c, seed=c)
    img[0, 0, 0] = -0.0
    img[1, 1, 0] = np.nan
    s = dev(img)
    for fx, fy in ((1, 0), (0, 1), (1, 1)):
        d = torch.empty_like(s)
        kr.flip(s, d, fx, fy)
        torch.cuda.synchronize()
        assert np.array_equal(d.cpu().numpy().view(np.uint32), oracle.flip(img, fx, fy).view(np.uint32))


@pytest.mark.parametrize("shape", SHAPES, ids=[f"{a}x{b}" for a, b in SHAPES])
def test_gray(shape):
    h, w = shape
    img = wl.uniform_u8(h, w, 3, seed=h * 7 + w)
    s = dev(img)
    say(f"gray {h}x{w}")
    d8 = torch.empty((h, w, 1), dtype=torch.uint8, device="cuda")
    kr.rgb_to_gray(s, d8)
    df = torch.empty((h, w, 1), dtype=torch.float32, device="cuda")
    kr.rgb_to_gray(s, df)
    dn = torch.empty((h, w, 1), dtype=torch.float32, device="cuda")
    kr.rgb_to_gray(s, dn, mean=[0.45], std=[0.226])
    torch.cuda.synchronize()
    assert_u8_equal(d8.cpu().numpy(), oracle.rgb_to_gray(img), "gray u8")
    assert_f32_close(df.cpu().numpy(), oracle.rgb_to_gray(img, "f64"), "gray f32")
    assert_f32_close(dn.cpu().numpy(), oracle.rgb_to_gray(img, "f64", [0.45], [0.226]), "gray norm", std=[0.226])


def test_gray_f32_source():
    img = wl.uniform_f32(99, 130, 3, seed=3)
    d = torch.empty((99, 130, 1), dtype=torch.float32, device="cuda")
    kr.rgb_to_gray(dev(img), d)
    torch.cuda.synchronize()
    assert_f32_close(d.cpu().numpy(), oracle.rgb_to_gray(img, "f64"), "gray f32 src")
