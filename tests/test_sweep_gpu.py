"""Seeded random sweep of the single-image operators against the oracle:
sizes from 1 to a few hundred pixels (several tiles and ragged edges), 1-4
channels, u8 and f32 sources, u8, f32 and normalised f32 outputs, both
borders with random border values, random affine maps (rotations up to 180
degrees, shrinks to 0.2x, zooms to 5x, shears, translations that push the
image partly or wholly out of view), random homographies, and sources that
are views into larger buffers.  u8 outputs must be bit-exact, f32 within
1e-3 on the 0..255 scale.  Every case prints its parameters first."""
from __future__ import annotations

import numpy as np
import pytest

import oracle
from paper_2505_12425_amd import workloads as wl
from tests.gpu_util import assert_f32_close, assert_u8_equal, empty, say

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

from paper_2505_12425_amd import kr  # noqa: E402

TH = 16
MEAN = (0.485, 0.456, 0.406, 0.5)
STD = (0.229, 0.224, 0.225, 0.25)


def random_source(rng, h, w, c, f32, as_view):
    """A device source (maybe a crop of a larger buffer) and its host copy."""
    img = (wl.uniform_f32 if f32 else wl.uniform_u8)(h, w, c, int(rng.integers(1 << 30)))
    if not as_view:
        return torch.from_numpy(img).cuda(), img
    ph, pw = h + int(rng.integers(0, 9)), w + int(rng.integers(1, 40))
    y, x = int(rng.integers(0, ph - h + 1)), int(rng.integers(0, pw - w + 1))
    par = (wl.uniform_f32 if f32 else wl.uniform_u8)(ph, pw, c, int(rng.integers(1 << 30)))
    par[y:y + h, x:x + w] = img
    dev = torch.from_numpy(par).cuda()
    return dev[y:y + h, x:x + w], img


def random_affine(rng, h, w):
    return wl.affine_compose(h, w, float(rng.uniform(-180, 180)), float(np.exp(rng.uniform(np.log(0.2), np.log(5)))),
                             float(rng.uniform(-0.4, 0.4)), float(rng.uniform(-1.2, 1.2) * w),
                             float(rng.uniform(-1.2, 1.2) * h))


def random_homography(rng, h, w):
    if h < 2 or w < 2:
        return np.array([[1.0, 0.1, 0.5], [-0.05, 0.9, 0.25], [1e-3, -2e-3, 1.0]])
    return wl.random_homography(h, w, rng, float(rng.uniform(0.02, 0.35)))


def run_case(rng, i):
    op = ["resize", "warp", "persp", "nearest"][i % 4]
    c = int(rng.integers(1, 5))
    f32src = bool(rng.random() < 0.25)
    h, w = int(rng.integers(1, 260)), int(rng.integers(1, 330))
    dh, dw = int(rng.integers(1, 300)), int(rng.integers(1, 360))
    as_view = bool(rng.random() < 0.4)
    border = int(rng.integers(0, 2))
    bval = float(rng.integers(0, 256))
    src, host = random_source(rng, h, w, c, f32src, as_view)
    outs = ["f32", "norm"] if f32src else ["u8", "f32", "norm"]
    m = random_affine(rng, h, w) if op == "warp" else (random_homography(rng, h, w) if op == "persp" else None)
    say(f"case {i}: {op} c={c} {h}x{w} -> {dh}x{dw} f32src={f32src} view={as_view} border={border} bval={bval}")
    for out in outs:
        mean, std = (MEAN[:c], STD[:c]) if out == "norm" else (None, None)
        d = empty(dh, dw, c, "u8" if out == "u8" else "f32")
        o = "u8" if out == "u8" else "f64"
        if op == "resize":
            kr.resize(src, d, border=border, border_value=bval, mean=mean, std=std)
            exp = oracle.resize(host, dh, dw, o, border, bval, mean, std, threads=TH)
        elif op == "nearest":
            kr.resize_nearest(src, d, mean=mean, std=std)
            exp = oracle.resize_nearest(host, dh, dw, o, mean, std, threads=TH)
        elif op == "warp":
            kr.warp_affine(src, d, m, border=border, border_value=bval, mean=mean, std=std)
            exp = oracle.warp(host, m, dh, dw, o, False, border, bval, mean, std, threads=TH)
        else:
            kr.warp_perspective(src, d, m, border=border, border_value=bval, mean=mean, std=std)
            exp = oracle.warp_perspective(host, m, dh, dw, o, False, border, bval, mean, std, threads=TH)
        torch.cuda.synchronize()
        got = d.cpu().numpy()
        what = f"case {i} {op} out={out}"
        if out == "u8":
            assert_u8_equal(got, exp, what)
        else:
            assert_f32_close(got, exp, what, std=std)


@pytest.mark.parametrize("block", range(4))
def test_random_sweep(block):
    rng = np.random.default_rng(2024 + block)
    for i in range(block * 40, block * 40 + 40):
        run_case(rng, i)


@pytest.mark.parametrize("block", range(3))
def test_random_batch_sweep(block):
    """Random batches (resizes and warps, views among the sources, u8 or
    normalised f32, interleaved or planar destinations) against the oracle
    item by item."""
    rng = np.random.default_rng(77 + block)
    for b in range(4):
        c = int(rng.choice([3, 4]))
        out = ["u8", "f32"][int(rng.integers(0, 2))]
        planar = bool(rng.random() < 0.5)
        border = int(rng.integers(0, 2))
        bval = float(rng.integers(0, 256))
        mean, std = (MEAN[:c], STD[:c]) if out == "f32" else (None, None)
        specs, exps = [], []
        n = int(rng.integers(1, 40))
        for i in range(n):
            h, w = int(rng.integers(1, 400)), int(rng.integers(1, 400))
            dh, dw = int(rng.integers(1, 300)), int(rng.integers(1, 300))
            src, host = random_source(rng, h, w, c, False, bool(rng.random() < 0.4))
            o = "u8" if out == "u8" else "f64"
            if rng.random() < 0.5:
                m = random_affine(rng, h, w)
                specs.append({"op": "warp", "src": src, "m": m})
                exps.append(oracle.warp(host, m, dh, dw, o, False, border, bval, mean, std, threads=TH))
            else:
                specs.append({"op": "resize", "src": src})
                exps.append(oracle.resize(host, dh, dw, o, border, bval, mean, std, threads=TH))
            shape = (c, dh, dw) if planar else (dh, dw, c)
            specs[-1]["dst"] = torch.empty(shape, dtype=torch.uint8 if out == "u8" else torch.float32, device="cuda")
        say(f"batch sweep {block}.{b}: {n} items c={c} out={out} planar={planar} border={border} bval={bval}")
        kr.resize_batch(specs, border=border, border_value=bval, mean=mean, std=std,
                        layout=kr.LAYOUT_CHW if planar else kr.LAYOUT_HWC)
        torch.cuda.synchronize()
        for i, (sp, exp) in enumerate(zip(specs, exps)):
            got = sp["dst"].cpu().numpy()
            if planar:
                got = np.ascontiguousarray(np.transpose(got, (1, 2, 0)))
            what = f"batch {block}.{b} item {i} ({sp['op']})"
            if out == "u8":
                assert_u8_equal(got, exp, what)
            else:
                assert_f32_close(got, exp, what, std=std)
