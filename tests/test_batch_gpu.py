"""GPU parity of the batched forms (one launch per operation over a work-list
of output tiles, and its graph-captured plan) through the C ABI.

Every item must equal the oracle (u8 bit-exact, f32 within 1e-3 on the 0..255
scale) and equal the single-image call on the same item bit for bit.
"""
from __future__ import annotations

import numpy as np
import pytest

import oracle
from paper_2505_12425_amd import workloads as wl
from tests.gpu_util import assert_f32_close, assert_u8_equal, say

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

from paper_2505_12425_amd import kr  # noqa: E402

MEAN, STD = wl.IMAGENET_MEAN, wl.IMAGENET_STD
TH = 16


def _single(spec, **kw):
    d = torch.empty_like(spec["dst"])
    if spec["op"] == "warp":
        kr.warp_affine(spec["src"], d, spec["m"], **kw)
    else:
        kr.resize(spec["src"], d, **kw)
    return d


def test_batch_256_mixed_sizes_to_224_normalized():
    shapes = wl.batch_shapes(256, 240, 2160, seed=0)
    say(f"batch resize 256 images -> 224x224 f32 normalized (first {shapes[:3]})")
    imgs = [wl.uniform_u8(h, w, 3, seed=i) for i, (h, w) in enumerate(shapes)]
    specs = [{"op": "resize", "src": torch.from_numpy(im).cuda(),
              "dst": torch.empty((224, 224, 3), dtype=torch.float32, device="cuda")} for im in imgs]
    kr.resize_batch(specs, border=kr.REPLICATE, mean=MEAN, std=STD)
    torch.cuda.synchronize()
    for i, (im, sp) in enumerate(zip(imgs, specs)):
        got = sp["dst"].cpu().numpy()
        exp = oracle.resize(im, 224, 224, "f64", oracle.REPLICATE, 0, MEAN, STD, threads=TH)
        assert_f32_close(got, exp, f"item {i} {im.shape}", std=STD)
        single = _single(sp, border=kr.REPLICATE, mean=MEAN, std=STD)
        torch.cuda.synchronize()
        assert np.array_equal(single.cpu().numpy(), got), f"item {i}: batch != single"


def test_batch_64_warps_1080p_u8():
    rng = np.random.default_rng(3)
    say("batch warp 64 x 1080p u8")
    imgs, specs = [], []
    for i in range(64):
        im = wl.uniform_u8(1080, 1920, 3, seed=100 + i)
        m = wl.random_affine_batch(1080, 1920, rng)
        imgs.append((im, m))
        specs.append({"op": "warp", "src": torch.from_numpy(im).cuda(), "m": m,
                      "dst": torch.empty((1080, 1920, 3), dtype=torch.uint8, device="cuda")})
    kr.resize_batch(specs, border=kr.CONSTANT, border_value=0)
    torch.cuda.synchronize()
    for i, ((im, m), sp) in enumerate(zip(imgs, specs)):
        got = sp["dst"].cpu().numpy()
        if i % 4 == 0:  # the oracle on every fourth image, all compared with the single call
            assert_u8_equal(got, oracle.warp(im, m, 1080, 1920, "u8", threads=TH), f"warp item {i}")
        single = _single(sp, border=kr.CONSTANT)
        torch.cuda.synchronize()
        assert np.array_equal(single.cpu().numpy(), got), f"item {i}: batch != single"


@pytest.mark.parametrize("c,out", [(3, "u8"), (3, "f32"), (4, "u8"), (1, "u8"), (2, "f32")])
def test_mixed_batch_and_plan_replays(c, out):
    rng = np.random.default_rng(7 + c)
    dt = torch.uint8 if out == "u8" else torch.float32
    say(f"mixed batch c={c} out={out}")
    specs, refs = [], []
    for i in range(24):
        h, w = int(rng.integers(20, 700)), int(rng.integers(20, 700))
        im = wl.uniform_u8(h, w, c, seed=300 + i)
        dh, dw = int(rng.integers(8, 500)), int(rng.integers(8, 500))
        if i % 3 == 0:
            m = wl.affine_compose(h, w, rng.uniform(-60, 60), rng.uniform(0.3, 2.0), rng.uniform(-0.3, 0.3),
                                  rng.uniform(-50, 50), rng.uniform(-50, 50))
            spec = {"op": "warp", "src": torch.from_numpy(im).cuda(), "m": m,
                    "dst": torch.empty((dh, dw, c), dtype=dt, device="cuda")}
            ref = oracle.warp(im, m, dh, dw, "u8" if out == "u8" else "f64", False, oracle.REPLICATE, 0)
        else:
            spec = {"op": "resize", "src": torch.from_numpy(im).cuda(),
                    "dst": torch.empty((dh, dw, c), dtype=dt, device="cuda")}
            ref = oracle.resize(im, dh, dw, "u8" if out == "u8" else "f64", oracle.REPLICATE, 0)
        specs.append(spec)
        refs.append(ref)

    def check_all(tag):
        for i, (sp, ref) in enumerate(zip(specs, refs)):
            got = sp["dst"].cpu().numpy()
            if out == "u8":
                assert_u8_equal(got, ref, f"{tag} item {i}")
            else:
                assert_f32_close(got, ref, f"{tag} item {i}")

    kr.resize_batch(specs, border=kr.REPLICATE)
    torch.cuda.synchronize()
    check_all("batch")
    eager = [sp["dst"].clone() for sp in specs]
    plan = kr.BatchPlan(specs, border=kr.REPLICATE)
    try:
        for rep in range(3):
            for sp in specs:
                sp["dst"].zero_()
            scratch = torch.randn(1 << 20, device="cuda")  # unrelated eager work between replays
            scratch.mul_(2.0)
            plan.launch()
            torch.cuda.synchronize()
            for i, sp in enumerate(specs):
                assert torch.equal(sp["dst"], eager[i]), f"replay {rep} item {i} differs from eager"
    finally:
        plan.close()


def test_batch_single_item_and_empty():
    im = wl.uniform_u8(37, 53, 3, seed=9)
    src = torch.from_numpy(im).cuda()
    dst = torch.empty((19, 77, 3), dtype=torch.uint8, device="cuda")
    kr.resize_batch([{"op": "resize", "src": src, "dst": dst}])
    torch.cuda.synchronize()
    assert_u8_equal(dst.cpu().numpy(), oracle.resize(im, 19, 77, "u8"), "single-item batch")
    kr.resize_batch([])  # nothing to do


def test_prepared_batch_calls_equal_resize_batch():
    """kr.prepare_batch marshals once and calls kr_resize_batch_ex again on
    every call: each call equals resize_batch, bit for bit."""
    rng = np.random.default_rng(5)
    specs, ref = [], []
    for i in range(12):
        h, w = int(rng.integers(20, 300)), int(rng.integers(20, 300))
        src = torch.from_numpy(wl.uniform_u8(h, w, 3, seed=200 + i)).cuda()
        op = "warp" if i % 3 == 0 else "resize"
        dh, dw = (h, w) if op == "warp" else (int(rng.integers(8, 200)), int(rng.integers(8, 200)))
        sp = {"op": op, "src": src, "dst": torch.empty((dh, dw, 3), dtype=torch.float32, device="cuda")}
        if op == "warp":
            sp["m"] = wl.random_affine_batch(h, w, rng)
        specs.append(sp)
        ref.append(dict(sp, dst=torch.empty_like(sp["dst"])))
    kr.resize_batch(ref, border=kr.CONSTANT, border_value=7.0, mean=MEAN, std=STD)
    call = kr.prepare_batch(specs, border=kr.CONSTANT, border_value=7.0, mean=MEAN, std=STD)
    for rep in range(3):
        for sp in specs:
            sp["dst"].fill_(-1.0)
        call()
        torch.cuda.synchronize()
        for a, b in zip(specs, ref):
            assert torch.equal(a["dst"], b["dst"]), f"call {rep}"
    kr.prepare_batch([])()  # nothing to do


@pytest.mark.parametrize("out", ["u8", "f32"])
def test_warp_batch_all_lds_classes(out):
    """Warps whose boxes fit the primary tile shape, only 32x32 tiles, or no
    tile at all (strong shrinks under rotation: global-gather path) share one
    batch; every item equals its single call bitwise and the oracle."""
    rng = np.random.default_rng(21)
    dt = torch.uint8 if out == "u8" else torch.float32
    specs, refs = [], []
    scales = [1.0, 0.9, 0.55, 0.5, 0.3, 0.2, 1.3, 0.25]
    for i, sc in enumerate(scales):
        h, w = 700 + 37 * i, 900 + 53 * i
        im = wl.uniform_u8(h, w, 3, seed=300 + i)
        m = wl.affine_compose(h, w, 40.0 + 2 * i, sc, 0.1, rng.uniform(-20, 20), rng.uniform(-20, 20))
        dh, dw = 480 + 16 * i, 640 + 8 * i
        specs.append({"op": "warp", "src": torch.from_numpy(im).cuda(), "m": m,
                      "dst": torch.empty((dh, dw, 3), dtype=dt, device="cuda")})
        refs.append((im, m, dh, dw))
    say(f"warp batch over LDS classes, out={out}")
    kr.resize_batch(specs, border=kr.CONSTANT, border_value=9)
    torch.cuda.synchronize()
    for i, (sp, (im, m, dh, dw)) in enumerate(zip(specs, refs)):
        got = sp["dst"].cpu().numpy()
        single = _single(sp, border=kr.CONSTANT, border_value=9)
        torch.cuda.synchronize()
        assert np.array_equal(single.cpu().numpy(), got), f"item {i} (scale {scales[i]}): batch != single"
        if out == "u8":
            assert_u8_equal(got, oracle.warp(im, m, dh, dw, "u8", border=oracle.CONSTANT, bval=9, threads=TH),
                            f"item {i}")
        else:
            assert_f32_close(got, oracle.warp(im, m, dh, dw, "f64", border=oracle.CONSTANT, bval=9, threads=TH),
                             f"item {i}")


@pytest.mark.parametrize("out", ["u8", "f32"])
def test_warp_batch_launch_box_budget(out):
    """Warps whose boxes each fit the batch LDS budget but not together: at a
    0.7x shrink the default 64x16 tiles need wide boxes at 0 degrees and tall
    ones at 90 degrees, and the launch's box (widest pitch times most rows)
    would exceed the budget, so the tall ones move to the gather path.  Every
    item equals its single call bitwise and the oracle."""
    dt = torch.uint8 if out == "u8" else torch.float32
    specs, refs = [], []
    for i, theta in enumerate([0.0, 90.0, 0.0, 90.0, 2.0, 88.0]):
        h, w = 260 + 6 * i, 340 + 10 * i
        im = wl.uniform_u8(h, w, 3, seed=500 + i)
        m = wl.affine_compose(h, w, theta, 0.7, 0.0, 3.0 * i, -2.0 * i)
        specs.append({"op": "warp", "src": torch.from_numpy(im).cuda(), "m": m,
                      "dst": torch.empty((h, w, 3), dtype=dt, device="cuda")})
        refs.append((im, m, h, w))
    say(f"warp batch, launch box over the budget, out={out}")
    kr.resize_batch(specs, border=kr.CONSTANT, border_value=5)
    torch.cuda.synchronize()
    for i, (sp, (im, m, dh, dw)) in enumerate(zip(specs, refs)):
        got = sp["dst"].cpu().numpy()
        single = _single(sp, border=kr.CONSTANT, border_value=5)
        torch.cuda.synchronize()
        assert np.array_equal(single.cpu().numpy(), got), f"item {i}: batch != single"
        if out == "u8":
            assert_u8_equal(got, oracle.warp(im, m, dh, dw, "u8", border=oracle.CONSTANT, bval=5, threads=TH),
                            f"item {i}")
        else:
            assert_f32_close(got, oracle.warp(im, m, dh, dw, "f64", border=oracle.CONSTANT, bval=5, threads=TH),
                             f"item {i}")


@pytest.mark.parametrize("c,out", [(3, "f32"), (3, "u8"), (4, "u8"), (4, "f32"), (1, "f32"), (2, "u8")])
def test_planar_layout_equals_interleaved(c, out):
    """CHW destinations hold exactly the HWC results, transposed, for a mixed
    batch of resizes and warps (single launch and plan); spot-checked against
    the oracle."""
    rng = np.random.default_rng(40 + c)
    dt = torch.uint8 if out == "u8" else torch.float32
    mean = (MEAN + (0.5,))[:c] if out == "f32" else None
    std = (STD + (0.25,))[:c] if out == "f32" else None
    hwc, chw, refs = [], [], []
    for i in range(12):
        h, w = int(rng.integers(50, 700)), int(rng.integers(50, 700))
        im = wl.uniform_u8(h, w, c, seed=700 + i)
        s = torch.from_numpy(im).cuda()
        th, tw = int(rng.choice([37, 224, 301])), int(rng.choice([64, 224, 255]))
        sp = {"op": "resize", "src": s}
        if i % 3 == 1:
            sp = {"op": "warp", "src": s, "m": wl.affine_compose(h, w, rng.uniform(-30, 30), min(th, tw) / max(h, w),
                                                                 0.05, (tw - w) / 2.0, (th - h) / 2.0)}
        hwc.append(dict(sp, dst=torch.empty((th, tw, c), dtype=dt, device="cuda")))
        chw.append(dict(sp, dst=torch.empty((c, th, tw), dtype=dt, device="cuda")))
        refs.append((im, sp.get("m"), th, tw))
    say(f"planar batch c={c} out={out}")
    kr.resize_batch(hwc, border=kr.REPLICATE, mean=mean, std=std)
    kr.resize_batch(chw, border=kr.REPLICATE, mean=mean, std=std, layout=kr.LAYOUT_CHW)
    torch.cuda.synchronize()
    for k, (a, b) in enumerate(zip(hwc, chw)):
        assert np.array_equal(a["dst"].cpu().numpy().transpose(2, 0, 1), b["dst"].cpu().numpy()), f"item {k}"
    plan = kr.BatchPlan(chw, border=kr.REPLICATE, mean=mean, std=std, layout=kr.LAYOUT_CHW)
    for sp in chw:
        sp["dst"].zero_()
    plan.launch()
    torch.cuda.synchronize()
    for k, (a, b) in enumerate(zip(hwc, chw)):
        assert np.array_equal(a["dst"].cpu().numpy().transpose(2, 0, 1), b["dst"].cpu().numpy()), f"plan item {k}"
    plan.close()
    im, m, th, tw = refs[0]
    got = chw[0]["dst"].cpu().numpy().transpose(1, 2, 0)
    if out == "u8":
        assert_u8_equal(got, oracle.resize(im, th, tw, "u8", oracle.REPLICATE, threads=TH), "item 0 vs oracle")
    else:
        assert_f32_close(got, oracle.resize(im, th, tw, "f64", oracle.REPLICATE, 0, mean, std, threads=TH),
                         "item 0 vs oracle", std=std)
