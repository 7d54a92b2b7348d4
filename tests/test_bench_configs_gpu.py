"""GPU parity of the benchmarked batch workloads, exactly as bench.py builds
them, in the form it times (the graph-captured plan), against the oracle.

* 256 RGB u8 images, H and W uniform in [240, 2160] (seed 0), bilinear to
  224x224, u8 -> f32 with ImageNet mean/std, REPLICATE border (HWC and the
  planar NCHW destination);
* 64 RGB u8 1920x1080 images (seeds 100 + i), each warped by its own
  random_affine_batch map drawn from one rng seeded 0, constant-0 border,
  u8 output.

Every item of every plan replay is compared with the oracle (u8 bit-exact;
f32 within 1e-3 on the 0..255 scale, i.e. |d| * 255 * std_c <= 1e-3 in
normalised units), and the plan's outputs equal the eager batch call's bit
for bit.
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


def test_batch_resize_256_plan_vs_oracle():
    shapes = wl.batch_shapes(256, 240, 2160, seed=0)
    imgs = [wl.uniform_u8(h, w, 3, seed=i) for i, (h, w) in enumerate(shapes)]
    srcs = [torch.from_numpy(im).cuda() for im in imgs]
    hwc = [{"op": "resize", "src": s, "dst": torch.empty((224, 224, 3), dtype=torch.float32, device="cuda")}
           for s in srcs]
    nchw = torch.empty((256, 3, 224, 224), dtype=torch.float32, device="cuda")
    chw = [{"op": "resize", "src": s, "dst": nchw[i]} for i, s in enumerate(srcs)]
    refs = [oracle.resize(im, 224, 224, "f64", oracle.REPLICATE, 0, MEAN, STD, threads=TH) for im in imgs]
    kr.resize_batch(hwc, border=kr.REPLICATE, mean=MEAN, std=STD)
    torch.cuda.synchronize()
    eager = [sp["dst"].clone() for sp in hwc]
    plan = kr.BatchPlan(hwc, border=kr.REPLICATE, mean=MEAN, std=STD)
    plan_chw = kr.BatchPlan(chw, border=kr.REPLICATE, mean=MEAN, std=STD, layout=kr.LAYOUT_CHW)
    try:
        for rep in range(2):
            say(f"256-image resize plan, replay {rep}")
            for sp in hwc:
                sp["dst"].fill_(-1.0)
            nchw.fill_(-1.0)
            plan.launch()
            plan_chw.launch()
            torch.cuda.synchronize()
            got = [sp["dst"].cpu().numpy() for sp in hwc]
            got_chw = nchw.cpu().numpy()
            for i in range(256):
                assert_f32_close(got[i], refs[i], f"plan replay {rep} item {i} {shapes[i]}", std=STD)
                assert np.array_equal(got[i], eager[i].cpu().numpy()), f"replay {rep} item {i}: plan != batch"
                assert np.array_equal(got_chw[i].transpose(1, 2, 0), got[i]), f"replay {rep} item {i}: CHW != HWC"
    finally:
        plan.close()
        plan_chw.close()


def test_batch_warp_64_plan_vs_oracle():
    rng = np.random.default_rng(0)
    imgs, mats = [], []
    for i in range(64):
        imgs.append(wl.uniform_u8(1080, 1920, 3, seed=100 + i))
        mats.append(wl.random_affine_batch(1080, 1920, rng))
    specs = [{"op": "warp", "src": torch.from_numpy(im).cuda(), "m": m,
              "dst": torch.empty((1080, 1920, 3), dtype=torch.uint8, device="cuda")} for im, m in zip(imgs, mats)]
    kr.resize_batch(specs, border=kr.CONSTANT, border_value=0)
    torch.cuda.synchronize()
    eager = [sp["dst"].clone() for sp in specs]
    plan = kr.BatchPlan(specs, border=kr.CONSTANT)
    try:
        for rep in range(2):
            say(f"64 x 1080p warp plan, replay {rep}")
            for sp in specs:
                sp["dst"].fill_(123)
            plan.launch()
            torch.cuda.synchronize()
            for i, (im, m) in enumerate(zip(imgs, mats)):
                got = specs[i]["dst"].cpu().numpy()
                if rep == 0:
                    assert_u8_equal(got, oracle.warp(im, m, 1080, 1920, "u8", threads=TH), f"warp plan item {i}")
                assert np.array_equal(got, eager[i].cpu().numpy()), f"replay {rep} item {i}: plan != batch"
    finally:
        plan.close()
