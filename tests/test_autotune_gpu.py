"""GPU checks of the autotuner through the C ABI: tuning leaves the correct
output in dst, and every compiled tile configuration -- each forced in turn
through a loaded tuning table -- gives bit-identical results, equal to the
oracle (u8 exact, f32 within 1e-3), for single images and batches."""
from __future__ import annotations

import os
import re

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

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
TH = 16


def compiled_cfgs(macro):
    text = open(os.path.join(ROOT, "paper_2505_12425_amd", "csrc", "tiled_launch.h")).read()
    text = text.replace("\\\n", " ")  # join continued macro lines
    body = re.search(rf"#define {macro}\(X\)(.*)", text).group(1)
    return [tuple(int(v) for v in g) for g in re.findall(r"X\((\d+), (\d+), (\d+), (\d+)\)", body)]


@pytest.fixture(autouse=True)
def clean_table():
    kr.autotune_clear()
    yield
    kr.autotune_clear()


def tuned_keys(batch):
    out = []
    for ln in kr.autotune_save().splitlines():
        if ln.startswith("#") or ln.startswith("key "):
            continue
        v = ln.split()
        if int(v[3]) == batch:
            out.append(" ".join(v[:6]))
    return out


@pytest.mark.parametrize("op,out", [("resize", "u8"), ("resize", "f32"), ("warp", "u8"), ("warp", "f32")])
def test_every_image_config_bit_exact(op, out):
    h, w = 1000, 1400
    im = wl.uniform_u8(h, w, 3, seed=41)
    dt = torch.uint8 if out == "u8" else torch.float32
    if op == "resize":
        dh, dw, m = 613, 777, None
        exp = oracle.resize(im, dh, dw, out if out == "u8" else "f64", oracle.REPLICATE, threads=TH)
        border = kr.REPLICATE
    else:
        dh, dw = 901, 1203
        m = wl.affine_compose(h, w, 23.0, 0.85, 0.1, (dw - w) / 2.0, (dh - h) / 2.0)
        exp = oracle.warp(im, m, dh, dw, out if out == "u8" else "f64", threads=TH)
        border = kr.CONSTANT
    src = torch.from_numpy(im).cuda()

    def run():
        d = torch.empty((dh, dw, 3), dtype=dt, device="cuda")
        if op == "warp":
            kr.warp_affine(src, d, m, border=border)
        else:
            kr.resize(src, d, border=border)
        torch.cuda.synchronize()
        return d.cpu().numpy()

    default = run()
    d = torch.empty((dh, dw, 3), dtype=dt, device="cuda")
    scrub = torch.empty(32 << 20, dtype=torch.uint8, device="cuda") if out == "u8" else None
    say(f"autotune {op} {out}: {kr.autotune_image(op, src, d, m, border=border, reps=3, scrub=scrub)}")
    torch.cuda.synchronize()
    tuned = d.cpu().numpy()
    if out == "u8":
        assert_u8_equal(tuned, exp, f"{op} tuned vs oracle")
    else:
        assert_f32_close(tuned, exp, f"{op} tuned vs oracle")
    assert np.array_equal(tuned, default)
    (key,) = tuned_keys(0)
    for px, txt, cpt, rpt in compiled_cfgs("KR_WARP_CFGS" if op == "warp" else "KR_RESIZE_CFGS"):
        for grid in (0, 1):  # one workgroup per tile, persistent
            kr.autotune_clear()
            kr.autotune_load(f"key {kr.build_key()}\n{key} {px} {txt} {cpt} {rpt} {grid}\n")
            got = run()
            assert np.array_equal(got, default), f"{op} {out} config {px}x{txt}x{cpt}x{rpt} grid={grid}"


@pytest.mark.parametrize("out", ["u8", "f32"])
def test_every_batch_config_bit_exact(out):
    rng = np.random.default_rng(31)
    dt = torch.uint8 if out == "u8" else torch.float32
    specs = []
    for i in range(20):
        h, w = int(rng.integers(60, 1300)), int(rng.integers(60, 1300))
        im = torch.from_numpy(wl.uniform_u8(h, w, 3, seed=900 + i)).cuda()
        t = int(rng.choice([32, 224, 333]))
        sp = {"op": "resize", "src": im, "dst": torch.empty((t, t, 3), dtype=dt, device="cuda")}
        if i % 2:
            sp["op"] = "warp"
            sp["m"] = wl.affine_compose(h, w, rng.uniform(-60, 60), t / max(h, w) * rng.uniform(0.6, 1.4),
                                        rng.uniform(-0.2, 0.2), (t - w) / 2.0, (t - h) / 2.0)
        specs.append(sp)
    kr.resize_batch(specs, border=kr.REPLICATE)
    torch.cuda.synchronize()
    default = [sp["dst"].cpu().numpy() for sp in specs]
    for sp in specs:
        sp["dst"].zero_()
    scrub = torch.empty(32 << 20, dtype=torch.uint8, device="cuda") if out == "f32" else None
    say(f"autotune batch {out}: {kr.autotune_batch(specs, border=kr.REPLICATE, reps=2, scrub=scrub)}")
    torch.cuda.synchronize()
    for k, sp in enumerate(specs):
        assert np.array_equal(sp["dst"].cpu().numpy(), default[k]), f"tuned batch item {k}"
    keys = tuned_keys(1)
    assert len(keys) == 2
    for key in keys:
        op = int(key.split()[0])
        for px, txt, cpt, rpt in compiled_cfgs("KR_BATCH_WARP_CFGS" if op == 1 else "KR_BATCH_RESIZE_CFGS"):
            for grid in (0, 1):  # one workgroup per tile, persistent
                kr.autotune_clear()
                kr.autotune_load(f"key {kr.build_key()}\n{key} {px} {txt} {cpt} {rpt} {grid}\n")
                for sp in specs:
                    sp["dst"].zero_()
                kr.resize_batch(specs, border=kr.REPLICATE)
                torch.cuda.synchronize()
                for k, sp in enumerate(specs):
                    assert np.array_equal(sp["dst"].cpu().numpy(), default[k]), \
                        f"batch op {op} config {px}x{txt}x{cpt}x{rpt} grid {grid} item {k}"
