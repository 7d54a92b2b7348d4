"""kr_resize_batch_noalloc (the batch entry point that allocates nothing: its
work-list lives in the library's own per-GPU device scratch) against
kr_resize_batch_ex with a caller workspace, through the C ABI.

Two calls in a row share the scratch, the second with fewer and smaller
items, so a stale work-list from the first call would show.  Outputs must be
bit-identical to the workspace entry point's (u8 and f32, HWC and CHW), and
spot-checked against the oracle.  Oversized batches are rejected on the host
before anything is enqueued.
"""
from __future__ import annotations

import ctypes

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


def _specs(n, seed, c, dt, layout, big):
    """n mixed resize / warp items (sizes up to `big`), fresh destinations."""
    rng = np.random.default_rng(seed)
    specs = []
    for i in range(n):
        h, w = int(rng.integers(16, big)), int(rng.integers(16, big))
        im = wl.uniform_u8(h, w, c, seed=seed * 1000 + i)
        dh, dw = int(rng.integers(8, big)), int(rng.integers(8, big))
        shape = (c, dh, dw) if layout == kr.LAYOUT_CHW else (dh, dw, c)
        sp = {"op": "resize", "src": torch.from_numpy(im).cuda(), "host": im,
              "dst": torch.empty(shape, dtype=dt, device="cuda")}
        if i % 3 == 1:
            sp["op"] = "warp"
            sp["m"] = wl.affine_compose(h, w, rng.uniform(-50, 50), rng.uniform(0.4, 1.8), rng.uniform(-0.2, 0.2),
                                        rng.uniform(-30, 30), rng.uniform(-30, 30))
        specs.append(sp)
    return specs


def _twin(specs):
    return [dict(sp, dst=torch.empty_like(sp["dst"])) for sp in specs]


@pytest.mark.parametrize("c,out,layout", [(3, "u8", kr.LAYOUT_HWC), (3, "f32", kr.LAYOUT_HWC),
                                          (4, "u8", kr.LAYOUT_CHW), (3, "f32", kr.LAYOUT_CHW)])
def test_noalloc_equals_workspace_entry_point(c, out, layout):
    dt = torch.uint8 if out == "u8" else torch.float32
    mean = (MEAN + (0.5,))[:c] if out == "f32" else None
    std = (STD + (0.25,))[:c] if out == "f32" else None
    for call, (n, big) in enumerate([(40, 900), (7, 300)]):  # the second call is smaller
        say(f"noalloc call {call}: {n} items c={c} out={out} layout={layout}")
        a = _specs(n, 50 + call + 10 * c, c, dt, layout, big)
        b = _twin(a)
        for sp in a + b:
            sp["dst"].fill_(77)
        kr.resize_batch(a, border=kr.REPLICATE, mean=mean, std=std, layout=layout)
        kr.resize_batch_noalloc(b, border=kr.REPLICATE, mean=mean, std=std, layout=layout)
        torch.cuda.synchronize()
        for i, (x, y) in enumerate(zip(a, b)):
            assert torch.equal(x["dst"], y["dst"]), f"call {call} item {i} ({x['op']}): noalloc != workspace"
        # the oracle on the first item of each operation
        for op in ("resize", "warp"):
            sp = next(s for s in b if s["op"] == op)
            im = sp["host"]
            got = sp["dst"].cpu().numpy()
            if layout == kr.LAYOUT_CHW:
                got = got.transpose(1, 2, 0)
            dh, dw = got.shape[:2]
            if op == "resize":
                ref = oracle.resize(im, dh, dw, "u8" if out == "u8" else "f64", oracle.REPLICATE, 0, mean, std)
            else:
                ref = oracle.warp(im, sp["m"], dh, dw, "u8" if out == "u8" else "f64", False, oracle.REPLICATE, 0,
                                  mean, std)
            if out == "u8":
                assert_u8_equal(got, ref, f"call {call} {op} vs oracle")
            else:
                assert_f32_close(got, ref, f"call {call} {op} vs oracle", std=std)


def test_noalloc_same_stream_back_to_back():
    """Two calls enqueued on one stream without a host synchronisation in
    between (stream order protects the shared scratch), then a third on
    another stream after synchronising."""
    a1 = _specs(30, 90, 3, torch.uint8, kr.LAYOUT_HWC, 700)
    a2 = _specs(5, 91, 3, torch.uint8, kr.LAYOUT_HWC, 200)
    ref1, ref2 = _twin(a1), _twin(a2)
    kr.resize_batch(ref1, border=kr.CONSTANT, border_value=3)
    kr.resize_batch(ref2, border=kr.CONSTANT, border_value=3)
    s = torch.cuda.Stream()
    with torch.cuda.stream(s):
        kr.resize_batch_noalloc(a1, border=kr.CONSTANT, border_value=3, stream=s)
        kr.resize_batch_noalloc(a2, border=kr.CONSTANT, border_value=3, stream=s)
    torch.cuda.synchronize()
    for i, (x, y) in enumerate(zip(a1 + a2, ref1 + ref2)):
        assert torch.equal(x["dst"], y["dst"]), f"item {i}: back-to-back noalloc != workspace"
    a3 = _twin(a2)
    kr.resize_batch_noalloc(a3, border=kr.CONSTANT, border_value=3)
    torch.cuda.synchronize()
    for i, (x, y) in enumerate(zip(a3, ref2)):
        assert torch.equal(x["dst"], y["dst"]), f"item {i}: default-stream noalloc != workspace"


def test_noalloc_rejects_oversized_batch():
    """More than KR_NOALLOC_MAX_ITEMS items: KR_ERR_WORKSPACE_TOO_SMALL from
    the host check, before any item is read or anything enqueued."""
    n = kr.NOALLOC_MAX_ITEMS + 1
    items = (kr.BatchItem * n)()
    st = kr.lib().kr_resize_batch_noalloc(items, n, 3, 0, 0, kr.REPLICATE, 0.0, None, kr.LAYOUT_HWC, None)
    assert st == 4, (st, kr.last_error())
    assert "at most" in kr.last_error()
    # a valid call still works afterwards
    a = _specs(3, 92, 3, torch.uint8, kr.LAYOUT_HWC, 100)
    b = _twin(a)
    kr.resize_batch(a)
    kr.resize_batch_noalloc(b)
    torch.cuda.synchronize()
    for x, y in zip(a, b):
        assert torch.equal(x["dst"], y["dst"])
