"""Host logic of bench.py (no GPU): the one-GPU rule of its command line, the
algorithmic-byte counters behind every roofline figure, and the rotation of
destinations that makes every launch write its output back to HBM."""
import json
import os
import subprocess
import sys

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)
import bench  # noqa: E402


def test_more_than_one_gpu_is_refused_with_a_message():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode == 2
    msg = json.loads(r.stdout.strip().splitlines()[-1])
    assert "one GPU" in msg["error"]


def test_resize_touched_bytes_closed_forms():
    # an exact 2x downscale reads every source pixel once: the whole image
    assert bench.resize_touched_bytes(2160, 3840, 1080, 1920) == 2160 * 3840 * 3
    # 4x along both axes: rows 4k + 1 and 4k + 2, columns 4k + 1 and 4k + 2
    h, w = 64, 256
    got = bench.resize_touched_bytes(h, w, h // 4, w // 4, c=4)
    # a touched row's taps, RGBA pixels 4k + 1 and 4k + 2, reach every 128-byte line of the row
    assert got == (h // 2) * (w * 4)
    # f32 elements: four times the bytes of the same u8 footprint
    assert bench.resize_touched_bytes(100, 128, 50, 64, esize=4) == 4 * bench.resize_touched_bytes(100, 128, 50, 64)


def test_warp_touched_bytes_identity_and_outside():
    ident = [1.0, 0.0, 0.0, 0.0, 1.0, 0.0]
    assert bench.warp_touched_bytes(40, 128, 40, 128, ident) == 40 * 128 * 3
    # a map sending every pixel far outside the source reads nothing
    away = [1.0, 0.0, 10000.0, 0.0, 1.0, 0.0]
    assert bench.warp_touched_bytes(40, 128, 40, 128, away) == 0


def test_nearest_touched_bytes_up_and_down():
    # upscale: every source pixel is someone's nearest
    assert bench.nearest_touched_bytes(1080, 1920, 2160, 3840) == 1080 * 1920 * 3
    # 2x downscale picks odd rows and columns: half the rows, all their lines
    assert bench.nearest_touched_bytes(64, 256, 32, 128) == 32 * 256 * 3


def test_rotating_destinations_cover_twice_the_cache():
    import torch
    t = torch.empty((1080, 1920, 3), dtype=torch.float32)
    rot = bench.Rotating(torch, t)
    n = len(rot.copies)
    assert n * t.numel() * 4 >= bench.OUT_ROTATE_BYTES and (n - 1) * t.numel() * 4 < bench.OUT_ROTATE_BYTES
    seen = [rot.next().data_ptr() for _ in range(2 * n)]
    assert len(set(seen)) == n and seen[:n] == seen[n:] and seen[0] == t.data_ptr()
    small = bench.Rotating(torch, torch.empty(16, dtype=torch.uint8))
    assert len(small.copies) == 128  # capped
    big = bench.Rotating(torch, torch.empty(1 << 29, dtype=torch.uint8))
    assert len(big.copies) == 2  # at least two
