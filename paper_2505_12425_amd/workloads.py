"""Seeded synthetic inputs shared by the tests, the benchmark and the oracle checks.

This module draws images, affine matrices, batch shapes and request streams.
It holds none of the resampling arithmetic: it neither interpolates nor maps
coordinates.  Everything is a pure function of its seed
(``numpy.random.default_rng``), so the GPU path and the oracle always see the
same inputs.

The paper benchmarks its operators on unspecified images (Sec. III); these
generators stand in for them with the shapes used here:

* uniform random u8 images;
* a smooth per-channel gradient, and the 4K mix (U + G + 1) >> 1 of both;
* random affine maps composed as T(c + t) R(theta) Sh(k) S(s) T(-c) about the
  image centre c = ((W - 1) / 2, (H - 1) / 2);
* batches of images with H, W uniform in a range;
* a Poisson request stream of resize (70 %) / warp (30 %) jobs whose pixel
  count is log-uniform in [0.1, 8] MP with aspect ratio log-uniform in [0.5, 2]
  and square targets from {224, 384, 512, 1024}.
"""
from __future__ import annotations

import math
from dataclasses import dataclass

import numpy as np

# Per-channel normalisation constants of the batched 224x224 workload, on the
# [0, 1] scale.
IMAGENET_MEAN = (0.485, 0.456, 0.406)
IMAGENET_STD = (0.229, 0.224, 0.225)


def uniform_u8(h: int, w: int, c: int = 3, seed: int = 0) -> np.ndarray:
    """HxWxC u8 image with i.i.d. uniform samples in [0, 255]."""
    rng = np.random.default_rng(seed)
    return rng.integers(0, 256, size=(h, w, c), dtype=np.uint8)


def uniform_f32(h: int, w: int, c: int = 3, seed: int = 0) -> np.ndarray:
    """HxWxC f32 image with i.i.d. uniform samples in [0, 255)."""
    rng = np.random.default_rng(seed)
    return (rng.random(size=(h, w, c)) * 255.0).astype(np.float32)


def gradient_u8(h: int, w: int, c: int = 3) -> np.ndarray:
    """Smooth gradient G(x, y, ch) = floor(255 (w_ch x / (W-1) + (1 - w_ch) y / (H-1)))
    with channel weights w = (1, 1/2, 0) (cycled for more channels)."""
    wts = [1.0, 0.5, 0.0, 0.25]
    xs = np.arange(w, dtype=np.float64) / max(w - 1, 1)
    ys = np.arange(h, dtype=np.float64) / max(h - 1, 1)
    out = np.empty((h, w, c), np.uint8)
    for ch in range(c):
        wc = wts[ch % len(wts)]
        g = np.floor(255.0 * (wc * xs[None, :] + (1.0 - wc) * ys[:, None]))
        out[:, :, ch] = np.clip(g, 0, 255).astype(np.uint8)
    return out


def mixed_u8(h: int, w: int, c: int = 3, seed: int = 0) -> np.ndarray:
    """(U + G + 1) >> 1: uniform noise averaged with the smooth gradient."""
    u = uniform_u8(h, w, c, seed).astype(np.uint16)
    g = gradient_u8(h, w, c).astype(np.uint16)
    return ((u + g + 1) >> 1).astype(np.uint8)


def affine_compose(h: int, w: int, theta_deg: float, scale: float, shear: float,
                   tx: float, ty: float) -> np.ndarray:
    """Forward (source -> destination) 2x3 map T(c + t) R(theta) Sh(k) S(s) T(-c)."""
    cx, cy = (w - 1) / 2.0, (h - 1) / 2.0
    th = math.radians(theta_deg)
    r = np.array([[math.cos(th), -math.sin(th), 0.0],
                  [math.sin(th), math.cos(th), 0.0],
                  [0.0, 0.0, 1.0]])
    sh = np.array([[1.0, shear, 0.0], [0.0, 1.0, 0.0], [0.0, 0.0, 1.0]])
    s = np.array([[scale, 0.0, 0.0], [0.0, scale, 0.0], [0.0, 0.0, 1.0]])
    t_in = np.array([[1.0, 0.0, -cx], [0.0, 1.0, -cy], [0.0, 0.0, 1.0]])
    t_out = np.array([[1.0, 0.0, cx + tx], [0.0, 1.0, cy + ty], [0.0, 0.0, 1.0]])
    m = t_out @ r @ sh @ s @ t_in
    return np.ascontiguousarray(m[:2, :])


def random_affine_4k(h: int, w: int, seed: int) -> np.ndarray:
    """Rotation U[-30, 30] deg, scale U[0.8, 1.2], translation U[-100, 100]^2 px,
    no shear (draw order: theta, scale, tx, ty)."""
    rng = np.random.default_rng(seed)
    th = rng.uniform(-30.0, 30.0)
    s = rng.uniform(0.8, 1.2)
    tx, ty = rng.uniform(-100.0, 100.0, size=2)
    return affine_compose(h, w, th, s, 0.0, tx, ty)


def random_affine_batch(h: int, w: int, rng: np.random.Generator) -> np.ndarray:
    """Rotation U[-45, 45] deg, scale U[0.5, 1.5], shear U[-0.2, 0.2],
    translation U[-0.1 W, 0.1 W] x U[-0.1 H, 0.1 H] (draw order: theta, scale,
    shear, tx, ty)."""
    th = rng.uniform(-45.0, 45.0)
    s = rng.uniform(0.5, 1.5)
    k = rng.uniform(-0.2, 0.2)
    tx = rng.uniform(-0.1 * w, 0.1 * w)
    ty = rng.uniform(-0.1 * h, 0.1 * h)
    return affine_compose(h, w, th, s, k, tx, ty)


def batch_shapes(n: int, lo: int = 240, hi: int = 2160, seed: int = 0):
    """n (H, W) pairs with H, W i.i.d. uniform integers in [lo, hi]."""
    rng = np.random.default_rng(seed)
    hs = rng.integers(lo, hi + 1, size=n)
    ws = rng.integers(lo, hi + 1, size=n)
    return [(int(a), int(b)) for a, b in zip(hs, ws)]


@dataclass
class Request:
    """One serving request: resize or warp of a resident u8 RGB source."""
    rid: int
    arrival_s: float
    op: int            # 0 = resize, 1 = warp
    src_h: int
    src_w: int
    dst_h: int
    dst_w: int
    m: tuple           # forward 2x3 map for warps, identity otherwise


def serving_requests(n: int, qps: float, seed: int = 0, targets=(224, 384, 512, 1024)):
    """Poisson arrivals at ``qps``; 70 % resize / 30 % warp; source pixel count
    log-uniform in [0.1, 8] MP, aspect log-uniform in [0.5, 2]; square target
    drawn uniformly from ``targets``.  Warps first fit the source to the target
    (scale by target / max side, centre), then apply a random jitter with the
    batched-warp ranges."""
    rng = np.random.default_rng(seed)
    gaps = rng.exponential(1.0 / qps, size=n)
    arrivals = np.cumsum(gaps) - gaps[0]
    reqs = []
    for i in range(n):
        op = 0 if rng.random() < 0.7 else 1
        p = math.exp(rng.uniform(math.log(0.1e6), math.log(8e6)))
        a = math.exp(rng.uniform(math.log(0.5), math.log(2.0)))
        w = max(1, int(round(math.sqrt(p * a))))
        h = max(1, int(round(math.sqrt(p / a))))
        t = int(targets[rng.integers(0, len(targets))])
        if op == 1:
            fit = t / max(h, w)
            th = rng.uniform(-45.0, 45.0)
            s = fit * rng.uniform(0.5, 1.5)
            k = rng.uniform(-0.2, 0.2)
            tx = rng.uniform(-0.1 * t, 0.1 * t)
            ty = rng.uniform(-0.1 * t, 0.1 * t)
            # about the source centre, then move that centre to the target centre
            m = affine_compose(h, w, th, s, k, tx + (t - w) / 2.0, ty + (t - h) / 2.0)
            mt = tuple(float(v) for v in m.reshape(6))
        else:
            mt = (1.0, 0.0, 0.0, 0.0, 1.0, 0.0)
        reqs.append(Request(i, float(arrivals[i]), op, h, w, t, t, mt))
    return reqs


def random_homography(h: int, w: int, rng: np.random.Generator, jitter: float = 0.15) -> np.ndarray:
    """Forward (source -> destination) 3x3 homography that moves the four image
    corners by independent uniform offsets of up to ``jitter`` times the image
    size (a camera tilt), found from the four correspondences."""
    src = np.array([[0, 0], [w - 1, 0], [0, h - 1], [w - 1, h - 1]], np.float64)
    dst = src + rng.uniform(-jitter, jitter, (4, 2)) * np.array([w, h])
    a, b = [], []
    for (x, y), (u, v) in zip(src, dst):
        a.append([x, y, 1, 0, 0, 0, -u * x, -u * y]); b.append(u)
        a.append([0, 0, 0, x, y, 1, -v * x, -v * y]); b.append(v)
    p = np.linalg.solve(np.array(a), np.array(b))
    return np.append(p, 1.0).reshape(3, 3)
