"""Helpers for the GPU parity tests: run libkr on numpy inputs through the C ABI
(via the ctypes binding) and compare with the oracle at the stated tolerances:
bit-exact for u8 output, <= 1e-3 absolute on the 0..255 scale for f32 output
(for normalised output: |d| * 255 * std_c <= 1e-3)."""
from __future__ import annotations

import sys

import numpy as np

F32_TOL = 1e-3


def say(msg: str) -> None:
    print(msg, flush=True)
    sys.stdout.flush()


def dev(a: np.ndarray):
    import torch
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def empty(h, w, c, out):
    import torch
    return torch.empty((h, w, c), dtype=torch.uint8 if out == "u8" else torch.float32, device="cuda")


def gpu_resize(img, dh, dw, out="u8", border=1, bval=0.0, mean=None, std=None):
    import torch
    from paper_2505_12425_amd import kr
    s = dev(img)
    d = empty(dh, dw, img.shape[2], out)
    kr.resize(s, d, border=border, border_value=bval, mean=mean, std=std)
    torch.cuda.synchronize()
    return d.cpu().numpy()


def gpu_warp(img, m, dh, dw, out="u8", inverse=False, border=0, bval=0.0, mean=None, std=None):
    import torch
    from paper_2505_12425_amd import kr
    s = dev(img)
    d = empty(dh, dw, img.shape[2], out)
    kr.warp_affine(s, d, m, inverse=inverse, border=border, border_value=bval, mean=mean, std=std)
    torch.cuda.synchronize()
    return d.cpu().numpy()


def assert_u8_equal(got: np.ndarray, exp: np.ndarray, what: str = "") -> None:
    assert got.shape == exp.shape, (got.shape, exp.shape)
    if not np.array_equal(got, exp):
        bad = np.argwhere(got != exp)
        i = tuple(bad[0])
        raise AssertionError(f"{what}: {len(bad)} u8 mismatches; first at {i}: got {got[i]} want {exp[i]}")


def assert_f32_close(got: np.ndarray, exp: np.ndarray, what: str = "", std=None) -> None:
    assert got.shape == exp.shape, (got.shape, exp.shape)
    err = np.abs(got.astype(np.float64) - exp)
    if std is not None:
        err = err * 255.0 * np.asarray(std, np.float64)[: got.shape[2]]
    worst = float(err.max()) if err.size else 0.0
    if not worst <= F32_TOL:
        i = np.unravel_index(int(np.argmax(err)), err.shape)
        raise AssertionError(f"{what}: f32 error {worst:.3g} > {F32_TOL} at {i}: got {got[i]} want {exp[i]}")
