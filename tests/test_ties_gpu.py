"""GPU parity at 11-bit weight ties: every kernel path against the oracle.

The u8 weights are w1 = round-half-even(2048 * frac) with w0 = 2048 - w1
(ties to even).  A resize axis has a tie at output d when 2048 r / (2 n_out)
is k + 1/2 (r the remainder of the exact half-pixel map), which needs n_out to
be a multiple of 2048: 6 -> 4096, 3 -> 2048 and 2051 -> 2048 tie at every
output.  A warp ties where 2048 * frac(xs) is k + 1/2: the inverse scale
1 + 2^-12 gives xs = x + x / 4096, a tie at every odd x.  Random sizes and maps
essentially never tie, so these cases are chosen to tie everywhere (the tie
counts are asserted on the host, in exact integers, before the GPU runs), with
both parities of k, so that rounding up and rounding down are both exercised.

Paths covered: the LDS-tiled kernel (C = 1-4: the integer rule of its resize
tables and the magic-constant rounding of its 2048-scaled warp coordinates),
its global-gather path (x shrink above 3), the perspective kernels, and batch
items (u8 bit-exact against the oracle and against the single-image call).
"""
from __future__ import annotations

from fractions import Fraction

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

CONST, REPL = 0, 1
MEAN, STD = wl.IMAGENET_MEAN, wl.IMAGENET_STD
TH = 16
TIE = 1.0 + 2.0 ** -12  # inverse scale: xs = x + x / 4096, a weight tie at every odd x


# ------------------------------------------------------------------ tie counts (host, exact)
def resize_axis_ties(n_in: int, n_out: int):
    """(ties rounding down, ties rounding up) over the outputs of one resize
    axis: 2048 r / den = k + 1/2 exactly, k even rounds down, k odd rounds up."""
    d = np.arange(n_out, dtype=np.int64)
    den = 2 * n_out
    r = np.mod((2 * d + 1) * n_in - n_out, den)
    t = 4096 * r
    tie = np.mod(t, 2 * den) == den
    k = (t - den) // (2 * den)
    return int(np.sum(tie & (k % 2 == 0))), int(np.sum(tie & (k % 2 == 1)))


def scaled_axis_ties(coords):
    """Same for exact dyadic source coordinates (Fractions)."""
    down = up = 0
    for v in coords:
        f = v - (v.numerator // v.denominator)
        s = 2048 * f
        if s.denominator == 2:
            k = s.numerator // 2
            if k % 2 == 0:
                down += 1
            else:
                up += 1
    return down, up


def assert_ties_both_ways(counts, what):
    down, up = counts
    say(f"{what}: {down} ties rounding down, {up} rounding up")
    assert down > 0 and up > 0, f"{what}: the case must tie both ways ({down}, {up})"


# ------------------------------------------------------------------ helpers
def _out(h, w, c, out):
    return torch.empty((h, w, c), dtype=torch.uint8 if out == "u8" else torch.float32, device="cuda")


def run_resize(img, dh, dw, out, border, bval, mean=None, std=None):
    s = dev(img)
    d = _out(dh, dw, img.shape[2], out)
    kr.resize(s, d, border=border, border_value=bval, mean=mean, std=std)
    torch.cuda.synchronize()
    return d.cpu().numpy()


def run_warp(img, m, dh, dw, out, border, bval, mean=None, std=None):
    s = dev(img)
    d = _out(dh, dw, img.shape[2], out)
    kr.warp_affine(s, d, m, inverse=True, border=border, border_value=bval, mean=mean, std=std)
    torch.cuda.synchronize()
    return d.cpu().numpy()


def run_persp(img, m9, dh, dw, out, border, bval):
    s = dev(img)
    d = _out(dh, dw, img.shape[2], out)
    kr.warp_perspective(s, d, m9, inverse=True, border=border, border_value=bval)
    torch.cuda.synchronize()
    return d.cpu().numpy()


def check_resize(img, dh, dw, border, bval, what):
    h, w, c = img.shape
    say(f"tie resize {what}: {h}x{w}x{c} -> {dh}x{dw} border={border} bval={bval}")
    assert_u8_equal(run_resize(img, dh, dw, "u8", border, bval),
                    oracle.resize(img, dh, dw, "u8", border, bval, threads=TH), f"tie resize u8 {what}")
    assert_f32_close(run_resize(img, dh, dw, "f32", border, bval),
                     oracle.resize(img, dh, dw, "f64", border, bval, threads=TH), f"tie resize f32 {what}")
    if c == 3:
        assert_f32_close(run_resize(img, dh, dw, "f32", border, bval, MEAN, STD),
                         oracle.resize(img, dh, dw, "f64", border, bval, MEAN, STD, threads=TH),
                         f"tie resize norm {what}", std=STD)


def check_warp(img, inv, dh, dw, border, bval, what):
    h, w, c = img.shape
    say(f"tie warp {what}: {h}x{w}x{c} -> {dh}x{dw} inv={inv} border={border} bval={bval}")
    assert_u8_equal(run_warp(img, inv, dh, dw, "u8", border, bval),
                    oracle.warp(img, inv, dh, dw, "u8", True, border, bval, threads=TH), f"tie warp u8 {what}")
    assert_f32_close(run_warp(img, inv, dh, dw, "f32", border, bval),
                     oracle.warp(img, inv, dh, dw, "f64", True, border, bval, threads=TH), f"tie warp f32 {what}")


# ------------------------------------------------------------------ resize
@pytest.mark.parametrize("c", [1, 2, 3, 4])
@pytest.mark.parametrize("border,bval", [(REPL, 0), (CONST, 77)])
def test_resize_row_ties(c, border, bval):
    """1x6 -> 1x4096 (every column a tie) and 6x1 -> 4096x1 (every row)."""
    assert_ties_both_ways(resize_axis_ties(6, 4096), "6 -> 4096")
    img = wl.uniform_u8(1, 6, c, seed=900 + c)
    check_resize(img, 1, 4096, border, bval, f"1x6 c={c}")
    img = wl.uniform_u8(6, 1, c, seed=910 + c)
    check_resize(img, 4096, 1, border, bval, f"6x1 c={c}")


@pytest.mark.parametrize("c", [1, 3, 4])
def test_resize_2d_ties(c):
    """3x6 -> 2048x4096: both weights of every output pixel are ties."""
    assert_ties_both_ways(resize_axis_ties(3, 2048), "3 -> 2048")
    img = wl.uniform_u8(3, 6, c, seed=920 + c)
    check_resize(img, 2048, 4096, REPL, 0, f"3x6 c={c}")
    check_resize(img, 2048, 4096, CONST, 200, f"3x6 c={c} const")


@pytest.mark.parametrize("c", [1, 3])
def test_resize_downscale_ties(c):
    """2051x2051 -> 2048x2048: a mild downscale through the staged (LDS)
    path of the tiled kernel, every weight a tie."""
    assert_ties_both_ways(resize_axis_ties(2051, 2048), "2051 -> 2048")
    img = wl.uniform_u8(2051, 2051, c, seed=930 + c)
    check_resize(img, 2048, 2048, REPL, 0, f"2051 c={c}")


def test_resize_gather_ties():
    """1x12290 -> 1x4096 shrinks x by more than 3: the tiled kernel's
    global-gather path, every column a tie."""
    assert_ties_both_ways(resize_axis_ties(12290, 4096), "12290 -> 4096")
    for c in (3, 4):
        img = wl.uniform_u8(2, 12290, c, seed=940 + c)
        check_resize(img, 2, 4096, REPL, 0, f"gather c={c}")


# ------------------------------------------------------------------ warp
def _affine_ties(inv, h, w):
    """Tie counts of the x and y axes of an exact dyadic inverse map over an h x w output."""
    A, B, C, D, E, F = (Fraction(v) for v in inv)
    xs = [A * x + B * y + C for y in range(h) for x in range(w)]
    ys = [D * x + E * y + F for y in range(h) for x in range(w)]
    return scaled_axis_ties(xs), scaled_axis_ties(ys)


WARP_TIE_MAPS = [
    # inverse maps whose fma chain is exact (dyadic, few bits), so the tie
    # counts below are those of the binary64 coordinates
    ("scale", [TIE, 0.0, 0.0, 0.0, TIE, 0.0]),
    ("scale+shift", [TIE, 0.0, -100.25, 0.0, TIE, 37.75]),
    ("shear", [1.0, 2.0 ** -12, 0.5, 2.0 ** -12, 1.0, -0.5]),
]


@pytest.mark.parametrize("name,inv", WARP_TIE_MAPS, ids=[n for n, _ in WARP_TIE_MAPS])
@pytest.mark.parametrize("c", [1, 3, 4])
@pytest.mark.parametrize("border,bval", [(CONST, 0), (CONST, 91), (REPL, 0)])
def test_warp_small_ties(name, inv, c, border, bval):
    """The oracle's own 32x40 tie case and two variants (negative source
    coordinates, ties from the off-diagonal terms)."""
    tx, ty = _affine_ties(inv, 32, 40)
    assert_ties_both_ways(tx, f"{name} x")
    if name != "shear":
        assert_ties_both_ways(ty, f"{name} y")
    img = wl.uniform_u8(32, 40, c, seed=950 + c)
    check_warp(img, inv, 32, 40, border, bval, f"{name} 32x40 c={c}")


@pytest.mark.parametrize("c", [1, 3, 4])
def test_warp_1080p_ties(c):
    """The tie map at 1920x1080 (many tiles, interior and edge tiles)."""
    inv = [TIE, 0.0, -3.0, 0.0, TIE, 2.0]
    img = wl.mixed_u8(1080, 1920, c, seed=960 + c)
    check_warp(img, inv, 1080, 1920, CONST, 0, f"1080p c={c}")
    check_warp(img, inv, 1080, 1920, REPL, 0, f"1080p c={c} repl")


@pytest.mark.parametrize("c", [1, 3])
def test_perspective_affine_ties(c):
    """Homographies with an affine third row: [A 0 0; 0 A 0; 0 0 1] and the
    same scaled by 2 ([2A 0 0; 0 2A 0; 0 0 2], an exact quotient by w = 2).
    The perspective result must equal the oracle's perspective warp, and the
    affine warp bit for bit."""
    img = wl.mixed_u8(700, 900, c, seed=970 + c)
    for m9 in ([TIE, 0.0, 0.0, 0.0, TIE, 0.0, 0.0, 0.0, 1.0],
               [2 * TIE, 0.0, 0.0, 0.0, 2 * TIE, 0.0, 0.0, 0.0, 2.0]):
        say(f"tie perspective c={c} m={m9}")
        got = run_persp(img, m9, 700, 900, "u8", CONST, 5)
        assert_u8_equal(got, oracle.warp_perspective(img, m9, 700, 900, "u8", True, CONST, 5, threads=TH),
                        f"tie perspective u8 c={c}")
        assert_u8_equal(got, oracle.warp(img, [TIE, 0, 0, 0, TIE, 0], 700, 900, "u8", True, CONST, 5, threads=TH),
                        f"tie perspective == affine c={c}")
        assert_f32_close(run_persp(img, m9, 700, 900, "f32", REPL, 0),
                         oracle.warp_perspective(img, m9, 700, 900, "f64", True, REPL, 0, threads=TH),
                         f"tie perspective f32 c={c}")


# ------------------------------------------------------------------ batches
@pytest.mark.parametrize("c", [3, 4])
@pytest.mark.parametrize("out", ["u8", "f32"])
def test_batch_ties(c, out):
    """Tie cases as items of one batch (staged resize, gather resize, warp):
    equal to the oracle and, bit for bit, to the single-image calls."""
    dt = torch.uint8 if out == "u8" else torch.float32
    ok = "u8" if out == "u8" else "f64"
    cases = [
        ("resize", wl.uniform_u8(1, 6, c, seed=980), (1, 4096), None),
        ("resize", wl.uniform_u8(3, 6, c, seed=981), (2048, 4096), None),
        ("resize", wl.uniform_u8(2051, 2051, c, seed=982), (2048, 2048), None),
        ("resize", wl.uniform_u8(2, 12290, c, seed=983), (2, 4096), None),
        ("warp", wl.uniform_u8(32, 40, c, seed=984), (32, 40), [TIE, 0.0, 0.0, 0.0, TIE, 0.0]),
        ("warp", wl.mixed_u8(1080, 1920, c, seed=985), (1080, 1920), [TIE, 0.0, -100.25, 0.0, TIE, 37.75]),
    ]
    specs, refs = [], []
    for op, im, (dh, dw), inv in cases:
        sp = {"op": op, "src": dev(im), "dst": torch.empty((dh, dw, c), dtype=dt, device="cuda")}
        if op == "warp":
            sp["m"] = inv
            sp["inverse"] = True
            refs.append(oracle.warp(im, inv, dh, dw, ok, True, REPL, 0, threads=TH))
        else:
            refs.append(oracle.resize(im, dh, dw, ok, REPL, 0, threads=TH))
        specs.append(sp)
    say(f"tie batch c={c} out={out}")
    kr.resize_batch(specs, border=REPL)
    torch.cuda.synchronize()
    for i, (sp, ref) in enumerate(zip(specs, refs)):
        got = sp["dst"].cpu().numpy()
        if out == "u8":
            assert_u8_equal(got, ref, f"tie batch item {i}")
        else:
            assert_f32_close(got, ref, f"tie batch item {i}")
        single = torch.empty_like(sp["dst"])
        if sp["op"] == "warp":
            kr.warp_affine(sp["src"], single, sp["m"], inverse=True, border=REPL)
        else:
            kr.resize(sp["src"], single, border=REPL)
        torch.cuda.synchronize()
        assert np.array_equal(single.cpu().numpy(), got), f"tie batch item {i}: batch != single"
