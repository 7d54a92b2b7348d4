"""Strength of the oracle pins: plant plausible slips in a copy of kro.c (on
the CPU, in a temporary directory) and check that tests/test_oracle.py fails
for every one of them.  The oracle in the tree is never modified."""
from __future__ import annotations

import os
import subprocess
import sys
import tempfile

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SRC = os.path.join(ROOT, "oracle", "kro.c")

MUTANTS = [
    ("swapped x weights", "int64_t wx0 = 2048 - wx1, wy0 = 2048 - wy1;",
     "int64_t wx0 = wx1, wy0 = 2048 - wy1; wx1 = 2048 - wx0;"),
    ("rounding constant", "(acc + (1 << 21)) >> 22", "(acc + (1 << 20)) >> 22"),
    ("truncation", "(acc + (1 << 21)) >> 22", "(acc) >> 22"),
    ("ties rounded up", "if (t % (2 * den) == 0 && (q & 1))", "if (0)"),
    ("half-pixel sign (y)", "int64_t ny = (int64_t)(2 * dy + 1) * sh - dh",
     "int64_t ny = (int64_t)(2 * dy + 1) * sh + dh"),
    ("off-by-one numerator (x)", "int64_t nx = (int64_t)(2 * dx + 1) * sw - dw",
     "int64_t nx = (int64_t)(2 * dx + 1) * sw - dw - 1"),
    ("wrong inverse term", "double xs = fma(im[0], (double)x, fma(im[1], (double)y, im[2]));",
     "double xs = fma(im[0], (double)x, fma(im[3], (double)y, im[2]));"),
    ("transposed x/y", "double ys = fma(im[3], (double)x, fma(im[4], (double)y, im[5]));",
     "double ys = fma(im[3], (double)y, fma(im[4], (double)x, im[5]));"),
    ("inverse translation sign", "double C = -(t1 + t2);", "double C = (t1 + t2);"),
    ("unfused evaluation", "double xs = fma(im[0], (double)x, fma(im[1], (double)y, im[2]));",
     "double xs = im[0]*(double)x + im[1]*(double)y + im[2];"),
    ("dropped tap", "+ wy1 * wx1 * tap_u8(s, sh, sw, c, x0 + 1, y0 + 1, ch, border, b);", ";"),
    ("border value ignored", "if (border == KRO_CONSTANT)\n            return bval;",
     "if (border == KRO_CONSTANT)\n            return 0;"),
    ("normalise order", "v = (v / 255.0 - mean[ch]) / stdv[ch];", "v = (v - mean[ch]) / stdv[ch] / 255.0;"),
    ("swapped inverse terms", "double A = m[4] / det, B = -m[1] / det, D = -m[3] / det, E = m[0] / det;",
     "double A = m[4] / det, B = -m[3] / det, D = -m[1] / det, E = m[0] / det;"),
    ("nearest without half-pixel", "int64_t sx = ((int64_t)(2 * dx + 1) * sw) / (2 * (int64_t)dw);",
     "int64_t sx = ((int64_t)(2 * dx) * sw) / (2 * (int64_t)dw);"),
    ("nearest row scale from columns", "int64_t sy = ((int64_t)(2 * dy + 1) * sh) / (2 * (int64_t)dh);",
     "int64_t sy = ((int64_t)(2 * dy + 1) * sh) / (2 * (int64_t)dw);"),
    ("nearest rounds up", "int64_t sx = ((int64_t)(2 * dx + 1) * sw) / (2 * (int64_t)dw);",
     "int64_t sx = ((int64_t)(2 * dx + 1) * sw + 2 * (int64_t)dw - 1) / (2 * (int64_t)dw); if (sx >= sw) sx = sw - 1;"),
    ("gray R/B weights swapped", "4899 * (int64_t)p[0] + 9617 * (int64_t)p[1] + 1868 * (int64_t)p[2]",
     "1868 * (int64_t)p[0] + 9617 * (int64_t)p[1] + 4899 * (int64_t)p[2]"),
    ("gray truncation", "((acc + (1 << 13)) >> 14)", "(acc >> 14)"),
    ("flip shifted by one", "int sx = flip_x ? w - 1 - x : x;", "int sx = flip_x ? (w - x) % w : x;"),
    ("perspective w row swapped", "double w = fma(im[6], (double)x, fma(im[7], (double)y, im[8]));",
     "double w = fma(im[7], (double)x, fma(im[6], (double)y, im[8]));"),
    ("homography cofactor sign", "double c01 = m[5] * m[6] - m[3] * m[8];",
     "double c01 = m[3] * m[8] - m[5] * m[6];"),
    ("perspective without division", "double xs = fma(im[0], (double)x, fma(im[1], (double)y, im[2])) / w;",
     "double xs = fma(im[0], (double)x, fma(im[1], (double)y, im[2]));"),
    ("wrong tap row (f64)", "+ fy * fx * tap(src, src_t, sh, sw, c, x0 + 1, y0 + 1, ch, border, bval);",
     "+ fy * fx * tap(src, src_t, sh, sw, c, x0 + 1, y0, ch, border, bval);"),
]


@pytest.mark.slow
@pytest.mark.parametrize("name,old,new", MUTANTS, ids=[m[0] for m in MUTANTS])
def test_pins_catch_mutant(name, old, new, tmp_path):
    src = open(SRC).read()
    assert old in src, name
    mut = tmp_path / "kro_mut.c"
    mut.write_text(src.replace(old, new, 1))
    lib = tmp_path / "libkro_mut.so"
    subprocess.run(["gcc", "-O2", "-std=c11", "-ffp-contract=off", "-fopenmp", "-fPIC", "-shared",
                    str(mut), "-o", str(lib), "-lm"], check=True)
    env = dict(os.environ, KRO_LIB=str(lib))
    r = subprocess.run([sys.executable, "-m", "pytest", "-x", "-q", "-p", "no:cacheprovider",
                        os.path.join(ROOT, "tests", "test_oracle.py")],
                       cwd=ROOT, env=env, capture_output=True, text=True)
    assert r.returncode != 0, f"mutant '{name}' survived the oracle pins"
