"""MI355X-native bilinear resize / affine warp library (kornia-rs image
transformation hot path, arXiv 2505.12425), built on hand-written HIP kernels
for gfx950 behind a C ABI (``include/kr.h``).

``paper_2505_12425_amd.kr`` is the thin ctypes binding over ``libkr.so``;
``paper_2505_12425_amd.workloads`` draws the seeded synthetic inputs.
Importing the package loads nothing; the binding loads the library on first
use and raises if it has not been built.
"""
__all__ = ["kr", "workloads"]
