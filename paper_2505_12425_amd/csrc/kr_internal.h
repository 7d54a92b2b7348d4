// kr_internal.h -- parameter blocks shared by libkr's host code and kernels.
// Not part of the public ABI (include/kr.h is).
#pragma once

#include <hip/hip_runtime.h>
#include <cstddef>
#include <cstdint>

#include "kr.h"

namespace kr {

enum { OP_RESIZE = 0, OP_WARP = 1, OP_PERSP = 2 };

// Output/epilogue parameters common to every kernel variant.
struct Epilogue {
    float alpha[4];  // f32 output: out_c = v * alpha[c] + beta[c] (1, 0 without normalisation)
    float beta[4];
    float bval_f;    // CONSTANT border value as a sample (f32 path)
    int bval_i;      // CONSTANT border value as an integer sample (u8 path)
    int border;      // KR_BORDER_CONSTANT or KR_BORDER_REPLICATE
    int planar;      // output layout: 0 = interleaved (HWC), 1 = planar (CHW, plane c at c * dh * dw)
    int gray;        // RGB source, one BT.601 gray channel out (the channel values are
                     // then unnormalised: alpha 1, beta 0; galpha, gbeta normalise the gray)
    float galpha, gbeta;
};

// One image as the kernels see it.  For warps, inv is the inverse map with
// its first row and second row kept as given (not pre-scaled); perspective
// warps add the inverse homography's third row in proj.
//
// Source addressing: pixel (x, y) is pixel number sk + y * sp + x counted
// from src, which is 16-byte aligned.  A contiguous image has sp = sw and
// sk = 0; a view into a larger buffer has its row pitch sp (in pixels) and
// src moved back by sk < 16 pixels to the 16-byte boundary at or below its
// first pixel.  Kernels read no pixel before number sk or after the last one
// (the dword-aligned loads of a pixel aside, which stay inside its aligned
// dwords).
struct ImageJob {
    const void *src;
    void *dst;
    int sh, sw, dh, dw;
    int sp, sk;
    double inv[6];
    double proj[3];
};

// Pixel numbers [lo, hi) that hold the source image (lo = sk).
__host__ __device__ inline int src_end(const ImageJob &j) { return j.sk + (j.sh - 1) * j.sp + j.sw; }

// Launchers (resample.hip).  All return the HIP error of the launch.
hipError_t launch_generic(int op, int c, kr_dtype st, kr_dtype dt, const ImageJob &j,
                          const Epilogue &e, hipStream_t s);
hipError_t launch_resize(int c, kr_dtype st, kr_dtype dt, const ImageJob &j, const Epilogue &e,
                         hipStream_t s);
hipError_t launch_warp(int c, kr_dtype st, kr_dtype dt, const ImageJob &j, const Epilogue &e,
                       hipStream_t s);
hipError_t launch_persp(int c, kr_dtype st, kr_dtype dt, const ImageJob &j, const Epilogue &e,
                        hipStream_t s);
// Affine warps whose inverse map permutes pixels (permute.hip): the map's
// whole-number coefficients, when A, B, D, E are -1, 0 or 1 with one non-zero
// per row and column and C, F are whole numbers.
bool permutation_map(const ImageJob &j, int (&m)[6]);
hipError_t launch_permute(int c, kr_dtype dt, const ImageJob &j, const int (&m)[6], const Epilogue &e, hipStream_t s);
// Resize of an RGB u8 source to one gray channel (e.gray set): the exact-2x
// kernel where it applies, the LDS-tiled kernel otherwise.
hipError_t launch_resize_gray(kr_dtype dt, const ImageJob &j, const Epilogue &e, hipStream_t s);
// The LDS-tiled kernels (u8 sources, 1-4 channels) directly.
hipError_t launch_tiled(int op, int c, kr_dtype dt, const ImageJob &j, const Epilogue &e, hipStream_t s);
hipError_t launch_copy(void *dst, const void *src, size_t bytes, hipStream_t s);
// Traffic-mix probe: shrink > 0 reads 2^shrink input chunks per output chunk,
// grow > 0 reads one input chunk for 2^grow output chunks (at most one of them
// non-zero).
hipError_t launch_stream(void *dst, size_t n_out, const void *src, int shrink, int grow, hipStream_t s);
// Flip and RGB -> gray (pointops.hip); the destination is contiguous, sh x sw.
hipError_t launch_flip(int c, kr_dtype t, const ImageJob &j, int fx, int fy, hipStream_t s);
hipError_t launch_gray(kr_dtype st, kr_dtype dt, const ImageJob &j, const Epilogue &e, hipStream_t s);
// Bilinear resize by exactly 2 in both axes from a u8 source (halfscale.hip):
// the 2x2 block means, the same bits as the general kernels.
bool is_half_scale(kr_dtype st, const ImageJob &j);
hipError_t launch_half(int c, kr_dtype dt, const ImageJob &j, const Epilogue &e, hipStream_t s);
// Nearest-neighbour resize (nearest.hip); any channel count and type pair.
hipError_t launch_nearest(int c, kr_dtype st, kr_dtype dt, const ImageJob &j, const Epilogue &e, hipStream_t s);

}  // namespace kr
