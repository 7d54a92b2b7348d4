// nearest.hip -- nearest-neighbour resize with half-pixel centres: output
// pixel (x, y) copies the source sample at column floor((2 x + 1) W_in /
// (2 W_out)) and row floor((2 y + 1) H_in / (2 H_out)) (exact integer
// quotients, from a rounded reciprocal plus an exact correction).
//
// A workgroup is 64 x 4 threads.  u8 output: a thread owns 4 consecutive
// pixels (12 contiguous bytes for RGB) of 2 rows; f32 output: one pixel of 8
// rows, so that each store instruction of a wave writes one contiguous run.
// A thread's column map is computed once.  u8 RGB samples are read with
// dword-aligned 8-byte loads (L1/L2 absorb the reuse between neighbouring
// outputs); the f32 path applies the per-channel epilogue v * alpha + beta.
#include "kr_internal.h"
#include "tiled.h"

namespace kr {

namespace {

constexpr int NN_TX = 64, NN_TY = 4;

template <bool DST_F32> struct NNShape {
    static constexpr int PXL = DST_F32 ? 1 : 4;  // pixels per thread and row
    static constexpr int RPT = DST_F32 ? 8 : 2;  // rows per thread
    static constexpr int COLS = NN_TX * PXL, ROWS = NN_TY * RPT;
};

struct NearestJob {
    const void *src;
    void *dst;
    int sh, sw, dh, dw;
    int sp, sk;     // source row pitch and first pixel, in pixels from src
    double rx, ry;  // 1 / (2 dw), 1 / (2 dh), rounded
};

template <int C, bool SRC_F32, bool DST_F32>
__global__ __launch_bounds__(NN_TX * NN_TY) void k_nearest(NearestJob j, Epilogue e)
{
    using S = NNShape<DST_F32>;
    constexpr int PXL = S::PXL;
    const int x = (blockIdx.x * NN_TX + threadIdx.x) * PXL;
    if (x >= j.dw)
        return;
    const int n = min(PXL, j.dw - x);
    size_t sx[PXL];
#pragma unroll
    for (int k = 0; k < PXL; k++) {
        int r;
        sx[k] = (size_t)floor_div_r((2 * min(x + k, j.dw - 1) + 1) * j.sw, 2 * j.dw, j.rx, r);
    }
    const size_t nbytes = ((size_t)j.sk + (size_t)(j.sh - 1) * j.sp + j.sw) * C * (SRC_F32 ? 4 : 1);
#pragma unroll
    for (int rr = 0; rr < S::RPT; rr++) {
        const int y = blockIdx.y * S::ROWS + threadIdx.y + rr * NN_TY;
        if (y >= j.dh)
            break;
        int r;
        const size_t row = (size_t)j.sk + (size_t)floor_div_r((2 * y + 1) * j.sh, 2 * j.dh, j.ry, r) * (size_t)j.sp;
        const size_t out = ((size_t)y * j.dw + x) * C;
        if constexpr (!DST_F32) {
            uint32_t P[4];
#pragma unroll
            for (int k = 0; k < 4; k++)
                P[k] = load_u8_px<C>(static_cast<const uint8_t *>(j.src), nbytes, row + sx[k]);
            store_u8_4<C>(static_cast<uint8_t *>(j.dst) + out, n, store4_aligned<C, false>(j.dw), P);
        } else {
            float o[C];
            if constexpr (!SRC_F32) {
                const uint32_t P = load_u8_px<C>(static_cast<const uint8_t *>(j.src), nbytes, row + sx[0]);
#pragma unroll
                for (int c = 0; c < C; c++)
                    o[c] = __builtin_fmaf((float)((P >> (8 * c)) & 0xFFu), e.alpha[c], e.beta[c]);
            } else {
                const float *src = static_cast<const float *>(j.src) + (row + sx[0]) * C;
#pragma unroll
                for (int c = 0; c < C; c++)
                    o[c] = __builtin_fmaf(src[c], e.alpha[c], e.beta[c]);
            }
            // non-temporal: no kernel of the call reads the output back
            float *d = static_cast<float *>(j.dst) + out;
#pragma unroll
            for (int c = 0; c < C; c++)
                __builtin_nontemporal_store(o[c], d + c);
        }
    }
}

template <int C>
hipError_t launch_c(const NearestJob &j, kr_dtype st, kr_dtype dt, const Epilogue &e, hipStream_t s)
{
    const dim3 block(NN_TX, NN_TY);
    if (dt == KR_F32) {
        using S = NNShape<true>;
        const dim3 grid((j.dw + S::COLS - 1) / S::COLS, (j.dh + S::ROWS - 1) / S::ROWS);
        if (st == KR_F32)
            hipLaunchKernelGGL((k_nearest<C, true, true>), grid, block, 0, s, j, e);
        else
            hipLaunchKernelGGL((k_nearest<C, false, true>), grid, block, 0, s, j, e);
    } else {
        using S = NNShape<false>;
        const dim3 grid((j.dw + S::COLS - 1) / S::COLS, (j.dh + S::ROWS - 1) / S::ROWS);
        hipLaunchKernelGGL((k_nearest<C, false, false>), grid, block, 0, s, j, e);
    }
    return hipGetLastError();
}

}  // namespace

hipError_t launch_nearest(int c, kr_dtype st, kr_dtype dt, const ImageJob &ij, const Epilogue &e, hipStream_t s)
{
    NearestJob j{ij.src, ij.dst, ij.sh, ij.sw, ij.dh, ij.dw, ij.sp, ij.sk, 1.0 / (2.0 * ij.dw), 1.0 / (2.0 * ij.dh)};
    switch (c) {
    case 1: return launch_c<1>(j, st, dt, e, s);
    case 2: return launch_c<2>(j, st, dt, e, s);
    case 3: return launch_c<3>(j, st, dt, e, s);
    default: return launch_c<4>(j, st, dt, e, s);
    }
}

}  // namespace kr
