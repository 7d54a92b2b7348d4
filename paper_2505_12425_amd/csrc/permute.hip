// permute.hip -- affine warps that only permute pixels: the inverse map sends
// every destination pixel centre to a source pixel centre, xs = A x + B y + C
// and ys = D x + E y + F with A, B, D, E in {-1, 0, 1}, one non-zero per row
// and per column (flips, rotations by multiples of 90 degrees, transposes,
// their combinations) and C, F whole numbers.  Every fraction is then zero,
// so the bilinear result is the one tap at (xs, ys) -- or the border rule
// for it -- exactly: u8 keeps the sample (its weight is 2^22 of 2^22), f32
// holds the sample's value before the epilogue (the other three weights are
// zero and add +0 to a non-negative sum).  The warp entry points route such
// maps of u8 sources here: same bits as the interpolating kernels, with no
// coordinate arithmetic per pixel.
//
// One workgroup per 64 x 64 destination tile.  The tile's source pixels form
// a 64 x 64 block; it is staged in LDS (one dword per pixel, rows read with
// consecutive lanes on consecutive pixels, out-of-image pixels replaced by
// the border rule), then read in destination order (a rotated or transposed
// walk through the block; the odd pitch keeps those reads on distinct banks)
// and stored as 4-pixel runs.
#include "kr_internal.h"
#include "tiled.h"

namespace kr {

namespace {

constexpr int PM_T = 64;           // tile side
constexpr int PM_PITCH = PM_T + 1;  // LDS pitch in dwords

struct PermJob {
    ImageJob j;
    int a, b, c, d, e, f;  // xs = a x + b y + c, ys = d x + e y + f
};

template <int C, bool F32>
__global__ __launch_bounds__(256) void k_permute(PermJob pj, Epilogue ep)
{
    __shared__ uint32_t blk[PM_T * PM_PITCH];
    const ImageJob &j = pj.j;
    const int ox0 = blockIdx.x * PM_T, oy0 = blockIdx.y * PM_T;
    // the source block: the images of the tile's corners span it
    const int sx0 = pj.a * ox0 + pj.b * oy0 + pj.c + min(pj.a, 0) * (PM_T - 1) + min(pj.b, 0) * (PM_T - 1);
    const int sy0 = pj.d * ox0 + pj.e * oy0 + pj.f + min(pj.d, 0) * (PM_T - 1) + min(pj.e, 0) * (PM_T - 1);
    const uint8_t *src = static_cast<const uint8_t *>(j.src);
    const size_t nbytes = (size_t)src_end(j) * C;
    const bool cst = ep.border == KR_BORDER_CONSTANT;
    const uint32_t b = (uint32_t)ep.bval_i;
    const uint32_t bpix = C == 1 ? b : (C == 2 ? b * 0x101u : (C == 3 ? b * 0x10101u : b * 0x1010101u));
    for (int i = threadIdx.x; i < PM_T * PM_T; i += 256) {
        const int r = i >> 6, q = i & 63;
        int x = sx0 + q, y = sy0 + r;
        uint32_t v;
        if ((unsigned)x < (unsigned)j.sw && (unsigned)y < (unsigned)j.sh) {
            v = load_u8_px<C>(src, nbytes, (size_t)j.sk + (size_t)y * j.sp + x);
        } else if (cst) {
            v = bpix;
        } else {
            x = clampi(x, 0, j.sw - 1);
            y = clampi(y, 0, j.sh - 1);
            v = load_u8_px<C>(src, nbytes, (size_t)j.sk + (size_t)y * j.sp + x);
        }
        blk[r * PM_PITCH + q] = v;
    }
    __syncthreads();
    // destination: 16 lanes x 4 pixels per row, 16 rows per pass
    const int lx = (threadIdx.x & 15) * 4, ly = threadIdx.x >> 4;
    const int x = ox0 + lx;
    if (x >= j.dw)
        return;
    const int n = min(4, j.dw - x);
    const bool aligned = store4_aligned<C, F32>(j.dw);
    for (int yy = ly; yy < PM_T; yy += 16) {
        const int y = oy0 + yy;
        if (y >= j.dh)
            break;
        uint32_t P[4];
#pragma unroll
        for (int k = 0; k < 4; k++) {
            const int xk = x + min(k, n - 1);
            const int sx = pj.a * xk + pj.b * y + pj.c - sx0;
            const int sy = pj.d * xk + pj.e * y + pj.f - sy0;
            P[k] = blk[sy * PM_PITCH + sx];
        }
        if constexpr (!F32) {
            store_u8_4<C>(static_cast<uint8_t *>(j.dst) + ((size_t)y * j.dw + x) * C, n, aligned, P);
        } else {
            float o[4][C];
#pragma unroll
            for (int k = 0; k < 4; k++)
#pragma unroll
                for (int c = 0; c < C; c++)
                    o[k][c] = __builtin_fmaf((float)((P[k] >> (8 * c)) & 0xFFu), ep.alpha[c], ep.beta[c]);
            store_f32_4<C>(static_cast<float *>(j.dst) + ((size_t)y * j.dw + x) * C, n, aligned, o);
        }
    }
}

template <bool F32>
hipError_t launch_c(int c, const PermJob &pj, const Epilogue &e, hipStream_t s)
{
    const dim3 grid((pj.j.dw + PM_T - 1) / PM_T, (pj.j.dh + PM_T - 1) / PM_T);
    switch (c) {
    case 1: hipLaunchKernelGGL((k_permute<1, F32>), grid, dim3(256), 0, s, pj, e); break;
    case 2: hipLaunchKernelGGL((k_permute<2, F32>), grid, dim3(256), 0, s, pj, e); break;
    case 3: hipLaunchKernelGGL((k_permute<3, F32>), grid, dim3(256), 0, s, pj, e); break;
    default: hipLaunchKernelGGL((k_permute<4, F32>), grid, dim3(256), 0, s, pj, e); break;
    }
    return hipGetLastError();
}

// v as an int in [-2^24, 2^24] when it is one exactly.
bool whole(double v, int &out)
{
    if (!(v >= -16777216.0 && v <= 16777216.0) || v != (double)(int)v)
        return false;
    out = (int)v;
    return true;
}

}  // namespace

bool permutation_map(const ImageJob &j, int (&m)[6])
{
    for (int i = 0; i < 6; i++)
        if (!whole(j.inv[i], m[i]))
            return false;
    for (int i : {0, 1, 3, 4})
        if (m[i] < -1 || m[i] > 1)
            return false;
    // one non-zero per row and per column: |det| = 1 with unit entries
    return (m[0] != 0) != (m[1] != 0) && (m[3] != 0) != (m[4] != 0) && (m[0] != 0) != (m[3] != 0);
}

hipError_t launch_permute(int c, kr_dtype dt, const ImageJob &j, const int (&m)[6], const Epilogue &e, hipStream_t s)
{
    const PermJob pj{j, m[0], m[1], m[2], m[3], m[4], m[5]};
    return dt == KR_F32 ? launch_c<true>(c, pj, e, s) : launch_c<false>(c, pj, e, s);
}

}  // namespace kr
