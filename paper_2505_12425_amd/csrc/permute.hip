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
// Tiles are chosen so that every tile's source block is 128 pixels wide and
// 64 rows tall: 128 RGB pixels are three whole 128-byte lines (four for
// RGBA).  The destination tile is 128 x 64 when the map keeps rows as rows
// (flips, shifts) and 64 wide x 128 tall when it swaps the axes (quarter
// turns, transposes); then two horizontally adjacent tiles each write half of
// a destination line, and the tile order (x fastest, each XCD a contiguous
// run) puts them on one XCD's L2 back to back.  The block is staged in LDS
// one dword per pixel: RGB and RGBA rows inside the image in 16-pixel groups
// aligned on the image's linear pixel index (48 or 64 contiguous bytes per
// lane, the group phase absorbed by a margin of 15 columns), every other
// case pixel by pixel with the border rule.  The tile is then read in
// destination order, four pixels per lane, and stored as 4-pixel runs.  With
// a pitch of 159 dwords (-4 mod 64 for four rows), the sixteen lanes of a
// destination row of a swapped tile walk down four source rows apart and
// the four rows a wave covers sit one column apart, so a wave's reads hit 64
// distinct banks.
#include "kr_internal.h"
#include "tiled.h"

namespace kr {

namespace {

constexpr int PM_SW = 128;          // source block width (pixels)
constexpr int PM_SH = 64;           // source block height (rows)
constexpr int PM_M = 15;            // LDS column of the block's first pixel
constexpr int PM_PITCH = 159;       // LDS pitch in dwords (> PM_M + PM_SW + 15, odd)
constexpr int PM_THREADS = 256;
constexpr int PM_GROUPS = 9;        // most 16-pixel groups a 128-pixel row touches

struct PermJob {
    ImageJob j;
    int a, b, c, d, e, f;  // xs = a x + b y + c, ys = d x + e y + f
    int tw, th;            // destination tile size (128 x 64 or 64 x 128)
    int ntx, ntiles;       // tiles per destination row, in all
};

// Rows [ya, ya + nrows) of the block, columns [xa, xb], all inside the
// image, in 16-pixel groups: every load issued before the first LDS write.
template <int C>
__device__ __forceinline__ void stage_groups(uint32_t *blk, const uint8_t *src, int lo, int hi, int sp, int xa, int xb,
                                             int ya, int nrows)
{
    constexpr int IT = (PM_SH * PM_GROUPS + PM_THREADS - 1) / PM_THREADS;
    GroupRegs<C> g[IT];
    int dst[IT], p0[IT];
#pragma unroll
    for (int it = 0; it < IT; it++) {
        const int k = (int)threadIdx.x + it * PM_THREADS;
        const int r = k / PM_GROUPS, gi = k - r * PM_GROUPS;
        dst[it] = -1;
        if (r < nrows) {
            const int rowbase = lo + (ya + r) * sp;
            const int gp = (((rowbase + xa) >> 4) + gi) << 4;
            if (gp <= rowbase + xb) {
                dst[it] = r * PM_PITCH + PM_M + (gp - rowbase - xa);
                p0[it] = gp;
                if (gp >= lo && gp + 16 <= hi)
                    load_group<C>(src, gp, g[it]);
            }
        }
    }
#pragma unroll
    for (int it = 0; it < IT; it++) {
        if (dst[it] >= 0) {
            if (p0[it] >= lo && p0[it] + 16 <= hi)
                write_group<C>(blk + dst[it], g[it]);
            else
                write_tail_group<C>(blk + dst[it], src, p0[it], lo, hi);
        }
    }
}

// The same block pixel by pixel, with the border rule off the image.
template <int C>
__device__ __forceinline__ void stage_pixels(uint32_t *blk, const ImageJob &j, const Epilogue &ep, int xa, int xb,
                                             int ya, int nrows)
{
    const uint8_t *src = static_cast<const uint8_t *>(j.src);
    const size_t nbytes = (size_t)src_end(j) * C;
    const bool cst = ep.border == KR_BORDER_CONSTANT;
    const uint32_t b = (uint32_t)ep.bval_i;
    const uint32_t bpix = C == 1 ? b : (C == 2 ? b * 0x101u : (C == 3 ? b * 0x10101u : b * 0x1010101u));
    const int ncols = xb - xa + 1;
    for (int i = threadIdx.x; i < nrows * PM_SW; i += PM_THREADS) {
        const int r = i >> 7, q = i & (PM_SW - 1);
        if (q >= ncols)
            continue;
        int x = xa + q, y = ya + r;
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
        blk[r * PM_PITCH + PM_M + q] = v;
    }
}

template <int C, bool F32, bool SWAP>
__global__ __launch_bounds__(PM_THREADS) void k_permute(PermJob pj, Epilogue ep)
{
    __shared__ uint32_t blk[PM_SH * PM_PITCH];
    const ImageJob &j = pj.j;
    constexpr int TW = SWAP ? PM_SH : PM_SW, TH = SWAP ? PM_SW : PM_SH;
    const int t = xcd_tile((int)blockIdx.x, pj.ntiles);
    const int ty = t / pj.ntx;
    const int ox0 = (t - ty * pj.ntx) * TW, oy0 = ty * TH;
    const int ox1 = min(ox0 + TW, j.dw) - 1, oy1 = min(oy0 + TH, j.dh) - 1;
    // the source rectangle of the (clipped) tile: the images of its corners
    const int xa = pj.a * (pj.a > 0 ? ox0 : ox1) + pj.b * (pj.b > 0 ? oy0 : oy1) + pj.c;
    const int xb = pj.a * (pj.a > 0 ? ox1 : ox0) + pj.b * (pj.b > 0 ? oy1 : oy0) + pj.c;
    const int ya = pj.d * (pj.d > 0 ? ox0 : ox1) + pj.e * (pj.e > 0 ? oy0 : oy1) + pj.f;
    const int yb = pj.d * (pj.d > 0 ? ox1 : ox0) + pj.e * (pj.e > 0 ? oy1 : oy0) + pj.f;
    const uint8_t *src = static_cast<const uint8_t *>(j.src);
    const int lo = j.sk, hi = src_end(j);
    const int nrows = yb - ya + 1;
    if (xa >= 0 && xb < j.sw && ya >= 0 && yb < j.sh)
        stage_groups<C>(blk, src, lo, hi, j.sp, xa, xb, ya, nrows);
    else
        stage_pixels<C>(blk, j, ep, xa, xb, ya, nrows);
    __syncthreads();
    // destination: TW / 4 lanes of 4 pixels per row
    constexpr int LR = TW / 4, RI = PM_THREADS / LR;
    const int lx = ((int)threadIdx.x % LR) * 4, ly = (int)threadIdx.x / LR;
    const int x = ox0 + lx;
    if (x > ox1)
        return;
    const int n = min(4, ox1 + 1 - x);
    const bool aligned = store4_aligned<C, F32>(j.dw);
    // LDS index of destination pixel (x, y): (ys - ya) * pitch + xs - xa + M
    const int dx = pj.a + pj.d * PM_PITCH;
    const int i0 = (pj.a * x + pj.c - xa + PM_M) + (pj.d * x + pj.f - ya) * PM_PITCH;
    const int iy = pj.b + pj.e * PM_PITCH;
    for (int yy = oy0 + ly; yy <= oy1; yy += RI) {
        const int base = i0 + iy * yy;
        uint32_t P[4];
#pragma unroll
        for (int k = 0; k < 4; k++)
            P[k] = blk[base + dx * min(k, n - 1)];
        if constexpr (!F32) {
            store_u8_4<C>(static_cast<uint8_t *>(j.dst) + ((size_t)yy * j.dw + x) * C, n, aligned, P);
        } else {
            float o[4][C];
#pragma unroll
            for (int k = 0; k < 4; k++)
#pragma unroll
                for (int c = 0; c < C; c++)
                    o[k][c] = __builtin_fmaf((float)((P[k] >> (8 * c)) & 0xFFu), ep.alpha[c], ep.beta[c]);
            store_f32_4<C, true>(static_cast<float *>(j.dst) + ((size_t)yy * j.dw + x) * C, n, aligned, o);
        }
    }
}

template <bool F32, bool SWAP>
hipError_t launch_c(int c, const PermJob &pj, const Epilogue &e, hipStream_t s)
{
    const dim3 grid(pj.ntiles);
    switch (c) {
    case 1: hipLaunchKernelGGL((k_permute<1, F32, SWAP>), grid, dim3(PM_THREADS), 0, s, pj, e); break;
    case 2: hipLaunchKernelGGL((k_permute<2, F32, SWAP>), grid, dim3(PM_THREADS), 0, s, pj, e); break;
    case 3: hipLaunchKernelGGL((k_permute<3, F32, SWAP>), grid, dim3(PM_THREADS), 0, s, pj, e); break;
    default: hipLaunchKernelGGL((k_permute<4, F32, SWAP>), grid, dim3(PM_THREADS), 0, s, pj, e); break;
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
    const bool swap = m[0] == 0;
    PermJob pj{j, m[0], m[1], m[2], m[3], m[4], m[5], 0, 0, 0, 0};
    pj.tw = swap ? PM_SH : PM_SW;
    pj.th = swap ? PM_SW : PM_SH;
    pj.ntx = (j.dw + pj.tw - 1) / pj.tw;
    const long long n = (long long)pj.ntx * ((j.dh + pj.th - 1) / pj.th);
    if (n <= 0)
        return hipSuccess;
    if (n > 0x7fffffff)
        return hipErrorInvalidValue;
    pj.ntiles = (int)n;
    if (dt == KR_F32)
        return swap ? launch_c<true, true>(c, pj, e, s) : launch_c<true, false>(c, pj, e, s);
    return swap ? launch_c<false, true>(c, pj, e, s) : launch_c<false, false>(c, pj, e, s);
}

}  // namespace kr
