// Wave bodies of the dot products on partly decompressed blocks
// (Algorithm 3 with Eqs. eqbbb0 and eqbbb, applied blockwise): one wave per
// dot product, the lanes walking the blocks of the line's block row (and of
// the column's block column) 64 at a time.  Shared by the standalone kernels
// and the persistent batch kernel.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "blaz_device.hpp"

namespace blaz {

// Lines 0..R of a block from its 28 scaled coefficients: inverse DCT of those
// lines, then the inverse normalization of Eq. eqbbb over them.  Returns line
// R in row[8].
template <int R>
__device__ __forceinline__ void partial_line(const double coef[kKept], double f, double row[8])
{
#pragma clang fp contract(fast)
    double y[64];  // only lines 0..R are computed
#pragma unroll
    for (int j = 0; j < 2; ++j) {
        double col[8], out[8];
#pragma unroll
        for (int i = 0; i < 8; ++i) col[i] = coef[kept_index(i, j)];
        idct8<1, 1>(col, out);
#pragma unroll
        for (int u = 0; u <= R; ++u) y[u * 8 + j] = out[u];
    }
#pragma unroll
    for (int j = 2; j < 8; ++j) {
        const double y0 = coef[kept_index(0, j)], y1 = coef[kept_index(1, j)];
#pragma unroll
        for (int u = 0; u <= R; ++u) y[u * 8 + j] = dct_t(0, u) * y0 + dct_t(1, u) * y1;
    }
#pragma unroll
    for (int u = 0; u <= R; ++u) idct8<1, 1>(y + u * 8, y + u * 8);
    // inverse normalization restricted to lines 0..R
    y[0] = f;
#pragma unroll
    for (int v = 1; v < 8; ++v) y[v] = y[v - 1] + y[v];
#pragma unroll
    for (int u = 1; u <= R; ++u) {
        y[u * 8] = y[(u - 1) * 8] + y[u * 8];
#pragma unroll
        for (int v = 1; v < 8; ++v) y[u * 8 + v] = (y[(u - 1) * 8 + v] + y[u * 8 + v - 1]) * 0.5 + y[u * 8 + v];
    }
#pragma unroll
    for (int k = 0; k < 8; ++k) row[k] = y[R * 8 + k];
}

// Line r (wave-uniform, 0..7) of block b; transpose_codes reads the block's
// coefficients transposed, which yields column r of the block instead
// (normalization, DCT, kept set and inverse are all symmetric under
// transposition).
template <bool kTranspose>
__device__ __forceinline__ void block_line(const double* f, const double* s, const uint8_t* phi,
                                           const uint32_t* codes, int64_t b, int r, double out[8])
{
    uint32_t w[kCodeWords];
#pragma unroll
    for (int q = 0; q < kCodeWords; ++q) w[q] = codes[b * kCodeWords + q];
    double c[kKept], coef[kKept];
    unpack_codes(w, s[b] / (double)phi[b], c);
#pragma unroll
    for (int t = 0; t < kKept; ++t)
        coef[t] = kTranspose ? c[kept_index(kept_col(t), kept_row(t))] : c[t];
    const double fb = f[b];
    switch (r) {
        case 0: partial_line<0>(coef, fb, out); break;
        case 1: partial_line<1>(coef, fb, out); break;
        case 2: partial_line<2>(coef, fb, out); break;
        case 3: partial_line<3>(coef, fb, out); break;
        case 4: partial_line<4>(coef, fb, out); break;
        case 5: partial_line<5>(coef, fb, out); break;
        case 6: partial_line<6>(coef, fb, out); break;
        default: partial_line<7>(coef, fb, out); break;
    }
}

__device__ __forceinline__ double wave_sum(double v)
{
#pragma unroll
    for (int off = 32; off >= 1; off /= 2) v += __shfl_xor(v, off, 64);
    return v;
}

// out[q] = <line xrow[q] of X, column ycol[q] of Y>; X is (nbr_x*8) x (nk*8),
// Y is (nk*8) x (nbc_y*8).  An index outside its matrix gives NaN.
__device__ __forceinline__ void dot_wave(int64_t q, int lane, const double* __restrict__ xf,
                                         const double* __restrict__ xs, const uint8_t* __restrict__ xphi,
                                         const uint32_t* __restrict__ xc, int64_t nbr_x, const double* __restrict__ yf,
                                         const double* __restrict__ ys, const uint8_t* __restrict__ yphi,
                                         const uint32_t* __restrict__ yc, int64_t nbc_y, int64_t nk,
                                         const int64_t* __restrict__ xrow, const int64_t* __restrict__ ycol,
                                         double* __restrict__ out)
{
    const int64_t i = xrow[q], j = ycol[q];
    const bool ok = i >= 0 && i < nbr_x * 8 && j >= 0 && j < nbc_y * 8;
    double acc = 0.0;
    if (ok) {
        const int64_t I = i >> 3, Jc = j >> 3;
        const int r = (int)(i & 7), c = (int)(j & 7);
        for (int64_t kb = lane; kb < nk; kb += 64) {
            double xl[8], yl[8];
            block_line<false>(xf, xs, xphi, xc, I * nk + kb, r, xl);
            block_line<true>(yf, ys, yphi, yc, kb * nbc_y + Jc, c, yl);
#pragma unroll
            for (int k = 0; k < 8; ++k) acc += xl[k] * yl[k];
        }
    }
    acc = wave_sum(acc);
    if (lane == 0) out[q] = ok ? acc : __builtin_nan("");
}

// out[q] = <line xrow[q] of X, v + q*ldv>; X is (nbr*8) x (nbc*8).
__device__ __forceinline__ void dot_dense_wave(int64_t q, int lane, const double* __restrict__ xf,
                                               const double* __restrict__ xs, const uint8_t* __restrict__ xphi,
                                               const uint32_t* __restrict__ xc, int64_t nbr, int64_t nbc,
                                               const int64_t* __restrict__ xrow, const double* __restrict__ v,
                                               int64_t ldv, double* __restrict__ out)
{
    const int64_t i = xrow[q];
    const bool ok = i >= 0 && i < nbr * 8;
    double acc = 0.0;
    if (ok) {
        const int64_t I = i >> 3;
        const int r = (int)(i & 7);
        const double* vq = v + q * ldv;
        for (int64_t kb = lane; kb < nbc; kb += 64) {
            double xl[8];
            block_line<false>(xf, xs, xphi, xc, I * nbc + kb, r, xl);
            const double2* vp = reinterpret_cast<const double2*>(vq + kb * 8);
#pragma unroll
            for (int k = 0; k < 4; ++k) {
                const double2 vv = vp[k];
                acc += xl[2 * k] * vv.x;
                acc += xl[2 * k + 1] * vv.y;
            }
        }
    }
    acc = wave_sum(acc);
    if (lane == 0) out[q] = ok ? acc : __builtin_nan("");
}

}  // namespace blaz
