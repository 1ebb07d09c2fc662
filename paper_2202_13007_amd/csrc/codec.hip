// Compression and decompression kernels (Section "Compression Scheme" and
// Eq. eqbbb of Section "Basic Linear Algebra Algorithms").
//
// Mapping: one lane per 8x8 block.  A block's 64 values live in the lane's
// VGPRs for the whole pipeline, so normalization, the two slope reductions,
// both 8-point transform passes and the max reduction are plain in-register
// arithmetic with no cross-lane traffic and no LDS round trips.  A wave owns
// 64 consecutive blocks of a block row, so each of the 8 row loads of a wave
// reads one contiguous 4 KiB segment (64 lanes x 64 B) of the matrix.
#include <hip/hip_runtime.h>

#include "blaz_device.hpp"
#include "blaz_internal.hpp"

namespace blaz {

typedef double f64x2 __attribute__((ext_vector_type(2)));

// Pairwise sum of the 64 values v(0..63) in row-major order: level 1 adds
// (v0+v1), (v2+v3), ..., each next level adds adjacent pairs.  This fixed
// order makes the slope s and the DC coefficient bit-reproducible.
template <typename F>
__device__ __forceinline__ double pairwise64(F v)
{
    double t[32];
#pragma unroll
    for (int i = 0; i < 32; ++i) t[i] = v(2 * i) + v(2 * i + 1);
#pragma unroll
    for (int n = 16; n >= 1; n /= 2) {
#pragma unroll
        for (int i = 0; i < n; ++i) t[i] = t[2 * i] + t[2 * i + 1];
    }
    return t[0];
}

template <bool kVec>
__device__ __forceinline__ void load_block(const double* __restrict__ src, int64_t lda, double x[64])
{
#pragma unroll
    for (int r = 0; r < 8; ++r) {
        const double* row = src + r * lda;
        if constexpr (kVec) {
#pragma unroll
            for (int c = 0; c < 8; c += 2) {
                const f64x2 v = __builtin_nontemporal_load(reinterpret_cast<const f64x2*>(row + c));
                x[r * 8 + c] = v[0];
                x[r * 8 + c + 1] = v[1];
            }
        } else {
#pragma unroll
            for (int c = 0; c < 8; ++c) x[r * 8 + c] = row[c];
        }
    }
}

template <bool kVec>
__device__ __forceinline__ void store_block(double* __restrict__ dst, int64_t lda, const double x[64])
{
#pragma unroll
    for (int r = 0; r < 8; ++r) {
        double* row = dst + r * lda;
        if constexpr (kVec) {
#pragma unroll
            for (int c = 0; c < 8; c += 2) {
                const f64x2 v = {x[r * 8 + c], x[r * 8 + c + 1]};
                __builtin_nontemporal_store(v, reinterpret_cast<f64x2*>(row + c));
            }
        } else {
#pragma unroll
            for (int c = 0; c < 8; ++c) row[c] = x[r * 8 + c];
        }
    }
}

// Normalization, Eq. eqnorm, in place.  Processing from the bottom-right
// corner backwards keeps every left and upper neighbour unmodified when it is
// read.  The interior term is ((M - Mup) + (M - Mleft)) * 0.5 exactly as
// written (no contraction is possible: there is no product).
__device__ __forceinline__ void normalize(double x[64])
{
#pragma unroll
    for (int u = 7; u >= 1; --u) {
#pragma unroll
        for (int v = 7; v >= 1; --v)
            x[u * 8 + v] = ((x[u * 8 + v] - x[(u - 1) * 8 + v]) + (x[u * 8 + v] - x[u * 8 + v - 1])) * 0.5;
    }
#pragma unroll
    for (int v = 7; v >= 1; --v) x[v] = x[v] - x[v - 1];
#pragma unroll
    for (int u = 7; u >= 1; --u) x[u * 8] = x[u * 8] - x[(u - 1) * 8];
    x[0] = 0.0;
}

template <bool kVec, bool kPsi>
__global__ __launch_bounds__(256) void compress_f64_kernel(const double* __restrict__ A, int64_t lda,
                                                           int64_t nbc, int64_t nblk, double* __restrict__ fo,
                                                           double* __restrict__ so, uint8_t* __restrict__ phio,
                                                           uint32_t* __restrict__ codes,
                                                           uint8_t* __restrict__ psi)
{
    const int64_t b = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (b >= nblk) return;
    const int64_t I = b / nbc;
    const int64_t J = b - I * nbc;

    double x[64];
    load_block<kVec>(A + (I * 8) * lda + J * 8, lda, x);
    const double f = x[0];

    // Normalization (Eq. eqnorm) and mean slope (Eqs. eqslope, eqslope2).
    normalize(x);
    int K = 0;
#pragma unroll
    for (int e = 1; e < 64; ++e) K += x[e] != 0.0 ? 1 : 0;
    const double S1 = pairwise64([&](int e) { return fabs(x[e]); });
    const double S = pairwise64([&](int e) { return x[e]; });
    const double s = K > 0 ? S1 / (double)K : 0.0;
    // D_00 = alpha_0^2 sum Delta' = 0.125 (sum Delta / s), the fixed order.
    const double dc = s != 0.0 ? 0.125 * (S / s) : 0.0;

    // Delta' = Delta / s.  The reciprocal is exact enough for the 63 other
    // coefficients; a slope so small that 1/s overflows falls back to division.
    if (s != 0.0 && fabs(s) >= 0x1p-1020) {
        const double r = 1.0 / s;
#pragma unroll
        for (int e = 0; e < 64; ++e) x[e] *= r;
    } else if (s != 0.0) {
#pragma unroll
        for (int e = 0; e < 64; ++e) x[e] = x[e] / s;
    }

    if constexpr (kPsi) {
        // Prediction, Eq. eqpredict: index of the nearest of 256 points
        // s - smax + k * (2 smax / 256), the smaller index on a tie.
        double smax = 0.0;
#pragma unroll
        for (int e = 0; e < 64; ++e) smax = fmax(smax, fabs(x[e]));
        uint32_t w[16];
#pragma unroll
        for (int q = 0; q < 16; ++q) w[q] = 0;
        if (smax != 0.0) {
            const double lo = s - smax;
            const double inv_step = 128.0 / smax;
#pragma unroll
            for (int e = 0; e < 64; ++e) {
                double k = ceil((x[e] - lo) * inv_step - 0.5);
                k = fmin(fmax(k, 0.0), 255.0);
                w[e / 4] |= (uint32_t)k << (8 * (e % 4));
            }
        }
        uint4* dst = reinterpret_cast<uint4*>(psi + b * 64);
#pragma unroll
        for (int q = 0; q < 4; ++q) dst[q] = make_uint4(w[4 * q], w[4 * q + 1], w[4 * q + 2], w[4 * q + 3]);
    }

    // Two-dimensional DCT-II (Eq. eqdct): rows, then columns, in place.
#pragma unroll
    for (int u = 0; u < 8; ++u) dct8<1, 1>(x + u * 8, x + u * 8);
#pragma unroll
    for (int v = 0; v < 8; ++v) dct8<8, 8>(x + v, x + v);
    x[0] = dc;

    // Quantization (Eq. eqphi): m over all 64 coefficients, phi = trunc(127/m)
    // clamped to 255, codes = trunc(phi * D) at the 28 kept positions.
    double m = 0.0;
#pragma unroll
    for (int e = 0; e < 64; ++e) m = fmax(m, fabs(x[e]));
    const double px = 127.0 / m;  // +inf when m == 0
    const int phi = px < 255.0 ? (int)px : 255;
    const double phid = (double)phi;
    uint32_t w[kCodeWords];
#pragma unroll
    for (int q = 0; q < kCodeWords; ++q) w[q] = 0;
#pragma unroll
    for (int t = 0; t < kKept; ++t) {
        const int c = (int)(phid * x[kept_row(t) * 8 + kept_col(t)]);  // truncation toward zero
        w[t / 4] |= ((uint32_t)c & 0xffu) << (8 * (t % 4));
    }

    fo[b] = f;
    so[b] = s;
    phio[b] = (uint8_t)phi;
    uint32_t* cw = codes + b * kCodeWords;
#pragma unroll
    for (int q = 0; q < kCodeWords; ++q) cw[q] = w[q];
}

template <bool kVec>
__global__ __launch_bounds__(256) void decompress_kernel(const double* __restrict__ f, const double* __restrict__ s,
                                                         const uint8_t* __restrict__ phi,
                                                         const uint32_t* __restrict__ codes, int64_t nbc,
                                                         int64_t nblk, double* __restrict__ A, int64_t lda)
{
    const int64_t b = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (b >= nblk) return;
    const int64_t I = b / nbc;
    const int64_t J = b - I * nbc;

    uint32_t w[kCodeWords];
#pragma unroll
    for (int q = 0; q < kCodeWords; ++q) w[q] = codes[b * kCodeWords + q];
    // Dhat = C / phi at the kept positions (zero elsewhere); the slope factor
    // of Eq. eqbbb is folded in by linearity of the inverse DCT.
    double coef[kKept];
    unpack_codes(w, s[b] / (double)phi[b], coef);
    double x[64];
    inverse_transform(coef, x);
    inverse_normalize(f[b], x);
    store_block<kVec>(A + (I * 8) * lda + J * 8, lda, x);
}

namespace detail {

static inline unsigned grid_for(int64_t nblk, int threads) { return (unsigned)((nblk + threads - 1) / threads); }

hipError_t launch_compress_f64(const double* A, int64_t lda, const blaz_matrix& m, uint8_t* psi, hipStream_t st)
{
    const int64_t nbc = m.cols / 8;
    const int64_t nblk = (m.rows / 8) * nbc;
    const bool vec = (reinterpret_cast<uintptr_t>(A) % 16 == 0) && (lda % 2 == 0);
    const unsigned grid = grid_for(nblk, 256);
    auto* cw = reinterpret_cast<uint32_t*>(m.codes);
    if (vec && psi)
        compress_f64_kernel<true, true><<<grid, 256, 0, st>>>(A, lda, nbc, nblk, m.f, m.s, m.phi, cw, psi);
    else if (vec)
        compress_f64_kernel<true, false><<<grid, 256, 0, st>>>(A, lda, nbc, nblk, m.f, m.s, m.phi, cw, psi);
    else if (psi)
        compress_f64_kernel<false, true><<<grid, 256, 0, st>>>(A, lda, nbc, nblk, m.f, m.s, m.phi, cw, psi);
    else
        compress_f64_kernel<false, false><<<grid, 256, 0, st>>>(A, lda, nbc, nblk, m.f, m.s, m.phi, cw, psi);
    return hipGetLastError();
}

hipError_t launch_decompress(const blaz_matrix& m, double* A, int64_t lda, hipStream_t st)
{
    const int64_t nbc = m.cols / 8;
    const int64_t nblk = (m.rows / 8) * nbc;
    const bool vec = (reinterpret_cast<uintptr_t>(A) % 16 == 0) && (lda % 2 == 0);
    const unsigned grid = grid_for(nblk, 256);
    const auto* cw = reinterpret_cast<const uint32_t*>(m.codes);
    if (vec)
        decompress_kernel<true><<<grid, 256, 0, st>>>(m.f, m.s, m.phi, cw, nbc, nblk, A, lda);
    else
        decompress_kernel<false><<<grid, 256, 0, st>>>(m.f, m.s, m.phi, cw, nbc, nblk, A, lda);
    return hipGetLastError();
}

}  // namespace detail
}  // namespace blaz
