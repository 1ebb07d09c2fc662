// Device helpers shared by the blaz kernels: the orthonormal DCT-II basis of
// Eq. eqdct (alphas as defined after Eq. eqdct2) and 8-point transforms on
// register arrays.  All loops are fully unrolled with compile-time indices so
// the 8x8 blocks stay in VGPRs.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace blaz {

constexpr int kKept = 28;          // coefficients kept per block
constexpr int kCodeWords = 7;      // 28 int8 codes = 7 dwords

// cos(a * pi / 16) for a = 0..8.
__host__ __device__ constexpr double cos16(int a)
{
    return a == 0 ? 1.0
         : a == 1 ? 0.98078528040323044912618223613424
         : a == 2 ? 0.92387953251128675612818318939679
         : a == 3 ? 0.83146961230254523707878837761791
         : a == 4 ? 0.70710678118654752440084436210485
         : a == 5 ? 0.55557023301960222474283081394853
         : a == 6 ? 0.38268343236508977172845998403040
         : a == 7 ? 0.19509032201612826784828486847702
         : 0.0;
}

// T(k, n) = alpha_k cos((2n + 1) k pi / 16): row k of the orthonormal 8-point
// DCT-II matrix, alpha_0 = sqrt(1/8), alpha_k = sqrt(1/4) = 1/2 otherwise.
__host__ __device__ constexpr double dct_t(int k, int n)
{
    int a = ((2 * n + 1) * k) % 32;  // angle a*pi/16, reduced mod 2 pi
    if (a > 16) a = 32 - a;          // cos(2 pi - x) = cos x
    double sgn = 1.0;
    if (a > 8) {                     // cos(pi - x) = -cos x
        a = 16 - a;
        sgn = -1.0;
    }
    const double alpha = k == 0 ? 0.35355339059327376220042218105242 : 0.5;
    return sgn * alpha * cos16(a);
}

// Forward 8-point orthonormal DCT-II, y_k = sum_n T(k, n) x_n, using the
// even/odd symmetry T(k, 7-n) = (-1)^k T(k, n) (36 flops instead of 64).
// x and y may alias.  SX/SY are element strides.
template <int SX, int SY, typename R>
__device__ __forceinline__ void dct8(const R* x, R* y)
{
#pragma clang fp contract(fast)
    R a[4], b[4];
#pragma unroll
    for (int n = 0; n < 4; ++n) {
        a[n] = x[n * SX] + x[(7 - n) * SX];
        b[n] = x[n * SX] - x[(7 - n) * SX];
    }
    const R e0 = a[0] + a[3], e1 = a[1] + a[2];
    const R d0 = a[0] - a[3], d1 = a[1] - a[2];
    R out[8];
    out[0] = R(dct_t(0, 0)) * e0 + R(dct_t(0, 1)) * e1;
    out[4] = R(dct_t(4, 0)) * e0 + R(dct_t(4, 1)) * e1;
    out[2] = R(dct_t(2, 0)) * d0 + R(dct_t(2, 1)) * d1;
    out[6] = R(dct_t(6, 0)) * d0 + R(dct_t(6, 1)) * d1;
#pragma unroll
    for (int k = 1; k < 8; k += 2)
        out[k] = R(dct_t(k, 0)) * b[0] + R(dct_t(k, 1)) * b[1] + R(dct_t(k, 2)) * b[2] + R(dct_t(k, 3)) * b[3];
#pragma unroll
    for (int k = 0; k < 8; ++k) y[k * SY] = out[k];
}

// Inverse 8-point DCT (DCT-III), x_n = sum_k T(k, n) y_k.  y and x may alias.
template <int SY, int SX, typename R>
__device__ __forceinline__ void idct8(const R* y, R* x)
{
#pragma clang fp contract(fast)
    R p[2], q[2], e[4], o[4];
#pragma unroll
    for (int n = 0; n < 2; ++n) {
        p[n] = R(dct_t(0, n)) * y[0] + R(dct_t(4, n)) * y[4 * SY];
        q[n] = R(dct_t(2, n)) * y[2 * SY] + R(dct_t(6, n)) * y[6 * SY];
    }
    e[0] = p[0] + q[0];
    e[3] = p[0] - q[0];
    e[1] = p[1] + q[1];
    e[2] = p[1] - q[1];
#pragma unroll
    for (int n = 0; n < 4; ++n)
        o[n] = R(dct_t(1, n)) * y[1 * SY] + R(dct_t(3, n)) * y[3 * SY] + R(dct_t(5, n)) * y[5 * SY] +
               R(dct_t(7, n)) * y[7 * SY];
    R out[8];
#pragma unroll
    for (int n = 0; n < 4; ++n) {
        out[n] = e[n] + o[n];
        out[7 - n] = e[n] - o[n];
    }
#pragma unroll
    for (int n = 0; n < 8; ++n) x[n * SX] = out[n];
}

// Inverse 8-point DCT of a vector whose only non-zero entries are y_0, y_1.
template <int SX, typename R>
__device__ __forceinline__ void idct8_two(R y0, R y1, R* x)
{
#pragma clang fp contract(fast)
    const R p = R(dct_t(0, 0)) * y0;
#pragma unroll
    for (int n = 0; n < 4; ++n) {
        const R o = R(dct_t(1, n)) * y1;
        x[n * SX] = p + o;
        x[(7 - n) * SX] = p - o;
    }
}

// Position of kept coefficient t (0..27) in the 8x8 block, row-major scan of
// the first two lines and first two columns.
__host__ __device__ constexpr int kept_row(int t) { return t < 16 ? t / 8 : 2 + (t - 16) / 2; }
__host__ __device__ constexpr int kept_col(int t) { return t < 16 ? t % 8 : (t - 16) % 2; }

// Index t of the kept coefficient at (i, j), or -1 if (i, j) is discarded.
__host__ __device__ constexpr int kept_index(int i, int j)
{
    return i < 2 ? i * 8 + j : (j < 2 ? 16 + (i - 2) * 2 + j : -1);
}

// The tunable rate: L kept lines (rows and columns 0..L-1 of the DCT),
// 16L - L^2 codes in row-major scan order, padded to whole dwords.  L = 2 is
// the paper's scheme (kKept, kCodeWords, kept_row/kept_col/kept_index).
template <int L>
struct KeptLines {
    static_assert(L >= 1 && L <= 8, "1 to 8 kept lines");
    static constexpr int kCount = 16 * L - L * L;
    static constexpr int kWords = (kCount + 3) / 4;
    // Position i*8+j of kept coefficient t: rows 0..L-1 are whole (8 each),
    // the rows below keep their first L columns.
    __host__ __device__ static constexpr int pos(int t)
    {
        return t < 8 * L ? t : (L + (t - 8 * L) / L) * 8 + (t - 8 * L) % L;
    }
    // Index t of position (i, j), or -1 if it is discarded.
    __host__ __device__ static constexpr int index(int i, int j)
    {
        return i < L ? i * 8 + j : (j < L ? 8 * L + (i - L) * L + j : -1);
    }
};

// Dequantized coefficients of one block, already multiplied by the slope:
// coef[t] = codes[t] * (s / phi).  The 28 codes arrive as 7 little-endian dwords.
__device__ __forceinline__ void unpack_codes(const uint32_t w[kCodeWords], double scale, double coef[kKept])
{
#pragma unroll
    for (int t = 0; t < kKept; ++t) {
        const int32_t c = (int32_t)(w[t / 4] << (24 - 8 * (t % 4))) >> 24;  // sign-extend byte t%4
        coef[t] = (double)c * scale;
    }
}

template <int L>
__device__ __forceinline__ void unpack_codes_lines(const uint32_t* w, double scale, double* coef)
{
#pragma unroll
    for (int t = 0; t < KeptLines<L>::kCount; ++t) {
        const int32_t c = (int32_t)(w[t / 4] << (24 - 8 * (t % 4))) >> 24;
        coef[t] = (double)c * scale;
    }
}

// The transforms and the inverse normalization may contract a*b + c into an
// FMA: their results are compared with a tolerance, never bit for bit.  The
// rest of the library is built with -ffp-contract=off.

// Full inverse transform of one block from its 28 scaled coefficients:
// P = T^T Dhat T, then the inverse of Eq. eqnorm.  out[64] row-major.
// Column pass first: columns 0 and 1 have 8 non-zeros, columns 2..7 only
// rows 0 and 1; then a full 8-point inverse per row.
__device__ __forceinline__ void inverse_transform(const double coef[kKept], double out[64])
{
    // column j, rows 0..7 of Dhat -> out[u*8 + j]
#pragma unroll
    for (int j = 0; j < 2; ++j) {
        double col[8];
#pragma unroll
        for (int i = 0; i < 8; ++i) col[i] = coef[kept_index(i, j)];
        idct8<1, 8>(col, out + j);
    }
#pragma unroll
    for (int j = 2; j < 8; ++j) idct8_two<8>(coef[kept_index(0, j)], coef[kept_index(1, j)], out + j);
#pragma unroll
    for (int u = 0; u < 8; ++u) idct8<1, 1>(out + u * 8, out + u * 8);
}

// The same for L kept lines: columns 0..L-1 hold 8 coefficients each, the
// other columns only their first L rows.
template <int L>
__device__ __forceinline__ void inverse_transform_lines(const double* coef, double out[64])
{
    using K = KeptLines<L>;
#pragma unroll
    for (int j = 0; j < 8; ++j) {
        double col[8];
#pragma unroll
        for (int i = 0; i < 8; ++i) col[i] = K::index(i, j) >= 0 ? coef[K::index(i, j)] : 0.0;
        if (j < L) {
            idct8<1, 8>(col, out + j);
        } else {
#pragma clang fp contract(fast)
#pragma unroll
            for (int u = 0; u < 8; ++u) {
                double acc = 0.0;
#pragma unroll
                for (int i = 0; i < L; ++i) acc += dct_t(i, u) * col[i];
                out[u * 8 + j] = acc;
            }
        }
    }
#pragma unroll
    for (int u = 0; u < 8; ++u) idct8<1, 1>(out + u * 8, out + u * 8);
}

// Inverse of the normalization (Eq. eqbbb with the subscripts of the exact
// inverse of Eq. eqnorm) in place: on entry d holds s * P, on exit the block.
__device__ __forceinline__ void inverse_normalize(double f, double d[64])
{
#pragma clang fp contract(fast)
    d[0] = f;
#pragma unroll
    for (int v = 1; v < 8; ++v) d[v] = d[v - 1] + d[v];
#pragma unroll
    for (int u = 1; u < 8; ++u) {
        d[u * 8] = d[(u - 1) * 8] + d[u * 8];
#pragma unroll
        for (int v = 1; v < 8; ++v) d[u * 8 + v] = (d[(u - 1) * 8 + v] + d[u * 8 + v - 1]) * 0.5 + d[u * 8 + v];
    }
}

}  // namespace blaz
