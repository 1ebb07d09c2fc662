// Compression with the transform stage on the matrix cores (FP32, or BF16
// hi + lo with three products), every other stage in binary64.
//
// Normalization (Eq. eqnorm), the mean slope (Eqs. eqslope, eqslope2),
// Delta' = Delta / s, the DC coefficient (fixed-order binary64, as in the
// plain kernel), m, phi and the truncation of the codes (Eq. eqphi) are
// exactly those of compress_f64_kernel.  Only the 63 other coefficients of
// the two-dimensional DCT-II (Eq. eqdct) change arithmetic: for the wave's
// 64 blocks they are one matrix product
//     D[b][c] = sum_e Delta'[b][e] K[e][c],   K[e][c] = T(i, u) T(j, v)
// with e = 8u + v the element and c = 8i + j the coefficient (the Kronecker
// form of the separable transform), 64 x 64 x 64 per wave on MFMA with FP32
// accumulation.  Delta' goes through LDS to reach the MFMA operand layout and
// D comes back through LDS to one block per lane for the quantization.
#include <hip/hip_runtime.h>

#include "blaz_codec.hpp"
#include "blaz_device.hpp"
#include "blaz_internal.hpp"

namespace blaz {

typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));

// bf16 bit pattern of a float, rounded to nearest even (finite inputs).
constexpr uint16_t bf16_bits(float f)
{
    uint32_t u = __builtin_bit_cast(uint32_t, f);
    u += 0x7FFFu + ((u >> 16) & 1u);
    return (uint16_t)(u >> 16);
}
constexpr float bf16_value(uint16_t h) { return __builtin_bit_cast(float, (uint32_t)h << 16); }

// K in FP32, [e][c]: the B operand of the FP32 16x16x4 MFMA takes one k = e
// row element per lane.
struct KronF32 {
    float v[64 * 64];
};
// K split into BF16 hi + lo, stored transposed [c][e]: the B operand of the
// BF16 16x16x32 MFMA takes 8 consecutive e of one column c per lane.
struct alignas(16) KronBF16 {
    uint16_t hi[64 * 64];
    uint16_t lo[64 * 64];
};

constexpr double kron(int e, int c) { return dct_t(c / 8, e / 8) * dct_t(c % 8, e % 8); }

constexpr KronF32 make_kron_f32()
{
    KronF32 k{};
    for (int e = 0; e < 64; ++e)
        for (int c = 0; c < 64; ++c) k.v[e * 64 + c] = (float)kron(e, c);
    return k;
}

constexpr KronBF16 make_kron_bf16()
{
    KronBF16 k{};
    for (int c = 0; c < 64; ++c)
        for (int e = 0; e < 64; ++e) {
            const double t = kron(e, c);
            const uint16_t h = bf16_bits((float)t);
            k.hi[c * 64 + e] = h;
            k.lo[c * 64 + e] = bf16_bits((float)(t - (double)bf16_value(h)));
        }
    return k;
}

__constant__ KronF32 kKronF32 = make_kron_f32();
__constant__ KronBF16 kKronBF16 = make_kron_bf16();

constexpr int kRowF = 65;  // floats per LDS row: consecutive rows start one bank apart
constexpr int kRowH = 72;  // bf16 per LDS row (144 B): 16 rows land on 16 distinct 4-bank groups

template <int kPrec, bool kVec, bool kPsi>
__global__ __launch_bounds__(kWave, 2) void compress_mixed_kernel(const double* __restrict__ A, int64_t lda,
                                                               int64_t nbc, int64_t nblk, double* __restrict__ fo,
                                                               double* __restrict__ so, uint8_t* __restrict__ phio,
                                                               uint32_t* __restrict__ codes,
                                                               uint8_t* __restrict__ psi)
{
    // One buffer for the row staging, the MFMA operand, the MFMA result and
    // the packed codes, used one after the other.
    __shared__ __align__(16) unsigned char smem[2 * 64 * kRowH * 2];
    const int lane = threadIdx.x;
    const int g = lane >> 4, l16 = lane & 15;
    const int64_t wave_base = (int64_t)blockIdx.x * kWave;

    double x[64];
    load_blocks<kVec>(A, lda, nbc, nblk, wave_base, lane, reinterpret_cast<double*>(smem), x);
    SlopeOut so_ = slope_of(x);
    if constexpr (kPsi) predict_block<true, false>(x, so_, psi, wave_base + lane, wave_base + lane < nblk);
    divide_by_slope(x, so_.s);

    f32x4 acc[4][4];
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < 4; ++j) acc[i][j] = f32x4{0.f, 0.f, 0.f, 0.f};

    if constexpr (kPrec == BLAZ_PREC_FP32) {
        // Operand A[b][e] = Delta'[b][e] in FP32, row b = lane.
        float* af = reinterpret_cast<float*>(smem);
#pragma unroll
        for (int e = 0; e < 64; ++e) af[lane * kRowF + e] = (float)x[e];
        __syncthreads();
        // 16x16x4: lane holds A[m = l%16][k = l/16] and B[k = l/16][n = l%16].
#pragma unroll
        for (int ks = 0; ks < 16; ++ks) {
            float a[4], bv[4];
#pragma unroll
            for (int mt = 0; mt < 4; ++mt) a[mt] = af[(mt * 16 + l16) * kRowF + ks * 4 + g];
#pragma unroll
            for (int nt = 0; nt < 4; ++nt) bv[nt] = kKronF32.v[(ks * 4 + g) * 64 + nt * 16 + l16];
#pragma unroll
            for (int mt = 0; mt < 4; ++mt)
#pragma unroll
                for (int nt = 0; nt < 4; ++nt)
                    acc[mt][nt] = __builtin_amdgcn_mfma_f32_16x16x4f32(a[mt], bv[nt], acc[mt][nt], 0, 0, 0);
        }
    } else {
        // Operand A[b][e] = Delta'[b][e] split into BF16 hi + lo.
        __bf16* ah = reinterpret_cast<__bf16*>(smem);
        __bf16* al = ah + 64 * kRowH;
#pragma unroll
        for (int e0 = 0; e0 < 64; e0 += 8) {
            bf16x8 h, l;
#pragma unroll
            for (int q = 0; q < 8; ++q) {
                const float xf = (float)x[e0 + q];
                const __bf16 hq = (__bf16)xf;
                h[q] = hq;
                l[q] = (__bf16)(float)(x[e0 + q] - (double)(float)hq);
            }
            *reinterpret_cast<bf16x8*>(&ah[lane * kRowH + e0]) = h;
            *reinterpret_cast<bf16x8*>(&al[lane * kRowH + e0]) = l;
        }
        __syncthreads();
        // 16x16x32: lane holds the 8 k-values 8*(l/16).. of row (A) or
        // column (B) l%16, for A and B alike.
#pragma unroll
        for (int ks = 0; ks < 2; ++ks) {
            bf16x8 a_hi[4], a_lo[4], b_hi[4], b_lo[4];
#pragma unroll
            for (int mt = 0; mt < 4; ++mt) {
                const int off = (mt * 16 + l16) * kRowH + ks * 32 + 8 * g;
                a_hi[mt] = *reinterpret_cast<const bf16x8*>(&ah[off]);
                a_lo[mt] = *reinterpret_cast<const bf16x8*>(&al[off]);
            }
#pragma unroll
            for (int nt = 0; nt < 4; ++nt) {
                const int off = (nt * 16 + l16) * 64 + ks * 32 + 8 * g;
                b_hi[nt] = __builtin_bit_cast(bf16x8, *reinterpret_cast<const uint4*>(&kKronBF16.hi[off]));
                b_lo[nt] = __builtin_bit_cast(bf16x8, *reinterpret_cast<const uint4*>(&kKronBF16.lo[off]));
            }
#pragma unroll
            for (int mt = 0; mt < 4; ++mt)
#pragma unroll
                for (int nt = 0; nt < 4; ++nt) {
                    acc[mt][nt] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a_lo[mt], b_hi[nt], acc[mt][nt], 0, 0, 0);
                    acc[mt][nt] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a_hi[mt], b_lo[nt], acc[mt][nt], 0, 0, 0);
                    acc[mt][nt] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a_hi[mt], b_hi[nt], acc[mt][nt], 0, 0, 0);
                }
        }
    }
    __syncthreads();  // every operand read is done before D overwrites the buffer

    // D[b][c]: value r of lane l in tile (mt, nt) is row b = 16 mt + 4 (l/16) + r,
    // column c = 16 nt + l%16 (16x16 FP32-accumulator layout).
    float* df = reinterpret_cast<float*>(smem);
#pragma unroll
    for (int mt = 0; mt < 4; ++mt)
#pragma unroll
        for (int nt = 0; nt < 4; ++nt)
#pragma unroll
            for (int r = 0; r < 4; ++r) df[(mt * 16 + 4 * g + r) * kRowF + nt * 16 + l16] = acc[mt][nt][r];
    __syncthreads();
#pragma unroll
    for (int c = 0; c < 64; ++c) x[c] = (double)df[lane * kRowF + c];
    x[0] = so_.dc;

    quantize_store(x, so_, nblk, wave_base, lane, smem, fo, so, phio, codes);
}

namespace detail {

template <int kPrec>
static void launch_mixed(const double* A, int64_t lda, int64_t nbc, int64_t nblk, const blaz_matrix& m, uint8_t* psi,
                         bool vec, hipStream_t st)
{
    const unsigned grid = (unsigned)((nblk + kWave - 1) / kWave);
    auto* cw = reinterpret_cast<uint32_t*>(m.codes);
    if (vec && psi)
        compress_mixed_kernel<kPrec, true, true><<<grid, kWave, 0, st>>>(A, lda, nbc, nblk, m.f, m.s, m.phi, cw, psi);
    else if (vec)
        compress_mixed_kernel<kPrec, true, false><<<grid, kWave, 0, st>>>(A, lda, nbc, nblk, m.f, m.s, m.phi, cw, psi);
    else if (psi)
        compress_mixed_kernel<kPrec, false, true><<<grid, kWave, 0, st>>>(A, lda, nbc, nblk, m.f, m.s, m.phi, cw, psi);
    else
        compress_mixed_kernel<kPrec, false, false><<<grid, kWave, 0, st>>>(A, lda, nbc, nblk, m.f, m.s, m.phi, cw, psi);
}

hipError_t launch_compress_mixed(const double* A, int64_t lda, const blaz_matrix& m, uint8_t* psi,
                                 blaz_precision prec, hipStream_t st)
{
    const int64_t nbc = m.cols / 8;
    const int64_t nblk = (m.rows / 8) * nbc;
    const bool vec = (reinterpret_cast<uintptr_t>(A) % 16 == 0) && (lda % 2 == 0);
    if (prec == BLAZ_PREC_FP32)
        launch_mixed<BLAZ_PREC_FP32>(A, lda, nbc, nblk, m, psi, vec, st);
    else
        launch_mixed<BLAZ_PREC_BF16X3>(A, lda, nbc, nblk, m, psi, vec, st);
    return hipGetLastError();
}

}  // namespace detail
}  // namespace blaz
