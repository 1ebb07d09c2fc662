// Compression with the transform stage on the matrix cores (FP32, or BF16
// hi + lo with three products), every other stage in binary64.
//
// Normalization (Eq. eqnorm), the mean slope (Eqs. eqslope, eqslope2),
// Delta' = Delta / s, the DC coefficient (fixed-order binary64, as in the
// plain kernel), m, phi and the truncation of the codes (Eq. eqphi) are
// exactly those of compress_f64_kernel.  Only the 63 other coefficients of
// the two-dimensional DCT-II (Eq. eqdct), D = T Delta' T^T, change
// arithmetic: both 8-point passes run on MFMA with FP32 accumulation.
//
// Four blocks at a time form a 16 x 16 operand X = [P Q; R S] (blocks side by
// side and one above the other).  The row pass is X diag(T^T, T^T), which is
// [P T^T  Q T^T; R T^T  S T^T], and the column pass is diag(T, T) times that,
// which is T (.) T^T of each block: two 16 x 16 x 16 products per four
// blocks, a quarter of the multiply-adds of the 64 x 64 Kronecker form.  The
// k index of each product is assigned to (lane group g, slot t) as
// k = 4 g + t, for A and B alike, which the sum over k allows.  With that
// assignment the row pass's result, which lane (g, n) holds as rows
// 4 g .. 4 g + 3 of column n, is exactly the B operand lane (g, n) supplies
// to the column pass, so the two passes chain in registers; the block
// diagonal constants are the same four values per lane for both passes.
// Delta' reaches the operand layout through LDS (rows of 4 values, 16-byte
// or 8-byte reads) and D returns through LDS to one block per lane for the
// quantization; both layouts are free of bank conflicts.
#include <hip/hip_runtime.h>

#include "blaz_codec.hpp"
#include "blaz_device.hpp"
#include "blaz_internal.hpp"

namespace blaz {

typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef short s16x4 __attribute__((ext_vector_type(4)));
typedef __bf16 bf16x4 __attribute__((ext_vector_type(4)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));

// FP32 staging of Delta' and of D: one block per 68 floats (4 floats of
// padding), row u as two 16-byte halves stored in the order
// h ^ ((u >> 2) & 1).  Writes (a lane's own block, 8 lanes per access
// phase on 8 blocks) and operand reads (8 lanes on 8 rows of one block)
// both touch 32 distinct banks.
constexpr int kPitchF = 68;
__device__ __forceinline__ int f32_slot(int blk, int u, int h) { return blk * kPitchF + 8 * u + 4 * (h ^ ((u >> 2) & 1)); }

// BF16 staging of Delta' (hi and lo arrays): one block per 72 bf16, row u as
// two 8-byte halves stored in the order h ^ ((u >> 1) & 1): 16-byte row
// writes and 8-byte operand reads without bank conflicts.
constexpr int kPitchH = 72;
__device__ __forceinline__ int bf16_slot(int blk, int u, int h) { return blk * kPitchH + 8 * u + 4 * (h ^ ((u >> 1) & 1)); }

__device__ __forceinline__ short bf16_bits_of(__bf16 h) { return __builtin_bit_cast(short, h); }

template <int kPrec, bool kVec, bool kPsi>
__global__ __launch_bounds__(kWave, 2) void compress_mixed_kernel(const double* __restrict__ A, int64_t lda,
                                                               int64_t nbc, int64_t nblk, double* __restrict__ fo,
                                                               double* __restrict__ so, uint8_t* __restrict__ phio,
                                                               uint32_t* __restrict__ codes,
                                                               uint8_t* __restrict__ psi)
{
    // One buffer for the row staging, the operand staging, D and the packed
    // codes, used one after the other.
    __shared__ __align__(16) unsigned char smem[2 * 64 * kPitchH * 2];
    static_assert(sizeof(smem) >= 64 * kPitchF * 4, "D fits the buffer");
    const int lane = threadIdx.x;
    const int g = lane >> 4, l16 = lane & 15;
    const int64_t wave_base = (int64_t)blockIdx.x * kWave;

    double x[64];
    load_blocks<kVec>(A, lda, nbc, nblk, wave_base, lane, reinterpret_cast<double*>(smem), x);
    SlopeOut so_ = slope_of(x);
    if constexpr (kPsi) predict_block<true, false>(x, so_, psi, wave_base + lane, wave_base + lane < nblk);
    divide_by_slope(x, so_.s);

    // The block-diagonal constants of lane (g, n = l16) at slot t: row
    // 4 g + t, column n of diag(T^T, T^T) (row pass, B operand) and row n,
    // column 4 g + t of diag(T, T) (column pass, A operand), both
    // T(n % 8, 4 (g % 2) + t) when the diagonal blocks agree (g / 2 == n / 8).
    double tc[4];
#pragma unroll
    for (int t = 0; t < 4; ++t) tc[t] = (g >> 1) == (l16 >> 3) ? dct_t(l16 & 7, 4 * (g & 1) + t) : 0.0;

    // Operand of the row pass for group G: lane (g, m = l16) supplies
    // X[m][4 g .. 4 g + 3] = half g % 2 of row m % 8 of block
    // 4 G + 2 (m / 8) + g / 2.  Result: lane (g, c) holds
    // D[4 (g % 2) + r][c % 8], r = 0..3, of block 4 G + 2 (g / 2) + c / 8.
    f32x4 dacc[16];
    const int xu = l16 & 7, xh = g & 1, xb = 2 * (l16 >> 3) + (g >> 1);
    if constexpr (kPrec == BLAZ_PREC_FP32) {
        float* sf = reinterpret_cast<float*>(smem);
        __syncthreads();  // the row staging is done with the buffer
#pragma unroll
        for (int u = 0; u < 8; ++u)
#pragma unroll
            for (int h = 0; h < 2; ++h)
                *reinterpret_cast<f32x4*>(&sf[f32_slot(lane, u, h)]) =
                    f32x4{(float)x[8 * u + 4 * h], (float)x[8 * u + 4 * h + 1], (float)x[8 * u + 4 * h + 2],
                          (float)x[8 * u + 4 * h + 3]};
        __syncthreads();
        float c[4];
#pragma unroll
        for (int t = 0; t < 4; ++t) c[t] = (float)tc[t];
#pragma unroll
        for (int G = 0; G < 16; ++G) {
            const f32x4 a = *reinterpret_cast<const f32x4*>(&sf[f32_slot(4 * G + xb, xu, xh)]);
            f32x4 r = f32x4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
            for (int t = 0; t < 4; ++t) r = __builtin_amdgcn_mfma_f32_16x16x4f32(a[t], c[t], r, 0, 0, 0);
            f32x4 d = f32x4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
            for (int t = 0; t < 4; ++t) d = __builtin_amdgcn_mfma_f32_16x16x4f32(c[t], r[t], d, 0, 0, 0);
            dacc[G] = d;
        }
    } else {
        // Delta' = hi + lo, hi = bf16(Delta'), lo = bf16(Delta' - hi), split in
        // FP32 (Delta' - hi is exact there; |Delta' - hi - lo| <= (2^-16 +
        // 2^-24) |Delta'|)
        __bf16* sh = reinterpret_cast<__bf16*>(smem);
        __bf16* sl = sh + 64 * kPitchH;
        __syncthreads();  // the row staging is done with the buffer
#pragma unroll
        for (int u = 0; u < 8; ++u) {
            bf16x8 h, l;
#pragma unroll
            for (int q = 0; q < 8; ++q) {
                const float xv = (float)x[8 * u + q];
                const __bf16 hq = (__bf16)xv;
                // slot of value q: its half q / 4 lands in position (q / 4) ^ ((u >> 1) & 1)
                const int pos = 4 * ((q >> 2) ^ ((u >> 1) & 1)) + (q & 3);
                h[pos] = hq;
                l[pos] = (__bf16)(xv - (float)hq);
            }
            *reinterpret_cast<bf16x8*>(&sh[lane * kPitchH + 8 * u]) = h;
            *reinterpret_cast<bf16x8*>(&sl[lane * kPitchH + 8 * u]) = l;
        }
        __syncthreads();
        s16x4 ch, cl;
#pragma unroll
        for (int t = 0; t < 4; ++t) {
            const __bf16 hq = (__bf16)(float)tc[t];
            ch[t] = bf16_bits_of(hq);
            cl[t] = bf16_bits_of((__bf16)(float)(tc[t] - (double)(float)hq));
        }
#pragma unroll
        for (int G = 0; G < 16; ++G) {
            const int off = bf16_slot(4 * G + xb, xu, xh);
            const s16x4 ah = __builtin_bit_cast(s16x4, *reinterpret_cast<const bf16x4*>(&sh[off]));
            const s16x4 al = __builtin_bit_cast(s16x4, *reinterpret_cast<const bf16x4*>(&sl[off]));
            f32x4 r = f32x4{0.f, 0.f, 0.f, 0.f};
            r = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(al, ch, r, 0, 0, 0);
            r = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(ah, cl, r, 0, 0, 0);
            r = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(ah, ch, r, 0, 0, 0);
            s16x4 rh, rl;
#pragma unroll
            for (int t = 0; t < 4; ++t) {
                const __bf16 hq = (__bf16)r[t];
                rh[t] = bf16_bits_of(hq);
                rl[t] = bf16_bits_of((__bf16)(r[t] - (float)hq));
            }
            f32x4 d = f32x4{0.f, 0.f, 0.f, 0.f};
            d = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(ch, rl, d, 0, 0, 0);
            d = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(cl, rh, d, 0, 0, 0);
            d = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(ch, rh, d, 0, 0, 0);
            dacc[G] = d;
        }
    }
    __syncthreads();  // every operand read is done before D overwrites the buffer

    // D back to one block per lane, each block stored transposed (row j of
    // the stored block is column j of D): lane (g, c) writes D[4 (g % 2) ..
    // 4 (g % 2) + 3][c % 8] as one 16-byte half.
    float* df = reinterpret_cast<float*>(smem);
#pragma unroll
    for (int G = 0; G < 16; ++G)
        *reinterpret_cast<f32x4*>(&df[f32_slot(4 * G + 2 * (g >> 1) + (l16 >> 3), l16 & 7, g & 1)]) = dacc[G];
    __syncthreads();
    float dv[64];  // D of the lane's block, row-major
#pragma unroll
    for (int j = 0; j < 8; ++j)
#pragma unroll
        for (int h = 0; h < 2; ++h) {
            const f32x4 v = *reinterpret_cast<const f32x4*>(&df[f32_slot(lane, j, h)]);
#pragma unroll
            for (int q = 0; q < 4; ++q) dv[8 * (4 * h + q) + j] = v[q];
        }

    // Quantization with quantize_store's values: m over the 63 non-DC
    // coefficients is taken in FP32 (widening to binary64 is exact and keeps
    // the order, so it is the binary64 max of the widened values) and joined
    // with |DC| in binary64; the codes are trunc(phi D) in binary64 of the
    // widened coefficients, the DC code of the binary64 DC.
    float mf = 0.0f;
#pragma unroll
    for (int e = 1; e < 64; ++e) mf = fmaxf(mf, fabsf(dv[e]));
    const int phi = phi_of(fmax((double)mf, fabs(so_.dc)));
    const double phid = (double)phi;
    uint32_t w[kCodeWords];
#pragma unroll
    for (int q = 0; q < kCodeWords; ++q) w[q] = 0;
#pragma unroll
    for (int t = 0; t < kKept; ++t) {
        const int e = kept_row(t) * 8 + kept_col(t);
        pack_code(w, t, phid, e == 0 ? so_.dc : (double)dv[e]);
    }
    store_record(w, phi, so_, nblk, wave_base, lane, smem, fo, so, phio, codes);
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
