// Compression and decompression kernels (Section "Compression Scheme" and
// Eq. eqbbb of Section "Basic Linear Algebra Algorithms").
//
// Mapping: one lane per 8x8 block.  A block's 64 values live in the lane's
// VGPRs for the whole pipeline, so normalization, the two slope reductions,
// both 8-point transform passes and the max reduction are plain in-register
// arithmetic with no cross-lane traffic.  A workgroup is one wave owning 64
// consecutive blocks; its HBM traffic is staged through LDS (below) so that
// every global access instruction covers a contiguous run.
#include <hip/hip_runtime.h>

#include "blaz_codec.hpp"
#include "blaz_device.hpp"
#include "blaz_internal.hpp"

namespace blaz {

template <bool kVec, bool kPsi>
__global__ __launch_bounds__(kWave) void compress_f64_kernel(const double* __restrict__ A, int64_t lda,
                                                             int64_t nbc, int64_t nblk, double* __restrict__ fo,
                                                             double* __restrict__ so, uint8_t* __restrict__ phio,
                                                             uint32_t* __restrict__ codes,
                                                             uint8_t* __restrict__ psi)
{
    __shared__ __align__(16) double tile[kWave * kSlot];
    const int lane = threadIdx.x;
    const int64_t wave_base = (int64_t)blockIdx.x * kWave;

    double x[64];
    load_blocks<kVec>(A, lda, nbc, nblk, wave_base, lane, tile, x);
    const SlopeOut so_ = normalize_and_slope(x);
    if constexpr (kPsi) predict_store(x, so_.s, psi, wave_base + lane, wave_base + lane < nblk);

    // Two-dimensional DCT-II (Eq. eqdct) of Delta': rows, then columns, in
    // place; the DC term is the fixed-order binary64 value.
#pragma unroll
    for (int u = 0; u < 8; ++u) dct8<1, 1>(x + u * 8, x + u * 8);
#pragma unroll
    for (int v = 0; v < 8; ++v) dct8<8, 8>(x + v, x + v);
    x[0] = so_.dc;

    quantize_store(x, so_, nblk, wave_base, lane, tile, fo, so, phio, codes);
}

// Output forms of the decompression: binary64 (the plain method), and the
// operand forms of the low-precision contractions in blaz_matmul: FP32, or
// BF16 hi + lo with hi = bf16(x), lo = bf16(x - hi).
struct OutF64 {
    double* p;
    __device__ void store2(int64_t off, double a, double b) const
    {
        __builtin_nontemporal_store(f64x2{a, b}, reinterpret_cast<f64x2*>(p + off));
    }
    __device__ void store(int64_t off, double a) const { p[off] = a; }
};
struct OutF32 {
    float* p;
    __device__ void store2(int64_t off, double a, double b) const
    {
        *reinterpret_cast<f32x2*>(p + off) = f32x2{(float)a, (float)b};
    }
    __device__ void store(int64_t off, double a) const { p[off] = (float)a; }
};
struct OutBF16Split {
    __bf16* hi;
    __bf16* lo;
    __device__ static __bf16 high(double x) { return (__bf16)(float)x; }
    __device__ static __bf16 low(double x, __bf16 h) { return (__bf16)(float)(x - (double)(float)h); }
    __device__ void store2(int64_t off, double a, double b) const
    {
        const __bf16 ha = high(a), hb = high(b);
        *reinterpret_cast<bf16x2*>(hi + off) = bf16x2{ha, hb};
        *reinterpret_cast<bf16x2*>(lo + off) = bf16x2{low(a, ha), low(b, hb)};
    }
    __device__ void store(int64_t off, double a) const
    {
        const __bf16 h = high(a);
        hi[off] = h;
        lo[off] = low(a, h);
    }
};

template <bool kVec, typename Out>
__global__ __launch_bounds__(kWave) void decompress_kernel(const double* __restrict__ f, const double* __restrict__ s,
                                                           const uint8_t* __restrict__ phi,
                                                           const uint32_t* __restrict__ codes, int64_t nbc,
                                                           int64_t nblk, Out out, int64_t lda)
{
    __shared__ __align__(16) double tile[kWave * kSlot];
    const int lane = threadIdx.x;
    const int64_t wave_base = (int64_t)blockIdx.x * kWave;
    const int64_t b = wave_base + lane;
    const bool valid = b < nblk;

    // The wave's codes: consecutive dwords into LDS, then each lane's 7.
    uint32_t* ct = reinterpret_cast<uint32_t*>(tile);
    const int64_t nwords = (nblk - wave_base < kWave ? nblk - wave_base : kWave) * kCodeWords;
    const uint32_t* csrc = codes + wave_base * kCodeWords;
#pragma unroll
    for (int k = 0; k < kCodeWords; ++k) {
        const int idx = lane + kWave * k;
        if (idx < nwords) ct[idx] = csrc[idx];
    }
    __syncthreads();
    uint32_t w[kCodeWords];
#pragma unroll
    for (int q = 0; q < kCodeWords; ++q) w[q] = ct[lane * kCodeWords + q];
    __syncthreads();

    const double fb = valid ? f[b] : 0.0;
    const double sb = valid ? s[b] : 0.0;
    const double pb = valid ? (double)phi[b] : 1.0;
    // Dhat = C / phi at the kept positions (zero elsewhere); the slope factor
    // of Eq. eqbbb is folded in by linearity of the inverse DCT.
    double coef[kKept];
    unpack_codes(w, sb / pb, coef);
    double x[64];
    inverse_transform(coef, x);
    inverse_normalize(fb, x);

    if constexpr (kVec) {
        const WaveChunks wc = wave_chunks(wave_base, lane, nbc, nblk, lda);
#pragma unroll
        for (int r = 0; r < 8; ++r) {
#pragma unroll
            for (int p = 0; p < 4; ++p)
                *reinterpret_cast<f64x2*>(&tile[lane * kSlot + 2 * p]) = f64x2{x[r * 8 + 2 * p], x[r * 8 + 2 * p + 1]};
            __syncthreads();
#pragma unroll
            for (int k = 0; k < 4; ++k) {
                const f64x2 v = *reinterpret_cast<const f64x2*>(&tile[((lane >> 2) + 16 * k) * kSlot + 2 * (lane & 3)]);
                if (wc.ok[k]) out.store2(wc.off[k] + r * lda, v[0], v[1]);
            }
            __syncthreads();
        }
    } else if (valid) {
        const int64_t I = b / nbc, J = b - (b / nbc) * nbc;
        const int64_t base = (I * 8) * lda + J * 8;
#pragma unroll
        for (int r = 0; r < 8; ++r)
#pragma unroll
            for (int c = 0; c < 8; ++c) out.store(base + r * lda + c, x[r * 8 + c]);
    }
}

namespace detail {

static inline unsigned grid_for(int64_t nblk) { return (unsigned)((nblk + kWave - 1) / kWave); }

hipError_t launch_compress_f64(const double* A, int64_t lda, const blaz_matrix& m, uint8_t* psi, hipStream_t st)
{
    const int64_t nbc = m.cols / 8;
    const int64_t nblk = (m.rows / 8) * nbc;
    const bool vec = (reinterpret_cast<uintptr_t>(A) % 16 == 0) && (lda % 2 == 0);
    const unsigned grid = grid_for(nblk);
    auto* cw = reinterpret_cast<uint32_t*>(m.codes);
    if (vec && psi)
        compress_f64_kernel<true, true><<<grid, kWave, 0, st>>>(A, lda, nbc, nblk, m.f, m.s, m.phi, cw, psi);
    else if (vec)
        compress_f64_kernel<true, false><<<grid, kWave, 0, st>>>(A, lda, nbc, nblk, m.f, m.s, m.phi, cw, psi);
    else if (psi)
        compress_f64_kernel<false, true><<<grid, kWave, 0, st>>>(A, lda, nbc, nblk, m.f, m.s, m.phi, cw, psi);
    else
        compress_f64_kernel<false, false><<<grid, kWave, 0, st>>>(A, lda, nbc, nblk, m.f, m.s, m.phi, cw, psi);
    return hipGetLastError();
}

template <typename Out>
static hipError_t launch_decompress_to(const blaz_matrix& m, Out out, bool vec, int64_t lda, hipStream_t st)
{
    const int64_t nbc = m.cols / 8;
    const int64_t nblk = (m.rows / 8) * nbc;
    const unsigned grid = grid_for(nblk);
    const auto* cw = reinterpret_cast<const uint32_t*>(m.codes);
    if (vec)
        decompress_kernel<true><<<grid, kWave, 0, st>>>(m.f, m.s, m.phi, cw, nbc, nblk, out, lda);
    else
        decompress_kernel<false><<<grid, kWave, 0, st>>>(m.f, m.s, m.phi, cw, nbc, nblk, out, lda);
    return hipGetLastError();
}

hipError_t launch_decompress(const blaz_matrix& m, double* A, int64_t lda, hipStream_t st)
{
    const bool vec = (reinterpret_cast<uintptr_t>(A) % 16 == 0) && (lda % 2 == 0);
    return launch_decompress_to(m, OutF64{A}, vec, lda, st);
}

hipError_t launch_decompress_f32(const blaz_matrix& m, float* A, int64_t lda, hipStream_t st)
{
    const bool vec = (reinterpret_cast<uintptr_t>(A) % 8 == 0) && (lda % 2 == 0);
    return launch_decompress_to(m, OutF32{A}, vec, lda, st);
}

hipError_t launch_decompress_bf16_split(const blaz_matrix& m, __bf16* hi, __bf16* lo, int64_t lda, hipStream_t st)
{
    const bool vec = (reinterpret_cast<uintptr_t>(hi) % 4 == 0) && (reinterpret_cast<uintptr_t>(lo) % 4 == 0) &&
                     (lda % 2 == 0);
    return launch_decompress_to(m, OutBF16Split{hi, lo}, vec, lda, st);
}

}  // namespace detail
}  // namespace blaz
