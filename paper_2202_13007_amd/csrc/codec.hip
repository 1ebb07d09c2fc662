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

template <bool kVec, bool kPsi, int L = 2, bool kPred = false>
__global__ __launch_bounds__(kWave) void compress_f64_kernel(const double* __restrict__ A, int64_t lda,
                                                             int64_t nbc, int64_t nblk, double* __restrict__ fo,
                                                             double* __restrict__ so, uint8_t* __restrict__ phio,
                                                             uint32_t* __restrict__ codes,
                                                             uint8_t* __restrict__ psi)
{
    __shared__ __align__(16) double tile[kWave * kSlot];
    compress_wave<kVec, kPsi, L, kPred>(A, lda, nbc, nblk, fo, so, phio, codes, psi, (int64_t)blockIdx.x * kWave,
                                        (int)threadIdx.x, tile);
}

template <bool kVec, typename Out, int L = 2>
__global__ __launch_bounds__(kWave) void decompress_kernel(const double* __restrict__ f, const double* __restrict__ s,
                                                           const uint8_t* __restrict__ phi,
                                                           const uint32_t* __restrict__ codes, int64_t nbc,
                                                           int64_t nblk, Out out, int64_t lda)
{
    __shared__ __align__(16) double tile[kWave * kSlot];
    decompress_wave<kVec, Out, L>(f, s, phi, codes, nbc, nblk, out, lda, (int64_t)blockIdx.x * kWave,
                                  (int)threadIdx.x, tile);
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
    if (m.lines != 0 && m.lines != 2)  // other rates: no prediction side output (rejected before)
        return dispatch_lines(m, [&](auto lc) {
            constexpr int L = decltype(lc)::value;
            if (vec)
                compress_f64_kernel<true, false, L><<<grid, kWave, 0, st>>>(A, lda, nbc, nblk, m.f, m.s, m.phi, cw,
                                                                           nullptr);
            else
                compress_f64_kernel<false, false, L><<<grid, kWave, 0, st>>>(A, lda, nbc, nblk, m.f, m.s, m.phi,
                                                                            cw, nullptr);
            return hipGetLastError();
        });
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

hipError_t launch_compress_predicted(const double* A, int64_t lda, const blaz_matrix& m, uint8_t* psi,
                                     hipStream_t st)
{
    const int64_t nbc = m.cols / 8;
    const int64_t nblk = (m.rows / 8) * nbc;
    const bool vec = (reinterpret_cast<uintptr_t>(A) % 16 == 0) && (lda % 2 == 0);
    const unsigned grid = grid_for(nblk);
    auto* cw = reinterpret_cast<uint32_t*>(m.codes);
    if (vec && psi)
        compress_f64_kernel<true, true, 2, true><<<grid, kWave, 0, st>>>(A, lda, nbc, nblk, m.f, m.s, m.phi, cw, psi);
    else if (vec)
        compress_f64_kernel<true, false, 2, true><<<grid, kWave, 0, st>>>(A, lda, nbc, nblk, m.f, m.s, m.phi, cw,
                                                                         psi);
    else if (psi)
        compress_f64_kernel<false, true, 2, true><<<grid, kWave, 0, st>>>(A, lda, nbc, nblk, m.f, m.s, m.phi, cw,
                                                                         psi);
    else
        compress_f64_kernel<false, false, 2, true><<<grid, kWave, 0, st>>>(A, lda, nbc, nblk, m.f, m.s, m.phi, cw,
                                                                          psi);
    return hipGetLastError();
}

template <typename Out>
static hipError_t launch_decompress_to(const blaz_matrix& m, Out out, bool vec, int64_t lda, hipStream_t st)
{
    const int64_t nbc = m.cols / 8;
    const int64_t nblk = (m.rows / 8) * nbc;
    const unsigned grid = grid_for(nblk);
    const auto* cw = reinterpret_cast<const uint32_t*>(m.codes);
    return dispatch_lines(m, [&](auto lc) {
        constexpr int L = decltype(lc)::value;
        if (vec)
            decompress_kernel<true, Out, L><<<grid, kWave, 0, st>>>(m.f, m.s, m.phi, cw, nbc, nblk, out, lda);
        else
            decompress_kernel<false, Out, L><<<grid, kWave, 0, st>>>(m.f, m.s, m.phi, cw, nbc, nblk, out, lda);
        return hipGetLastError();
    });
}

hipError_t launch_decompress(const blaz_matrix& m, double* A, int64_t lda, hipStream_t st)
{
    const bool vec = (reinterpret_cast<uintptr_t>(A) % 16 == 0) && (lda % 2 == 0);
    return launch_decompress_to(m, OutF64{A}, vec, lda, st);
}

hipError_t launch_decompress_f32(const blaz_matrix& m, float* A, int64_t lda, hipStream_t st)
{
    // each block row is two 16-byte stores: 16-byte aligned rows
    const bool vec = (reinterpret_cast<uintptr_t>(A) % 16 == 0) && (lda % 4 == 0);
    return launch_decompress_to(m, OutF32{A}, vec, lda, st);
}

hipError_t launch_decompress_bf16_split(const blaz_matrix& m, __bf16* hi, __bf16* lo, int64_t lda, hipStream_t st)
{
    // each block row is one 16-byte store per array: 16-byte aligned rows
    const bool vec = (reinterpret_cast<uintptr_t>(hi) % 16 == 0) && (reinterpret_cast<uintptr_t>(lo) % 16 == 0) &&
                     (lda % 8 == 0);
    return launch_decompress_to(m, OutBF16Split{hi, lo}, vec, lda, st);
}

}  // namespace detail
}  // namespace blaz
