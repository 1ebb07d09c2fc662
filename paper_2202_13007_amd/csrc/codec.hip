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

// One matrix's share of a two-matrix decompression launch.
template <typename Out>
struct DecompressJob {
    const double* f;
    const double* s;
    const uint8_t* phi;
    const uint32_t* codes;
    int64_t nbc, nblk;
    Out out;
    int64_t lda;
};

// The rebuilds of both operands of a product in one launch: workgroups
// 0 .. waves_a-1 take the first matrix, the rest the second.  A small
// product's two rebuilds are each a single latency-bound wave; side by side
// they take the time of one.
template <bool kVec, typename Out, int L = 2>
__global__ __launch_bounds__(kWave) void decompress_pair_kernel(DecompressJob<Out> a, DecompressJob<Out> b,
                                                                unsigned waves_a)
{
    __shared__ __align__(16) double tile[kWave * kSlot];
    const bool first = blockIdx.x < waves_a;
    const DecompressJob<Out>& j = first ? a : b;
    const int64_t wave = first ? (int64_t)blockIdx.x : (int64_t)(blockIdx.x - waves_a);
    decompress_wave<kVec, Out, L>(j.f, j.s, j.phi, j.codes, j.nbc, j.nblk, j.out, j.lda, wave * kWave,
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

// Both operands in one launch when they share the kept lines and the store
// path; otherwise one launch each.
template <typename Out>
static hipError_t launch_decompress_pair_to(const blaz_matrix& ma, Out outa, bool veca, int64_t lda,
                                            const blaz_matrix& mb, Out outb, bool vecb, int64_t ldb, hipStream_t st)
{
    const auto lines = [](const blaz_matrix& m) { return m.lines >= 1 && m.lines <= 8 ? m.lines : 2; };
    if (lines(ma) != lines(mb) || veca != vecb) {
        if (hipError_t e = launch_decompress_to(ma, outa, veca, lda, st)) return e;
        return launch_decompress_to(mb, outb, vecb, ldb, st);
    }
    const auto job = [](const blaz_matrix& m, Out out, int64_t ld) {
        const int64_t nbc = m.cols / 8;
        return DecompressJob<Out>{m.f, m.s, m.phi, reinterpret_cast<const uint32_t*>(m.codes), nbc,
                                  (m.rows / 8) * nbc, out, ld};
    };
    const DecompressJob<Out> ja = job(ma, outa, lda), jb = job(mb, outb, ldb);
    const unsigned wa = grid_for(ja.nblk), grid = wa + grid_for(jb.nblk);
    if (grid == 0) return hipSuccess;
    return dispatch_lines(ma, [&](auto lc) {
        constexpr int L = decltype(lc)::value;
        if (veca)
            decompress_pair_kernel<true, Out, L><<<grid, kWave, 0, st>>>(ja, jb, wa);
        else
            decompress_pair_kernel<false, Out, L><<<grid, kWave, 0, st>>>(ja, jb, wa);
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

static bool vec_f64(const double* A, int64_t lda) { return (reinterpret_cast<uintptr_t>(A) % 16 == 0) && (lda % 2 == 0); }
static bool vec_f32(const float* A, int64_t lda) { return (reinterpret_cast<uintptr_t>(A) % 16 == 0) && (lda % 4 == 0); }
static bool vec_bf16(const __bf16* hi, const __bf16* lo, int64_t lda)
{
    return (reinterpret_cast<uintptr_t>(hi) % 16 == 0) && (reinterpret_cast<uintptr_t>(lo) % 16 == 0) && (lda % 8 == 0);
}

hipError_t launch_decompress_pair(const blaz_matrix& a, double* A, int64_t lda, const blaz_matrix& b, double* B,
                                  int64_t ldb, hipStream_t st)
{
    return launch_decompress_pair_to(a, OutF64{A}, vec_f64(A, lda), lda, b, OutF64{B}, vec_f64(B, ldb), ldb, st);
}

hipError_t launch_decompress_pair_f32(const blaz_matrix& a, float* A, int64_t lda, const blaz_matrix& b, float* B,
                                      int64_t ldb, hipStream_t st)
{
    return launch_decompress_pair_to(a, OutF32{A}, vec_f32(A, lda), lda, b, OutF32{B}, vec_f32(B, ldb), ldb, st);
}

hipError_t launch_decompress_pair_bf16_split(const blaz_matrix& a, __bf16* Ahi, __bf16* Alo, int64_t lda,
                                             const blaz_matrix& b, __bf16* Bhi, __bf16* Blo, int64_t ldb,
                                             hipStream_t st)
{
    return launch_decompress_pair_to(a, OutBF16Split{Ahi, Alo}, vec_bf16(Ahi, Alo, lda), lda, b,
                                     OutBF16Split{Bhi, Blo}, vec_bf16(Bhi, Blo, ldb), ldb, st);
}

}  // namespace detail
}  // namespace blaz
