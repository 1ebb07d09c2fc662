// Launchers of the blaz kernels, called by the C ABI in api.hip after the
// arguments have been validated.  Each returns the HIP error of its launch.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <type_traits>

#include "libblaz.h"

namespace blaz {

// One product of a grouped binary64 contraction (device image): C (M x N,
// ldc) = A (M x K, lda) B (K x N, ldb), row-major binary64, owning the
// workgroups tile0 .. tile0 + tiles - 1 of the launch (tile0 a multiple of 8).
struct GemmGroupItem {
    const double* A;
    int64_t lda;
    const double* B;
    int64_t ldb;
    double* C;
    int64_t ldc;
    int64_t M, N, K;
    int64_t tile0;
};

// One matrix of a grouped rebuild (device image): its blocks decompressed
// into out (leading dimension ld), by the waves wave0 .. wave0 + ceil(nblk /
// 64) - 1 of the launch.
struct RebuildJob {
    const double* f;
    const double* s;
    const uint8_t* phi;
    const uint32_t* codes;
    int64_t nbc, nblk;
    double* out;
    int64_t ld;
    int64_t wave0;
};

namespace detail {

// Calls f(std::integral_constant<int, L>) for the kept lines L of a
// descriptor (0 stands for the paper's 2), so that every rate gets its own
// kernel instance.
template <typename F>
inline hipError_t dispatch_lines(const blaz_matrix& m, F&& f)
{
    switch (m.lines) {
        case 1: return f(std::integral_constant<int, 1>{});
        case 3: return f(std::integral_constant<int, 3>{});
        case 4: return f(std::integral_constant<int, 4>{});
        case 5: return f(std::integral_constant<int, 5>{});
        case 6: return f(std::integral_constant<int, 6>{});
        case 7: return f(std::integral_constant<int, 7>{});
        case 8: return f(std::integral_constant<int, 8>{});
        default: return f(std::integral_constant<int, 2>{});
    }
}

// Compute units of the current device (cached per device; 0 on error).
int device_cu_count();
// blaz_matmul's output tile for an m x n product (128 once that gives every
// compute unit a workgroup, else 64).
int default_gemm_tile(int64_t m, int64_t n);

hipError_t launch_compress_f64(const double* A, int64_t lda, const blaz_matrix& m, uint8_t* psi, hipStream_t st);
// Compression whose transform takes the predicted slopes (two kept lines).
hipError_t launch_compress_predicted(const double* A, int64_t lda, const blaz_matrix& m, uint8_t* psi,
                                     hipStream_t st);
// Compression with the transform stage in FP32 or BF16x3 on MFMA.
hipError_t launch_compress_mixed(const double* A, int64_t lda, const blaz_matrix& m, uint8_t* psi,
                                 blaz_precision prec, hipStream_t st);
hipError_t launch_decompress(const blaz_matrix& m, double* A, int64_t lda, hipStream_t st);
// Decompression into the operand forms of the low-precision contractions.
hipError_t launch_decompress_f32(const blaz_matrix& m, float* A, int64_t lda, hipStream_t st);
hipError_t launch_decompress_bf16_split(const blaz_matrix& m, __bf16* hi, __bf16* lo, int64_t lda, hipStream_t st);
// Both operands of a product (a, then b) rebuilt in one launch, in the same
// output form: one launch when they have the same kept lines, else two.
hipError_t launch_decompress_pair(const blaz_matrix& a, double* A, int64_t lda, const blaz_matrix& b, double* B,
                                  int64_t ldb, hipStream_t st);
hipError_t launch_decompress_pair_f32(const blaz_matrix& a, float* A, int64_t lda, const blaz_matrix& b, float* B,
                                      int64_t ldb, hipStream_t st);
hipError_t launch_decompress_pair_bf16_split(const blaz_matrix& a, __bf16* Ahi, __bf16* Alo, int64_t lda,
                                             const blaz_matrix& b, __bf16* Bhi, __bf16* Blo, int64_t ldb,
                                             hipStream_t st);
hipError_t launch_add(const blaz_matrix& x, const blaz_matrix& y, const blaz_matrix& z, bool negate_y,
                      hipStream_t st);
hipError_t launch_scale(const blaz_matrix& x, double c, const blaz_matrix& z, hipStream_t st);
// Data-condition counts of a compressed matrix, added to counters[0..3].
hipError_t launch_diagnose(const blaz_matrix& x, uint64_t* counters, hipStream_t st);
hipError_t launch_dot(const blaz_matrix& x, const int64_t* xrow, const blaz_matrix& y, const int64_t* ycol,
                      int64_t count, double* out, hipStream_t st);
hipError_t launch_dot_dense(const blaz_matrix& x, const int64_t* xrow, const double* v, int64_t ldv,
                            int64_t count, double* out, hipStream_t st);
// C (m x n, ldc) = A (m x k, lda) * B (k x n, ldb), all row-major binary64.
// tile: 64 or 128 (the output tile of one workgroup).
hipError_t launch_gemm_f64(const double* A, int64_t lda, const double* B, int64_t ldb, double* C, int64_t ldc,
                           int64_t m, int64_t n, int64_t k, int tile, hipStream_t st);
// Grouped binary64 products: workgroups = the last item's tile0 plus its
// tiles; tile 64 or 128 for every item of the launch.
hipError_t launch_gemm_group(const GemmGroupItem* items, int n_items, int64_t workgroups, int tile, hipStream_t st);
// Grouped rebuild of the operands of grouped products (two kept lines,
// 16-byte aligned rows with an even ld): waves = the last job's wave0 plus
// its waves.
hipError_t launch_rebuild_group(const RebuildJob* jobs, int n_jobs, int64_t waves, hipStream_t st);
// The same product with FP32 operands on FP32 MFMA (FP32 accumulation):
// A (m x k, lda) k-contiguous, B^T (n x k) in the blocked form of
// launch_convert_f32_blocked.  k a multiple of 4, lda too.
hipError_t launch_gemm_f32(const float* A, int64_t lda, const float* Bt, double* C, int64_t ldc, int64_t m, int64_t n,
                           int64_t k, int tile, hipStream_t st);
// The same product with A = Ahi + Alo (m x k) and B^T = Bthi + Btlo (n x k)
// in BF16: C = Ahi B_hi + Ahi B_lo + Alo B_hi on BF16 MFMA, FP32 accumulation.
// B^T is in the blocked form of launch_convert_bf16_split_blocked.
hipError_t launch_gemm_bf16x3(const __bf16* Ahi, const __bf16* Alo, int64_t lda, const __bf16* Bthi,
                              const __bf16* Btlo, double* C, int64_t ldc, int64_t m, int64_t n, int64_t k, int tile,
                              hipStream_t st);
// 32-k chunks of the blocked B^T forms, and their elements per array: tiles
// of 64 rows (n) x 32 k (4 KB in BF16, 8 KB in FP32), the padding zero.
inline int64_t bf16_k_chunks(int64_t k) { return (k + 31) / 32; }
inline int64_t bf16_blocked_elems(int64_t k, int64_t n) { return ((n + 63) / 64) * 64 * bf16_k_chunks(k) * 32; }
inline int64_t f32_k_chunks(int64_t k) { return (k + 31) / 32; }
inline int64_t f32_blocked_elems(int64_t k, int64_t n) { return ((n + 63) / 64) * 64 * f32_k_chunks(k) * 32; }
// Dense binary64 B (k x n, ldb) to B^T in FP32 in blocked form: tile
// (n / 64, k / 32) of 64 rows x 32 k (k contiguous) at
// ((n / 64) * f32_k_chunks(k) + k / 32) * 2048 elements.
hipError_t launch_convert_f32_blocked(const double* B, int64_t ldb, float* out, int64_t k, int64_t n, hipStream_t st);
// Dense binary64 B (k x n, ldb) to B^T split into BF16 hi + lo in blocked
// form: tile (n / 64, k / 32) of 64 rows x 32 k (k contiguous) at
// ((n / 64) * bf16_k_chunks(k) + k / 32) * 2048 elements.
hipError_t launch_convert_bf16_split_blocked(const double* B, int64_t ldb, __bf16* hi, __bf16* lo, int64_t k,
                                             int64_t n, hipStream_t st);
// The same blocked forms from row-major k x n operands already in FP32, or
// split into BF16 hi + lo (ld a multiple of 8, 16-byte aligned rows).
hipError_t launch_transpose_f32_blocked(const float* in, int64_t ld, float* out, int64_t k, int64_t n, hipStream_t st);
hipError_t launch_transpose_bf16_pair_blocked(const __bf16* hi_in, const __bf16* lo_in, int64_t ld, __bf16* hi,
                                              __bf16* lo, int64_t k, int64_t n, hipStream_t st);

}  // namespace detail
}  // namespace blaz
