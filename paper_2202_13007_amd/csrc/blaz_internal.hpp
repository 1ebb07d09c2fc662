// Launchers of the blaz kernels, called by the C ABI in api.hip after the
// arguments have been validated.  Each returns the HIP error of its launch.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "libblaz.h"

namespace blaz {
namespace detail {

hipError_t launch_compress_f64(const double* A, int64_t lda, const blaz_matrix& m, uint8_t* psi, hipStream_t st);
hipError_t launch_decompress(const blaz_matrix& m, double* A, int64_t lda, hipStream_t st);
hipError_t launch_add(const blaz_matrix& x, const blaz_matrix& y, const blaz_matrix& z, bool negate_y,
                      hipStream_t st);
hipError_t launch_scale(const blaz_matrix& x, double c, const blaz_matrix& z, hipStream_t st);
hipError_t launch_dot(const blaz_matrix& x, const int64_t* xrow, const blaz_matrix& y, const int64_t* ycol,
                      int64_t count, double* out, hipStream_t st);
hipError_t launch_dot_dense(const blaz_matrix& x, const int64_t* xrow, const double* v, int64_t ldv,
                            int64_t count, double* out, hipStream_t st);
// C (m x n, ldc) = A (m x k, lda) * B (k x n, ldb), all row-major binary64.
hipError_t launch_gemm_f64(const double* A, int64_t lda, const double* B, int64_t ldb, double* C, int64_t ldc,
                           int64_t m, int64_t n, int64_t k, hipStream_t st);

}  // namespace detail
}  // namespace blaz
