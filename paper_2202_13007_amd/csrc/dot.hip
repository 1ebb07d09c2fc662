// Dot products on partly decompressed blocks: Algorithm 3 with Eqs. eqbbb0
// and eqbbb, applied blockwise along the line of X (and the column of Y).
//
// Mapping: one 256-thread workgroup per group of 8 consecutive queries; its
// four waves are the four parts of the group (each takes every fourth run
// of 64 blocks of the line), and the part sums are added in a fixed order
// through LDS.  Each lane rebuilds only lines 0..(i mod 8) of its X blocks
// -- the IPREDICT_LINES step -- and only columns 0..(j mod 8) of its Y
// blocks, or, for a group on the 8 lines of one block row, every block once
// for the whole group.
#include <hip/hip_runtime.h>

#include "blaz_device.hpp"
#include "blaz_dot.hpp"
#include "blaz_internal.hpp"

namespace blaz {

__device__ __forceinline__ void combine_parts(const double (&part)[kDotParts][kDotGroup], int64_t q0, int64_t nq,
                                              const int64_t* xrow, const int64_t* ycol, int64_t xlines,
                                              int64_t ylines, double* out)
{
    const int t = threadIdx.x;
    if (t < nq) {
        double r = part[0][t];
#pragma unroll
        for (int w = 1; w < kDotParts; ++w) r = r + part[w][t];
        out[q0 + t] = dot_valid(xrow, ycol, q0 + t, xlines, ylines) ? r : __builtin_nan("");
    }
}

__global__ __launch_bounds__(256) void dot_kernel(DotOperand X, int64_t nbr_x, DotOperand Y, int64_t nbc_y,
                                                  int64_t nk, const int64_t* __restrict__ xrow,
                                                  const int64_t* __restrict__ ycol, int64_t count,
                                                  double* __restrict__ out)
{
    __shared__ double part[kDotParts][kDotGroup];
    const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int64_t q0 = (int64_t)blockIdx.x * kDotGroup;
    const int64_t nq = count - q0 < kDotGroup ? count - q0 : kDotGroup;
    double S[kDotGroup];
    dot_part(w, lane, q0, nq, X, nbr_x, Y, nbc_y, nk, xrow, ycol, S);
    if (lane == 0)
#pragma unroll
        for (int t = 0; t < kDotGroup; ++t) part[w][t] = S[t];
    __syncthreads();
    combine_parts(part, q0, nq, xrow, ycol, nbr_x * 8, nbc_y * 8, out);
}

__global__ __launch_bounds__(256) void dot_dense_kernel(DotOperand X, int64_t nbr, int64_t nbc,
                                                        const int64_t* __restrict__ xrow,
                                                        const double* __restrict__ v, int64_t ldv, int64_t count,
                                                        double* __restrict__ out)
{
    __shared__ double part[kDotParts][kDotGroup];
    const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int64_t q0 = (int64_t)blockIdx.x * kDotGroup;
    const int64_t nq = count - q0 < kDotGroup ? count - q0 : kDotGroup;
    double S[kDotGroup];
    dot_dense_part(w, lane, q0, nq, X, nbr, nbc, xrow, v, ldv, S);
    if (lane == 0)
#pragma unroll
        for (int t = 0; t < kDotGroup; ++t) part[w][t] = S[t];
    __syncthreads();
    combine_parts(part, q0, nq, xrow, nullptr, nbr * 8, 0, out);
}

namespace detail {

static DotOperand operand(const blaz_matrix& m)
{
    return DotOperand{m.f, m.s, m.phi, reinterpret_cast<const uint32_t*>(m.codes)};
}

hipError_t launch_dot(const blaz_matrix& x, const int64_t* xrow, const blaz_matrix& y, const int64_t* ycol,
                      int64_t count, double* out, hipStream_t st)
{
    const unsigned grid = (unsigned)((count + kDotGroup - 1) / kDotGroup);
    dot_kernel<<<grid, 256, 0, st>>>(operand(x), x.rows / 8, operand(y), y.cols / 8, x.cols / 8, xrow, ycol, count,
                                     out);
    return hipGetLastError();
}

hipError_t launch_dot_dense(const blaz_matrix& x, const int64_t* xrow, const double* v, int64_t ldv, int64_t count,
                            double* out, hipStream_t st)
{
    const unsigned grid = (unsigned)((count + kDotGroup - 1) / kDotGroup);
    dot_dense_kernel<<<grid, 256, 0, st>>>(operand(x), x.rows / 8, x.cols / 8, xrow, v, ldv, count, out);
    return hipGetLastError();
}

}  // namespace detail
}  // namespace blaz
