// Dot products on partly decompressed blocks: Algorithm 3 with Eqs. eqbbb0
// and eqbbb, applied blockwise along the line of X (and the column of Y).
//
// Mapping: one wave per dot product; the lanes walk the blocks of the line's
// block row (and of the column's block column) 64 at a time, each lane
// rebuilding only the lines 0..(i mod 8) of its X block -- the
// IPREDICT_LINES step of Algorithm 3 -- and only the columns 0..(j mod 8) of
// its Y block.  Partial sums are reduced across the wave at the end.
#include <hip/hip_runtime.h>

#include "blaz_device.hpp"
#include "blaz_dot.hpp"
#include "blaz_internal.hpp"

namespace blaz {

__global__ __launch_bounds__(256) void dot_kernel(const double* __restrict__ xf, const double* __restrict__ xs,
                                                  const uint8_t* __restrict__ xphi,
                                                  const uint32_t* __restrict__ xc, int64_t nbr_x,
                                                  const double* __restrict__ yf, const double* __restrict__ ys,
                                                  const uint8_t* __restrict__ yphi,
                                                  const uint32_t* __restrict__ yc, int64_t nbc_y, int64_t nk,
                                                  const int64_t* __restrict__ xrow,
                                                  const int64_t* __restrict__ ycol, int64_t count,
                                                  double* __restrict__ out)
{
    const int64_t q = (int64_t)blockIdx.x * (blockDim.x / 64) + (threadIdx.x >> 6);
    if (q >= count) return;  // uniform across the wave
    dot_wave(q, threadIdx.x & 63, xf, xs, xphi, xc, nbr_x, yf, ys, yphi, yc, nbc_y, nk, xrow, ycol, out);
}

__global__ __launch_bounds__(256) void dot_dense_kernel(const double* __restrict__ xf,
                                                        const double* __restrict__ xs,
                                                        const uint8_t* __restrict__ xphi,
                                                        const uint32_t* __restrict__ xc, int64_t nbr,
                                                        int64_t nbc, const int64_t* __restrict__ xrow,
                                                        const double* __restrict__ v, int64_t ldv, int64_t count,
                                                        double* __restrict__ out)
{
    const int64_t q = (int64_t)blockIdx.x * (blockDim.x / 64) + (threadIdx.x >> 6);
    if (q >= count) return;
    dot_dense_wave(q, threadIdx.x & 63, xf, xs, xphi, xc, nbr, nbc, xrow, v, ldv, out);
}

namespace detail {

hipError_t launch_dot(const blaz_matrix& x, const int64_t* xrow, const blaz_matrix& y, const int64_t* ycol,
                      int64_t count, double* out, hipStream_t st)
{
    const unsigned grid = (unsigned)((count + 3) / 4);
    dot_kernel<<<grid, 256, 0, st>>>(x.f, x.s, x.phi, reinterpret_cast<const uint32_t*>(x.codes), x.rows / 8, y.f,
                                     y.s, y.phi, reinterpret_cast<const uint32_t*>(y.codes), y.cols / 8, x.cols / 8,
                                     xrow, ycol, count, out);
    return hipGetLastError();
}

hipError_t launch_dot_dense(const blaz_matrix& x, const int64_t* xrow, const double* v, int64_t ldv, int64_t count,
                            double* out, hipStream_t st)
{
    const unsigned grid = (unsigned)((count + 3) / 4);
    dot_dense_kernel<<<grid, 256, 0, st>>>(x.f, x.s, x.phi, reinterpret_cast<const uint32_t*>(x.codes), x.rows / 8,
                                           x.cols / 8, xrow, v, ldv, count, out);
    return hipGetLastError();
}

}  // namespace detail
}  // namespace blaz
