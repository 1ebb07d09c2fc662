// Operations on compressed blocks: addition (Algorithm 1), subtraction (the
// addition applied to x and -y) and multiplication by a constant
// (Algorithm 2).
//
// Mapping: one lane per block.  The per-block work is a handful of binary64
// divisions and 28 multiply-adds, so a lane can own a whole record; a wave
// then reads 64 consecutive records, i.e. contiguous runs of f, s, phi and
// codes, and the kernels stay bound by HBM rather than by instruction issue.
#include <hip/hip_runtime.h>

#include "blaz_device.hpp"
#include "blaz_internal.hpp"
#include "blaz_ops.hpp"

namespace blaz {

template <bool kNegY, int L>
__global__ __launch_bounds__(256) void add_kernel(const double* f1, const double* s1, const uint8_t* phi1,
                                                  const uint32_t* c1, const double* f2, const double* s2,
                                                  const uint8_t* phi2, const uint32_t* c2, int64_t nblk, double* fo,
                                                  double* so, uint8_t* phio, uint32_t* co)
{
    const int64_t b = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (b >= nblk) return;
    add_block<L>(b, kNegY, f1, s1, phi1, c1, f2, s2, phi2, c2, fo, so, phio, co);
}

// Algorithm 2 in place: only f and s change.
__global__ __launch_bounds__(256) void scale_inplace_kernel(double* f, double* s, double c, int64_t nblk)
{
    const int64_t b = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (b >= nblk) return;
    f[b] = f[b] * c;
    s[b] = s[b] * c;
}

// Algorithm 2 out of place: f and s times c, phi and the codes copied
// (kW dwords of codes per block).
template <int kW>
__global__ __launch_bounds__(256) void scale_kernel(const double* __restrict__ f1, const double* __restrict__ s1,
                                                    const uint8_t* phi1,
                                                    const uint32_t* __restrict__ c1, double c, int64_t nblk,
                                                    double* __restrict__ fo, double* __restrict__ so,
                                                    uint8_t* __restrict__ phio, uint32_t* __restrict__ co)
{
    const int64_t b = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (b < nblk) {
        fo[b] = f1[b] * c;
        so[b] = s1[b] * c;
        phio[b] = phi1[b];
    }
    // The codes are copied as one flat dword stream (kW dwords per block) so
    // that consecutive lanes touch consecutive dwords.
    const int64_t total = nblk * kW;
    const int64_t base = (int64_t)blockIdx.x * blockDim.x * kW + threadIdx.x;
#pragma unroll
    for (int q = 0; q < kW; ++q) {
        const int64_t i = base + (int64_t)q * blockDim.x;
        if (i < total) co[i] = c1[i];
    }
}

// Data conditions of a compressed matrix (see blaz_diagnose): one lane per
// block, the wave's counts summed across lanes and added by lane 0.
template <int L>
__global__ __launch_bounds__(256) void diagnose_kernel(const double* __restrict__ f, const double* __restrict__ s,
                                                       const uint8_t* __restrict__ phi,
                                                       const uint32_t* __restrict__ codes, int64_t nblk,
                                                       unsigned long long* __restrict__ counters)
{
    constexpr int kW = KeptLines<L>::kWords, kN = KeptLines<L>::kCount;
    const int64_t b = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    int c[4] = {0, 0, 0, 0};
    if (b < nblk) {
        const double fb = f[b], sb = s[b];
        c[0] = sb == 0.0;
        c[1] = sb != 0.0 && phi[b] == 255;
        c[3] = !(__builtin_isfinite(fb) && __builtin_isfinite(sb));
#pragma unroll
        for (int t = 0; t < kN; ++t) {
            const int32_t v = (int32_t)(codes[b * kW + t / 4] << (24 - 8 * (t % 4))) >> 24;
            c[2] += v >= 127 || v <= -127;
        }
    }
#pragma unroll
    for (int k = 0; k < 4; ++k) {
#pragma unroll
        for (int off = 32; off >= 1; off /= 2) c[k] += __shfl_xor(c[k], off, 64);
    }
    if ((threadIdx.x & 63) == 0) {
#pragma unroll
        for (int k = 0; k < 4; ++k)
            if (c[k]) atomicAdd(counters + k, (unsigned long long)c[k]);
    }
}

namespace detail {

hipError_t launch_diagnose(const blaz_matrix& x, uint64_t* counters, hipStream_t st)
{
    const int64_t nblk = (x.rows / 8) * (x.cols / 8);
    const unsigned grid = (unsigned)((nblk + 255) / 256);
    return dispatch_lines(x, [&](auto lc) {
        diagnose_kernel<decltype(lc)::value><<<grid, 256, 0, st>>>(
            x.f, x.s, x.phi, reinterpret_cast<const uint32_t*>(x.codes), nblk,
            reinterpret_cast<unsigned long long*>(counters));
        return hipGetLastError();
    });
}


hipError_t launch_add(const blaz_matrix& x, const blaz_matrix& y, const blaz_matrix& z, bool negate_y,
                      hipStream_t st)
{
    const int64_t nblk = (x.rows / 8) * (x.cols / 8);
    const unsigned grid = (unsigned)((nblk + 255) / 256);
    auto cw = [](const blaz_matrix& m) { return reinterpret_cast<uint32_t*>(m.codes); };
    return dispatch_lines(x, [&](auto lc) {
        constexpr int L = decltype(lc)::value;
        if (negate_y)
            add_kernel<true, L><<<grid, 256, 0, st>>>(x.f, x.s, x.phi, cw(x), y.f, y.s, y.phi, cw(y), nblk, z.f,
                                                      z.s, z.phi, cw(z));
        else
            add_kernel<false, L><<<grid, 256, 0, st>>>(x.f, x.s, x.phi, cw(x), y.f, y.s, y.phi, cw(y), nblk, z.f,
                                                       z.s, z.phi, cw(z));
        return hipGetLastError();
    });
}

hipError_t launch_scale(const blaz_matrix& x, double c, const blaz_matrix& z, hipStream_t st)
{
    const int64_t nblk = (x.rows / 8) * (x.cols / 8);
    const unsigned grid = (unsigned)((nblk + 255) / 256);
    if (z.f == x.f && z.s == x.s && z.phi == x.phi && z.codes == x.codes)
        scale_inplace_kernel<<<grid, 256, 0, st>>>(z.f, z.s, c, nblk);
    else
        return dispatch_lines(x, [&](auto lc) {
            scale_kernel<KeptLines<decltype(lc)::value>::kWords><<<grid, 256, 0, st>>>(
                x.f, x.s, x.phi, reinterpret_cast<const uint32_t*>(x.codes), c, nblk, z.f, z.s, z.phi,
                reinterpret_cast<uint32_t*>(z.codes));
            return hipGetLastError();
        });
    return hipGetLastError();
}

}  // namespace detail
}  // namespace blaz
