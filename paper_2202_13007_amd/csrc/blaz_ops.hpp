// Per-block bodies of the operations on compressed records: addition
// (Algorithm 1), subtraction (Algorithm 1 on x and -y) and multiplication by
// a constant (Algorithm 2).  Shared by the standalone kernels and the
// persistent batch kernel.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "blaz_device.hpp"

namespace blaz {

// z = x + y (or x - y) for block b.  z may alias x or y: every input of the
// block is read before it is written.  L: kept lines of the records (the
// paper's 2 by default); pad bytes of the result are zero.
template <int L = 2>
__device__ __forceinline__ void add_block(int64_t b, bool neg_y, const double* f1, const double* s1,
                                          const uint8_t* phi1, const uint32_t* c1, const double* f2,
                                          const double* s2, const uint8_t* phi2, const uint32_t* c2, double* fo,
                                          double* so, uint8_t* phio, uint32_t* co)
{
    // Algorithm 1 first sums f and s: f = f1 + f2, s = s1 + s2 (y negated for subtraction,
    // which is exact).
    const double fy = neg_y ? -f2[b] : f2[b];
    const double sy = neg_y ? -s2[b] : s2[b];
    const double sx = s1[b];
    const double f = f1[b] + fy;
    const double s = sx + sy;
    // Then phi (Eq. eq55): phi = phi1 phi2 / (phi1 + phi2), integer division,
    // kept >= 1 so that the block can be decompressed.
    const int p1 = phi1[b], p2 = phi2[b];
    int p = p1 + p2 > 0 ? (p1 * p2) / (p1 + p2) : 1;
    p = p < 1 ? 1 : p;

    constexpr int kW = KeptLines<L>::kWords, kN = KeptLines<L>::kCount;
    uint32_t wx[kW], wy[kW], wo[kW];
#pragma unroll
    for (int q = 0; q < kW; ++q) {
        wx[q] = c1[b * kW + q];
        wy[q] = c2[b * kW + q];
        wo[q] = 0;
    }
    if (s != 0.0) {
        // Weights: alpha_k = s_k / s, beta_k = (alpha_k / phi_k) * phi.
        const double a1 = sx / s;
        const double a2 = sy / s;
        const double b1 = a1 / (double)p1 * (double)p;
        const double b2 = a2 / (double)p2 * (double)p;
        // Codes: C = trunc(beta1 C1 + beta2 C2), saturated to +-127.
        // Two products then one sum, never fused (the library is built with
        // -ffp-contract=off), so the result is reproducible bit for bit.
#pragma unroll
        for (int t = 0; t < kN; ++t) {
            const int32_t cx = (int32_t)(wx[t / 4] << (24 - 8 * (t % 4))) >> 24;
            const int32_t cy = (int32_t)(wy[t / 4] << (24 - 8 * (t % 4))) >> 24;
            const double v = b1 * (double)cx + b2 * (double)cy;
            const double tv = fmin(fmax(trunc(v), -127.0), 127.0);
            wo[t / 4] |= ((uint32_t)(int32_t)tv & 0xffu) << (8 * (t % 4));
        }
    }
    fo[b] = f;
    so[b] = s;
    phio[b] = (uint8_t)p;
#pragma unroll
    for (int q = 0; q < kW; ++q) co[b * kW + q] = wo[q];
}

// z = c x for block b (Algorithm 2): f and s scaled, phi and codes copied
// unless z is x.
__device__ __forceinline__ void scale_block(int64_t b, double c, const double* f1, const double* s1,
                                            const uint8_t* phi1, const uint32_t* c1, double* fo, double* so,
                                            uint8_t* phio, uint32_t* co)
{
    const double f = f1[b] * c;
    const double s = s1[b] * c;
    if (co != c1) {
        phio[b] = phi1[b];
#pragma unroll
        for (int q = 0; q < kCodeWords; ++q) co[b * kCodeWords + q] = c1[b * kCodeWords + q];
    }
    fo[b] = f;
    so[b] = s;
}

}  // namespace blaz
