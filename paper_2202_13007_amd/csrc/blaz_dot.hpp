// Bodies of the dot products on partly decompressed blocks (Algorithm 3 with
// Eqs. eqbbb0 and eqbbb, applied blockwise), shared by the standalone kernels
// and the persistent batch kernel.
//
// Work unit: a group of 8 consecutive queries q0..q0+7.  The blocks of a
// line (the n/8 blocks of its block row; for a column of Y, of its block
// column) are dealt to 256 slots, slot = kb mod 256; slot 64w + l belongs to
// lane l of "part" w (0..3) and accumulates its blocks in increasing kb.  A
// part's 64 slot sums are added by an xor butterfly, and the result of a
// query is ((S0 + S1) + S2) + S3.  The standalone kernel runs the four parts
// on the four waves of a workgroup; the batch kernel runs them one after the
// other on its single wave; both therefore produce the same bits.
//
// Lines are rebuilt by LineStream, line 0 first (the IPREDICT_LINES step):
// after the column pass of the inverse DCT, line u needs only its own 8
// coefficients and line u-1.  A query on line r stops after line r.  When a
// group is "aligned" -- its queries are the 8 lines of one block row in
// order (and, for two compressed operands, the 8 columns of one block column
// of Y) -- each block is rebuilt once for all 8 queries instead of once per
// query (36 line rebuilds become 8).  The arithmetic of line u is written out
// operation by operation (explicit fma, nothing left to contraction), so a
// query gets the same bits on either path.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "blaz_device.hpp"

namespace blaz {

constexpr int kDotParts = 4;                 // parts per query group (waves of the standalone kernel)
constexpr int kDotSlots = kDotParts * 64;    // slots a line's blocks are dealt to
constexpr int kDotGroup = 8;                 // queries per group

// Inverse 8-point DCT with every operation explicit: x_n = sum_k T(k, n) y_k
// through the even/odd split of the basis.
__device__ __forceinline__ void idct8_explicit(const double y[8], double x[8])
{
    double p[2], q[2];
#pragma unroll
    for (int n = 0; n < 2; ++n) {
        p[n] = __builtin_fma(dct_t(0, n), y[0], dct_t(4, n) * y[4]);
        q[n] = __builtin_fma(dct_t(2, n), y[2], dct_t(6, n) * y[6]);
    }
    const double e[4] = {p[0] + q[0], p[1] + q[1], p[1] - q[1], p[0] - q[0]};
#pragma unroll
    for (int n = 0; n < 4; ++n) {
        double o = dct_t(1, n) * y[1];
        o = __builtin_fma(dct_t(3, n), y[3], o);
        o = __builtin_fma(dct_t(5, n), y[5], o);
        o = __builtin_fma(dct_t(7, n), y[7], o);
        x[n] = e[n] + o;
        x[7 - n] = e[n] - o;
    }
}

struct LineStream {
    double c0[8], c1[8];  // columns 0 and 1 after the column inverse DCT, by line
    double a[6], b[6];    // lines 0 and 1 of columns 2..7, their only non-zero coefficients
    double prev[8];       // the last line produced
    double f;

    // coef: the 28 kept coefficients already scaled by s / phi.
    __device__ __forceinline__ void init(const double coef[kKept], double fb)
    {
        double col[8];
#pragma unroll
        for (int i = 0; i < 8; ++i) col[i] = coef[kept_index(i, 0)];
        idct8_explicit(col, c0);
#pragma unroll
        for (int i = 0; i < 8; ++i) col[i] = coef[kept_index(i, 1)];
        idct8_explicit(col, c1);
#pragma unroll
        for (int j = 2; j < 8; ++j) {
            a[j - 2] = coef[kept_index(0, j)];
            b[j - 2] = coef[kept_index(1, j)];
        }
        f = fb;
    }

    // Line u of the block (call with u = 0, 1, 2, ... in order; u must fold
    // to a constant, i.e. the caller's loop is unrolled).
    __device__ __forceinline__ void line(int u, double x[8])
    {
        double y[8], d[8];
        y[0] = c0[u];
        y[1] = c1[u];
#pragma unroll
        for (int j = 2; j < 8; ++j) y[j] = __builtin_fma(dct_t(0, u), a[j - 2], dct_t(1, u) * b[j - 2]);
        idct8_explicit(y, d);
        if (u == 0) {
            x[0] = f;
#pragma unroll
            for (int v = 1; v < 8; ++v) x[v] = x[v - 1] + d[v];
        } else {
            x[0] = prev[0] + d[0];
#pragma unroll
            for (int v = 1; v < 8; ++v) x[v] = __builtin_fma(prev[v] + x[v - 1], 0.5, d[v]);
        }
#pragma unroll
        for (int v = 0; v < 8; ++v) prev[v] = x[v];
    }
};

// The 28 scaled coefficients and f of block b; kTranspose reads them
// transposed, which makes the stream produce the block's columns (the
// normalization, the transform, the kept set and their inverses are all
// symmetric under transposition).
template <bool kTranspose>
__device__ __forceinline__ void load_block(const double* f, const double* s, const uint8_t* phi,
                                           const uint32_t* codes, int64_t b, double coef[kKept], double& fb)
{
    uint32_t w[kCodeWords];
#pragma unroll
    for (int q = 0; q < kCodeWords; ++q) w[q] = codes[b * kCodeWords + q];
    double c[kKept];
    unpack_codes(w, s[b] / (double)phi[b], c);
#pragma unroll
    for (int t = 0; t < kKept; ++t) coef[t] = kTranspose ? c[kept_index(kept_col(t), kept_row(t))] : c[t];
    fb = f[b];
}

// Lines 0..R of the stream, straight-line code; x = line R.
template <int R>
__device__ __forceinline__ void stream_to(LineStream& st, double x[8])
{
#pragma unroll
    for (int u = 0; u <= R; ++u) st.line(u, x);
}

// Line r (wave-uniform, 0..7) of a block: the stream stopped after line r.
template <bool kTranspose>
__device__ __forceinline__ void block_line(const double* f, const double* s, const uint8_t* phi,
                                           const uint32_t* codes, int64_t b, int r, double x[8])
{
    double coef[kKept], fb;
    load_block<kTranspose>(f, s, phi, codes, b, coef, fb);
    LineStream st;
    st.init(coef, fb);
    switch (r) {
        case 0: stream_to<0>(st, x); break;
        case 1: stream_to<1>(st, x); break;
        case 2: stream_to<2>(st, x); break;
        case 3: stream_to<3>(st, x); break;
        case 4: stream_to<4>(st, x); break;
        case 5: stream_to<5>(st, x); break;
        case 6: stream_to<6>(st, x); break;
        default: stream_to<7>(st, x); break;
    }
}

// acc + x[0]*v[0] + ... + x[7]*v[7], left to right, products rounded; v in
// global memory, 16-byte aligned.
__device__ __forceinline__ double dot8_global(double acc, const double x[8], const double* __restrict__ v)
{
    const double2* vp = reinterpret_cast<const double2*>(v);
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        const double2 vv = vp[k];
        acc = acc + x[2 * k] * vv.x;
        acc = acc + x[2 * k + 1] * vv.y;
    }
    return acc;
}

__device__ __forceinline__ double dot8(double acc, const double x[8], const double y[8])
{
#pragma unroll
    for (int k = 0; k < 8; ++k) acc = acc + x[k] * y[k];
    return acc;
}

__device__ __forceinline__ double wave_sum(double v)
{
#pragma unroll
    for (int off = 32; off >= 1; off /= 2) v += __shfl_xor(v, off, 64);
    return v;
}

// The group's 8 indices idx[q0 .. q0+nq-1], lane t holding entry t (-1 past nq).
__device__ __forceinline__ int64_t group_indices(const int64_t* idx, int64_t q0, int64_t nq, int lane)
{
    return lane < nq ? idx[q0 + lane] : -1;
}

// Entry t of the group's indices, as a wave-uniform value.
__device__ __forceinline__ int64_t index_of(int64_t v, int t)
{
    const uint32_t lo = __builtin_amdgcn_readlane((uint32_t)v, t);
    const uint32_t hi = __builtin_amdgcn_readlane((uint32_t)((uint64_t)v >> 32), t);
    return (int64_t)(((uint64_t)hi << 32) | lo);
}

// First index of an aligned run of 8 (the lines 8I..8I+7 in order) among the
// group's indices v (see group_indices), or -1.  lines = extent of the axis.
__device__ __forceinline__ int64_t aligned_run(int64_t v, int64_t nq, int64_t lines)
{
    if (nq != kDotGroup) return -1;
    const int64_t i0 = index_of(v, 0);
    if (i0 < 0 || i0 >= lines || (i0 & 7) != 0) return -1;
#pragma unroll
    for (int t = 1; t < kDotGroup; ++t)
        if (index_of(v, t) != i0 + t) return -1;
    return i0;
}

struct DotOperand {
    const double* f;
    const double* s;
    const uint8_t* phi;
    const uint32_t* c;
};

// Part w of the group at q0: S[t] = butterfly sum of this part's slot sums
// for query q0 + t (t < nq; the others are left 0).
//   X: lines of (nbr_x*8) x (nk*8); Y: columns of (nk*8) x (nbc_y*8).
__device__ __forceinline__ void dot_part(int w, int lane, int64_t q0, int64_t nq, const DotOperand& X, int64_t nbr_x,
                                         const DotOperand& Y, int64_t nbc_y, int64_t nk,
                                         const int64_t* __restrict__ xrow, const int64_t* __restrict__ ycol,
                                         double S[kDotGroup])
{
#pragma unroll
    for (int t = 0; t < kDotGroup; ++t) S[t] = 0.0;
    const int64_t xi = group_indices(xrow, q0, nq, lane), yj = group_indices(ycol, q0, nq, lane);
    const int64_t i0 = aligned_run(xi, nq, nbr_x * 8);
    const int64_t j0 = i0 < 0 ? -1 : aligned_run(yj, nq, nbc_y * 8);
    if (j0 >= 0) {
        const int64_t I = i0 >> 3, J = j0 >> 3;
        double acc[kDotGroup];
#pragma unroll
        for (int t = 0; t < kDotGroup; ++t) acc[t] = 0.0;
        for (int64_t kb = 64 * w + lane; kb < nk; kb += kDotSlots) {
            double coef[kKept], fb;
            LineStream sx, sy;
            load_block<false>(X.f, X.s, X.phi, X.c, I * nk + kb, coef, fb);
            sx.init(coef, fb);
            load_block<true>(Y.f, Y.s, Y.phi, Y.c, kb * nbc_y + J, coef, fb);
            sy.init(coef, fb);
#pragma unroll
            for (int u = 0; u < kDotGroup; ++u) {
                double x[8], y[8];
                sx.line(u, x);
                sy.line(u, y);
                acc[u] = dot8(acc[u], x, y);
            }
        }
#pragma unroll
        for (int t = 0; t < kDotGroup; ++t) S[t] = wave_sum(acc[t]);
        return;
    }
    for (int t = 0; t < nq; ++t) {
        const int64_t i = index_of(xi, t), j = index_of(yj, t);
        if (i < 0 || i >= nbr_x * 8 || j < 0 || j >= nbc_y * 8) continue;
        const int64_t I = i >> 3, J = j >> 3;
        const int r = (int)(i & 7), c = (int)(j & 7);
        double acc = 0.0;
        for (int64_t kb = 64 * w + lane; kb < nk; kb += kDotSlots) {
            double x[8], y[8];
            block_line<false>(X.f, X.s, X.phi, X.c, I * nk + kb, r, x);
            block_line<true>(Y.f, Y.s, Y.phi, Y.c, kb * nbc_y + J, c, y);
            acc = dot8(acc, x, y);
        }
        const double s = wave_sum(acc);
#pragma unroll
        for (int u = 0; u < kDotGroup; ++u)
            if (u == t) S[u] = s;
    }
}

// Part w for lines of X (nbr*8 x nbc*8) against dense vectors v + q*ldv.
__device__ __forceinline__ void dot_dense_part(int w, int lane, int64_t q0, int64_t nq, const DotOperand& X,
                                               int64_t nbr, int64_t nbc, const int64_t* __restrict__ xrow,
                                               const double* __restrict__ v, int64_t ldv, double S[kDotGroup])
{
#pragma unroll
    for (int t = 0; t < kDotGroup; ++t) S[t] = 0.0;
    const int64_t xi = group_indices(xrow, q0, nq, lane);
    const int64_t i0 = aligned_run(xi, nq, nbr * 8);
    if (i0 >= 0) {
        const int64_t I = i0 >> 3;
        double acc[kDotGroup];
#pragma unroll
        for (int t = 0; t < kDotGroup; ++t) acc[t] = 0.0;
        if (ldv == 0) {  // one shared vector: its 8 entries per block loaded once for the 8 lines
            for (int64_t kb = 64 * w + lane; kb < nbc; kb += kDotSlots) {
                double coef[kKept], fb, vb[8];
                LineStream sx;
                load_block<false>(X.f, X.s, X.phi, X.c, I * nbc + kb, coef, fb);
                const double2* vp = reinterpret_cast<const double2*>(v + kb * 8);
#pragma unroll
                for (int k = 0; k < 4; ++k) {
                    const double2 vv = vp[k];
                    vb[2 * k] = vv.x;
                    vb[2 * k + 1] = vv.y;
                }
                sx.init(coef, fb);
#pragma unroll
                for (int u = 0; u < kDotGroup; ++u) {
                    double x[8];
                    sx.line(u, x);
                    acc[u] = dot8(acc[u], x, vb);  // the order and roundings of dot8_global
                }
            }
        } else {
            for (int64_t kb = 64 * w + lane; kb < nbc; kb += kDotSlots) {
                double coef[kKept], fb;
                LineStream sx;
                load_block<false>(X.f, X.s, X.phi, X.c, I * nbc + kb, coef, fb);
                sx.init(coef, fb);
#pragma unroll
                for (int u = 0; u < kDotGroup; ++u) {
                    double x[8];
                    sx.line(u, x);
                    acc[u] = dot8_global(acc[u], x, v + (q0 + u) * ldv + kb * 8);
                }
            }
        }
#pragma unroll
        for (int t = 0; t < kDotGroup; ++t) S[t] = wave_sum(acc[t]);
        return;
    }
    for (int t = 0; t < nq; ++t) {
        const int64_t i = index_of(xi, t);
        if (i < 0 || i >= nbr * 8) continue;
        const int64_t I = i >> 3;
        const int r = (int)(i & 7);
        const double* vq = v + (q0 + t) * ldv;
        double acc = 0.0;
        for (int64_t kb = 64 * w + lane; kb < nbc; kb += kDotSlots) {
            double x[8];
            block_line<false>(X.f, X.s, X.phi, X.c, I * nbc + kb, r, x);
            acc = dot8_global(acc, x, vq + kb * 8);
        }
        const double s = wave_sum(acc);
#pragma unroll
        for (int u = 0; u < kDotGroup; ++u)
            if (u == t) S[u] = s;
    }
}

// Query q0 + t is valid (its indices are inside the operands).
__device__ __forceinline__ bool dot_valid(const int64_t* xrow, const int64_t* ycol, int64_t q, int64_t xlines,
                                          int64_t ylines)
{
    const int64_t i = xrow[q];
    if (i < 0 || i >= xlines) return false;
    if (!ycol) return true;
    const int64_t j = ycol[q];
    return j >= 0 && j < ylines;
}

// A wave-uniform double moved to scalar registers (the part sums are the same
// in every lane after the butterfly; keeping the running totals scalar frees
// vector registers for the line streams).
__device__ __forceinline__ double to_scalar(double v)
{
    const uint64_t b = __builtin_bit_cast(uint64_t, v);
    const uint32_t lo = __builtin_amdgcn_readfirstlane((uint32_t)b);
    const uint32_t hi = __builtin_amdgcn_readfirstlane((uint32_t)(b >> 32));
    return __builtin_bit_cast(double, ((uint64_t)hi << 32) | lo);
}

// One wave runs the four parts of a group in order and writes the results
// (the batch kernel's form; same sums, same order as the four-wave kernels).
__device__ __forceinline__ void dot_group_one_wave(int lane, int64_t q0, int64_t count, const DotOperand& X,
                                                   int64_t nbr_x, const DotOperand& Y, int64_t nbc_y, int64_t nk,
                                                   const int64_t* __restrict__ xrow,
                                                   const int64_t* __restrict__ ycol, double* __restrict__ out)
{
    const int64_t nq = count - q0 < kDotGroup ? count - q0 : kDotGroup;
    double T[kDotGroup], S[kDotGroup];
    dot_part(0, lane, q0, nq, X, nbr_x, Y, nbc_y, nk, xrow, ycol, T);
#pragma unroll
    for (int t = 0; t < kDotGroup; ++t) T[t] = to_scalar(T[t]);
#pragma nounroll
    for (int w = 1; w < kDotParts; ++w) {
        dot_part(w, lane, q0, nq, X, nbr_x, Y, nbc_y, nk, xrow, ycol, S);
#pragma unroll
        for (int t = 0; t < kDotGroup; ++t) T[t] = to_scalar(T[t] + S[t]);
    }
    if (lane == 0)
        for (int t = 0; t < nq; ++t)
            out[q0 + t] = dot_valid(xrow, ycol, q0 + t, nbr_x * 8, nbc_y * 8) ? T[t] : __builtin_nan("");
}

__device__ __forceinline__ void dot_dense_group_one_wave(int lane, int64_t q0, int64_t count, const DotOperand& X,
                                                         int64_t nbr, int64_t nbc, const int64_t* __restrict__ xrow,
                                                         const double* __restrict__ v, int64_t ldv,
                                                         double* __restrict__ out)
{
    const int64_t nq = count - q0 < kDotGroup ? count - q0 : kDotGroup;
    double T[kDotGroup], S[kDotGroup];
    dot_dense_part(0, lane, q0, nq, X, nbr, nbc, xrow, v, ldv, T);
#pragma unroll
    for (int t = 0; t < kDotGroup; ++t) T[t] = to_scalar(T[t]);
#pragma nounroll
    for (int w = 1; w < kDotParts; ++w) {
        dot_dense_part(w, lane, q0, nq, X, nbr, nbc, xrow, v, ldv, S);
#pragma unroll
        for (int t = 0; t < kDotGroup; ++t) T[t] = to_scalar(T[t] + S[t]);
    }
    if (lane == 0)
        for (int t = 0; t < nq; ++t)
            out[q0 + t] = dot_valid(xrow, nullptr, q0 + t, nbr * 8, 0) ? T[t] : __builtin_nan("");
}

}  // namespace blaz
