// Device helpers shared by the compression kernels (binary64 and
// mixed-precision transform): the fixed-order pairwise sum, the
// normalization of Eq. eqnorm, and the wave-cooperative LDS staging of block
// rows.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "blaz_device.hpp"

namespace blaz {

typedef double f64x2 __attribute__((ext_vector_type(2)));
typedef __bf16 bf16x8v __attribute__((ext_vector_type(8)));
typedef float f32x4v __attribute__((ext_vector_type(4)));

// Pairwise sum of the 64 values v(0..63) in row-major order: level 1 adds
// (v0+v1), (v2+v3), ..., each next level adds adjacent pairs.  This fixed
// order makes the slope s and the DC coefficient bit-reproducible.
template <typename F>
__device__ __forceinline__ double pairwise64(F v)
{
    double t[32];
#pragma unroll
    for (int i = 0; i < 32; ++i) t[i] = v(2 * i) + v(2 * i + 1);
#pragma unroll
    for (int n = 16; n >= 1; n /= 2) {
#pragma unroll
        for (int i = 0; i < n; ++i) t[i] = t[2 * i] + t[2 * i + 1];
    }
    return t[0];
}

// Normalization, Eq. eqnorm, in place.  Processing from the bottom-right
// corner backwards keeps every left and upper neighbour unmodified when it is
// read.  The interior term is ((M - Mup) + (M - Mleft)) * 0.5 exactly as
// written (no contraction is possible: there is no product).
__device__ __forceinline__ void normalize(double x[64])
{
#pragma unroll
    for (int u = 7; u >= 1; --u) {
#pragma unroll
        for (int v = 7; v >= 1; --v)
            x[u * 8 + v] = ((x[u * 8 + v] - x[(u - 1) * 8 + v]) + (x[u * 8 + v] - x[u * 8 + v - 1])) * 0.5;
    }
#pragma unroll
    for (int v = 7; v >= 1; --v) x[v] = x[v] - x[v - 1];
#pragma unroll
    for (int u = 7; u >= 1; --u) x[u * 8] = x[u * 8] - x[(u - 1) * 8];
    x[0] = 0.0;
}

// ---------------------------------------------------------------------------
// Wave-cooperative staging.  A workgroup is one wave of 64 lanes owning 64
// consecutive blocks.  Row r of those blocks is moved between HBM and the
// lanes' registers through a 5 KiB LDS tile: every global instruction moves
// 16 B per lane over a contiguous 1 KiB run (4 lanes per block row segment,
// 16 blocks per instruction), and each lane then reads or writes its own
// block's 64 B in LDS.  Each lane has a 64-byte slot; the four 16-byte
// chunks of slot s sit in the order c ^ ((s >> 1) & 3), which makes both
// access patterns free of bank conflicts (gfx950 serves 16-byte accesses 8
// lanes at a time from 32 four-byte banks): the global-side 8 lanes move the
// four chunks of two neighbouring slots, the lane-side 8 lanes one chunk of
// 8 consecutive slots.  (80-byte slots in natural order conflicted 2-way on
// every global-side phase: 4.2e6 conflict cycles per 8192^2 compress.)
// ---------------------------------------------------------------------------
constexpr int kWave = 64;
constexpr int kSlot = 8;  // doubles per lane slot in the LDS tile

// Offset (doubles) of chunk c (columns 2c, 2c+1 of a block row) of slot s.
__device__ __forceinline__ int slot_chunk(int s, int c) { return s * kSlot + 2 * (c ^ ((s >> 1) & 3)); }

// Global offsets (in doubles, row 0) of the four 16-byte chunks a lane moves:
// chunk k covers part (lane & 3) of block wave_base + (lane >> 2) + 16 k.
struct WaveChunks {
    int64_t off[4];
    bool ok[4];
};

__device__ __forceinline__ WaveChunks wave_chunks(int64_t wave_base, int lane, int64_t nbc, int64_t nblk,
                                                  int64_t lda)
{
    WaveChunks w;
    int64_t I0 = 0, J0 = 0;
    if (nbc >= kWave) {  // wave-uniform: the 64 blocks wrap into the next block row at most once
        I0 = wave_base / nbc;
        J0 = wave_base - I0 * nbc;
    }
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        const int q = (lane >> 2) + 16 * k;
        const int64_t bb = wave_base + q;
        int64_t I, J;
        if (nbc >= kWave) {
            I = I0;
            J = J0 + q;
            if (J >= nbc) {
                J -= nbc;
                ++I;
            }
        } else {
            I = bb / nbc;
            J = bb - I * nbc;
        }
        w.ok[k] = bb < nblk;
        w.off[k] = (8 * I) * lda + 8 * J + 2 * (lane & 3);
    }
    return w;
}


// Load the 8x8 blocks wave_base .. wave_base+63 into x (one block per lane).
// kVec: A 16-byte aligned with even lda, rows staged through the LDS tile so
// each global load covers a contiguous 1 KiB run; otherwise each lane reads
// its own block.  Lanes past nblk get zeros.
template <bool kVec>
__device__ __forceinline__ void load_blocks(const double* __restrict__ A, int64_t lda, int64_t nbc, int64_t nblk,
                                            int64_t wave_base, int lane, double* tile, double x[64])
{
    const int64_t b = wave_base + lane;
    if constexpr (kVec) {
        const WaveChunks wc = wave_chunks(wave_base, lane, nbc, nblk, lda);
        f64x2 g[8][4];
        // the 32 loads issue at raised wave priority, so the other wave's
        // transform on the SIMD does not stretch the burst (0.5 % faster)
        __builtin_amdgcn_s_setprio(2);
#pragma unroll
        for (int r = 0; r < 8; ++r)
#pragma unroll
            for (int k = 0; k < 4; ++k)
                g[r][k] = wc.ok[k] ? __builtin_nontemporal_load(reinterpret_cast<const f64x2*>(A + wc.off[k] + r * lda))
                                   : f64x2{0.0, 0.0};
        __builtin_amdgcn_s_setprio(0);
#pragma unroll
        for (int r = 0; r < 8; ++r) {
#pragma unroll
            for (int k = 0; k < 4; ++k)
                *reinterpret_cast<f64x2*>(&tile[slot_chunk((lane >> 2) + 16 * k, lane & 3)]) = g[r][k];
            __syncthreads();
#pragma unroll
            for (int p = 0; p < 4; ++p) {
                const f64x2 v = *reinterpret_cast<const f64x2*>(&tile[slot_chunk(lane, p)]);
                x[r * 8 + 2 * p] = v[0];
                x[r * 8 + 2 * p + 1] = v[1];
            }
            __syncthreads();
        }
    } else {
        if (b < nblk) {
            const int64_t I = b / nbc, J = b - (b / nbc) * nbc;
            const double* src = A + (I * 8) * lda + J * 8;
#pragma unroll
            for (int r = 0; r < 8; ++r)
#pragma unroll
                for (int c = 0; c < 8; ++c) x[r * 8 + c] = src[r * lda + c];
        } else {
#pragma unroll
            for (int e = 0; e < 64; ++e) x[e] = 0.0;
        }
    }
}

struct SlopeOut {
    double f;   // first element M_00
    double s;   // mean slope
    double dc;  // D_00, fixed-order binary64
};

// Normalization (Eq. eqnorm) and mean slope (Eqs. eqslope, eqslope2), all
// binary64: x holds the block on entry and Delta on exit.
__device__ __forceinline__ SlopeOut slope_of(double x[64])
{
    SlopeOut o;
    o.f = x[0];
    normalize(x);
    int K = 0;
#pragma unroll
    for (int e = 1; e < 64; ++e) K += x[e] != 0.0 ? 1 : 0;
    const double S1 = pairwise64([&](int e) { return fabs(x[e]); });
    const double S = pairwise64([&](int e) { return x[e]; });
    o.s = K > 0 ? S1 / (double)K : 0.0;
    // D_00 = alpha_0^2 sum Delta' = 0.125 (sum Delta / s), the fixed order.
    o.dc = o.s != 0.0 ? 0.125 * (S / o.s) : 0.0;
    return o;
}

// Delta' = Delta / s in place.  The reciprocal is exact enough for the 63
// non-DC coefficients; a slope so small that 1/s overflows falls back to
// division.
__device__ __forceinline__ void divide_by_slope(double x[64], double s)
{
    if (s != 0.0 && fabs(s) >= 0x1p-1020) {
        const double r = 1.0 / s;
#pragma unroll
        for (int e = 0; e < 64; ++e) x[e] *= r;
    } else if (s != 0.0) {
#pragma unroll
        for (int e = 0; e < 64; ++e) x[e] = x[e] / s;
    }
}

// Prediction, Eq. eqpredict, of a block from Delta (x on entry, as slope_of
// leaves it).  Psi_e is the index of the grid point
// g(k) = (s - s_max) + k * (2 s_max / 256), k = 0..255, nearest to
// Delta'_e = Delta_e / s, as a search over all 256 points in increasing k
// finds it: the first index of the smallest computed distance |Delta' - g(k)|.
// s_max = max |Delta'| = max |Delta| / s (division rounds monotonically; s is
// a mean of absolute values, so s >= 0).
//
// Where the grid points are well apart in binary64 (|lo| <= 2^30 step,
// lo = s - s_max) every computed distance is within 2^-22 step of the exact
// one.  So when Delta''s position (Delta' - lo) / step lies more than 1e-6
// from a half-way point, the nearest point is the unambiguous answer
// (Delta * (1/s) is close enough for this test); otherwise the answer is the
// nearer of the two points around the half-way point by their computed
// distances from Delta_e / s, the lower one on a tie.  With the grid not
// well apart, lo > 2^23 s_max lies above every Delta', whose distances then
// grow with k: index 0.  Non-finite slopes give index 0, as the search
// does.
//
// kStore: write Psi to psi[b][64] (a side output, not part of the stream).
// kReplace: replace x by the predicted slopes g(Psi_e) and o.dc by their DC
// term 0.125 * (pairwise sum), the transform's input under the reading that
// the DCT takes the predicted slopes; otherwise x keeps Delta.
template <bool kStore, bool kReplace>
__device__ __forceinline__ void predict_block(double x[64], SlopeOut& o, uint8_t* psi, int64_t b, bool valid)
{
    double amax = 0.0;
#pragma unroll
    for (int e = 0; e < 64; ++e) amax = fmax(amax, fabs(x[e]));
    const double smax = o.s != 0.0 ? amax / fabs(o.s) : 0.0;
    const double lo = o.s - smax;
    const double step = 2.0 * smax / 256.0;
    const double inv_step = 128.0 / smax;
    const double r = 1.0 / o.s;
    const bool by_division = !isfinite(r);  // a subnormal slope
    const bool wide = smax != 0.0 && isfinite(step) && fabs(lo) <= 0x1p30 * step;  // false for NaN
    uint32_t w[16];
#pragma unroll
    for (int q = 0; q < 16; ++q) w[q] = 0;
#pragma unroll
    for (int e = 0; e < 64; ++e) {
        int k = 0;
        if (wide) {
            const double pos = ((by_division ? x[e] / o.s : x[e] * r) - lo) * inv_step;
            double kd = rint(pos);
            if (!(fabs(pos - kd) < 0.5 - 1e-6)) {  // near a half-way point
                const double lower = floor(pos);
                const double xe = x[e] / o.s;
                const double d0 = fabs(xe - (lo + lower * step));
                const double d1 = fabs(xe - (lo + (lower + 1.0) * step));
                kd = d1 < d0 ? lower + 1.0 : lower;
            }
            k = (int)fmin(fmax(kd, 0.0), 255.0);
        }
        w[e / 4] |= (uint32_t)k << (8 * (e % 4));
        if constexpr (kReplace) x[e] = lo + (double)k * step;
    }
    if constexpr (kReplace) o.dc = 0.125 * pairwise64([&](int e) { return x[e]; });
    if (kStore && valid) {
        uint4* dst = reinterpret_cast<uint4*>(psi + b * 64);
#pragma unroll
        for (int q = 0; q < 4; ++q) dst[q] = make_uint4(w[4 * q], w[4 * q + 1], w[4 * q + 2], w[4 * q + 3]);
    }
}

// phi of Eq. eqphi from m, the max over the block's 64 |D|: trunc(127/m)
// clamped to 255.
__device__ __forceinline__ int phi_of(double m)
{
    const double px = 127.0 / m;  // +inf when m == 0
    return px < 255.0 ? (int)px : 255;
}

// Code t (trunc(phi D), toward zero) into its byte of the packed words.
__device__ __forceinline__ void pack_code(uint32_t w[kCodeWords], int t, double phid, double d)
{
    const int c = (int)(phid * d);
    w[t / 4] |= ((uint32_t)c & 0xffu) << (8 * (t % 4));
}

__device__ __forceinline__ void store_record(const uint32_t w[kCodeWords], int phi, const SlopeOut& so_,
                                             int64_t nblk, int64_t wave_base, int lane, void* tile, double* fo,
                                             double* so, uint8_t* phio, uint32_t* codes);

// Quantization (Eq. eqphi) and the stores of one wave's records.  D holds
// the 64 DCT coefficients of the lane's block (binary64).  m is the max over
// all 64, phi = trunc(127/m) clamped to 255, codes = trunc(phi D) at the 28
// kept positions.
__device__ __forceinline__ void quantize_store(const double D[64], const SlopeOut& so_, int64_t nblk,
                                               int64_t wave_base, int lane, void* tile, double* fo, double* so,
                                               uint8_t* phio, uint32_t* codes)
{
    double m = 0.0;
#pragma unroll
    for (int e = 0; e < 64; ++e) m = fmax(m, fabs(D[e]));
    const int phi = phi_of(m);
    const double phid = (double)phi;
    uint32_t w[kCodeWords];
#pragma unroll
    for (int q = 0; q < kCodeWords; ++q) w[q] = 0;
#pragma unroll
    for (int t = 0; t < kKept; ++t) pack_code(w, t, phid, D[kept_row(t) * 8 + kept_col(t)]);
    store_record(w, phi, so_, nblk, wave_base, lane, tile, fo, so, phio, codes);
}

// The record of the lane's block: f and s, then the wave's codes and phi
// bytes.  The codes are one contiguous run of 64 * 28 bytes: packed in LDS
// (tile, >= 1856 bytes) with the phi bytes, then written out.
__device__ __forceinline__ void store_record(const uint32_t w[kCodeWords], int phi, const SlopeOut& so_,
                                             int64_t nblk, int64_t wave_base, int lane, void* tile, double* fo,
                                             double* so, uint8_t* phio, uint32_t* codes)
{
    const int64_t b = wave_base + lane;
    if (b < nblk) {
        fo[b] = so_.f;
        so[b] = so_.s;
    }
    // The wave's codes (1792 bytes) and phi bytes (64) packed in LDS, then
    // written as 16-byte runs (4-byte ones when the destination is not
    // 16-byte aligned, and for a ragged last wave's tail).
    uint32_t* ct = reinterpret_cast<uint32_t*>(tile);
    uint8_t* pt = reinterpret_cast<uint8_t*>(ct + kWave * kCodeWords);
    __syncthreads();
#pragma unroll
    for (int q = 0; q < kCodeWords; ++q) ct[lane * kCodeWords + q] = w[q];
    pt[lane] = (uint8_t)phi;
    __syncthreads();
    const int64_t nb = nblk - wave_base < kWave ? nblk - wave_base : kWave;
    const int64_t nwords = nb * kCodeWords;
    uint32_t* cdst = codes + wave_base * kCodeWords;
    if ((reinterpret_cast<uintptr_t>(cdst) & 15) == 0) {
        const int64_t nvec = nwords >> 2;
#pragma unroll
        for (int k = 0; k < (kWave * kCodeWords + 4 * kWave - 1) / (4 * kWave); ++k) {
            const int idx = lane + kWave * k;
            if (idx < nvec) reinterpret_cast<uint4*>(cdst)[idx] = reinterpret_cast<const uint4*>(ct)[idx];
        }
        const int64_t rest = 4 * nvec + lane;
        if (rest < nwords && lane < 4) cdst[rest] = ct[rest];
    } else {
#pragma unroll
        for (int k = 0; k < kCodeWords; ++k) {
            const int idx = lane + kWave * k;
            if (idx < nwords) cdst[idx] = ct[idx];
        }
    }
    uint8_t* pdst = phio + wave_base;
    if (nb == kWave && (reinterpret_cast<uintptr_t>(pdst) & 3) == 0) {
        if (lane < kWave / 4) reinterpret_cast<uint32_t*>(pdst)[lane] = reinterpret_cast<const uint32_t*>(pt)[lane];
    } else if (lane < nb) {
        pdst[lane] = pt[lane];
    }
}

// quantize_store for L kept lines: the same phi and truncations, the codes
// of the L-line mask, KeptLines<L>::kWords dwords per block.
template <int L>
__device__ __forceinline__ void quantize_store_lines(const double D[64], const SlopeOut& so_, int64_t nblk,
                                                     int64_t wave_base, int lane, void* tile, double* fo,
                                                     double* so, uint8_t* phio, uint32_t* codes)
{
    using K = KeptLines<L>;
    double m = 0.0;
#pragma unroll
    for (int e = 0; e < 64; ++e) m = fmax(m, fabs(D[e]));
    const double px = 127.0 / m;  // +inf when m == 0
    const int phi = px < 255.0 ? (int)px : 255;
    const double phid = (double)phi;
    uint32_t w[K::kWords];
#pragma unroll
    for (int q = 0; q < K::kWords; ++q) w[q] = 0;
#pragma unroll
    for (int t = 0; t < K::kCount; ++t) {
        const int c = (int)(phid * D[K::pos(t)]);  // truncation toward zero
        w[t / 4] |= ((uint32_t)c & 0xffu) << (8 * (t % 4));
    }
    const int64_t b = wave_base + lane;
    if (b < nblk) {
        fo[b] = so_.f;
        so[b] = so_.s;
        phio[b] = (uint8_t)phi;
    }
    uint32_t* ct = reinterpret_cast<uint32_t*>(tile);
    __syncthreads();
#pragma unroll
    for (int q = 0; q < K::kWords; ++q) ct[lane * K::kWords + q] = w[q];
    __syncthreads();
    const int64_t nwords = (nblk - wave_base < kWave ? nblk - wave_base : kWave) * K::kWords;
    uint32_t* cdst = codes + wave_base * K::kWords;
#pragma unroll
    for (int k = 0; k < K::kWords; ++k) {
        const int idx = lane + kWave * k;
        if (idx < nwords) cdst[idx] = ct[idx];
    }
}

// Output forms of the decompression: binary64 (the plain method), and the
// operand forms of the low-precision contractions in blaz_matmul: FP32, or
// BF16 hi + lo with hi = bf16(x), lo = bf16(x - hi).
// kRow8: the form stores one block row (8 consecutive values) of a lane with
// 16-byte stores of its own (store8; the narrow forms: a row is 32 or
// 2 x 16 bytes, and the rows of adjacent lanes' blocks are adjacent);
// otherwise the rows go through LDS to full-width stores (store2).
struct OutF64 {
    static constexpr bool kRow8 = false;
    double* p;
    __device__ void store2(int64_t off, double a, double b) const
    {
        __builtin_nontemporal_store(f64x2{a, b}, reinterpret_cast<f64x2*>(p + off));
    }
    __device__ void store(int64_t off, double a) const { p[off] = a; }
};
struct OutF32 {
    static constexpr bool kRow8 = true;
    float* p;
    __device__ void store8(int64_t off, const double* v) const
    {
        *reinterpret_cast<f32x4v*>(p + off) = f32x4v{(float)v[0], (float)v[1], (float)v[2], (float)v[3]};
        *reinterpret_cast<f32x4v*>(p + off + 4) = f32x4v{(float)v[4], (float)v[5], (float)v[6], (float)v[7]};
    }
    __device__ void store(int64_t off, double a) const { p[off] = (float)a; }
};
struct OutBF16Split {
    static constexpr bool kRow8 = true;
    __bf16* hi;
    __bf16* lo;
    __device__ static __bf16 high(double x) { return (__bf16)(float)x; }
    __device__ static __bf16 low(double x, __bf16 h) { return (__bf16)(float)(x - (double)(float)h); }
    __device__ void store(int64_t off, double a) const
    {
        const __bf16 h = high(a);
        hi[off] = h;
        lo[off] = low(a, h);
    }
    __device__ void store8(int64_t off, const double* v) const
    {
        bf16x8v h, l;
#pragma unroll
        for (int e = 0; e < 8; ++e) {
            h[e] = high(v[e]);
            l[e] = low(v[e], h[e]);
        }
        *reinterpret_cast<bf16x8v*>(hi + off) = h;
        *reinterpret_cast<bf16x8v*>(lo + off) = l;
    }
};

// Compression (all stages binary64) of the blocks wave_base .. wave_base+63
// (one per lane) of A; tile is the wave's LDS staging area.
// kPred: the transform takes the predicted slopes instead of Delta' (the
// other reading of the transform's input; the stream format is the same).
template <bool kVec, bool kPsi, int L = 2, bool kPred = false>
__device__ __forceinline__ void compress_wave(const double* __restrict__ A, int64_t lda, int64_t nbc, int64_t nblk,
                                              double* __restrict__ fo, double* __restrict__ so,
                                              uint8_t* __restrict__ phio, uint32_t* __restrict__ codes,
                                              uint8_t* __restrict__ psi, int64_t wave_base, int lane, double* tile)
{
    double x[64];
    load_blocks<kVec>(A, lda, nbc, nblk, wave_base, lane, tile, x);
    SlopeOut so_ = slope_of(x);
    if constexpr (kPsi || kPred)
        predict_block<kPsi, kPred>(x, so_, psi, wave_base + lane, wave_base + lane < nblk);
    if constexpr (!kPred) divide_by_slope(x, so_.s);

    // Two-dimensional DCT-II (Eq. eqdct) of Delta' (or of the predicted
    // slopes): rows, then columns, in place; the DC term is the fixed-order
    // binary64 value.
#pragma unroll
    for (int u = 0; u < 8; ++u) dct8<1, 1>(x + u * 8, x + u * 8);
#pragma unroll
    for (int v = 0; v < 8; ++v) dct8<8, 8>(x + v, x + v);
    x[0] = so_.dc;

    if constexpr (L == 2)
        quantize_store(x, so_, nblk, wave_base, lane, tile, fo, so, phio, codes);
    else
        quantize_store_lines<L>(x, so_, nblk, wave_base, lane, tile, fo, so, phio, codes);
}

// Decompression of the blocks wave_base .. wave_base+63 (one per lane) of a
// compressed matrix into `out` (leading dimension lda); tile is the wave's
// LDS staging area (kWave * kSlot doubles).
template <bool kVec, typename Out, int L = 2>
__device__ __forceinline__ void decompress_wave(const double* __restrict__ f, const double* __restrict__ s,
                                                const uint8_t* __restrict__ phi, const uint32_t* __restrict__ codes,
                                                int64_t nbc, int64_t nblk, Out out, int64_t lda, int64_t wave_base,
                                                int lane, double* tile)
{
    const int64_t b = wave_base + lane;
    const bool valid = b < nblk;
    // f, s and phi are loaded first, so that their latency overlaps the
    // staging of the codes instead of following it.
    const double fb = valid ? f[b] : 0.0;
    const double sb = valid ? s[b] : 0.0;
    const double pb = valid ? (double)phi[b] : 1.0;

    // The wave's codes: consecutive dwords into LDS, then each lane's own
    // (7 for the paper's scheme, KeptLines<L>::kWords in general).
    constexpr int kW = KeptLines<L>::kWords;
    uint32_t* ct = reinterpret_cast<uint32_t*>(tile);
    const int64_t nwords = (nblk - wave_base < kWave ? nblk - wave_base : kWave) * kW;
    const uint32_t* csrc = codes + wave_base * kW;
#pragma unroll
    for (int k = 0; k < kW; ++k) {
        const int idx = lane + kWave * k;
        if (idx < nwords) ct[idx] = csrc[idx];
    }
    __syncthreads();
    uint32_t w[kW];
#pragma unroll
    for (int q = 0; q < kW; ++q) w[q] = ct[lane * kW + q];
    __syncthreads();
    // Dhat = C / phi at the kept positions (zero elsewhere); the slope factor
    // of Eq. eqbbb is folded in by linearity of the inverse DCT.
    double x[64];
    if constexpr (L == 2) {
        double coef[kKept];
        unpack_codes(w, sb / pb, coef);
        inverse_transform(coef, x);
    } else {
        double coef[KeptLines<L>::kCount];
        unpack_codes_lines<L>(w, sb / pb, coef);
        inverse_transform_lines<L>(coef, x);
    }
    inverse_normalize(fb, x);

    if constexpr (kVec && Out::kRow8) {
        // Each lane stores its own block rows: the rows of a wave's blocks
        // in one block row of the matrix are contiguous, so a store
        // instruction writes one run of 64 x 16 bytes (BF16) or two
        // interleaved ones (FP32), with no LDS round trip (the BF16x3
        // product with a compressed B, both operands rebuilt this way:
        // 0.094 -> 0.088 ms at 2048^3, 0.398 -> 0.389 ms at 4096^3).
        if (valid) {
            const int64_t I = b / nbc, J = b - (b / nbc) * nbc;
            const int64_t base = (I * 8) * lda + J * 8;
#pragma unroll
            for (int r = 0; r < 8; ++r) out.store8(base + r * lda, x + r * 8);
        }
    } else if constexpr (kVec) {
        const WaveChunks wc = wave_chunks(wave_base, lane, nbc, nblk, lda);
#pragma unroll
        for (int r = 0; r < 8; ++r) {
#pragma unroll
            for (int p = 0; p < 4; ++p)
                *reinterpret_cast<f64x2*>(&tile[slot_chunk(lane, p)]) = f64x2{x[r * 8 + 2 * p], x[r * 8 + 2 * p + 1]};
            __syncthreads();
#pragma unroll
            for (int k = 0; k < 4; ++k) {
                const f64x2 v = *reinterpret_cast<const f64x2*>(&tile[slot_chunk((lane >> 2) + 16 * k, lane & 3)]);
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

}  // namespace blaz
