// Dense contraction of blaz_matmul on the matrix cores.
//
// The paper's matrix multiplication rebuilds every block once and then
// multiplies (last paragraph of Section "Basic Linear Algebra Algorithms").
// The rebuild is the decompression kernel; this file holds the product
// C = A B of the rebuilt operands in three arithmetics, all writing binary64:
//   FP64    v_mfma_f64_16x16x4_f64 on binary64 operands (the plain method)
//   FP32    v_mfma_f32_16x16x4_f32 on FP32 operands, FP32 accumulation
//   BF16x3  v_mfma_f32_16x16x32_bf16 on A = Ahi + Alo, B = Bhi + Blo:
//           C = Alo Bhi + Ahi Blo + Ahi Bhi (the Alo Blo term, ~2^-16
//           relative, is dropped), FP32 accumulation
//
// Tiling: a workgroup computes a BMxBM tile of C (BM = 128 or 64; the 64
// tile gives small products four times as many workgroups).  FP64 and FP32
// run four waves, each owning a quadrant as (BM/32)x(BM/32) MFMA tiles of
// 16x16; K advances through double-buffered LDS tiles, and the stage after
// next is loaded into registers during the current stage's MFMAs, so HBM/L2
// latency overlaps the matrix math.  BF16x3 fills its LDS tiles straight from
// memory (global_load_lds) and runs eight waves on the 128 tile.  The MFMAs
// run at raised wave priority.  Workgroup ids are remapped so that each XCD
// (the hardware deals workgroups to the 8 XCDs round-robin) works on a
// contiguous group of tiles that share rows of A and columns of B in its own
// L2.  The file also holds the preparation of B for the FP32 and BF16x3
// products: conversion of a dense binary64 B, or transposition of a
// compressed B rebuilt in the operand precision, into blocked B^T tiles.
#include <hip/hip_runtime.h>

#include "blaz_internal.hpp"

namespace blaz {

typedef double f64x2 __attribute__((ext_vector_type(2)));
typedef double f64x4 __attribute__((ext_vector_type(4)));
typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));

// s_waitcnt immediate (gfx9 encoding) that waits for every outstanding
// vector memory operation and leaves the export and LDS counters free:
// vmcnt = 0 (bits 3:0 and 15:14), expcnt = 7 (bits 6:4), lgkmcnt = 15
// (bits 11:8).
constexpr int kWaitVmcnt0 = 0x0F70;

// Elements of padding per LDS row of the FP64 operand tiles.  gfx950's LDS
// serves 128 B per clock from 32 four-byte banks, 64-bit accesses in groups
// of 16 lanes and 32-bit ones in groups of 32 (this model reproduces the
// measured conflict counts of the FP64 and FP32 layouts tried).  A 16-lane
// group of the transposed A store writes column m, m+1 of rows k, k+2, ...,
// k+14; with a 131-double row (3 doubles of padding) those rows start 12
// banks apart and all 16 stores hit distinct banks (counted: 0 conflicts; a
// 130-double row gives 2-way conflicts on them, 0.8 % slower at 4096^3).  B
// rows take even padding so that their 16-byte stores stay aligned; the
// fragment reads (16 consecutive doubles of one row per group) never
// conflict.
constexpr int kPadA64 = 3;
constexpr int kPadB64 = 2;

// Tile (tm, tn) for workgroup `wg` of `nwg`: contiguous ranges per XCD, then
// groups of 4 tile rows walked column by column for L2 reuse.
__device__ __forceinline__ void tile_of(int wg, int nwg, int ntm, int ntn, int& tm, int& tn)
{
    if (nwg % 8 == 0) wg = (wg % 8) * (nwg / 8) + wg / 8;
    constexpr int kGroup = 4;
    const int per_group = kGroup * ntn;
    const int g = wg / per_group;
    const int first = g * kGroup;
    const int rows = min(ntm - first, kGroup);
    const int r = wg - g * per_group;
    tm = first + r % rows;
    tn = r / rows;
}

// The 16x16x4 MFMA for each operand type, and where value r of lane l lands
// in the 16x16 result (probed on gfx950: the FP64 form places value r of
// lane l in row 4r + l/16, the FP32 form in row 4(l/16) + r; column l%16).
template <typename T>
struct Mfma16x16x4;
template <>
struct Mfma16x16x4<double> {
    using acc_t = f64x4;
    using vec_t = f64x2;  // 16-byte global/LDS vector
    static constexpr int kBK = 16;
    __device__ static acc_t op(double a, double b, acc_t c) { return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0); }
    __device__ static int row(int g, int r) { return 4 * r + g; }
};

// Output tile (tm, tn) of C = A B with A (M x K, lda) and B (K x N, ldb)
// row-major binary64; C binary64.  Run by one 256-thread workgroup.  LDS
// rows hold kBM + kPadA64 (A) and kBN + kPadB64 (B) elements.
template <typename T, int kBM>
__device__ __forceinline__ void gemm_tile(const T* __restrict__ A, int64_t lda, const T* __restrict__ B, int64_t ldb,
                                          double* __restrict__ C, int64_t ldc, int64_t M, int64_t N, int64_t K,
                                          int tm, int tn)
{
    using MF = Mfma16x16x4<T>;
    using acc_t = typename MF::acc_t;
    using vec_t = typename MF::vec_t;
    constexpr int kBN = kBM;
    constexpr int TW = kBM / 32;          // MFMA tiles per wave and dimension
    constexpr int BK = MF::kBK;
    constexpr int V = 16 / sizeof(T);     // elements per 16-byte vector
    constexpr int AV = BK / V;            // vectors per A tile row
    constexpr int BV = kBN / V;           // vectors per B tile row
    constexpr int RV = kBM * AV / 256;    // vectors of A (and of B) per thread
    static_assert(kBM * AV == BK * BV && RV * 256 == kBM * AV, "whole vectors per thread");

    __shared__ __align__(16) T As[2][BK][kBM + kPadA64];  // A tiles stored k-major (transposed), double-buffered
    __shared__ __align__(16) T Bs[2][BK][kBN + kPadB64];  // 16-byte row stores
    static_assert((kBN + kPadB64) * sizeof(T) % 16 == 0, "B rows keep 16-byte alignment");

    const int64_t row0 = (int64_t)tm * kBM, col0 = (int64_t)tn * kBN;

    const int tid = threadIdx.x;
    const int lane = tid & 63, wave = tid >> 6;
    const int wm = wave >> 1, wn = wave & 1;

    vec_t ra[RV], rb[RV];
    auto load_stage = [&](int64_t k0) {
#pragma unroll
        for (int r = 0; r < RV; ++r) {
            const int q = tid + 256 * r;
            const int am = q / AV, ak = (q % AV) * V;
            const int64_t gr = row0 + am, gk = k0 + ak;
            ra[r] = (gr < M && gk < K) ? *reinterpret_cast<const vec_t*>(A + gr * lda + gk) : vec_t{};
            const int bk = q / BV, bn = (q % BV) * V;
            const int64_t hk = k0 + bk, hn = col0 + bn;
            rb[r] = (hk < K && hn < N) ? *reinterpret_cast<const vec_t*>(B + hk * ldb + hn) : vec_t{};
        }
    };
    auto store_stage = [&](int buf) {
#pragma unroll
        for (int r = 0; r < RV; ++r) {
            const int q = tid + 256 * r;
            const int am = q / AV, ak = (q % AV) * V;
#pragma unroll
            for (int e = 0; e < V; ++e) As[buf][ak + e][am] = ra[r][e];
            const int bk = q / BV, bn = (q % BV) * V;
            *reinterpret_cast<vec_t*>(&Bs[buf][bk][bn]) = rb[r];
        }
    };

    acc_t acc[TW][TW];
#pragma unroll
    for (int i = 0; i < TW; ++i)
#pragma unroll
        for (int j = 0; j < TW; ++j) acc[i][j] = acc_t{};

    // Pipeline: stage kt is read from LDS buffer kt%2 while stage kt+1 (loaded
    // into registers one step earlier) is written to the other buffer and
    // stage kt+2 is fetched from memory; one barrier per step.
    const int nk = (int)((K + BK - 1) / BK);
    load_stage(0);
    store_stage(0);
    if (nk > 1) load_stage(BK);
    __syncthreads();
    for (int kt = 0; kt < nk; ++kt) {
        const int cur = kt & 1;
        __builtin_amdgcn_s_setprio(1);
#pragma unroll
        for (int kk = 0; kk < BK; kk += 4) {
            // A operand: lane holds A[m = lane%16][k = lane/16]; B operand:
            // lane holds B[k = lane/16][n = lane%16].
            T a[TW], b[TW];
#pragma unroll
            for (int i = 0; i < TW; ++i) a[i] = As[cur][kk + (lane >> 4)][wm * (kBM / 2) + i * 16 + (lane & 15)];
#pragma unroll
            for (int j = 0; j < TW; ++j) b[j] = Bs[cur][kk + (lane >> 4)][wn * (kBN / 2) + j * 16 + (lane & 15)];
#pragma unroll
            for (int i = 0; i < TW; ++i)
#pragma unroll
                for (int j = 0; j < TW; ++j) acc[i][j] = MF::op(a[i], b[j], acc[i][j]);
        }
        __builtin_amdgcn_s_setprio(0);
        if (kt + 1 < nk) {
            store_stage(cur ^ 1);
            if (kt + 2 < nk) load_stage((int64_t)(kt + 2) * BK);
        }
        __syncthreads();
    }

#pragma unroll
    for (int i = 0; i < TW; ++i)
#pragma unroll
        for (int j = 0; j < TW; ++j) {
            const int64_t gc = col0 + wn * (kBN / 2) + j * 16 + (lane & 15);
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int64_t gr = row0 + wm * (kBM / 2) + i * 16 + MF::row(lane >> 4, r);
                if (gr < M && gc < N) C[gr * ldc + gc] = (double)acc[i][j][r];
            }
        }
}

template <typename T, int kBM>
__global__ __launch_bounds__(256) void gemm_kernel(const T* __restrict__ A, int64_t lda, const T* __restrict__ B,
                                                   int64_t ldb, double* __restrict__ C, int64_t ldc, int64_t M,
                                                   int64_t N, int64_t K)
{
    const int ntm = (int)((M + kBM - 1) / kBM);
    const int ntn = (int)((N + kBM - 1) / kBM);
    int tm, tn;
    tile_of(blockIdx.x, gridDim.x, ntm, ntn, tm, tn);
    gemm_tile<T, kBM>(A, lda, B, ldb, C, ldc, M, N, K, tm, tn);
}

// Many binary64 products in one launch: product p owns the workgroups
// tile0 .. tile0 + ntm * ntn - 1, tile0 a multiple of 8, so that the
// XCD-aware tile order of each product is the standalone kernel's (the
// workgroups between two products exit at once).  A workgroup finds its
// product by binary search over tile0.
template <int kBM>
__global__ __launch_bounds__(256) void gemm_group_kernel(const GemmGroupItem* __restrict__ items, int n_items)
{
    const int64_t wg = blockIdx.x;
    int lo = 0, hi = n_items - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (items[mid].tile0 <= wg) lo = mid;
        else hi = mid - 1;
    }
    const GemmGroupItem it = items[lo];
    const int ntm = (int)((it.M + kBM - 1) / kBM);
    const int ntn = (int)((it.N + kBM - 1) / kBM);
    const int64_t local = wg - it.tile0;
    if (local >= (int64_t)ntm * ntn) return;  // padding up to the next product's multiple of 8
    int tm, tn;
    tile_of((int)local, ntm * ntn, ntm, ntn, tm, tn);
    gemm_tile<double, kBM>(it.A, it.lda, it.B, it.ldb, it.C, it.ldc, it.M, it.N, it.K, tm, tn);
}

// FP32: A (M x K, lda) with k contiguous and B^T (N x K) in blocked form:
// tiles of 64 rows (n) x 32 k, 8 KB each, tile (n / 64, k / 32) at
// ((n / 64) * nkc + k / 32) * 2048 elements, nkc = ceil(K / 32), row-major
// inside.  K advances in steps of 32; an LDS tile row is its 32 floats
// (128 B) as eight 16-byte chunks, chunk c of row r in slot c ^ ((r >> 1) & 7).
// A lane's chunk c holds k = 4c .. 4c+3 of its row, and MFMA step s of chunk
// c uses k = 4c + s in every lane group alike, so one 16-byte LDS read feeds
// four v_mfma_f32_16x16x4f32 (measured 5 % faster than the k-major tiles
// with transposed stores: 130 against 124 TFLOP/s at 8192^3).
constexpr int kBKf = 32;

__device__ __forceinline__ int f32_tile_slot(int row, int chunk)
{
    return row * kBKf + ((chunk ^ ((row >> 1) & 7)) << 2);
}

template <int kBM>
__global__ __launch_bounds__(256) void gemm_f32_kernel(const float* __restrict__ A, int64_t lda,
                                                       const float* __restrict__ Bt, int64_t nkc,
                                                       double* __restrict__ C, int64_t ldc, int64_t M, int64_t N,
                                                       int64_t K)
{
    constexpr int kBN = kBM;
    constexpr int TW = kBM / 32;
    constexpr int CPR = kBKf / 4;      // 16-byte chunks per tile row
    constexpr int RC = kBM * CPR / 256;  // chunks of each operand tile per thread
    __shared__ __align__(16) float As[2][kBM * kBKf];
    __shared__ __align__(16) float Bs[2][kBN * kBKf];

    const int ntm = (int)((M + kBM - 1) / kBM);
    const int ntn = (int)((N + kBN - 1) / kBN);
    int tm, tn;
    tile_of(blockIdx.x, gridDim.x, ntm, ntn, tm, tn);
    const int64_t row0 = (int64_t)tm * kBM, col0 = (int64_t)tn * kBN;

    const int tid = threadIdx.x;
    const int lane = tid & 63, wave = tid >> 6;
    const int wm = wave >> 1, wn = wave & 1;

    f32x4 ra[RC], rb[RC];
    auto load_stage = [&](int64_t k0) {
#pragma unroll
        for (int r = 0; r < RC; ++r) {
            const int q = tid + 256 * r;
            const int row = q / CPR, ck = q % CPR;
            const int64_t gk = k0 + 4 * ck, ga = row0 + row, gb = col0 + row;
            ra[r] = (ga < M && gk < K) ? *reinterpret_cast<const f32x4*>(A + ga * lda + gk) : f32x4{0.f, 0.f, 0.f, 0.f};
            const int64_t ob = (((gb >> 6) * nkc + (gk >> 5)) * 64 + (gb & 63)) * kBKf + (gk & 31);
            rb[r] = (gb < N && gk < K) ? *reinterpret_cast<const f32x4*>(Bt + ob) : f32x4{0.f, 0.f, 0.f, 0.f};
        }
    };
    auto store_stage = [&](int buf) {
#pragma unroll
        for (int r = 0; r < RC; ++r) {
            const int q = tid + 256 * r;
            const int off = f32_tile_slot(q / CPR, q % CPR);
            *reinterpret_cast<f32x4*>(&As[buf][off]) = ra[r];
            *reinterpret_cast<f32x4*>(&Bs[buf][off]) = rb[r];
        }
    };

    f32x4 acc[TW][TW];
#pragma unroll
    for (int i = 0; i < TW; ++i)
#pragma unroll
        for (int j = 0; j < TW; ++j) acc[i][j] = f32x4{0.f, 0.f, 0.f, 0.f};

    // The pipeline of gemm_kernel: compute on one LDS buffer while the next
    // stage is stored to the other and the one after is fetched.
    const int nk = (int)((K + kBKf - 1) / kBKf);
    load_stage(0);
    store_stage(0);
    if (nk > 1) load_stage(kBKf);
    __syncthreads();
    for (int kt = 0; kt < nk; ++kt) {
        const int cur = kt & 1;
        __builtin_amdgcn_s_setprio(1);
#pragma unroll
        for (int cc = 0; cc < CPR; cc += 4) {
            const int c = cc + (lane >> 4);
            f32x4 a4[TW], b4[TW];
#pragma unroll
            for (int i = 0; i < TW; ++i)
                a4[i] = *reinterpret_cast<const f32x4*>(&As[cur][f32_tile_slot(wm * (kBM / 2) + i * 16 + (lane & 15), c)]);
#pragma unroll
            for (int j = 0; j < TW; ++j)
                b4[j] = *reinterpret_cast<const f32x4*>(&Bs[cur][f32_tile_slot(wn * (kBN / 2) + j * 16 + (lane & 15), c)]);
#pragma unroll
            for (int s = 0; s < 4; ++s)
#pragma unroll
                for (int i = 0; i < TW; ++i)
#pragma unroll
                    for (int j = 0; j < TW; ++j)
                        acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x4f32(a4[i][s], b4[j][s], acc[i][j], 0, 0, 0);
        }
        __builtin_amdgcn_s_setprio(0);
        if (kt + 1 < nk) {
            store_stage(cur ^ 1);
            if (kt + 2 < nk) load_stage((int64_t)(kt + 2) * kBKf);
        }
        __syncthreads();
    }

    // Value r of lane l holds row 4*(l/16) + r, column l%16 (FP32 16x16 form).
#pragma unroll
    for (int i = 0; i < TW; ++i)
#pragma unroll
        for (int j = 0; j < TW; ++j) {
            const int64_t gc = col0 + wn * (kBN / 2) + j * 16 + (lane & 15);
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int64_t gr = row0 + wm * (kBM / 2) + i * 16 + 4 * (lane >> 4) + r;
                if (gr < M && gc < N) C[gr * ldc + gc] = (double)acc[i][j][r];
            }
        }
}

// BF16x3: A hi/lo (M x K, lda) with k contiguous, and B^T hi/lo (N x K) in
// blocked form: tiles of 64 rows (n) x 32 k, each 4 KB contiguous, tile
// (n / 64, k / 32) at ((n / 64) * nkc + k / 32) * 2048 elements, nkc =
// ceil(K / 32), row-major inside (k contiguous).  One 16-byte load gives an
// MFMA lane its 8 k-values, and a workgroup's B tile for one K step is two
// contiguous 4 KB blocks.
// K advances in steps of 32.  An LDS tile row is the row's 32 bf16 (64 B, no
// padding) as four 16-byte chunks; chunk c of row r sits in slot
// c ^ ((r >> 1) & 3).  Both the tile fills (4 lanes per row) and the
// fragment reads (one chunk of 16 consecutive rows per 16 lanes) are then
// free of bank conflicts on gfx950 (counted: 0, against 2 conflict cycles
// per access cycle with 80-byte padded rows).
// The tiles are filled by global_load_lds_dwordx4: one instruction of a
// wave writes 1 KB of LDS, 16 bytes per lane in lane order, here 16 tile
// rows, so lane l fetches the chunk that belongs in slot l & 3 of row
// l >> 2.  No registers or LDS store instructions are spent on staging
// (measured against staging through registers: 12 % faster at 4096^3, 5 %
// at 8192^3, 29 % for the 64 tile at 8192^3).  A
// lane whose chunk lies outside the matrix (row >= M or N, k >= K) fetches
// 16 zero bytes instead, so that the fills stay free of branches (with
// branches the compiler waits for every fill before the fragment reads).
constexpr int kBKb = 32;
constexpr int kRowB = kBKb;

__device__ __forceinline__ int bf16_tile_slot(int row, int chunk)
{
    return row * kRowB + ((chunk ^ ((row >> 1) & 3)) << 3);
}

typedef __attribute__((address_space(3))) void* lds_ptr_t;

// Source of the fills for chunks outside the matrix: 16 zero bytes.
__device__ __align__(16) const __bf16 kZeroChunk[8] = {};

// kWaves waves in a 2 x (kWaves / 2) grid, each computing a (kBM / 2) x
// (2 kBN / kWaves) piece of the tile: 4 waves for the 64 tile, 8 for the 128
// tile (64 x 32 per wave: four waves per SIMD instead of two at the same
// 64 KB of LDS; against four 64 x 64 waves the kernel is 5-8 % faster at
// 2048^3-8192^3, the product with its operand preparation 1-8 %).
template <int kBM, int kWaves>
__global__ __launch_bounds__(64 * kWaves) void gemm_bf16x3_kernel(const __bf16* __restrict__ Ahi,
                                                                  const __bf16* __restrict__ Alo, int64_t lda,
                                                                  const __bf16* __restrict__ Bhi,
                                                                  const __bf16* __restrict__ Blo, int64_t nkc,
                                                                  double* __restrict__ C, int64_t ldc, int64_t M,
                                                                  int64_t N, int64_t K)
{
    constexpr int kBN = kBM;
    constexpr int WNW = kWaves / 2;      // waves along n
    constexpr int PM = kBM / 2;          // rows of a wave's piece
    constexpr int PN = kBN / WNW;        // columns of a wave's piece
    constexpr int TWM = PM / 16, TWN = PN / 16;
    constexpr int RC = kBM / 16 / kWaves;  // 1 KB fills of each operand tile per wave
    static_assert(RC >= 1 && RC * 16 * kWaves == kBM && TWN >= 1, "whole fills and MFMA tiles per wave");
    // double-buffered operand tiles: [buffer][A hi, A lo, B hi, B lo], one
    // array (with four, the compiler waits for the other buffer's fills
    // before every fragment read)
    __shared__ __align__(16) __bf16 T[2][4][kBM * kRowB];

    const int ntm = (int)((M + kBM - 1) / kBM);
    const int ntn = (int)((N + kBN - 1) / kBN);
    int tm, tn;
    tile_of(blockIdx.x, gridDim.x, ntm, ntn, tm, tn);
    const int64_t row0 = (int64_t)tm * kBM, col0 = (int64_t)tn * kBN;

    const int tid = threadIdx.x;
    const int lane = tid & 63, wave = tid >> 6;
    const int wm = wave / WNW, wn = wave % WNW;

    // Fill of stage k0 into buffer buf: fill r of wave w covers tile rows
    // (w * RC + r) * 16 .. +15 of each of the four tiles.
    auto fill_stage = [&](int buf, int64_t k0) {
#pragma unroll
        for (int r = 0; r < RC; ++r) {
            const int rb = (wave * RC + r) * 16;
            const int row = rb + (lane >> 2);
            const int chunk = (lane & 3) ^ ((row >> 1) & 3);
            const int64_t gk = k0 + chunk * 8, ga = row0 + row, gb = col0 + row;
            const bool oka = ga < M && gk < K, okb = gb < N && gk < K;
            const int64_t oa = ga * lda + gk;
            const int64_t ob = (((gb >> 6) * nkc + (gk >> 5)) * 64 + (gb & 63)) * 32 + (gk & 31);
            // byte addresses, selected as integers (a pointer select becomes a branch)
            const uintptr_t z = reinterpret_cast<uintptr_t>(kZeroChunk);
            const uintptr_t pah = oka ? reinterpret_cast<uintptr_t>(Ahi + oa) : z;
            const uintptr_t pal = oka ? reinterpret_cast<uintptr_t>(Alo + oa) : z;
            const uintptr_t pbh = okb ? reinterpret_cast<uintptr_t>(Bhi + ob) : z;
            const uintptr_t pbl = okb ? reinterpret_cast<uintptr_t>(Blo + ob) : z;
            __builtin_amdgcn_global_load_lds(reinterpret_cast<const void*>(pah), (lds_ptr_t)&T[buf][0][rb * kRowB], 16, 0, 0);
            __builtin_amdgcn_global_load_lds(reinterpret_cast<const void*>(pal), (lds_ptr_t)&T[buf][1][rb * kRowB], 16, 0, 0);
            __builtin_amdgcn_global_load_lds(reinterpret_cast<const void*>(pbh), (lds_ptr_t)&T[buf][2][rb * kRowB], 16, 0, 0);
            __builtin_amdgcn_global_load_lds(reinterpret_cast<const void*>(pbl), (lds_ptr_t)&T[buf][3][rb * kRowB], 16, 0, 0);
        }
    };

    f32x4 acc[TWM][TWN];
#pragma unroll
    for (int i = 0; i < TWM; ++i)
#pragma unroll
        for (int j = 0; j < TWN; ++j) acc[i][j] = f32x4{0.f, 0.f, 0.f, 0.f};

    // Compute on one LDS buffer while the next stage fills the other.  The
    // fill of buffer b for stage kt+1 starts after the barrier that ends
    // stage kt-1, the last reader of b (here after this stage's fragment
    // reads are issued); every wave waits for its own fills (vmcnt) before
    // the barrier that publishes them.  The MFMAs run at raised wave
    // priority, so that a SIMD's waves that have their fragments issue
    // their products ahead of the others' reads and fills (with both: 2.5 %
    // faster at 8192^3, level at 4096^3).
    const int nk = (int)((K + kBKb - 1) / kBKb);
    fill_stage(0, 0);
    __builtin_amdgcn_s_waitcnt(kWaitVmcnt0);
    __syncthreads();
    for (int kt = 0; kt < nk; ++kt) {
        const int cur = kt & 1;
        // Operands of a 16x16x32 MFMA: lane l holds the 8 k-values
        // 8*(l/16) .. 8*(l/16)+7 of row (A) or column (B) l%16; any fixed
        // assignment of k to (lane group, element) works as long as A and B
        // use the same one.
        bf16x8 ah[TWM], al[TWM], bh[TWN], bl[TWN];
#pragma unroll
        for (int i = 0; i < TWM; ++i) {
            const int off = bf16_tile_slot(wm * PM + i * 16 + (lane & 15), lane >> 4);
            ah[i] = *reinterpret_cast<const bf16x8*>(&T[cur][0][off]);
            al[i] = *reinterpret_cast<const bf16x8*>(&T[cur][1][off]);
        }
#pragma unroll
        for (int j = 0; j < TWN; ++j) {
            const int off = bf16_tile_slot(wn * PN + j * 16 + (lane & 15), lane >> 4);
            bh[j] = *reinterpret_cast<const bf16x8*>(&T[cur][2][off]);
            bl[j] = *reinterpret_cast<const bf16x8*>(&T[cur][3][off]);
        }
        if (kt + 1 < nk) fill_stage(cur ^ 1, (int64_t)(kt + 1) * kBKb);
        __builtin_amdgcn_s_setprio(1);
#pragma unroll
        for (int i = 0; i < TWM; ++i)
#pragma unroll
            for (int j = 0; j < TWN; ++j) {
                acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(al[i], bh[j], acc[i][j], 0, 0, 0);
                acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah[i], bl[j], acc[i][j], 0, 0, 0);
                acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah[i], bh[j], acc[i][j], 0, 0, 0);
            }
        __builtin_amdgcn_s_setprio(0);
        __builtin_amdgcn_s_waitcnt(kWaitVmcnt0);
        __syncthreads();
    }

    // Value r of lane l holds row 4*(l/16) + r, column l%16 (BF16 16x16 form).
#pragma unroll
    for (int i = 0; i < TWM; ++i)
#pragma unroll
        for (int j = 0; j < TWN; ++j) {
            const int64_t gc = col0 + wn * PN + j * 16 + (lane & 15);
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int64_t gr = row0 + wm * PM + i * 16 + 4 * (lane >> 4) + r;
                if (gr < M && gc < N) C[gr * ldc + gc] = (double)acc[i][j][r];
            }
        }
}

// Loads the 64 (k) x 64 (n) binary64 tile of B at (k0, n0) into t, zeros
// beyond k and n: 16-byte loads, 32 lanes per row, all eight of a thread in
// flight before the LDS stores (21 % faster at 4096^2 and 30 % at 8192^2
// than one 8-byte load per lane).  n, ldb and B's address are even / 16-byte
// aligned, so a column pair never straddles n.
__device__ __forceinline__ void load_b_tile(const double* __restrict__ B, int64_t ldb, int64_t k, int64_t n, int64_t k0,
                                            int64_t n0, double (&t)[64][65])
{
    const int c2 = threadIdx.x & 31, ry = threadIdx.x >> 5;  // 32 column pairs x 8 rows
    f64x2 v[8];
#pragma unroll
    for (int r = 0; r < 8; ++r) {
        const int kk = ry + 8 * r;
        const bool ok = k0 + kk < k && n0 + 2 * c2 < n;
        v[r] = ok ? *reinterpret_cast<const f64x2*>(B + (k0 + kk) * ldb + n0 + 2 * c2) : f64x2{0.0, 0.0};
    }
#pragma unroll
    for (int r = 0; r < 8; ++r) {
        t[ry + 8 * r][2 * c2] = v[r][0];
        t[ry + 8 * r][2 * c2 + 1] = v[r][1];
    }
    __syncthreads();
}

// Dense binary64 (k x n, ldb) to its transpose in FP32 in the blocked form
// the FP32 contraction reads (64 x 32 tiles, see above), through a 64 (k) x
// 64 (n) LDS tile: the reads run along n, and each of the tile's two 32-k
// chunks is written as one contiguous 8 KB block (zeros beyond n and k,
// inside the padded workspace).
__global__ __launch_bounds__(256) void convert_f32_blocked_kernel(const double* __restrict__ B, int64_t ldb,
                                                                  float* __restrict__ out, int64_t k, int64_t n,
                                                                  int64_t nkc)
{
    __shared__ double t[64][65];
    // one-dimensional grid over the 64 x 64 tiles, n fastest (a grid's y
    // extent is limited to 65536, which would bound k)
    const int64_t ntn = (n + 63) / 64;
    const int64_t nb = (int64_t)blockIdx.x % ntn, k0 = ((int64_t)blockIdx.x / ntn) * 64, n0 = nb * 64;
    load_b_tile(B, ldb, k, n, k0, n0, t);
#pragma unroll
    for (int c = 0; c < 2; ++c) {
        const int64_t chunk = k0 / 32 + c;
        if (chunk >= nkc) break;
#pragma unroll
        for (int h = 0; h < 2; ++h) {  // 64 rows x 8 pieces of 4 k, two passes
            const int p = threadIdx.x + 256 * h, nl = p >> 3, kq = (p & 7) * 4;
            f32x4 v;
#pragma unroll
            for (int e = 0; e < 4; ++e) v[e] = (float)t[32 * c + kq + e][nl];
            *reinterpret_cast<f32x4*>(out + ((nb * nkc + chunk) * 64 + nl) * 32 + kq) = v;
        }
    }
}

// Dense binary64 (k x n, ldb) to its transpose split into BF16 hi + lo in
// the blocked form the BF16x3 contraction reads (64 x 32 tiles, see above),
// through a 64 (k) x 64 (n) LDS tile: the reads run along n, and each of the
// tile's two 32-k chunks is written as one contiguous 4 KB block per array
// (zeros beyond n and k, inside the padded workspace).
__global__ __launch_bounds__(256) void convert_bf16_split_blocked_kernel(const double* __restrict__ B, int64_t ldb,
                                                                         __bf16* __restrict__ hi,
                                                                         __bf16* __restrict__ lo, int64_t k,
                                                                         int64_t n, int64_t nkc)
{
    __shared__ double t[64][65];
    // one-dimensional grid over the 64 x 64 tiles, n fastest (a grid's y
    // extent is limited to 65536, which would bound k)
    const int64_t ntn = (n + 63) / 64;
    const int64_t nb = (int64_t)blockIdx.x % ntn, k0 = ((int64_t)blockIdx.x / ntn) * 64, n0 = nb * 64;
    load_b_tile(B, ldb, k, n, k0, n0, t);
    const int nl = threadIdx.x >> 2, kq = (threadIdx.x & 3) * 8;  // 64 rows x 4 pieces of 8 k
#pragma unroll
    for (int c = 0; c < 2; ++c) {
        const int64_t chunk = k0 / 32 + c;
        if (chunk >= nkc) break;
        bf16x8 h, l;
#pragma unroll
        for (int e = 0; e < 8; ++e) {
            const double x = t[32 * c + kq + e][nl];
            // hi = bf16(x), lo = bf16(x - hi), as the rebuild of A splits
            const __bf16 hb = (__bf16)(float)x;
            h[e] = hb;
            l[e] = (__bf16)(float)(x - (double)(float)hb);
        }
        const int64_t off = ((nb * nkc + chunk) * 64 + nl) * 32 + kq;
        *reinterpret_cast<bf16x8*>(hi + off) = h;
        *reinterpret_cast<bf16x8*>(lo + off) = l;
    }
}

namespace detail {

static unsigned gemm_grid(int64_t m, int64_t n, int tile)
{
    return (unsigned)(((m + tile - 1) / tile) * ((n + tile - 1) / tile));
}

// Row-major k x n operands already in the contraction's precision (a
// compressed B rebuilt straight into FP32, or into BF16 hi + lo) to the
// blocked B^T form of the converters above, through a 64 (k) x 64 (n) LDS
// tile.  Half the bytes of going through binary64: the rebuild writes 4
// bytes per element instead of 8, and this pass reads them.  The LDS rows
// hold 66 bf16 or 65 floats, so that the column reads of the four (BF16) or
// eight (FP32) k-pieces fall in different banks.
__global__ __launch_bounds__(256) void transpose_bf16_pair_blocked_kernel(const __bf16* __restrict__ hi_in,
                                                                          const __bf16* __restrict__ lo_in,
                                                                          int64_t ld, __bf16* __restrict__ hi,
                                                                          __bf16* __restrict__ lo, int64_t k,
                                                                          int64_t n, int64_t nkc)
{
    __shared__ uint32_t th[64][33], tl[64][33];  // 64 k-rows of 64 bf16 (+ 2 of padding)
    // one-dimensional grid over the 64 x 64 tiles, n fastest (a grid's y
    // extent is limited to 65536, which would bound k)
    const int64_t ntn = (n + 63) / 64;
    const int64_t nb = (int64_t)blockIdx.x % ntn, k0 = ((int64_t)blockIdx.x / ntn) * 64, n0 = nb * 64;
#pragma unroll
    for (int r = 0; r < 2; ++r) {  // 64 rows x 8 pieces of 8 bf16
        const int q = threadIdx.x + 256 * r, row = q >> 3, pc = q & 7;
        const bool ok = k0 + row < k && n0 + 8 * pc < n;
        const int64_t o = (k0 + row) * ld + n0 + 8 * pc;
        const uint4 vh = ok ? *reinterpret_cast<const uint4*>(hi_in + o) : uint4{0, 0, 0, 0};
        const uint4 vl = ok ? *reinterpret_cast<const uint4*>(lo_in + o) : uint4{0, 0, 0, 0};
        th[row][4 * pc] = vh.x, th[row][4 * pc + 1] = vh.y, th[row][4 * pc + 2] = vh.z, th[row][4 * pc + 3] = vh.w;
        tl[row][4 * pc] = vl.x, tl[row][4 * pc + 1] = vl.y, tl[row][4 * pc + 2] = vl.z, tl[row][4 * pc + 3] = vl.w;
    }
    __syncthreads();
    const auto* bh = reinterpret_cast<const uint16_t*>(&th[0][0]);
    const auto* bl = reinterpret_cast<const uint16_t*>(&tl[0][0]);
    const int nl = threadIdx.x >> 2, kq = (threadIdx.x & 3) * 8;  // 64 rows x 4 pieces of 8 k
#pragma unroll
    for (int c = 0; c < 2; ++c) {
        const int64_t chunk = k0 / 32 + c;
        if (chunk >= nkc) break;
        uint32_t h[4], l[4];
#pragma unroll
        for (int e = 0; e < 4; ++e) {
            const int r0 = 32 * c + kq + 2 * e;  // two k-values per dword
            h[e] = bh[r0 * 66 + nl] | ((uint32_t)bh[(r0 + 1) * 66 + nl] << 16);
            l[e] = bl[r0 * 66 + nl] | ((uint32_t)bl[(r0 + 1) * 66 + nl] << 16);
        }
        const int64_t off = ((nb * nkc + chunk) * 64 + nl) * 32 + kq;
        *reinterpret_cast<uint4*>(hi + off) = uint4{h[0], h[1], h[2], h[3]};
        *reinterpret_cast<uint4*>(lo + off) = uint4{l[0], l[1], l[2], l[3]};
    }
}

__global__ __launch_bounds__(256) void transpose_f32_blocked_kernel(const float* __restrict__ in, int64_t ld,
                                                                    float* __restrict__ out, int64_t k, int64_t n,
                                                                    int64_t nkc)
{
    __shared__ float t[64][65];
    // one-dimensional grid over the 64 x 64 tiles, n fastest (a grid's y
    // extent is limited to 65536, which would bound k)
    const int64_t ntn = (n + 63) / 64;
    const int64_t nb = (int64_t)blockIdx.x % ntn, k0 = ((int64_t)blockIdx.x / ntn) * 64, n0 = nb * 64;
#pragma unroll
    for (int r = 0; r < 4; ++r) {  // 64 rows x 16 pieces of 4 floats
        const int q = threadIdx.x + 256 * r, row = q >> 4, pc = q & 15;
        const bool ok = k0 + row < k && n0 + 4 * pc < n;
        const f32x4 v = ok ? *reinterpret_cast<const f32x4*>(in + (k0 + row) * ld + n0 + 4 * pc) : f32x4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
        for (int e = 0; e < 4; ++e) t[row][4 * pc + e] = v[e];
    }
    __syncthreads();
#pragma unroll
    for (int c = 0; c < 2; ++c) {
        const int64_t chunk = k0 / 32 + c;
        if (chunk >= nkc) break;
#pragma unroll
        for (int h = 0; h < 2; ++h) {  // 64 rows x 8 pieces of 4 k, two passes
            const int p = threadIdx.x + 256 * h, nl = p >> 3, kq = (p & 7) * 4;
            f32x4 v;
#pragma unroll
            for (int e = 0; e < 4; ++e) v[e] = t[32 * c + kq + e][nl];
            *reinterpret_cast<f32x4*>(out + ((nb * nkc + chunk) * 64 + nl) * 32 + kq) = v;
        }
    }
}

hipError_t launch_gemm_f64(const double* A, int64_t lda, const double* B, int64_t ldb, double* C, int64_t ldc,
                           int64_t m, int64_t n, int64_t k, int tile, hipStream_t st)
{
    if (tile == 64)
        gemm_kernel<double, 64><<<gemm_grid(m, n, 64), 256, 0, st>>>(A, lda, B, ldb, C, ldc, m, n, k);
    else
        gemm_kernel<double, 128><<<gemm_grid(m, n, 128), 256, 0, st>>>(A, lda, B, ldb, C, ldc, m, n, k);
    return hipGetLastError();
}

hipError_t launch_gemm_group(const GemmGroupItem* items, int n_items, int64_t workgroups, int tile, hipStream_t st)
{
    if (n_items == 0 || workgroups == 0) return hipSuccess;
    if (tile == 64)
        gemm_group_kernel<64><<<(unsigned)workgroups, 256, 0, st>>>(items, n_items);
    else
        gemm_group_kernel<128><<<(unsigned)workgroups, 256, 0, st>>>(items, n_items);
    return hipGetLastError();
}

hipError_t launch_gemm_f32(const float* A, int64_t lda, const float* Bt, double* C, int64_t ldc, int64_t m, int64_t n,
                           int64_t k, int tile, hipStream_t st)
{
    const int64_t nkc = f32_k_chunks(k);
    if (tile == 64)
        gemm_f32_kernel<64><<<gemm_grid(m, n, 64), 256, 0, st>>>(A, lda, Bt, nkc, C, ldc, m, n, k);
    else
        gemm_f32_kernel<128><<<gemm_grid(m, n, 128), 256, 0, st>>>(A, lda, Bt, nkc, C, ldc, m, n, k);
    return hipGetLastError();
}

hipError_t launch_gemm_bf16x3(const __bf16* Ahi, const __bf16* Alo, int64_t lda, const __bf16* Bthi,
                              const __bf16* Btlo, double* C, int64_t ldc, int64_t m, int64_t n, int64_t k, int tile,
                              hipStream_t st)
{
    const int64_t nkc = bf16_k_chunks(k);
    if (tile == 64)
        gemm_bf16x3_kernel<64, 4><<<gemm_grid(m, n, 64), 256, 0, st>>>(Ahi, Alo, lda, Bthi, Btlo, nkc, C, ldc, m, n, k);
    else
        gemm_bf16x3_kernel<128, 8><<<gemm_grid(m, n, 128), 512, 0, st>>>(Ahi, Alo, lda, Bthi, Btlo, nkc, C, ldc, m, n, k);
    return hipGetLastError();
}

hipError_t launch_convert_f32_blocked(const double* B, int64_t ldb, float* out, int64_t k, int64_t n, hipStream_t st)
{
    if (k == 0 || n == 0) return hipSuccess;
    const unsigned grid = (unsigned)(((n + 63) / 64) * ((k + 63) / 64));
    convert_f32_blocked_kernel<<<grid, 256, 0, st>>>(B, ldb, out, k, n, f32_k_chunks(k));
    return hipGetLastError();
}

hipError_t launch_convert_bf16_split_blocked(const double* B, int64_t ldb, __bf16* hi, __bf16* lo, int64_t k,
                                             int64_t n, hipStream_t st)
{
    if (k == 0 || n == 0) return hipSuccess;
    const unsigned grid = (unsigned)(((n + 63) / 64) * ((k + 63) / 64));
    convert_bf16_split_blocked_kernel<<<grid, 256, 0, st>>>(B, ldb, hi, lo, k, n, bf16_k_chunks(k));
    return hipGetLastError();
}

hipError_t launch_transpose_bf16_pair_blocked(const __bf16* hi_in, const __bf16* lo_in, int64_t ld, __bf16* hi,
                                              __bf16* lo, int64_t k, int64_t n, hipStream_t st)
{
    if (k == 0 || n == 0) return hipSuccess;
    const unsigned grid = (unsigned)(((n + 63) / 64) * ((k + 63) / 64));
    transpose_bf16_pair_blocked_kernel<<<grid, 256, 0, st>>>(hi_in, lo_in, ld, hi, lo, k, n, bf16_k_chunks(k));
    return hipGetLastError();
}

hipError_t launch_transpose_f32_blocked(const float* in, int64_t ld, float* out, int64_t k, int64_t n, hipStream_t st)
{
    if (k == 0 || n == 0) return hipSuccess;
    const unsigned grid = (unsigned)(((n + 63) / 64) * ((k + 63) / 64));
    transpose_f32_blocked_kernel<<<grid, 256, 0, st>>>(in, ld, out, k, n, f32_k_chunks(k));
    return hipGetLastError();
}

}  // namespace detail
}  // namespace blaz
