// Dense contraction of blaz_matmul on the matrix cores.
//
// The paper's matrix multiplication rebuilds every block once and then
// multiplies (last paragraph of Section "Basic Linear Algebra Algorithms").
// The rebuild is the decompression kernel; this file holds the product
// C = A B of the rebuilt operands: binary64 in, binary64 out, on
// v_mfma_f64_16x16x4_f64.
//
// Tiling: a 256-thread workgroup computes a 128x128 tile of C; its four
// waves each own a 64x64 quadrant as 4x4 MFMA tiles of 16x16.  K advances in
// steps of 16 through LDS; the next step's global loads are issued into
// registers before the current step's MFMAs, so HBM/L2 latency overlaps the
// matrix math.  Workgroup ids are remapped so that each XCD (the hardware
// deals workgroups to the 8 XCDs round-robin) works on a contiguous group of
// tiles that share rows of A and columns of B in its own L2.
#include <hip/hip_runtime.h>

#include "blaz_internal.hpp"

namespace blaz {

typedef double f64x4 __attribute__((ext_vector_type(4)));

constexpr int kBM = 128, kBN = 128, kBK = 16;
constexpr int kPad = 16;  // doubles; 1152-byte LDS rows put k and k+1 on disjoint banks

// Tile (tm, tn) for workgroup `wg` of `nwg`: contiguous ranges per XCD, then
// groups of 8 tile rows walked column by column for L2 reuse.
__device__ __forceinline__ void tile_of(int wg, int nwg, int ntm, int ntn, int& tm, int& tn)
{
    if (nwg % 8 == 0) wg = (wg % 8) * (nwg / 8) + wg / 8;
    constexpr int kGroup = 8;
    const int per_group = kGroup * ntn;
    const int g = wg / per_group;
    const int first = g * kGroup;
    const int rows = min(ntm - first, kGroup);
    const int r = wg - g * per_group;
    tm = first + r % rows;
    tn = r / rows;
}

__global__ __launch_bounds__(256) void gemm_f64_kernel(const double* __restrict__ A, int64_t lda,
                                                       const double* __restrict__ B, int64_t ldb,
                                                       double* __restrict__ C, int64_t ldc, int64_t M, int64_t N,
                                                       int64_t K)
{
    __shared__ double As[kBK][kBM + kPad];  // A tile stored k-major (transposed)
    __shared__ double Bs[kBK][kBN + kPad];

    const int ntm = (int)((M + kBM - 1) / kBM);
    const int ntn = (int)((N + kBN - 1) / kBN);
    int tm, tn;
    tile_of(blockIdx.x, gridDim.x, ntm, ntn, tm, tn);
    const int64_t row0 = (int64_t)tm * kBM, col0 = (int64_t)tn * kBN;

    const int tid = threadIdx.x;
    const int lane = tid & 63, wave = tid >> 6;
    const int wm = wave >> 1, wn = wave & 1;

    // Global -> register staging: 4 double2 of A and 4 of B per thread.
    double2 ra[4], rb[4];
    auto load_stage = [&](int64_t k0) {
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            const int q = tid + 256 * r;
            const int am = q >> 3, ak = (q & 7) * 2;          // A: 128 rows x 8 double2
            const int64_t gr = row0 + am, gk = k0 + ak;
            ra[r] = (gr < M && gk < K) ? *reinterpret_cast<const double2*>(A + gr * lda + gk) : double2{0.0, 0.0};
            const int bk = q >> 6, bn = (q & 63) * 2;         // B: 16 rows x 64 double2
            const int64_t hk = k0 + bk, hn = col0 + bn;
            rb[r] = (hk < K && hn < N) ? *reinterpret_cast<const double2*>(B + hk * ldb + hn) : double2{0.0, 0.0};
        }
    };
    auto store_stage = [&]() {
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            const int q = tid + 256 * r;
            const int am = q >> 3, ak = (q & 7) * 2;
            As[ak][am] = ra[r].x;
            As[ak + 1][am] = ra[r].y;
            const int bk = q >> 6, bn = (q & 63) * 2;
            *reinterpret_cast<double2*>(&Bs[bk][bn]) = rb[r];
        }
    };

    f64x4 acc[4][4];
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < 4; ++j) acc[i][j] = f64x4{0.0, 0.0, 0.0, 0.0};

    const int nk = (int)((K + kBK - 1) / kBK);
    load_stage(0);
    for (int kt = 0; kt < nk; ++kt) {
        __syncthreads();
        store_stage();
        __syncthreads();
        if (kt + 1 < nk) load_stage((int64_t)(kt + 1) * kBK);
#pragma unroll
        for (int kk = 0; kk < kBK; kk += 4) {
            // A operand of a 16x16x4 MFMA: lane holds A[m = lane%16][k = lane/16];
            // B operand: lane holds B[k = lane/16][n = lane%16].
            double a[4], b[4];
#pragma unroll
            for (int i = 0; i < 4; ++i) a[i] = As[kk + (lane >> 4)][wm * 64 + i * 16 + (lane & 15)];
#pragma unroll
            for (int j = 0; j < 4; ++j) b[j] = Bs[kk + (lane >> 4)][wn * 64 + j * 16 + (lane & 15)];
#pragma unroll
            for (int i = 0; i < 4; ++i)
#pragma unroll
                for (int j = 0; j < 4; ++j) acc[i][j] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[i], b[j], acc[i][j], 0, 0, 0);
        }
    }

    // Accumulator layout of v_mfma_f64_16x16x4_f64: value r (0..3) of a lane
    // holds D[4*r + lane/16][lane%16] (unlike the FP32/BF16 16x16 forms,
    // whose value r holds row 4*(lane/16) + r).
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            const int64_t gc = col0 + wn * 64 + j * 16 + (lane & 15);
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int64_t gr = row0 + wm * 64 + i * 16 + 4 * r + (lane >> 4);
                if (gr < M && gc < N) C[gr * ldc + gc] = acc[i][j][r];
            }
        }
}

namespace detail {

hipError_t launch_gemm_f64(const double* A, int64_t lda, const double* B, int64_t ldb, double* C, int64_t ldc,
                           int64_t m, int64_t n, int64_t k, hipStream_t st)
{
    const int64_t tiles = ((m + kBM - 1) / kBM) * ((n + kBN - 1) / kBN);
    gemm_f64_kernel<<<(unsigned)tiles, 256, 0, st>>>(A, lda, B, ldb, C, ldc, m, n, k);
    return hipGetLastError();
}

}  // namespace detail
}  // namespace blaz
