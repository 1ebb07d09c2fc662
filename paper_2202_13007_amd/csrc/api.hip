// The C ABI of libblaz (include/libblaz.h): argument validation, then the
// kernel launches.  Nothing here allocates, synchronizes or keeps state.
#include <hip/hip_runtime.h>

#include <atomic>
#include <cstdint>
#include <mutex>

#include "blaz_internal.hpp"
#include "blaz_validate.hpp"

#define BLAZ_API extern "C" __attribute__((visibility("default")))

using namespace blaz::validate;
using blaz::detail::launch_add;


BLAZ_API int64_t blaz_block_count(int64_t rows, int64_t cols)
{
    if (blaz_status st = check_shape(rows, cols)) return st;
    return (rows / 8) * (cols / 8);
}

BLAZ_API size_t blaz_compressed_bytes(int64_t rows, int64_t cols)
{
    if (check_shape(rows, cols) != BLAZ_OK) return 0;
    return (size_t)((rows / 8) * (cols / 8) * kRecordBytes);
}

BLAZ_API int64_t blaz_code_stride(int64_t lines)
{
    if (!valid_lines(lines)) return BLAZ_ERR_ARG;
    return code_stride(lines == 0 ? 2 : (int)lines);
}

BLAZ_API size_t blaz_compressed_bytes_lines(int64_t rows, int64_t cols, int64_t lines)
{
    if (check_shape(rows, cols) != BLAZ_OK || !valid_lines(lines)) return 0;
    return (size_t)((rows / 8) * (cols / 8) * (17 + code_stride(lines == 0 ? 2 : (int)lines)));
}

BLAZ_API blaz_status blaz_compress(const double* A, int64_t lda, const blaz_matrix* out, blaz_precision prec,
                                   uint8_t* psi, hipStream_t stream)
{
    bool empty;
    if (blaz_status st = validate_compress(A, lda, out, prec, psi, &empty)) return st;
    if (empty) return BLAZ_OK;
    if (prec == BLAZ_PREC_FP64) return hip_status(blaz::detail::launch_compress_f64(A, lda, *out, psi, stream));
    return hip_status(blaz::detail::launch_compress_mixed(A, lda, *out, psi, prec, stream));
}

BLAZ_API blaz_status blaz_compress_predicted(const double* A, int64_t lda, const blaz_matrix* out, uint8_t* psi,
                                             hipStream_t stream)
{
    bool empty;
    if (blaz_status st = validate_compress(A, lda, out, BLAZ_PREC_FP64, psi, &empty)) return st;
    if (lines_of(*out) != 2) return BLAZ_ERR_UNSUPPORTED;
    if (empty) return BLAZ_OK;
    return hip_status(blaz::detail::launch_compress_predicted(A, lda, *out, psi, stream));
}

BLAZ_API blaz_status blaz_decompress(const blaz_matrix* in, double* A, int64_t lda, hipStream_t stream)
{
    bool empty;
    if (blaz_status st = validate_decompress(in, A, lda, &empty)) return st;
    if (empty) return BLAZ_OK;
    return hip_status(blaz::detail::launch_decompress(*in, A, lda, stream));
}

static blaz_status add_or_sub(const blaz_matrix* x, const blaz_matrix* y, const blaz_matrix* z, bool sub,
                              hipStream_t stream)
{
    bool empty;
    if (blaz_status st = validate_add(x, y, z, &empty)) return st;
    if (empty) return BLAZ_OK;
    return hip_status(launch_add(*x, *y, *z, sub, stream));
}

BLAZ_API blaz_status blaz_add(const blaz_matrix* x, const blaz_matrix* y, const blaz_matrix* z, hipStream_t stream)
{
    return add_or_sub(x, y, z, false, stream);
}

BLAZ_API blaz_status blaz_sub(const blaz_matrix* x, const blaz_matrix* y, const blaz_matrix* z, hipStream_t stream)
{
    return add_or_sub(x, y, z, true, stream);
}

BLAZ_API blaz_status blaz_scale(const blaz_matrix* x, double c, const blaz_matrix* z, hipStream_t stream)
{
    bool empty;
    if (blaz_status st = validate_scale(x, z, &empty)) return st;
    if (empty) return BLAZ_OK;
    return hip_status(blaz::detail::launch_scale(*x, c, *z, stream));
}

BLAZ_API blaz_status blaz_diagnose(const blaz_matrix* x, uint64_t* counters, hipStream_t stream)
{
    if (blaz_status st = check_matrix(x)) return st;
    if (nblocks(*x) == 0) return BLAZ_OK;
    if (!counters) return BLAZ_ERR_NULL;
    if (!aligned(counters, 8)) return BLAZ_ERR_ALIGN;
    if (overlaps_matrix(span(counters, 32), *x)) return BLAZ_ERR_ARG;
    return hip_status(blaz::detail::launch_diagnose(*x, counters, stream));
}

BLAZ_API blaz_status blaz_dot(const blaz_matrix* x, const int64_t* xrow, const blaz_matrix* y, const int64_t* ycol,
                              int64_t count, double* out, hipStream_t stream)
{
    bool empty;
    if (blaz_status st = validate_dot(x, xrow, y, ycol, count, out, &empty)) return st;
    if (empty) return BLAZ_OK;
    return hip_status(blaz::detail::launch_dot(*x, xrow, *y, ycol, count, out, stream));
}

BLAZ_API blaz_status blaz_dot_dense(const blaz_matrix* x, const int64_t* xrow, const double* v, int64_t ldv,
                                    int64_t count, double* out, hipStream_t stream)
{
    bool empty;
    if (blaz_status st = validate_dot_dense(x, xrow, v, ldv, count, out, &empty)) return st;
    if (empty) return BLAZ_OK;
    return hip_status(blaz::detail::launch_dot_dense(*x, xrow, v, ldv, count, out, stream));
}

// Workspace regions of blaz_matmul, each 256-byte aligned: the rebuilt A
// and the prepared B in the contraction's operand form, plus, for a
// compressed B and a contraction that is not binary64, a staging area where
// B is rebuilt row-major in the operand precision (FP32, or BF16 hi and lo).
struct MatmulWorkspace {
    size_t a_bytes, b_bytes, tmp_bytes;
    size_t total() const { return a_bytes + b_bytes + tmp_bytes; }
};

static MatmulWorkspace matmul_workspace(int64_t m, int64_t n, int64_t k, bool b_compressed, blaz_precision prec)
{
    const size_t mk = (size_t)m * (size_t)k, kn = (size_t)k * (size_t)n;
    MatmulWorkspace w{0, 0, 0};
    switch (prec) {
        case BLAZ_PREC_FP64:
            w.a_bytes = round_up(mk * 8, 256);
            w.b_bytes = b_compressed ? round_up(kn * 8, 256) : 0;
            break;
        case BLAZ_PREC_FP32:
            w.a_bytes = round_up(mk * 4, 256);
            w.b_bytes = round_up((size_t)blaz::detail::f32_blocked_elems(k, n) * 4, 256);  // blocked B^T
            w.tmp_bytes = b_compressed ? round_up(kn * 4, 256) : 0;  // B rebuilt in FP32
            break;
        case BLAZ_PREC_BF16X3:
            w.a_bytes = 2 * round_up(mk * 2, 256);  // hi, lo
            w.b_bytes = 2 * round_up((size_t)blaz::detail::bf16_blocked_elems(k, n) * 2, 256);  // blocked B^T
            w.tmp_bytes = b_compressed ? round_up(kn * 4, 256) : 0;  // B rebuilt in BF16 hi, lo
            break;
    }
    return w;
}

static bool valid_precision(blaz_precision prec)
{
    return prec == BLAZ_PREC_FP64 || prec == BLAZ_PREC_FP32 || prec == BLAZ_PREC_BF16X3;
}

BLAZ_API size_t blaz_matmul_workspace_bytes(int64_t m, int64_t n, int64_t k, int b_compressed, blaz_precision prec)
{
    if (check_shape(m, k) != BLAZ_OK || check_shape(k, n) != BLAZ_OK || !valid_precision(prec)) return 0;
    return matmul_workspace(m, n, k, b_compressed != 0, prec).total();
}

namespace blaz {
namespace detail {

int device_cu_count()
{
    // looked up once per device: not a stream operation, so later calls may
    // be made while a stream is being captured into a graph
    static std::atomic<int> cu_count[64];
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) return 0;
    int cus = dev < 64 ? cu_count[dev].load() : 0;
    if (cus == 0) {
        if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess) return 0;
        if (dev < 64) cu_count[dev].store(cus);
    }
    return cus;
}

}  // namespace detail
}  // namespace blaz

// Every launch of a product fits one dispatch: the contraction's grid of
// output tiles (512 lanes per workgroup for the BF16x3 128 tile, 256
// otherwise), the rebuild of A (and of a compressed B) in 64-block waves,
// and the low-precision preparation of B in 64 x 64 tiles of 256 lanes.
static bool matmul_fits_dispatch(int64_t m, int64_t n, int64_t k, bool b_compressed, blaz_precision prec, int tile)
{
    const int64_t tiles = ((m + tile - 1) / tile) * ((n + tile - 1) / tile);
    const int lanes = (prec == BLAZ_PREC_BF16X3 && tile == 128) ? 512 : 256;
    if (!fits_dispatch(tiles, lanes)) return false;
    if (k == 0) return true;
    const int64_t waves = ((m / 8) * (k / 8) + 63) / 64 + (b_compressed ? ((k / 8) * (n / 8) + 63) / 64 : 0);
    if (!fits_dispatch(waves, 64)) return false;
    if (prec != BLAZ_PREC_FP64 && !fits_dispatch(((n + 63) / 64) * ((k + 63) / 64), 256)) return false;
    return true;
}

// The library's tile choice: the 128 tile once it gives every compute unit a
// workgroup, the 64 tile (four times as many workgroups) below that.
int blaz::detail::default_gemm_tile(int64_t m, int64_t n)
{
    const int64_t tiles128 = ((m + 127) / 128) * ((n + 127) / 128);
    const int cus = blaz::detail::device_cu_count();
    return tiles128 >= (cus > 0 ? cus : 256) ? 128 : 64;
}
using blaz::detail::default_gemm_tile;

static blaz_status matmul_impl(const blaz_matrix* a, const blaz_matrix* b, const double* bdense, int64_t n,
                               int64_t ldb, double* c, int64_t ldc, blaz_precision prec, void* workspace,
                               size_t ws_bytes, int32_t tile, hipStream_t stream)
{
    if (tile != 0 && tile != 64 && tile != 128) return BLAZ_ERR_ARG;
    if (blaz_status st = check_matrix(a)) return st;
    if (b && bdense) return BLAZ_ERR_ARG;  // exactly one form of B
    if (!b && !bdense && a->cols > 0) return BLAZ_ERR_NULL;
    if (!valid_precision(prec)) return BLAZ_ERR_ARG;
    const int64_t m = a->rows, k = a->cols;
    if (b) {
        if (blaz_status st = check_matrix(b)) return st;
        if (b->rows != k || b->cols != n) return BLAZ_ERR_MISMATCH;
    }
    if (check_shape(k, n) != BLAZ_OK) return BLAZ_ERR_SHAPE;
    if (m == 0 || n == 0) return BLAZ_OK;
    if (!c) return BLAZ_ERR_NULL;
    if (blaz_status st = check_dense(m, n, ldc)) return st;
    if (!aligned(c, 8)) return BLAZ_ERR_ALIGN;
    if (!b && k > 0) {
        if (blaz_status st = check_dense(k, n, ldb)) return st;
        if (!aligned(bdense, 16) || ldb % 2 != 0) return BLAZ_ERR_ALIGN;
    }
    const MatmulWorkspace wl = matmul_workspace(m, n, k, b != nullptr, prec);
    const size_t need = wl.total();
    if (k > 0 && (!workspace || ws_bytes < need)) return BLAZ_ERR_WORKSPACE;
    if (k > 0 && !aligned(workspace, 256)) return BLAZ_ERR_ALIGN;
    const Range rc = span(c, dense_span(m, n, ldc));
    if (overlaps_matrix(rc, *a) || (b && overlaps_matrix(rc, *b)) ||
        (bdense && overlap(rc, span(bdense, dense_span(k, n, ldb)))) ||
        (k > 0 && overlap(rc, span(workspace, (int64_t)need))))
        return BLAZ_ERR_ARG;
    // the rebuilds write the workspace while the inputs are read
    if (k > 0) {
        const Range rw = span(workspace, (int64_t)need);
        if (overlaps_matrix(rw, *a) || (b && overlaps_matrix(rw, *b)) ||
            (bdense && overlap(rw, span(bdense, dense_span(k, n, ldb)))))
            return BLAZ_ERR_ARG;
    }
    // k == 0: the product is the zero matrix; the contraction kernel with an
    // empty K loop writes exactly that and reads nothing.
    if (tile == 0) tile = default_gemm_tile(m, n);
    if (!matmul_fits_dispatch(m, n, k, b != nullptr, prec, tile)) return BLAZ_ERR_SHAPE;
    if (k == 0) return hip_status(blaz::detail::launch_gemm_f64(nullptr, 0, nullptr, 0, c, ldc, m, n, 0, tile, stream));

    char* ws = static_cast<char*>(workspace);
    char* wa = ws;
    char* wb = ws + wl.a_bytes;
    char* wtmp = ws + wl.a_bytes + wl.b_bytes;
    using namespace blaz::detail;

    // With B compressed too, both rebuilds go into one launch.
    if (prec == BLAZ_PREC_FP64) {
        double* A64 = reinterpret_cast<double*>(wa);
        const double* bop = bdense;
        int64_t ldbop = ldb;
        if (b) {
            double* B64 = reinterpret_cast<double*>(wb);
            if (hipError_t e = launch_decompress_pair(*a, A64, k, *b, B64, n, stream)) return hip_status(e);
            bop = B64;
            ldbop = n;
        } else if (hipError_t e = launch_decompress(*a, A64, k, stream)) {
            return hip_status(e);
        }
        return hip_status(launch_gemm_f64(A64, k, bop, ldbop, c, ldc, m, n, k, tile, stream));
    }

    // Low-precision contractions: a dense B is converted to the operand
    // form; a compressed B is rebuilt row-major in the operand precision
    // (the same values and the same split as converting its binary64
    // rebuild) and then transposed into the operand form.
    if (prec == BLAZ_PREC_FP32) {
        float* A32 = reinterpret_cast<float*>(wa);
        float* B32 = reinterpret_cast<float*>(wb);
        if (b) {
            float* T32 = reinterpret_cast<float*>(wtmp);
            if (hipError_t e = launch_decompress_pair_f32(*a, A32, k, *b, T32, n, stream)) return hip_status(e);
            if (hipError_t e = launch_transpose_f32_blocked(T32, n, B32, k, n, stream)) return hip_status(e);
        } else {
            if (hipError_t e = launch_decompress_f32(*a, A32, k, stream)) return hip_status(e);
            if (hipError_t e = launch_convert_f32_blocked(bdense, ldb, B32, k, n, stream)) return hip_status(e);
        }
        return hip_status(launch_gemm_f32(A32, k, B32, c, ldc, m, n, k, tile, stream));
    }
    __bf16* Ahi = reinterpret_cast<__bf16*>(wa);
    __bf16* Alo = reinterpret_cast<__bf16*>(wa + wl.a_bytes / 2);
    __bf16* Bhi = reinterpret_cast<__bf16*>(wb);
    __bf16* Blo = reinterpret_cast<__bf16*>(wb + wl.b_bytes / 2);
    if (b) {
        __bf16* Thi = reinterpret_cast<__bf16*>(wtmp);
        __bf16* Tlo = Thi + k * n;
        if (hipError_t e = launch_decompress_pair_bf16_split(*a, Ahi, Alo, k, *b, Thi, Tlo, n, stream))
            return hip_status(e);
        if (hipError_t e = launch_transpose_bf16_pair_blocked(Thi, Tlo, n, Bhi, Blo, k, n, stream))
            return hip_status(e);
    } else {
        if (hipError_t e = launch_decompress_bf16_split(*a, Ahi, Alo, k, stream)) return hip_status(e);
        if (hipError_t e = launch_convert_bf16_split_blocked(bdense, ldb, Bhi, Blo, k, n, stream))
            return hip_status(e);
    }
    return hip_status(launch_gemm_bf16x3(Ahi, Alo, k, Bhi, Blo, c, ldc, m, n, k, tile, stream));
}

BLAZ_API blaz_status blaz_matmul(const blaz_matrix* a, const blaz_matrix* b, const double* bdense, int64_t n,
                                 int64_t ldb, double* c, int64_t ldc, blaz_precision prec, void* workspace,
                                 size_t ws_bytes, hipStream_t stream)
{
    return matmul_impl(a, b, bdense, n, ldb, c, ldc, prec, workspace, ws_bytes, 0, stream);
}

BLAZ_API blaz_status blaz_matmul_tiled(const blaz_matrix* a, const blaz_matrix* b, const double* bdense, int64_t n,
                                       int64_t ldb, double* c, int64_t ldc, blaz_precision prec, void* workspace,
                                       size_t ws_bytes, int32_t tile, hipStream_t stream)
{
    return matmul_impl(a, b, bdense, n, ldb, c, ldc, prec, workspace, ws_bytes, tile, stream);
}

// ---------------------------------------------------------------------------
// The product without a caller workspace.  Its workspace is `scratch`, a
// file-scope device array that every device the library runs on holds until
// the process ends; host code reaches it only through the address that
// hipGetSymbolAddress returns for the current device.
// ---------------------------------------------------------------------------
static __device__ __align__(256) unsigned char scratch[BLAZ_STATIC_SCRATCH_BYTES];

// This device's address of `scratch`, looked up on the first call on the
// device (with that device current) and kept per device.
static blaz_status static_scratch(void** out)
{
    constexpr int kMaxDevices = 64;
    static std::atomic<void*> addr[kMaxDevices];
    static std::mutex lookup;
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) return BLAZ_ERR_HIP;
    if (dev < 0 || dev >= kMaxDevices) return BLAZ_ERR_UNSUPPORTED;
    void* p = addr[dev].load(std::memory_order_acquire);
    if (!p) {
        std::lock_guard<std::mutex> hold(lookup);
        p = addr[dev].load(std::memory_order_acquire);
        if (!p) {
            if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess || !p) return BLAZ_ERR_HIP;
            addr[dev].store(p, std::memory_order_release);
        }
    }
    *out = p;
    return BLAZ_OK;
}

BLAZ_API blaz_status blaz_matmul_static(const blaz_matrix* a, const blaz_matrix* b, const double* bdense, int64_t n,
                                        int64_t ldb, double* c, int64_t ldc, blaz_precision prec, hipStream_t stream)
{
    // a request whose workspace would not fit is refused before the lookup
    if (a && check_matrix(a) == BLAZ_OK && valid_precision(prec) && check_shape(a->cols, n) == BLAZ_OK &&
        matmul_workspace(a->rows, n, a->cols, b != nullptr, prec).total() > BLAZ_STATIC_SCRATCH_BYTES)
        return BLAZ_ERR_TOO_LARGE;
    void* ws = nullptr;
    if (blaz_status st = static_scratch(&ws)) return st;
    return matmul_impl(a, b, bdense, n, ldb, c, ldc, prec, ws, BLAZ_STATIC_SCRATCH_BYTES, 0, stream);
}

// The compressed-output product: the contraction writes C into a staging
// region after the contraction's own workspace, then C is compressed.
static size_t matmul_compressed_workspace(int64_t m, int64_t n, int64_t k, bool b_compressed, blaz_precision prec)
{
    return matmul_workspace(m, n, k, b_compressed, prec).total() + round_up((size_t)m * (size_t)n * 8, 256);
}

BLAZ_API size_t blaz_matmul_compressed_workspace_bytes(int64_t m, int64_t n, int64_t k, int b_compressed,
                                                       blaz_precision prec)
{
    if (check_shape(m, k) != BLAZ_OK || check_shape(k, n) != BLAZ_OK || !valid_precision(prec)) return 0;
    return matmul_compressed_workspace(m, n, k, b_compressed != 0, prec);
}

BLAZ_API blaz_status blaz_matmul_compressed(const blaz_matrix* a, const blaz_matrix* b, const double* bdense,
                                            int64_t n, int64_t ldb, blaz_matrix* c, blaz_precision prec,
                                            void* workspace, size_t ws_bytes, int32_t tile, hipStream_t stream)
{
    if (tile != 0 && tile != 64 && tile != 128) return BLAZ_ERR_ARG;
    if (blaz_status st = check_matrix(a)) return st;
    if (blaz_status st = check_matrix(c)) return st;
    if (b && bdense) return BLAZ_ERR_ARG;
    if (!b && !bdense && a->cols > 0) return BLAZ_ERR_NULL;
    if (!valid_precision(prec)) return BLAZ_ERR_ARG;
    const int64_t m = a->rows, k = a->cols;
    if (b) {
        if (blaz_status st = check_matrix(b)) return st;
        if (b->rows != k || b->cols != n) return BLAZ_ERR_MISMATCH;
    }
    if (check_shape(k, n) != BLAZ_OK) return BLAZ_ERR_SHAPE;
    if (c->rows != m || c->cols != n) return BLAZ_ERR_MISMATCH;
    if (m == 0 || n == 0) return BLAZ_OK;
    if (!b && k > 0) {
        if (blaz_status st = check_dense(k, n, ldb)) return st;
        if (!aligned(bdense, 16) || ldb % 2 != 0) return BLAZ_ERR_ALIGN;
    }
    const size_t mm = matmul_workspace(m, n, k, b != nullptr, prec).total();
    const size_t need = matmul_compressed_workspace(m, n, k, b != nullptr, prec);
    if (!workspace || ws_bytes < need) return BLAZ_ERR_WORKSPACE;
    if (!aligned(workspace, 256)) return BLAZ_ERR_ALIGN;
    const Range rw = span(workspace, (int64_t)need);
    if (overlaps_matrix(rw, *c) || overlaps_matrix(rw, *a) || (b && overlaps_matrix(rw, *b)) ||
        (bdense && overlap(rw, span(bdense, dense_span(k, n, ldb)))))
        return BLAZ_ERR_ARG;
    Range rc[4];
    ranges(*c, rc);
    for (const Range& r : rc)
        if (overlaps_matrix(r, *a) || (b && overlaps_matrix(r, *b)) ||
            (bdense && overlap(r, span(bdense, dense_span(k, n, ldb)))))
            return BLAZ_ERR_ARG;
    double* stage = reinterpret_cast<double*>(static_cast<char*>(workspace) + mm);
    if (blaz_status st = matmul_impl(a, b, bdense, n, ldb, stage, n, prec, workspace, mm, tile, stream)) return st;
    return hip_status(blaz::detail::launch_compress_f64(stage, n, *c, nullptr, stream));
}

BLAZ_API const char* blaz_status_string(blaz_status status)
{
    switch (status) {
        case BLAZ_OK: return "success";
        case BLAZ_ERR_NULL: return "a required pointer is NULL";
        case BLAZ_ERR_SHAPE: return "invalid shape: dimensions must be non-negative multiples of 8 and ld >= cols";
        case BLAZ_ERR_MISMATCH: return "operand shapes do not agree";
        case BLAZ_ERR_ALIGN: return "a pointer or leading dimension is not suitably aligned";
        case BLAZ_ERR_ARG: return "invalid argument (count, enum value, or overlapping buffers)";
        case BLAZ_ERR_UNSUPPORTED: return "request not supported by the library";
        case BLAZ_ERR_WORKSPACE: return "workspace missing or too small";
        case BLAZ_ERR_HIP: return "the HIP runtime reported an error";
        case BLAZ_ERR_TOO_LARGE:
            return "the request needs more than the library's static scratch (BLAZ_STATIC_SCRATCH_BYTES); "
                   "pass a workspace to blaz_matmul instead";
    }
    return "unknown status";
}
