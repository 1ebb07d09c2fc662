// Grouped binary64 products: many matrix multiplications (every block
// rebuilt once, then the product; last paragraph of Section "Basic Linear
// Algebra Algorithms") in at most three launches.  The plan lists one
// rebuild job per compressed operand (the rebuild launch's waves are dealt to
// the jobs by a prefix sum) and one contraction item per product (the
// contraction launch's workgroups are dealt by a prefix sum of output tiles,
// each product's first workgroup a multiple of 8 so that its tile order is the
// standalone kernel's).  The same device code as blaz_matmul runs for every
// block and every tile, so each product is bit for bit blaz_matmul's.
#include <hip/hip_runtime.h>

#include <cstring>

#include "blaz_codec.hpp"
#include "blaz_internal.hpp"
#include "blaz_validate.hpp"

#define BLAZ_API extern "C" __attribute__((visibility("default")))

namespace blaz {

// The operands of many products rebuilt in one launch: wave w finds its
// job by binary search over wave0 and decompresses that job's 64 blocks with
// the decompression kernel's device code.
__global__ __launch_bounds__(kWave) void rebuild_group_kernel(const RebuildJob* __restrict__ jobs, int n_jobs)
{
    __shared__ __align__(16) double tile[kWave * kSlot];
    const int64_t w = blockIdx.x;
    int lo = 0, hi = n_jobs - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (jobs[mid].wave0 <= w) lo = mid;
        else hi = mid - 1;
    }
    const RebuildJob j = jobs[lo];
    decompress_wave<true, OutF64, 2>(j.f, j.s, j.phi, j.codes, j.nbc, j.nblk, OutF64{j.out}, j.ld,
                                     (w - j.wave0) * kWave, (int)threadIdx.x, tile);
}

namespace detail {

hipError_t launch_rebuild_group(const RebuildJob* jobs, int n_jobs, int64_t waves, hipStream_t st)
{
    if (n_jobs == 0 || waves == 0) return hipSuccess;
    rebuild_group_kernel<<<(unsigned)waves, kWave, 0, st>>>(jobs, n_jobs);
    return hipGetLastError();
}

}  // namespace detail
}  // namespace blaz

using namespace blaz;
using namespace blaz::validate;

namespace {

constexpr int64_t kMaxGroupItems = int64_t(1) << 24;

size_t plan_bytes_for(int64_t n_items)
{
    return n_items > 0 ? (size_t)n_items * (2 * sizeof(RebuildJob) + sizeof(GemmGroupItem)) : 0;
}

int64_t waves_of(const blaz_matrix& m) { return (nblocks(m) + 63) / 64; }

RebuildJob job_of(const blaz_matrix& m, double* out, int64_t ld, int64_t wave0)
{
    return RebuildJob{m.f, m.s, m.phi, reinterpret_cast<const uint32_t*>(m.codes), m.cols / 8, nblocks(m), out, ld,
                      wave0};
}

// blaz_matmul's checks for one product with the binary64 contraction, the
// workspace aside; the group takes the paper's records (two kept lines).
blaz_status check_item(const blaz_matmul_item& it, bool* empty)
{
    *empty = true;
    if (it.reserved != 0 || (it.tile != 0 && it.tile != 64 && it.tile != 128)) return BLAZ_ERR_ARG;
    if (blaz_status st = check_matrix(&it.a)) return st;
    const bool bc = it.b.rows != 0 || it.b.cols != 0;
    if (bc && it.bdense) return BLAZ_ERR_ARG;
    if (!bc && !it.bdense && it.a.cols > 0) return BLAZ_ERR_NULL;
    const int64_t m = it.a.rows, k = it.a.cols, n = it.n;
    if (bc) {
        if (blaz_status st = check_matrix(&it.b)) return st;
        if (it.b.rows != k || it.b.cols != n) return BLAZ_ERR_MISMATCH;
    }
    if (check_shape(k, n) != BLAZ_OK) return BLAZ_ERR_SHAPE;
    if (lines_of(it.a) != 2 || (bc && lines_of(it.b) != 2)) return BLAZ_ERR_UNSUPPORTED;
    if (m == 0 || n == 0) return BLAZ_OK;
    if (!it.c) return BLAZ_ERR_NULL;
    if (blaz_status st = check_dense(m, n, it.ldc)) return st;
    if (!aligned(it.c, 8)) return BLAZ_ERR_ALIGN;
    if (!bc && k > 0) {
        if (blaz_status st = check_dense(k, n, it.ldb)) return st;
        if (!aligned(it.bdense, 16) || it.ldb % 2 != 0) return BLAZ_ERR_ALIGN;
    }
    const Range rc = span(it.c, dense_span(m, n, it.ldc));
    if (overlaps_matrix(rc, it.a) || (bc && overlaps_matrix(rc, it.b)) ||
        (it.bdense && k > 0 && overlap(rc, span(it.bdense, dense_span(k, n, it.ldb)))))
        return BLAZ_ERR_ARG;
    *empty = false;
    return BLAZ_OK;
}

}  // namespace

BLAZ_API size_t blaz_matmul_group_plan_bytes(int64_t n_items)
{
    if (n_items < 0 || n_items > kMaxGroupItems) return 0;
    return plan_bytes_for(n_items);
}

BLAZ_API blaz_status blaz_matmul_group_plan(const blaz_matmul_item* items, int64_t n_items, void* workspace,
                                            size_t ws_bytes, void* plan, size_t plan_bytes,
                                            blaz_matmul_group_info* info)
{
    if (!info) return BLAZ_ERR_NULL;
    std::memset(info, 0, sizeof *info);
    if (n_items < 0 || n_items > kMaxGroupItems) return BLAZ_ERR_ARG;
    if (n_items == 0) return BLAZ_OK;
    if (!items || !plan) return BLAZ_ERR_NULL;
    if (plan_bytes < plan_bytes_for(n_items)) return BLAZ_ERR_WORKSPACE;
    if (!aligned(plan, 8)) return BLAZ_ERR_ALIGN;

    // first pass: validate, count, size the workspace
    size_t ws = 0;
    int64_t jobs = 0, waves = 0, n128 = 0, n64 = 0, wg128 = 0, wg64 = 0;
    for (int64_t i = 0; i < n_items; ++i) {
        const blaz_matmul_item& it = items[i];
        bool empty;
        if (blaz_status st = check_item(it, &empty)) {
            info->rebuild_jobs = i;
            return st;
        }
        if (empty) continue;
        const int64_t m = it.a.rows, k = it.a.cols, n = it.n;
        const bool bc = it.b.rows != 0 || it.b.cols != 0;
        if (k > 0) {
            ws += round_up((size_t)m * (size_t)k * 8, 256);
            ++jobs;
            waves += waves_of(it.a);
            if (bc) {
                ws += round_up((size_t)k * (size_t)n * 8, 256);
                ++jobs;
                waves += waves_of(it.b);
            }
        }
        const int tile = it.tile != 0 ? it.tile : blaz::detail::default_gemm_tile(m, n);
        const int64_t tiles = ((m + tile - 1) / tile) * ((n + tile - 1) / tile);
        if (tile == 128) {
            ++n128;
            wg128 = (wg128 + 7) / 8 * 8 + tiles;
        } else {
            ++n64;
            wg64 = (wg64 + 7) / 8 * 8 + tiles;
        }
    }
    // every launch fits one dispatch's 32-bit work-item count
    if (!fits_dispatch(waves, 64) || !fits_dispatch(wg128, 256) || !fits_dispatch(wg64, 256)) {
        info->rebuild_jobs = n_items;
        return BLAZ_ERR_SHAPE;
    }
    info->workspace_bytes = ws;
    if (ws > 0) {
        if (!workspace || ws_bytes < ws) return BLAZ_ERR_WORKSPACE;
        if (!aligned(workspace, 256)) return BLAZ_ERR_ALIGN;
    }
    // the workspace may not overlap any product's operands or output
    if (ws > 0) {
        const Range rw = span(workspace, (int64_t)ws);
        for (int64_t i = 0; i < n_items; ++i) {
            const blaz_matmul_item& it = items[i];
            const int64_t m = it.a.rows, k = it.a.cols, n = it.n;
            if (m == 0 || n == 0) continue;
            const bool bc = it.b.rows != 0 || it.b.cols != 0;
            if (overlaps_matrix(rw, it.a) || (bc && overlaps_matrix(rw, it.b)) ||
                overlap(rw, span(it.c, dense_span(m, n, it.ldc))) ||
                (it.bdense && k > 0 && overlap(rw, span(it.bdense, dense_span(k, n, it.ldb))))) {
                info->rebuild_jobs = i;
                return BLAZ_ERR_ARG;
            }
        }
    }

    // The products run concurrently: no product's output may overlap another
    // product's operands or output (operands may be shared).
    {
        std::vector<Tagged> writes, reads;
        for (int64_t i = 0; i < n_items; ++i) {
            const blaz_matmul_item& it = items[i];
            const int64_t m = it.a.rows, k = it.a.cols, n = it.n;
            if (m == 0 || n == 0) continue;
            writes.push_back({span(it.c, dense_span(m, n, it.ldc)), i});
            push_matrix(reads, it.a, i);
            if (it.b.rows != 0 || it.b.cols != 0)
                push_matrix(reads, it.b, i);
            else if (it.bdense && k > 0)
                reads.push_back({span(it.bdense, dense_span(k, n, it.ldb)), i});
        }
        const int64_t bad = cross_item_conflict(writes, reads);
        if (bad >= 0) {
            info->rebuild_jobs = bad;
            return BLAZ_ERR_ARG;
        }
    }

    // second pass: the plan image [jobs][items on 128 tiles][items on 64 tiles]
    RebuildJob* pj = static_cast<RebuildJob*>(plan);
    GemmGroupItem* p128 = reinterpret_cast<GemmGroupItem*>(pj + jobs);
    GemmGroupItem* p64 = p128 + n128;
    char* wsp = static_cast<char*>(workspace);
    int64_t j = 0, w = 0, i128 = 0, i64 = 0, t128 = 0, t64 = 0;
    for (int64_t i = 0; i < n_items; ++i) {
        const blaz_matmul_item& it = items[i];
        const int64_t m = it.a.rows, k = it.a.cols, n = it.n;
        if (m == 0 || n == 0) continue;
        const bool bc = it.b.rows != 0 || it.b.cols != 0;
        const double* A = nullptr;
        const double* B = it.bdense;
        int64_t ldb = it.ldb;
        if (k > 0) {
            double* A64 = reinterpret_cast<double*>(wsp);
            wsp += round_up((size_t)m * (size_t)k * 8, 256);
            pj[j++] = job_of(it.a, A64, k, w);
            w += waves_of(it.a);
            A = A64;
            if (bc) {
                double* B64 = reinterpret_cast<double*>(wsp);
                wsp += round_up((size_t)k * (size_t)n * 8, 256);
                pj[j++] = job_of(it.b, B64, n, w);
                w += waves_of(it.b);
                B = B64;
                ldb = n;
            }
        }
        const int tile = it.tile != 0 ? it.tile : blaz::detail::default_gemm_tile(m, n);
        const int64_t tiles = ((m + tile - 1) / tile) * ((n + tile - 1) / tile);
        if (tile == 128) {
            t128 = (t128 + 7) / 8 * 8;
            p128[i128++] = GemmGroupItem{A, k, B, ldb, it.c, it.ldc, m, n, k, t128};
            t128 += tiles;
        } else {
            t64 = (t64 + 7) / 8 * 8;
            p64[i64++] = GemmGroupItem{A, k, B, ldb, it.c, it.ldc, m, n, k, t64};
            t64 += tiles;
        }
    }
    info->rebuild_jobs = jobs;
    info->rebuild_waves = waves;
    info->items128 = n128;
    info->workgroups128 = wg128;
    info->items64 = n64;
    info->workgroups64 = wg64;
    info->plan_bytes = (size_t)jobs * sizeof(RebuildJob) + (size_t)(n128 + n64) * sizeof(GemmGroupItem);
    return BLAZ_OK;
}

BLAZ_API blaz_status blaz_matmul_group_run(const void* plan_dev, const blaz_matmul_group_info* info,
                                           hipStream_t stream)
{
    if (!info) return BLAZ_ERR_NULL;
    const blaz_matmul_group_info g = *info;
    if (g.rebuild_jobs < 0 || g.rebuild_waves < 0 || g.items128 < 0 || g.items64 < 0 || g.workgroups128 < 0 ||
        g.workgroups64 < 0 || g.rebuild_jobs > 2 * kMaxGroupItems || g.items128 + g.items64 > kMaxGroupItems)
        return BLAZ_ERR_ARG;
    if (g.rebuild_jobs + g.items128 + g.items64 == 0) return BLAZ_OK;
    if (!plan_dev) return BLAZ_ERR_NULL;
    if (!aligned(plan_dev, 8)) return BLAZ_ERR_ALIGN;
    if (!fits_dispatch(g.rebuild_waves, 64) || !fits_dispatch(g.workgroups128, 256) ||
        !fits_dispatch(g.workgroups64, 256))
        return BLAZ_ERR_SHAPE;
    const RebuildJob* pj = static_cast<const RebuildJob*>(plan_dev);
    const GemmGroupItem* p128 = reinterpret_cast<const GemmGroupItem*>(pj + g.rebuild_jobs);
    const GemmGroupItem* p64 = p128 + g.items128;
    using namespace blaz::detail;
    if (hipError_t e = launch_rebuild_group(pj, (int)g.rebuild_jobs, g.rebuild_waves, stream)) return hip_status(e);
    if (hipError_t e = launch_gemm_group(p128, (int)g.items128, g.workgroups128, 128, stream)) return hip_status(e);
    return hip_status(launch_gemm_group(p64, (int)g.items64, g.workgroups64, 64, stream));
}
