// Batching: a flat queue of 64-block chunks (or groups of 8 dot products)
// over many operations on matrices of any sizes, drained by one persistent
// launch.
//
// The blocks of the method are independent (each operation is applied
// blockwise, end of Section "Basic Linear Algebra Algorithms"), so a batch is
// a list of items, each cut into chunks: a chunk is the unit one workgroup of
// the standalone kernels handles -- 64 consecutive blocks of a compress,
// decompress, add, sub or scale, or a group of 8 consecutive dot products
// (whose four parts the batch wave runs one after the other).  The plan stores every
// item's first chunk index (a prefix sum); a fixed grid of one-wave
// workgroups pops chunk indices from an atomic counter, finds the item by
// binary search and runs the same device body as the standalone kernel, until
// the counter passes the end of the queue.  Every wave reaches that exit, so
// the grid always drains.  Chunks of different items run at the same time, so
// the plan refuses items that read or write another item's output.
#include <hip/hip_runtime.h>

#include <cstring>

#include "blaz_codec.hpp"
#include "blaz_dot.hpp"
#include "blaz_internal.hpp"
#include "blaz_ops.hpp"
#include "blaz_validate.hpp"

#define BLAZ_API extern "C" __attribute__((visibility("default")))

namespace blaz {

// Device image of one planned item.
struct BatchItemDev {
    int32_t op;
    int32_t reserved;
    int64_t chunk0;  // first chunk of this item in the queue
    int64_t nbc;     // block columns (codec ops, x); DOT_DENSE: block columns of x
    int64_t nblk;    // blocks (codec ops)
    double* dense;
    int64_t ld;
    double* xf;
    double* xs;
    uint8_t* xphi;
    uint32_t* xc;
    double* yf;
    double* ys;
    uint8_t* yphi;
    uint32_t* yc;
    double* zf;
    double* zs;
    uint8_t* zphi;
    uint32_t* zc;
    double c;
    const int64_t* xrow;
    const int64_t* ycol;
    double* out;
    int64_t nbr_x;  // DOT, DOT_DENSE: block rows of x
    int64_t nbc_y;  // DOT: block columns of y
    int64_t nk;     // DOT: block columns of x = block rows of y
    int64_t count;  // DOT, DOT_DENSE: dot products
};

__global__ void batch_reset_kernel(unsigned long long* counter) { *counter = 0ull; }

__device__ __forceinline__ int64_t wave_uniform(int64_t v)
{
    const uint32_t lo = __builtin_amdgcn_readfirstlane((uint32_t)v);
    const uint32_t hi = __builtin_amdgcn_readfirstlane((uint32_t)((uint64_t)v >> 32));
    return (int64_t)(((uint64_t)hi << 32) | lo);
}

// Drains the queue; returns the value of the wave's last claim.
__device__ __forceinline__ int64_t batch_body(const BatchItemDev* __restrict__ items, int32_t n_items, int64_t total,
                                              unsigned long long* counter, int32_t per_claim)
{
    __shared__ __align__(16) double tile[kWave * kSlot];
    const int lane = threadIdx.x;
    int64_t chunk = 0, claim_end = 0, claimed = 0;
    for (;;) {
        __syncthreads();  // the previous chunk is done with the LDS tile
        if (chunk >= claim_end) {  // claim the next per_claim consecutive chunks
            unsigned long long got = 0;
            if (lane == 0) got = atomicAdd(counter, (unsigned long long)per_claim);
            chunk = claimed = wave_uniform((int64_t)got);
            claim_end = chunk + per_claim;
        }
        if (chunk >= total) return claimed;
        // last item whose first chunk is <= chunk
        int lo = 0, hi = n_items - 1;
        while (lo < hi) {
            const int mid = (lo + hi + 1) >> 1;
            if (items[mid].chunk0 <= chunk) lo = mid;
            else hi = mid - 1;
        }
        const BatchItemDev& it = items[lo];
        const int64_t local = chunk - it.chunk0;
        const int64_t wave_base = local * kWave;
        switch (it.op) {
            case BLAZ_OP_COMPRESS:
                compress_wave<true, false>(it.dense, it.ld, it.nbc, it.nblk, it.xf, it.xs, it.xphi, it.xc, nullptr,
                                           wave_base, lane, tile);
                break;
            case BLAZ_OP_DECOMPRESS:
                decompress_wave<true>(it.xf, it.xs, it.xphi, it.xc, it.nbc, it.nblk, OutF64{it.dense}, it.ld,
                                      wave_base, lane, tile);
                break;
            case BLAZ_OP_ADD:
            case BLAZ_OP_SUB: {
                const int64_t b = wave_base + lane;
                if (b < it.nblk)
                    add_block(b, it.op == BLAZ_OP_SUB, it.xf, it.xs, it.xphi, it.xc, it.yf, it.ys, it.yphi, it.yc,
                              it.zf, it.zs, it.zphi, it.zc);
                break;
            }
            case BLAZ_OP_SCALE: {
                const int64_t b = wave_base + lane;
                if (b < it.nblk) scale_block(b, it.c, it.xf, it.xs, it.xphi, it.xc, it.zf, it.zs, it.zphi, it.zc);
                break;
            }
            case BLAZ_OP_DOT:
                dot_group_one_wave(lane, local * kDotGroup, it.count, DotOperand{it.xf, it.xs, it.xphi, it.xc},
                                   it.nbr_x, DotOperand{it.yf, it.ys, it.yphi, it.yc}, it.nbc_y, it.nk, it.xrow,
                                   it.ycol, it.out);
                break;
            default:  // BLAZ_OP_DOT_DENSE
                dot_dense_group_one_wave(lane, local * kDotGroup, it.count, DotOperand{it.xf, it.xs, it.xphi, it.xc},
                                         it.nbr_x, it.nbc, it.xrow, it.dense, it.ld, it.out);
                break;
        }
        ++chunk;
    }
}

__global__ __launch_bounds__(kWave, 2) void batch_kernel(const BatchItemDev* __restrict__ items, int32_t n_items,
                                                         int64_t total, unsigned long long* __restrict__ counter,
                                                         int32_t per_claim)
{
    batch_body(items, n_items, total, counter, per_claim);
}

// Resident runs read the plan's counts from a device state record written
// before the launch executes, so one captured graph serves every plan that
// is copied into the same buffers.  The run is a single launch: every wave
// checks the counts against the plan buffer's capacity (workgroup 0
// publishes the status), and the wave that made the run's last claim
// resets the work counter, so the record is ready for the next run without
// a reset launch.  Which claim is last follows from counting: with T
// chunks, C chunks per claim and W waves, ceil(T / C) claims succeed; the
// wave holding a claim that runs past T (there is one when C does not
// divide T) leaves without claiming again, and every other wave leaves
// after one claim at or past T.  So the run makes
// N = ceil(T / C) + W - [C does not divide T] claims, the last one returning
// (N - 1) C, and no claim can follow it.
__global__ __launch_bounds__(kWave, 2) void batch_resident_kernel(const BatchItemDev* __restrict__ items,
                                                                  blaz_batch_state* state, int64_t capacity,
                                                                  int32_t per_claim)
{
    const int64_t np = state->n_plan, tot = state->total_chunks;
    const bool ok = np >= 0 && np <= capacity && tot >= 0 && (np > 0 || tot == 0);
    if (blockIdx.x == 0 && threadIdx.x == 0) state->status = ok ? BLAZ_OK : BLAZ_ERR_ARG;
    if (!ok) return;
    auto* counter = reinterpret_cast<unsigned long long*>(&state->counter);
    const int64_t last = batch_body(items, (int32_t)np, tot, counter, per_claim);
    const int64_t claims = (tot + per_claim - 1) / per_claim + (int64_t)gridDim.x - (tot % per_claim != 0 ? 1 : 0);
    if (threadIdx.x == 0 && last == (claims - 1) * per_claim) atomicExch(counter, 0ull);
}

}  // namespace blaz

using namespace blaz;
using namespace blaz::validate;

static void set_matrix(const blaz_matrix& m, double*& f, double*& s, uint8_t*& phi, uint32_t*& c)
{
    f = m.f;
    s = m.s;
    phi = m.phi;
    c = reinterpret_cast<uint32_t*>(m.codes);
}

BLAZ_API size_t blaz_batch_plan_bytes(int64_t n_items)
{
    return n_items > 0 ? (size_t)n_items * sizeof(BatchItemDev) : 0;
}

BLAZ_API blaz_status blaz_batch_plan(const blaz_batch_item* items, int64_t n_items, void* plan, size_t plan_bytes,
                                     int64_t* n_plan, int64_t* total_chunks)
{
    if (!n_plan || !total_chunks) return BLAZ_ERR_NULL;
    *n_plan = 0;
    *total_chunks = 0;
    if (n_items < 0 || n_items > (int64_t(1) << 30)) return BLAZ_ERR_ARG;
    if (n_items == 0) return BLAZ_OK;
    if (!items || !plan) return BLAZ_ERR_NULL;
    if (plan_bytes < blaz_batch_plan_bytes(n_items)) return BLAZ_ERR_WORKSPACE;
    if (!aligned(plan, 8)) return BLAZ_ERR_ALIGN;
    BatchItemDev* out = static_cast<BatchItemDev*>(plan);
    int64_t np = 0, chunks = 0;
    for (int64_t i = 0; i < n_items; ++i) {
        const blaz_batch_item& it = items[i];
        bool empty = true;
        blaz_status st = BLAZ_OK;
        if (it.reserved != 0) st = BLAZ_ERR_ARG;
        BatchItemDev d;
        std::memset(&d, 0, sizeof d);
        d.op = it.op;
        int64_t n = 0;
        if (st == BLAZ_OK) switch (it.op) {
            case BLAZ_OP_COMPRESS:
                st = validate_compress(it.dense, it.ld, &it.x, BLAZ_PREC_FP64, nullptr, &empty);
                set_matrix(it.x, d.xf, d.xs, d.xphi, d.xc);
                d.nblk = nblocks(it.x);
                d.nbc = it.x.cols / 8;
                n = (d.nblk + kWave - 1) / kWave;
                break;
            case BLAZ_OP_DECOMPRESS:
                st = validate_decompress(&it.x, it.dense, it.ld, &empty);
                set_matrix(it.x, d.xf, d.xs, d.xphi, d.xc);
                d.nblk = nblocks(it.x);
                d.nbc = it.x.cols / 8;
                n = (d.nblk + kWave - 1) / kWave;
                break;
            case BLAZ_OP_ADD:
            case BLAZ_OP_SUB:
                st = validate_add(&it.x, &it.y, &it.z, &empty);
                set_matrix(it.x, d.xf, d.xs, d.xphi, d.xc);
                set_matrix(it.y, d.yf, d.ys, d.yphi, d.yc);
                set_matrix(it.z, d.zf, d.zs, d.zphi, d.zc);
                d.nblk = nblocks(it.x);
                n = (d.nblk + kWave - 1) / kWave;
                break;
            case BLAZ_OP_SCALE:
                st = validate_scale(&it.x, &it.z, &empty);
                set_matrix(it.x, d.xf, d.xs, d.xphi, d.xc);
                set_matrix(it.z, d.zf, d.zs, d.zphi, d.zc);
                d.nblk = nblocks(it.x);
                d.c = it.c;
                n = (d.nblk + kWave - 1) / kWave;
                break;
            case BLAZ_OP_DOT:
                st = validate_dot(&it.x, it.xrow, &it.y, it.ycol, it.count, it.out, &empty);
                set_matrix(it.x, d.xf, d.xs, d.xphi, d.xc);
                set_matrix(it.y, d.yf, d.ys, d.yphi, d.yc);
                d.nbr_x = it.x.rows / 8;
                d.nbc_y = it.y.cols / 8;
                d.nk = it.x.cols / 8;
                d.count = it.count;
                n = (it.count + kDotGroup - 1) / kDotGroup;
                break;
            case BLAZ_OP_DOT_DENSE:
                st = validate_dot_dense(&it.x, it.xrow, it.dense, it.ld, it.count, it.out, &empty);
                set_matrix(it.x, d.xf, d.xs, d.xphi, d.xc);
                d.nbr_x = it.x.rows / 8;
                d.nbc = it.x.cols / 8;
                d.count = it.count;
                n = (it.count + kDotGroup - 1) / kDotGroup;
                break;
            default:
                st = BLAZ_ERR_ARG;
        }
        // batches carry the paper's records (two kept lines) only
        if (st == BLAZ_OK && !empty) {
            const bool uses_y = it.op == BLAZ_OP_ADD || it.op == BLAZ_OP_SUB || it.op == BLAZ_OP_DOT;
            const bool uses_z = it.op == BLAZ_OP_ADD || it.op == BLAZ_OP_SUB || it.op == BLAZ_OP_SCALE;
            if (lines_of(it.x) != 2 || (uses_y && lines_of(it.y) != 2) || (uses_z && lines_of(it.z) != 2))
                st = BLAZ_ERR_UNSUPPORTED;
        }
        // batched compress / decompress use the LDS-staged row path only
        if (st == BLAZ_OK && !empty && (it.op == BLAZ_OP_COMPRESS || it.op == BLAZ_OP_DECOMPRESS) &&
            (!aligned(it.dense, 16) || it.ld % 2 != 0))
            st = BLAZ_ERR_ALIGN;
        if (st != BLAZ_OK) {
            *n_plan = i;
            *total_chunks = 0;
            return st;
        }
        if (empty) continue;
        d.dense = it.dense;
        d.ld = it.ld;
        d.xrow = it.xrow;
        d.ycol = it.ycol;
        d.out = it.out;
        d.chunk0 = chunks;
        chunks += n;
        out[np++] = d;
    }
    // The items run concurrently: no item may read or write another item's
    // output (inputs may be shared).
    std::vector<Tagged> writes, reads;
    for (int64_t i = 0; i < n_items; ++i) {
        const blaz_batch_item& it = items[i];
        switch (it.op) {
            case BLAZ_OP_COMPRESS:
                if (nblocks(it.x) == 0) break;
                push_matrix(writes, it.x, i);
                reads.push_back({span(it.dense, dense_span(it.x.rows, it.x.cols, it.ld)), i});
                break;
            case BLAZ_OP_DECOMPRESS:
                if (nblocks(it.x) == 0) break;
                writes.push_back({span(it.dense, dense_span(it.x.rows, it.x.cols, it.ld)), i});
                push_matrix(reads, it.x, i);
                break;
            case BLAZ_OP_ADD:
            case BLAZ_OP_SUB:
                if (nblocks(it.x) == 0) break;
                push_matrix(writes, it.z, i);
                push_matrix(reads, it.x, i);
                push_matrix(reads, it.y, i);
                break;
            case BLAZ_OP_SCALE:
                if (nblocks(it.x) == 0) break;
                push_matrix(writes, it.z, i);
                push_matrix(reads, it.x, i);
                break;
            case BLAZ_OP_DOT:
                if (it.count == 0) break;
                writes.push_back({span(it.out, 8 * it.count), i});
                push_matrix(reads, it.x, i);
                push_matrix(reads, it.y, i);
                reads.push_back({span(it.xrow, 8 * it.count), i});
                reads.push_back({span(it.ycol, 8 * it.count), i});
                break;
            default:  // BLAZ_OP_DOT_DENSE
                if (it.count == 0) break;
                writes.push_back({span(it.out, 8 * it.count), i});
                push_matrix(reads, it.x, i);
                reads.push_back({span(it.xrow, 8 * it.count), i});
                reads.push_back({span(it.dense, it.ld == 0 ? 8 * it.x.cols : dense_span(it.count, it.x.cols, it.ld)),
                                 i});
                break;
        }
    }
    const int64_t bad = cross_item_conflict(writes, reads);
    if (bad >= 0) {
        *n_plan = bad;
        *total_chunks = 0;
        return BLAZ_ERR_ARG;
    }
    *n_plan = np;
    *total_chunks = chunks;
    return BLAZ_OK;
}

BLAZ_API blaz_status blaz_batch_run(const void* plan_dev, int64_t n_plan, int64_t total_chunks, uint64_t* counter,
                                    int64_t workgroups, int32_t chunks_per_claim, hipStream_t stream)
{
    if (n_plan < 0 || total_chunks < 0 || workgroups < 0 || n_plan > (int64_t(1) << 30)) return BLAZ_ERR_ARG;
    if (chunks_per_claim < 0 || chunks_per_claim > 64) return BLAZ_ERR_ARG;
    if (chunks_per_claim == 0) chunks_per_claim = 1;
    if (n_plan == 0 || total_chunks == 0) return BLAZ_OK;
    if (!plan_dev || !counter) return BLAZ_ERR_NULL;
    if (!aligned(plan_dev, 8) || !aligned(counter, 8)) return BLAZ_ERR_ALIGN;
    if (workgroups == 0) {
        const int cus = blaz::detail::device_cu_count();
        if (cus == 0) return BLAZ_ERR_HIP;
        workgroups = 8 * (int64_t)cus;
    }
    if (workgroups > total_chunks) workgroups = total_chunks;
    if (workgroups > (int64_t(1) << 20)) workgroups = int64_t(1) << 20;
    auto* cnt = reinterpret_cast<unsigned long long*>(counter);
    batch_reset_kernel<<<1, 1, 0, stream>>>(cnt);
    if (hipGetLastError() != hipSuccess) return BLAZ_ERR_HIP;
    batch_kernel<<<(unsigned)workgroups, kWave, 0, stream>>>(static_cast<const BatchItemDev*>(plan_dev),
                                                             (int32_t)n_plan, total_chunks, cnt, chunks_per_claim);
    return hipGetLastError() == hipSuccess ? BLAZ_OK : BLAZ_ERR_HIP;
}

BLAZ_API blaz_status blaz_batch_run_resident(const void* plan_dev, int64_t capacity, blaz_batch_state* state,
                                             int64_t workgroups,
                                             int32_t chunks_per_claim, hipStream_t stream)
{
    if (capacity <= 0 || capacity > (int64_t(1) << 30) || workgroups < 0) return BLAZ_ERR_ARG;
    if (chunks_per_claim < 0 || chunks_per_claim > 64) return BLAZ_ERR_ARG;
    if (chunks_per_claim == 0) chunks_per_claim = 1;
    if (!plan_dev || !state) return BLAZ_ERR_NULL;
    if (!aligned(plan_dev, 8) || !aligned(state, 8)) return BLAZ_ERR_ALIGN;
    if (workgroups == 0) {
        const int cus = blaz::detail::device_cu_count();
        if (cus == 0) return BLAZ_ERR_HIP;
        workgroups = 8 * (int64_t)cus;
    }
    if (workgroups > (int64_t(1) << 20)) workgroups = int64_t(1) << 20;
    batch_resident_kernel<<<(unsigned)workgroups, kWave, 0, stream>>>(static_cast<const BatchItemDev*>(plan_dev), state,
                                                                      capacity, chunks_per_claim);
    return hipGetLastError() == hipSuccess ? BLAZ_OK : BLAZ_ERR_HIP;
}
