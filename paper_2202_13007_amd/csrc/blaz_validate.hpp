// Host-side argument checks shared by the C-ABI entry points: shapes,
// NULL and alignment of descriptors, and byte-range overlap tests.  None of
// them touches device memory or calls the HIP runtime.
#pragma once

#include <algorithm>
#include <cstdint>
#include <vector>

#include "libblaz.h"

namespace blaz {
namespace validate {

constexpr int64_t kRecordBytes = 45;  // f (8) + s (8) + phi (1) + 28 codes (two kept lines)

// A dispatch's grid size is a 32-bit count of work-items (lanes), so every
// launch must stay at or below 2^32 - 1 lanes.
constexpr int64_t kMaxLanes = (int64_t(1) << 32) - 1;
inline bool fits_dispatch(int64_t workgroups, int64_t lanes_per_workgroup)
{
    return workgroups >= 0 && workgroups <= kMaxLanes / lanes_per_workgroup;
}
// Blocks per compressed matrix: the one-lane-per-block kernels (add, sub,
// scale, diagnose) round the block count up to whole 256-lane workgroups,
// the codec kernels to whole 64-lane waves, so 2^32 - 256 blocks (about
// 193 GB compressed) is the largest count every kernel launches as one grid.
constexpr int64_t kMaxBlocks = (int64_t(1) << 32) - 256;
// Dot products per call: eight per 256-lane workgroup, 32 lanes each.
constexpr int64_t kMaxDots = kMaxBlocks / 32;

inline bool aligned(const void* p, uintptr_t a) { return reinterpret_cast<uintptr_t>(p) % a == 0; }

inline blaz_status check_shape(int64_t rows, int64_t cols)
{
    if (rows < 0 || cols < 0 || rows % 8 != 0 || cols % 8 != 0) return BLAZ_ERR_SHAPE;
    if (rows > 0 && cols > 0 && (rows / 8) > kMaxBlocks / (cols / 8)) return BLAZ_ERR_SHAPE;
    return BLAZ_OK;
}

inline int64_t nblocks(const blaz_matrix& m) { return (m.rows / 8) * (m.cols / 8); }

// Kept lines L of a descriptor (0 stands for the paper's 2) and the bytes of
// codes per block: 16L - L^2 codes padded to whole dwords.
inline int lines_of(const blaz_matrix& m) { return m.lines == 0 ? 2 : (int)m.lines; }
inline bool valid_lines(int64_t lines) { return lines >= 0 && lines <= 8; }
inline int64_t code_stride(int lines) { return 4 * ((16 * lines - lines * lines + 3) / 4); }

struct Range {
    uintptr_t lo, hi;
};
inline Range span(const void* p, int64_t bytes)
{
    const auto a = reinterpret_cast<uintptr_t>(p);
    return {a, a + (uintptr_t)(bytes > 0 ? bytes : 0)};
}
// A range whose end passes the top of the address space (no allocation can
// hold it) counts as overlapping everything, so that the call is refused.
inline bool wraps(Range r) { return r.hi < r.lo; }
inline bool overlap(Range a, Range b) { return wraps(a) || wraps(b) || (a.lo < b.hi && b.lo < a.hi); }

// The byte ranges of a compressed matrix's four arrays.
inline void ranges(const blaz_matrix& m, Range r[4])
{
    const int64_t n = nblocks(m);
    r[0] = span(m.f, 8 * n);
    r[1] = span(m.s, 8 * n);
    r[2] = span(m.phi, n);
    r[3] = span(m.codes, code_stride(lines_of(m)) * n);
}

// A descriptor is valid if its shape and kept lines are and, when it holds
// blocks, its four arrays are present, aligned and end below the top of the
// address space.
inline blaz_status check_matrix(const blaz_matrix* m)
{
    if (!m) return BLAZ_ERR_NULL;
    if (!valid_lines(m->lines)) return BLAZ_ERR_ARG;
    if (blaz_status st = check_shape(m->rows, m->cols)) return st;
    if (nblocks(*m) == 0) return BLAZ_OK;
    if (!m->f || !m->s || !m->phi || !m->codes) return BLAZ_ERR_NULL;
    if (!aligned(m->f, 8) || !aligned(m->s, 8) || !aligned(m->codes, 4)) return BLAZ_ERR_ALIGN;
    Range r[4];
    ranges(*m, r);
    for (auto& x : r)
        if (wraps(x)) return BLAZ_ERR_ARG;
    return BLAZ_OK;
}

inline bool overlaps_matrix(Range a, const blaz_matrix& m)
{
    Range r[4];
    ranges(m, r);
    for (auto& x : r)
        if (overlap(a, x)) return true;
    return false;
}

// z must either be exactly x (same four arrays) or not overlap it at all.
inline bool same_or_disjoint(const blaz_matrix& z, const blaz_matrix& x)
{
    if (z.f == x.f && z.s == x.s && z.phi == x.phi && z.codes == x.codes) return true;
    Range rz[4];
    ranges(z, rz);
    for (auto& r : rz)
        if (overlaps_matrix(r, x)) return false;
    return true;
}

// Bytes spanned by a rows x cols row-major matrix with leading dimension ld
// (one that passed check_dense, so the product cannot overflow).
inline int64_t dense_span(int64_t rows, int64_t cols, int64_t ld) { return rows == 0 ? 0 : ((rows - 1) * ld + cols) * 8; }

// A dense rows x cols operand with leading dimension ld: ld >= cols, and the
// offset of its last element below 2^60 elements, so that every element
// offset the kernels form (and every byte span above) fits in int64.
constexpr int64_t kMaxDenseElems = int64_t(1) << 60;
inline blaz_status check_dense(int64_t rows, int64_t cols, int64_t ld)
{
    if (ld < cols) return BLAZ_ERR_SHAPE;
    if (rows > 1 && ld > (kMaxDenseElems - cols) / (rows - 1)) return BLAZ_ERR_SHAPE;
    return BLAZ_OK;
}

inline blaz_status hip_status(hipError_t e) { return e == hipSuccess ? BLAZ_OK : BLAZ_ERR_HIP; }

// Work that runs concurrently (the items of a batch, the products of a
// group): no item's output may overlap another item's output or inputs,
// while inputs may be shared.  writes and reads are byte ranges tagged with
// their item.  The writes, sorted by address, must be disjoint; then a read
// can only meet the last write that starts below its end.  Returns the
// larger item index of a conflicting pair, or -1.
struct Tagged {
    Range r;
    int64_t item;
};
inline int64_t cross_item_conflict(std::vector<Tagged>& writes, const std::vector<Tagged>& reads)
{
    std::sort(writes.begin(), writes.end(), [](const Tagged& x, const Tagged& y) { return x.r.lo < y.r.lo; });
    for (size_t q = 1; q < writes.size(); ++q)
        if (overlap(writes[q - 1].r, writes[q].r)) return std::max(writes[q - 1].item, writes[q].item);
    for (const Tagged& rd : reads) {
        if (rd.r.hi == rd.r.lo) continue;
        auto after = std::lower_bound(writes.begin(), writes.end(), rd.r.hi,
                                      [](const Tagged& w, uintptr_t hi) { return w.r.lo < hi; });
        if (after == writes.begin()) continue;
        const Tagged& w = *(after - 1);
        if (w.item != rd.item && overlap(w.r, rd.r)) return std::max(w.item, rd.item);
    }
    return -1;
}

// The four arrays of a compressed matrix, tagged.
inline void push_matrix(std::vector<Tagged>& v, const blaz_matrix& m, int64_t item)
{
    Range r[4];
    ranges(m, r);
    for (const Range& x : r) v.push_back({x, item});
}

inline size_t round_up(size_t x, size_t a) { return (x + a - 1) / a * a; }


// ---------------------------------------------------------------------------
// Per-operation checks.  Each returns BLAZ_OK and sets *empty when the call
// has nothing to do, or the first violated rule's status.
// ---------------------------------------------------------------------------

inline blaz_status validate_compress(const double* A, int64_t lda, const blaz_matrix* out, blaz_precision prec,
                                     const uint8_t* psi, bool* empty)
{
    *empty = true;
    if (blaz_status st = check_matrix(out)) return st;
    if (prec != BLAZ_PREC_FP64 && prec != BLAZ_PREC_FP32 && prec != BLAZ_PREC_BF16X3) return BLAZ_ERR_ARG;
    if (lines_of(*out) != 2 && (prec != BLAZ_PREC_FP64 || psi)) return BLAZ_ERR_UNSUPPORTED;
    const int64_t nblk = nblocks(*out);
    if (nblk == 0) return BLAZ_OK;
    if (!A) return BLAZ_ERR_NULL;
    if (blaz_status st = check_dense(out->rows, out->cols, lda)) return st;
    if (!aligned(A, 8) || (psi && !aligned(psi, 16))) return BLAZ_ERR_ALIGN;
    const Range ra = span(A, dense_span(out->rows, out->cols, lda));
    if (overlaps_matrix(ra, *out)) return BLAZ_ERR_ARG;
    if (psi && (overlap(span(psi, 64 * nblk), ra) || overlaps_matrix(span(psi, 64 * nblk), *out))) return BLAZ_ERR_ARG;
    *empty = false;
    return BLAZ_OK;
}

inline blaz_status validate_decompress(const blaz_matrix* in, const double* A, int64_t lda, bool* empty)
{
    *empty = true;
    if (blaz_status st = check_matrix(in)) return st;
    if (nblocks(*in) == 0) return BLAZ_OK;
    if (!A) return BLAZ_ERR_NULL;
    if (blaz_status st = check_dense(in->rows, in->cols, lda)) return st;
    if (!aligned(A, 8)) return BLAZ_ERR_ALIGN;
    if (overlaps_matrix(span(A, dense_span(in->rows, in->cols, lda)), *in)) return BLAZ_ERR_ARG;
    *empty = false;
    return BLAZ_OK;
}

inline blaz_status validate_add(const blaz_matrix* x, const blaz_matrix* y, const blaz_matrix* z, bool* empty)
{
    *empty = true;
    for (const blaz_matrix* m : {x, y, z})
        if (blaz_status st = check_matrix(m)) return st;
    if (x->rows != y->rows || x->cols != y->cols || x->rows != z->rows || x->cols != z->cols ||
        lines_of(*x) != lines_of(*y) || lines_of(*x) != lines_of(*z))
        return BLAZ_ERR_MISMATCH;
    if (nblocks(*x) == 0) return BLAZ_OK;
    if (!same_or_disjoint(*z, *x) || !same_or_disjoint(*z, *y)) return BLAZ_ERR_ARG;
    *empty = false;
    return BLAZ_OK;
}

inline blaz_status validate_scale(const blaz_matrix* x, const blaz_matrix* z, bool* empty)
{
    *empty = true;
    for (const blaz_matrix* m : {x, z})
        if (blaz_status st = check_matrix(m)) return st;
    if (x->rows != z->rows || x->cols != z->cols || lines_of(*x) != lines_of(*z)) return BLAZ_ERR_MISMATCH;
    if (nblocks(*x) == 0) return BLAZ_OK;
    if (!same_or_disjoint(*z, *x)) return BLAZ_ERR_ARG;
    *empty = false;
    return BLAZ_OK;
}

inline blaz_status validate_dot(const blaz_matrix* x, const int64_t* xrow, const blaz_matrix* y, const int64_t* ycol,
                                int64_t count, const double* out, bool* empty)
{
    *empty = true;
    for (const blaz_matrix* m : {x, y})
        if (blaz_status st = check_matrix(m)) return st;
    if (x->cols != y->rows) return BLAZ_ERR_MISMATCH;
    if (lines_of(*x) != 2 || lines_of(*y) != 2) return BLAZ_ERR_UNSUPPORTED;
    if (count < 0 || count > kMaxDots) return BLAZ_ERR_ARG;
    if (count == 0) return BLAZ_OK;
    if (!xrow || !ycol || !out) return BLAZ_ERR_NULL;
    if (!aligned(xrow, 8) || !aligned(ycol, 8) || !aligned(out, 8)) return BLAZ_ERR_ALIGN;
    const Range ro = span(out, 8 * count);
    if (overlaps_matrix(ro, *x) || overlaps_matrix(ro, *y)) return BLAZ_ERR_ARG;
    // out is written while other queries still read their indexes
    if (overlap(ro, span(xrow, 8 * count)) || overlap(ro, span(ycol, 8 * count))) return BLAZ_ERR_ARG;
    *empty = false;
    return BLAZ_OK;
}

inline blaz_status validate_dot_dense(const blaz_matrix* x, const int64_t* xrow, const double* v, int64_t ldv,
                                      int64_t count, const double* out, bool* empty)
{
    *empty = true;
    if (blaz_status st = check_matrix(x)) return st;
    if (lines_of(*x) != 2) return BLAZ_ERR_UNSUPPORTED;
    if (count < 0 || count > kMaxDots || ldv < 0) return BLAZ_ERR_ARG;
    if (ldv != 0)
        if (blaz_status st = check_dense(count, x->cols, ldv)) return st;
    if (count == 0) return BLAZ_OK;
    if (!xrow || !v || !out) return BLAZ_ERR_NULL;
    if (!aligned(xrow, 8) || !aligned(out, 8) || !aligned(v, 16) || ldv % 2 != 0) return BLAZ_ERR_ALIGN;
    const Range ro = span(out, 8 * count);
    if (overlaps_matrix(ro, *x)) return BLAZ_ERR_ARG;
    // out is written while other queries still read their indexes and vectors
    const Range rv = span(v, ldv == 0 ? 8 * x->cols : dense_span(count, x->cols, ldv));
    if (overlap(ro, span(xrow, 8 * count)) || overlap(ro, rv)) return BLAZ_ERR_ARG;
    *empty = false;
    return BLAZ_OK;
}

}  // namespace validate
}  // namespace blaz
