// Driver for a sanitizer build (AddressSanitizer and UndefinedBehaviorSanitizer)
// of the library's host-side argument checks (blaz_validate.hpp): every
// per-operation check runs on valid and invalid descriptors, including shapes
// and leading dimensions at and beyond the limits, whose arithmetic must not
// overflow.  Device pointers are fake addresses and are never dereferenced.
// Exits 0 when every expected status comes back.
#include <cstdint>
#include <cstdio>
#include <limits>

#include "blaz_validate.hpp"

using namespace blaz::validate;

static int failures = 0;
#define EXPECT(expr, want)                                                                  \
    do {                                                                                    \
        const int got_ = (int)(expr);                                                       \
        if (got_ != (int)(want)) {                                                          \
            std::fprintf(stderr, "line %d: %s gave %d, want %d\n", __LINE__, #expr, got_, (int)(want)); \
            ++failures;                                                                     \
        }                                                                                   \
    } while (0)

template <typename T>
static T* fake(uintptr_t a) { return reinterpret_cast<T*>(a); }

static blaz_matrix mat(int64_t rows, int64_t cols, uintptr_t base, int64_t lines = 0)
{
    const int64_t nb = (rows > 0 && cols > 0) ? (rows / 8) * (cols / 8) : 0;
    blaz_matrix m{};
    m.rows = rows;
    m.cols = cols;
    m.f = fake<double>(base);
    m.s = fake<double>(base + 8 * (uintptr_t)nb + 64);
    m.phi = fake<uint8_t>(base + 16 * (uintptr_t)nb + 128);
    m.codes = fake<int8_t>(base + (uintptr_t)((17 * nb + 256 + 15) / 16 * 16));
    m.lines = lines;
    return m;
}

int main()
{
    const int64_t big = std::numeric_limits<int64_t>::max();
    bool empty = false;
    // shapes
    EXPECT(check_shape(8, 8), BLAZ_OK);
    EXPECT(check_shape(big - 7, 8), BLAZ_ERR_SHAPE);
    EXPECT(check_shape(big / 8 * 8, big / 8 * 8), BLAZ_ERR_SHAPE);
    EXPECT(check_shape(8 * 256, 8 * ((int64_t(1) << 24) - 1)), BLAZ_OK);
    EXPECT(check_shape(8 * 257, 8 * ((int64_t(1) << 24) - 1)), BLAZ_ERR_SHAPE);
    EXPECT(check_shape(-8, 8), BLAZ_ERR_SHAPE);
    EXPECT(check_dense(16, 16, big), BLAZ_ERR_SHAPE);
    EXPECT(check_dense(2, big - 1, big), BLAZ_ERR_SHAPE);
    EXPECT(check_dense(1, 16, big), BLAZ_OK);
    EXPECT(fits_dispatch(kMaxLanes / 256, 256), true);
    EXPECT(fits_dispatch(kMaxLanes / 256 + 1, 256), false);
    EXPECT(fits_dispatch(big, 64), false);

    // compress / decompress
    blaz_matrix x = mat(16, 16, 0x100000);
    const double* A = fake<const double>(0x200000);
    EXPECT(validate_compress(A, 16, &x, BLAZ_PREC_FP64, nullptr, &empty), BLAZ_OK);
    EXPECT(empty, false);
    EXPECT(validate_compress(A, big, &x, BLAZ_PREC_FP64, nullptr, &empty), BLAZ_ERR_SHAPE);
    EXPECT(validate_compress(A, 8, &x, BLAZ_PREC_FP64, nullptr, &empty), BLAZ_ERR_SHAPE);
    EXPECT(validate_compress(fake<const double>(0x100000), 16, &x, BLAZ_PREC_FP64, nullptr, &empty), BLAZ_ERR_ARG);
    EXPECT(validate_compress(A, 16, &x, (blaz_precision)7, nullptr, &empty), BLAZ_ERR_ARG);
    EXPECT(validate_compress(A, 16, &x, BLAZ_PREC_FP64, fake<const uint8_t>(0x300008), &empty), BLAZ_ERR_ALIGN);
    blaz_matrix x3 = mat(16, 16, 0x100000, 3);
    EXPECT(validate_compress(A, 16, &x3, BLAZ_PREC_FP32, nullptr, &empty), BLAZ_ERR_UNSUPPORTED);
    blaz_matrix e = mat(0, 16, 0);
    EXPECT(validate_compress(nullptr, 0, &e, BLAZ_PREC_FP64, nullptr, &empty), BLAZ_OK);
    EXPECT(empty, true);
    EXPECT(validate_decompress(&x, fake<const double>(0x200000), 16, &empty), BLAZ_OK);
    EXPECT(validate_decompress(&x, fake<const double>(0x200000), big, &empty), BLAZ_ERR_SHAPE);
    EXPECT(validate_decompress(&x, fake<const double>(0x200004), 16, &empty), BLAZ_ERR_ALIGN);

    // add / scale: aliasing rules
    blaz_matrix y = mat(16, 16, 0x400000), z = mat(16, 16, 0x500000);
    EXPECT(validate_add(&x, &y, &z, &empty), BLAZ_OK);
    EXPECT(validate_add(&x, &y, &x, &empty), BLAZ_OK);
    blaz_matrix zp = mat(16, 16, 0x100008);
    EXPECT(validate_add(&x, &y, &zp, &empty), BLAZ_ERR_ARG);
    blaz_matrix w = mat(16, 24, 0x600000);
    EXPECT(validate_add(&x, &w, &z, &empty), BLAZ_ERR_MISMATCH);
    EXPECT(validate_scale(&x, &x, &empty), BLAZ_OK);
    EXPECT(validate_scale(&x, &zp, &empty), BLAZ_ERR_ARG);
    blaz_matrix huge = mat(8 * 257, 8 * ((int64_t(1) << 24) - 1), uintptr_t(1) << 44);
    EXPECT(validate_scale(&huge, &huge, &empty), BLAZ_ERR_SHAPE);

    // dots: count limits (the output far from the index arrays, which it must
    // not overlap even at the largest count)
    const int64_t* idx = fake<const int64_t>(0x700000);
    const double* far_out = fake<const double>(uintptr_t(1) << 40);
    EXPECT(validate_dot(&x, idx, &y, idx, kMaxDots, far_out, &empty), BLAZ_OK);
    EXPECT(validate_dot(&x, idx, &y, idx, kMaxDots + 1, far_out, &empty), BLAZ_ERR_ARG);
    EXPECT(validate_dot(&x, idx, &y, idx, -1, far_out, &empty), BLAZ_ERR_ARG);
    EXPECT(validate_dot(&x, idx, &w, idx, 4, far_out, &empty), BLAZ_OK);
    EXPECT(validate_dot(&w, idx, &x, idx, 4, far_out, &empty), BLAZ_ERR_MISMATCH);
    EXPECT(validate_dot_dense(&x, idx, fake<const double>(0x900000), 16, 4, fake<const double>(0x800000), &empty),
           BLAZ_OK);
    EXPECT(validate_dot_dense(&x, idx, fake<const double>(0x900000), big, 4, fake<const double>(0x800000), &empty),
           BLAZ_ERR_SHAPE);
    EXPECT(validate_dot_dense(&x, idx, fake<const double>(0x900000), 17, 4, fake<const double>(0x800000), &empty),
           BLAZ_ERR_ALIGN);
    EXPECT(validate_dot_dense(&x, idx, fake<const double>(0x900000), 0, kMaxDots + 1, fake<const double>(0x800000),
                              &empty),
           BLAZ_ERR_ARG);
    // the output may not overlap the index arrays or the vectors
    EXPECT(validate_dot(&x, idx, &y, idx, 4, fake<const double>(0x700008), &empty), BLAZ_ERR_ARG);
    EXPECT(validate_dot_dense(&x, idx, fake<const double>(0x900000), 16, 4, fake<const double>(0x900000 + 8 * 60),
                              &empty),
           BLAZ_ERR_ARG);
    if (failures) return 1;
    std::printf("validation sanitizer run: ok\n");
    return 0;
}
