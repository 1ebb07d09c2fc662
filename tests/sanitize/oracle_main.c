/*
 * Driver for a sanitizer build of the oracle (AddressSanitizer and
 * UndefinedBehaviorSanitizer, host code only).  It runs every whole-matrix
 * entry point of oracle/blaz_oracle.c on small seeded inputs that include the
 * designed corner cases (constant and all-zero blocks, huge, tiny and
 * subnormal magnitudes, a single non-zero slope, sign-consistent blocks) and
 * on every tunable rate, in heap buffers sized exactly to the shapes, so that
 * any out-of-bounds access or undefined operation aborts the run.  It checks
 * a few invariants of the records and exits 0.
 */
#include <math.h>
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

void oracle_set_threads(int n);
int oracle_kept_count(int lines);
void oracle_compress(const double *A, int64_t rows, int64_t cols, int64_t lda, double *f, double *s, uint8_t *phi,
                     int8_t *codes, uint8_t *psi, double *code_x, double *phi_x);
void oracle_compress_predicted(const double *A, int64_t rows, int64_t cols, int64_t lda, double *f, double *s,
                               uint8_t *phi, int8_t *codes, uint8_t *psi, double *code_x, double *phi_x);
void oracle_compress_blocks(const double *A, int64_t cols, int64_t lda, const int64_t *blocks, int64_t count,
                            double *f, double *s, uint8_t *phi, int8_t *codes, double *code_x, double *phi_x,
                            int predicted);
void oracle_decompress(const double *f, const double *s, const uint8_t *phi, const int8_t *codes, int64_t rows,
                       int64_t cols, double *A, int64_t lda);
void oracle_compress_lines(const double *A, int64_t rows, int64_t cols, int64_t lda, int lines, int64_t cstride,
                           double *f, double *s, uint8_t *phi, int8_t *codes, double *code_x, double *phi_x);
void oracle_decompress_lines(const double *f, const double *s, const uint8_t *phi, const int8_t *codes,
                             int64_t rows, int64_t cols, int lines, int64_t cstride, double *A, int64_t lda);
void oracle_add_codes(int64_t nblk, int ncodes, int64_t cstride, const double *f1, const double *s1,
                      const uint8_t *phi1, const int8_t *c1, const double *f2, const double *s2,
                      const uint8_t *phi2, const int8_t *c2, double *f, double *s, uint8_t *phi, int8_t *codes);
void oracle_scale_codes(int64_t nblk, int ncodes, int64_t cstride, const double *f1, const double *s1,
                        const uint8_t *phi1, const int8_t *c1, double c, double *f, double *s, uint8_t *phi,
                        int8_t *codes);
void oracle_dot(const double *xf, const double *xs, const uint8_t *xphi, const int8_t *xc, int64_t n,
                const double *yf, const double *ys, const uint8_t *yphi, const int8_t *yc, int64_t cols_y,
                const int64_t *xrow, const int64_t *ycol, int64_t count, double *out);
void oracle_dot_dense(const double *xf, const double *xs, const uint8_t *xphi, const int8_t *xc, int64_t n,
                      const int64_t *xrow, const double *v, int64_t ldv, int64_t count, double *out);
void oracle_gemm(const double *A, int64_t lda, const double *B, int64_t ldb, double *C, int64_t ldc, int64_t m,
                 int64_t n, int64_t k);

static uint64_t state = 0x9E3779B97F4A7C15ull;
static double uniform(void)  /* splitmix64 */
{
    uint64_t z = (state += 0x9E3779B97F4A7C15ull);
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    z ^= z >> 31;
    return (double)(z >> 11) * 0x1p-53;
}

static void *xmalloc(size_t n)
{
    void *p = malloc(n ? n : 1);
    if (!p) exit(2);
    memset(p, 0, n ? n : 1);
    return p;
}

#define CHECK(c)                                                        \
    do {                                                                \
        if (!(c)) {                                                     \
            fprintf(stderr, "check failed at line %d: %s\n", __LINE__, #c); \
            return 1;                                                   \
        }                                                               \
    } while (0)

/* One block row of designed blocks followed by a smooth field. */
static void fill(double *A, int64_t rows, int64_t cols)
{
    for (int64_t i = 0; i < rows; ++i)
        for (int64_t j = 0; j < cols; ++j)
            A[i * cols + j] = sin(0.07 * (double)i + 0.11 * (double)j) + 1e-3 * (uniform() - 0.5);
    const int64_t nbc = cols / 8;
    for (int64_t J = 0; J < nbc; ++J)
        for (int u = 0; u < 8; ++u)
            for (int v = 0; v < 8; ++v) {
                double x;
                switch (J % 8) {
                    case 0: x = 2.5; break;                                   /* constant */
                    case 1: x = 0.0; break;                                   /* zero */
                    case 2: x = 1e300 * sin(u + 2.0 * v); break;              /* huge */
                    case 3: x = 1e-310 * cos((double)(u - v)); break;         /* subnormal */
                    case 4: x = (u == 7 && v == 7) ? 1e-3 : 0.0; break;       /* one slope */
                    case 5: x = 0.37 * (u + 1) * (v + 1); break;              /* sign-consistent */
                    case 6: x = ((u + v) % 2) ? -1.0 : 1.0; break;            /* checkerboard */
                    default: x = -exp(0.1 * (u + v)); break;
                }
                A[(size_t)u * cols + J * 8 + v] = x;
            }
}

int main(void)
{
    const int64_t rows = 48, cols = 64, nb = (rows / 8) * (cols / 8);
    for (int threads = 1; threads <= 2; ++threads) {
        oracle_set_threads(threads);
        double *A = xmalloc(sizeof(double) * rows * cols), *Bk = xmalloc(sizeof(double) * rows * cols);
        fill(A, rows, cols);
        double *f = xmalloc(8 * nb), *s = xmalloc(8 * nb), *cx = xmalloc(8 * 28 * nb), *px = xmalloc(8 * nb);
        uint8_t *phi = xmalloc(nb), *psi = xmalloc(64 * nb);
        int8_t *codes = xmalloc(28 * nb);
        oracle_compress(A, rows, cols, cols, f, s, phi, codes, psi, cx, px);
        for (int64_t b = 0; b < nb; ++b) CHECK(phi[b] >= 1);
        oracle_compress_predicted(A, rows, cols, cols, f, s, phi, codes, psi, cx, px);
        oracle_compress(A, rows, cols, cols, f, s, phi, codes, NULL, NULL, NULL);
        oracle_decompress(f, s, phi, codes, rows, cols, Bk, cols);
        /* constant block 0 rebuilds exactly */
        CHECK(Bk[0] == 2.5 && Bk[7 * cols + 7] == 2.5);

        int64_t pick[5] = {0, 1, 7, nb - 1, 13};
        double *f5 = xmalloc(40), *s5 = xmalloc(40), *cx5 = xmalloc(8 * 28 * 5), *px5 = xmalloc(40);
        uint8_t *phi5 = xmalloc(5);
        int8_t *c5 = xmalloc(28 * 5);
        oracle_compress_blocks(A, cols, cols, pick, 5, f5, s5, phi5, c5, cx5, px5, 0);
        oracle_compress_blocks(A, cols, cols, pick, 5, f5, s5, phi5, c5, cx5, px5, 1);

        /* Algorithms 1 and 2, every tunable rate */
        for (int L = 1; L <= 8; ++L) {
            const int n = oracle_kept_count(L);
            const int64_t stride = 4 * ((n + 3) / 4);
            double *fl = xmalloc(8 * nb), *sl = xmalloc(8 * nb), *cxl = xmalloc(8 * (size_t)n * nb),
                   *pxl = xmalloc(8 * nb), *fz = xmalloc(8 * nb), *sz = xmalloc(8 * nb);
            uint8_t *phil = xmalloc(nb), *phiz = xmalloc(nb);
            int8_t *cl = xmalloc((size_t)stride * nb), *cz = xmalloc((size_t)stride * nb);
            oracle_compress_lines(A, rows, cols, cols, L, stride, fl, sl, phil, cl, cxl, pxl);
            oracle_decompress_lines(fl, sl, phil, cl, rows, cols, L, stride, Bk, cols);
            oracle_add_codes(nb, n, stride, fl, sl, phil, cl, fl, sl, phil, cl, fz, sz, phiz, cz);
            oracle_scale_codes(nb, n, stride, fz, sz, phiz, cz, -1.5, fz, sz, phiz, cz);
            oracle_add_codes(nb, n, stride, fl, sl, phil, cl, fz, sz, phiz, cz, fz, sz, phiz, cz);
            for (int64_t b = 0; b < nb; ++b) {
                CHECK(phiz[b] >= 1);
                for (int t = 0; t < n; ++t) CHECK(cz[b * stride + t] >= -127 && cz[b * stride + t] <= 127);
            }
            free(fl); free(sl); free(cxl); free(pxl); free(fz); free(sz); free(phil); free(phiz); free(cl); free(cz);
        }

        /* dot products and the product on decompressed values */
        int64_t xr[4] = {0, 7, 8, rows - 1}, yc[4] = {0, 5, 63, 17};
        double out[4];
        double *V = xmalloc(sizeof(double) * 4 * cols);
        for (int64_t i = 0; i < 4 * cols; ++i) V[i] = 2.0 * uniform() - 1.0;
        /* Y = the first 64 x 48 of a 64 x 64 field: x (48 x 64) times y (64 x 48) */
        double *Y = xmalloc(sizeof(double) * cols * rows);
        for (int64_t i = 0; i < cols * rows; ++i) Y[i] = cos(0.01 * (double)i);
        const int64_t nby = (cols / 8) * (rows / 8);
        double *fy = xmalloc(8 * nby), *sy = xmalloc(8 * nby);
        uint8_t *phiy = xmalloc(nby);
        int8_t *cy = xmalloc(28 * nby);
        oracle_compress(Y, cols, rows, rows, fy, sy, phiy, cy, NULL, NULL, NULL);
        int64_t ycols[4] = {0, 5, 47, 17};
        (void)yc;
        oracle_dot(f, s, phi, codes, cols, fy, sy, phiy, cy, rows, xr, ycols, 4, out);
        oracle_dot_dense(f, s, phi, codes, cols, xr, V, cols, 4, out);
        oracle_dot_dense(f, s, phi, codes, cols, xr, V, 0, 4, out);
        double *Xd = xmalloc(sizeof(double) * rows * cols), *Yd = xmalloc(sizeof(double) * cols * rows),
               *C = xmalloc(sizeof(double) * rows * rows);
        oracle_decompress(f, s, phi, codes, rows, cols, Xd, cols);
        oracle_decompress(fy, sy, phiy, cy, cols, rows, Yd, rows);
        oracle_gemm(Xd, cols, Yd, rows, C, rows, rows, rows, cols);
        oracle_gemm(Xd, cols, Yd, rows, C, rows, rows, rows, 0);
        CHECK(C[0] == 0.0);

        free(A); free(Bk); free(f); free(s); free(cx); free(px); free(phi); free(psi); free(codes);
        free(f5); free(s5); free(cx5); free(px5); free(phi5); free(c5); free(V); free(Y); free(fy); free(sy);
        free(phiy); free(cy); free(Xd); free(Yd); free(C);
    }
    printf("oracle sanitizer run: ok\n");
    return 0;
}
