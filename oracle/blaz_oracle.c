/*
 * blaz_oracle.c -- plain, slow FP64 CPU oracle for the blaz method
 * (M. Martel, "Compressed Matrix Computations", arXiv 2202.13007).
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product library calls, links or
 * loads this file; only the tests, the smoke check and the CPU-baseline leg
 * of the benchmark do.  It shares no code, header, table or constant with the
 * HIP implementation: the DCT basis below is evaluated with libm cos() and
 * sqrt() at run time.
 *
 * Every stage is written in the paper's order and notation, one block at a
 * time, with direct sums (no fast or separable transform).  Where the paper is
 * silent about a detail the reading taken is stated at the function.
 *
 * Compressed layout (struct-of-arrays, 45 bytes per 8x8 block = 360 bits):
 *   f[nblk]        binary64, first element of the block
 *   s[nblk]        binary64, mean slope
 *   phi[nblk]      uint8, re-scaling factor
 *   codes[nblk*28] int8, the 28 kept DCT coefficients, kept positions
 *                  (rows 0-1 and columns 0-1) in row-major scan order
 * (the tunable-rate functions *_lines / *_codes keep 16L - L^2 codes per
 * block at a caller-given stride).
 * Block (I, J) of a rows x cols matrix has flat index I*(cols/8) + J.
 *
 * Threads: the whole-matrix loops below hand whole blocks (or whole output
 * rows, or whole queries) to OpenMP threads; every block's arithmetic is the
 * same sequential code whatever the thread count, so the results do not
 * depend on it.  oracle_set_threads() fixes the count (1 = serial).
 *
 * Build: gcc -O2 -ffp-contract=off -fopenmp -fPIC -shared (no fast-math).
 */
#include <math.h>
#include <omp.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define NB 8            /* block side */
#define NKEPT 28        /* coefficients kept by the quantization */

void oracle_set_threads(int n) { omp_set_num_threads(n > 0 ? n : 1); }
int oracle_max_threads(void) { return omp_get_max_threads(); }

/* ------------------------------------------------------------------------ */
/* Helpers                                                                   */
/* ------------------------------------------------------------------------ */

/* Pairwise sum of 64 values taken in row-major order: the first level adds
 * (x0+x1), (x2+x3), ..., each following level adds adjacent pairs of the
 * previous level.  The paper does not fix a summation order for the slope
 * (Eq. eqslope) or for the DC coefficient; this order is the one both sides
 * use so that s and the DC code are reproducible bit for bit. */
static double pairwise64(const double x[64])
{
    double t[64];
    memcpy(t, x, sizeof t);
    for (int n = 64; n > 1; n /= 2)
        for (int i = 0; i < n / 2; ++i)
            t[i] = t[2 * i] + t[2 * i + 1];
    return t[0];
}

/* alpha_i of the orthonormal DCT-II (Section "Basic Linear Algebra
 * Algorithms", the definition following Eq. eqdct2): sqrt(1/8) for i = 0,
 * sqrt(1/4) otherwise. */
static double alpha(int i) { return i == 0 ? sqrt(1.0 / 8.0) : sqrt(1.0 / 4.0); }

/* cos((2u+1) i pi / 16), the DCT-II kernel of Eq. eqdct. */
static double dct_cos(int i, int u) { return cos((2.0 * u + 1.0) * i * M_PI / 16.0); }

/* Is (i, j) one of the coefficients kept by the quantization.  The paper
 * keeps the first two lines and the first two columns, 28 values (Section
 * "Block Transform and Quantization").  The tunable rate its conclusion asks
 * for is read as the number L of kept lines: rows 0..L-1 and columns
 * 0..L-1, 16L - L^2 coefficients; L = 2 is the paper's scheme. */
static int kept_lines(int i, int j, int lines) { return i < lines || j < lines; }
int oracle_kept_count(int lines) { return 16 * lines - lines * lines; }

/* ------------------------------------------------------------------------ */
/* Compression stages for one 8x8 block (Section "Compression Scheme")       */
/* ------------------------------------------------------------------------ */

/* Normalization, Eq. (1) eqnorm.  The interior term is evaluated exactly as
 * printed: ((M_ij - M_i-1,j) + (M_ij - M_i,j-1)) / 2. */
void oracle_normalize(const double M[64], double delta[64])
{
    for (int i = 0; i < NB; ++i)
        for (int j = 0; j < NB; ++j) {
            double d;
            if (i == 0 && j == 0)
                d = 0.0;
            else if (i == 0)
                d = M[0 * NB + j] - M[0 * NB + j - 1];
            else if (j == 0)
                d = M[i * NB + 0] - M[(i - 1) * NB + 0];
            else
                d = ((M[i * NB + j] - M[(i - 1) * NB + j]) + (M[i * NB + j] - M[i * NB + j - 1])) / 2.0;
            delta[i * NB + j] = d;
        }
}

/* Mean slope, Eqs. eqslope and eqslope2: s = (1/K) sum |Delta_ij| with K the
 * number of non-zero Delta_ij.  A block whose Delta is all zero (a constant
 * block) has K = 0; the paper leaves s undefined there and we take s = 0.
 * The sum uses the pairwise order of pairwise64(). */
void oracle_slope(const double delta[64], int *K_out, double *s_out)
{
    double a[64];
    int K = 0;
    for (int e = 0; e < 64; ++e) {
        a[e] = fabs(delta[e]);
        if (delta[e] != 0.0)
            ++K;
    }
    double S1 = pairwise64(a);
    *K_out = K;
    *s_out = K > 0 ? S1 / (double)K : 0.0;
}

/* Delta' = (1/s) Delta (third equation of the slope paragraph).  With s = 0
 * (constant block) Delta' = 0. */
void oracle_divide_by_slope(const double delta[64], double s, double dprime[64])
{
    for (int e = 0; e < 64; ++e)
        dprime[e] = s != 0.0 ? delta[e] / s : 0.0;
}

/* Prediction, Eq. eqpredict (Section "Prediction").  s_max = max |Delta'|;
 * S = 256 equidistant points starting at s - s_max with spacing
 * 2 s_max / 256; Psi_ij is the index of the point nearest to Delta'_ij, the
 * smallest index on a tie.  Readings: the equation prints Delta_ij where the
 * text says Delta' (Delta' is used); the spacing 2 s_max / 256 and the raw
 * mean slope s as the centre are the readings that reproduce Example 4.
 * With s_max = 0 every Psi_ij is 0.  Brute force over all 256 points. */
void oracle_predict(const double dprime[64], double s, uint8_t psi[64])
{
    double smax = 0.0;
    for (int e = 0; e < 64; ++e)
        if (fabs(dprime[e]) > smax)
            smax = fabs(dprime[e]);
    for (int e = 0; e < 64; ++e) {
        if (smax == 0.0) {
            psi[e] = 0;
            continue;
        }
        double lo = s - smax;
        double step = 2.0 * smax / 256.0;
        int best = 0;
        double best_err = fabs(dprime[e] - lo);
        for (int k = 1; k < 256; ++k) {
            double sk = lo + k * step;
            double err = fabs(dprime[e] - sk);
            if (err < best_err) {
                best_err = err;
                best = k;
            }
        }
        psi[e] = (uint8_t)best;
    }
}

/* Two-dimensional DCT-II, Eq. eqdct, orthonormal alphas.  The transform is
 * applied to Delta' (the normalized block): that is the reading under which
 * Example 5 (phi = 20 and all 64 printed integers) is reproduced; the
 * equation's Psi_ij inside the double sum is read as Delta'_uv.
 *
 * D_00 = alpha_0^2 sum_uv Delta'_uv is the one coefficient whose exact value
 * lands on a truncation boundary for whole classes of blocks (when every
 * non-zero Delta has the same sign, sum Delta' = K exactly).  Its evaluation
 * order is therefore fixed: D_00 = 0.125 * (pairwise(Delta) / s), equal to
 * alpha_0^2 sum Delta' in exact arithmetic.  All other coefficients are the
 * direct double sum of Eq. eqdct. */
void oracle_dct(const double delta[64], double s, const double dprime[64], double D[64])
{
    for (int i = 0; i < NB; ++i)
        for (int j = 0; j < NB; ++j) {
            if (i == 0 && j == 0)
                continue;
            double acc = 0.0;
            for (int u = 0; u < NB; ++u)
                for (int v = 0; v < NB; ++v)
                    acc += dprime[u * NB + v] * dct_cos(i, u) * dct_cos(j, v);
            D[i * NB + j] = alpha(i) * alpha(j) * acc;
        }
    D[0] = s != 0.0 ? 0.125 * (pairwise64(delta) / s) : 0.0;
}

/* Reading B of the transform's input.  The paragraph on the transform names
 * the normalized block, Eq. eqdct and Example 5 name Psi; read literally as
 * "the slopes Psi predicts", the DCT takes the grid points Eq. eqpredict
 * selects, sp_ij = (s - s_max) + Psi_ij * (2 s_max / 256), instead of
 * Delta'.  (The default, reading A, takes Delta' and reproduces all 64
 * printed values of Example 5; reading B reproduces 62, giving -52 for the
 * printed -51 at (0,1) and (1,0).)  The grid points are evaluated as in
 * oracle_predict.  With s_max = 0 every sp_ij is s, which is then 0. */
void oracle_predicted_slopes(const double dprime[64], double s, const uint8_t psi[64], double sp[64])
{
    double smax = 0.0;
    for (int e = 0; e < 64; ++e)
        if (fabs(dprime[e]) > smax)
            smax = fabs(dprime[e]);
    double lo = s - smax;
    double step = 2.0 * smax / 256.0;
    for (int e = 0; e < 64; ++e)
        sp[e] = lo + psi[e] * step;
}

/* Eq. eqdct of an arbitrary 8x8 input x: the 63 non-DC coefficients by the
 * direct double sum, D_00 = alpha_0^2 sum x = 0.125 * pairwise(x), the fixed
 * order the GPU reproduces. */
void oracle_dct_of(const double x[64], double D[64])
{
    for (int i = 0; i < NB; ++i)
        for (int j = 0; j < NB; ++j) {
            if (i == 0 && j == 0)
                continue;
            double acc = 0.0;
            for (int u = 0; u < NB; ++u)
                for (int v = 0; v < NB; ++v)
                    acc += x[u * NB + v] * dct_cos(i, u) * dct_cos(j, v);
            D[i * NB + j] = alpha(i) * alpha(j) * acc;
        }
    D[0] = 0.125 * pairwise64(x);
}

/* Quantization (Section "Block Transform and Quantization", Eq. eqphi).
 * m = max |D_ij| over the whole 8x8 matrix D; phi = 127/m stored in 8 bits:
 * truncated (Example 5: 127/6.125 = 20.73 gives 20), clamped to 255 (phi can
 * exceed 255 when few Delta are non-zero), and 255 when m = 0.  The kept
 * coefficients are truncated toward zero: C = trunc(phi * D) (Example 5:
 * 20 * D_01 = -51.996 is printed -51).  phi_x and code_x return the values
 * before truncation. */
void oracle_quantize_lines(const double D[64], int lines, double *m_out, double *phi_x, int *phi_out,
                           double *code_x, int8_t *codes);

void oracle_quantize(const double D[64], double *m_out, double *phi_x, int *phi_out,
                     double code_x[NKEPT], int8_t codes[NKEPT])
{
    oracle_quantize_lines(D, 2, m_out, phi_x, phi_out, code_x, codes);
}

/* The same with the kept set of L lines (16L - L^2 codes, row-major scan). */
void oracle_quantize_lines(const double D[64], int lines, double *m_out, double *phi_x, int *phi_out,
                           double *code_x, int8_t *codes)
{
    double m = 0.0;
    for (int e = 0; e < 64; ++e)
        if (fabs(D[e]) > m)
            m = fabs(D[e]);
    int phi;
    double px = m > 0.0 ? 127.0 / m : INFINITY;
    if (!(px < 255.0))
        phi = 255;
    else
        phi = (int)trunc(px);
    int t = 0;
    for (int i = 0; i < NB; ++i)
        for (int j = 0; j < NB; ++j)
            if (kept_lines(i, j, lines)) {
                double x = (double)phi * D[i * NB + j];
                code_x[t] = x;
                codes[t] = (int8_t)trunc(x);
                ++t;
            }
    *m_out = m;
    *phi_x = px;
    *phi_out = phi;
}

/* Every intermediate of one block's compression, for the tests. */
typedef struct {
    double f;
    double delta[64];
    int K;
    double s;
    double dprime[64];
    uint8_t psi[64];
    double D[64];
    double m;
    double phi_x;
    int phi;
    double code_x[NKEPT];
    int8_t codes[NKEPT];
} oracle_block_trace;

size_t oracle_trace_size(void) { return sizeof(oracle_block_trace); }

/* The five stages in the paper's order for one block.  The first element is
 * stored as f (Section "Block Normalization", after Eq. eqnorm). */
void oracle_compress_block(const double M[64], oracle_block_trace *tr)
{
    tr->f = M[0];
    oracle_normalize(M, tr->delta);
    oracle_slope(tr->delta, &tr->K, &tr->s);
    oracle_divide_by_slope(tr->delta, tr->s, tr->dprime);
    oracle_predict(tr->dprime, tr->s, tr->psi);
    oracle_dct(tr->delta, tr->s, tr->dprime, tr->D);
    oracle_quantize(tr->D, &tr->m, &tr->phi_x, &tr->phi, tr->code_x, tr->codes);
}

/* The same stages with the DCT of the predicted slopes (reading B); the
 * trace's D holds that transform. */
void oracle_compress_block_predicted(const double M[64], oracle_block_trace *tr)
{
    double sp[64];
    tr->f = M[0];
    oracle_normalize(M, tr->delta);
    oracle_slope(tr->delta, &tr->K, &tr->s);
    oracle_divide_by_slope(tr->delta, tr->s, tr->dprime);
    oracle_predict(tr->dprime, tr->s, tr->psi);
    oracle_predicted_slopes(tr->dprime, tr->s, tr->psi, sp);
    oracle_dct_of(sp, tr->D);
    oracle_quantize(tr->D, &tr->m, &tr->phi_x, &tr->phi, tr->code_x, tr->codes);
}

typedef void (*block_fn)(const double M[64], oracle_block_trace *tr);

/* ------------------------------------------------------------------------ */
/* Decompression (Section "Dot product", Eqs. eqbbb0 and eqbbb)              */
/* ------------------------------------------------------------------------ */

/* Inverse DCT: P_uv = sum_ij alpha_i alpha_j D_ij cos(..i..u) cos(..j..v). */
void oracle_idct(const double D[64], double P[64])
{
    for (int u = 0; u < NB; ++u)
        for (int v = 0; v < NB; ++v) {
            double acc = 0.0;
            for (int i = 0; i < NB; ++i)
                for (int j = 0; j < NB; ++j)
                    acc += alpha(i) * alpha(j) * D[i * NB + j] * dct_cos(i, u) * dct_cos(j, v);
            P[u * NB + v] = acc;
        }
}

/* Inverse of the normalization, Eq. eqbbb: B_00 = f, then each element is
 * its predecessor(s) plus s * P.  Reading: the printed equation indexes P at
 * (0,j-1), (i-1,0) and (i-1,j-1); the exact inverse of Eq. eqnorm uses P at
 * (i,j) itself, which is what is implemented (the printed subscripts do not
 * reconstruct even an unquantized block). */
void oracle_inverse_normalize(double f, double s, const double P[64], double B[64])
{
    for (int i = 0; i < NB; ++i)
        for (int j = 0; j < NB; ++j) {
            double b;
            if (i == 0 && j == 0)
                b = f;
            else if (i == 0)
                b = B[0 * NB + j - 1] + s * P[0 * NB + j];
            else if (j == 0)
                b = B[(i - 1) * NB + 0] + s * P[i * NB + 0];
            else
                b = (B[(i - 1) * NB + j] + B[i * NB + j - 1]) / 2.0 + s * P[i * NB + j];
            B[i * NB + j] = b;
        }
}

/* Dequantization: the kept coefficients are C/phi, the discarded ones are
 * replaced by zeros (Section "Dot product", first paragraph). */
void oracle_dequantize_lines(int phi, int lines, const int8_t *codes, double D[64]);

void oracle_dequantize(int phi, const int8_t codes[NKEPT], double D[64]) { oracle_dequantize_lines(phi, 2, codes, D); }

void oracle_dequantize_lines(int phi, int lines, const int8_t *codes, double D[64])
{
    int t = 0;
    for (int i = 0; i < NB; ++i)
        for (int j = 0; j < NB; ++j) {
            if (kept_lines(i, j, lines)) {
                D[i * NB + j] = (double)codes[t] / (double)phi;
                ++t;
            } else {
                D[i * NB + j] = 0.0;
            }
        }
}

/* Full decompression of one block: dequantize, IDCT, inverse normalization. */
void oracle_decompress_block_lines(double f, double s, int phi, int lines, const int8_t *codes, double B[64])
{
    double D[64], P[64];
    oracle_dequantize_lines(phi, lines, codes, D);
    oracle_idct(D, P);
    oracle_inverse_normalize(f, s, P, B);
}

void oracle_decompress_block(double f, double s, int phi, const int8_t codes[NKEPT], double B[64])
{
    oracle_decompress_block_lines(f, s, phi, 2, codes, B);
}

/* ------------------------------------------------------------------------ */
/* Whole matrices (blockwise generalisation, end of Section "Basic Linear    */
/* Algebra Algorithms")                                                      */
/* ------------------------------------------------------------------------ */

static void load_block(const double *A, int64_t lda, int64_t I, int64_t J, double M[64])
{
    for (int i = 0; i < NB; ++i)
        for (int j = 0; j < NB; ++j)
            M[i * NB + j] = A[(I * NB + i) * lda + J * NB + j];
}

/* Compress a rows x cols row-major matrix (leading dimension lda).  psi,
 * code_x and phi_x are optional (NULL) debug outputs: Psi per element
 * ([nblk][64]), phi*D before truncation ([nblk][28]) and 127/m
 * ([nblk]). */
static void compress_with(block_fn block, const double *A, int64_t rows, int64_t cols, int64_t lda,
                          double *f, double *s, uint8_t *phi, int8_t *codes,
                          uint8_t *psi, double *code_x, double *phi_x)
{
    int64_t nbc = cols / NB, nbr = rows / NB;
#pragma omp parallel for schedule(static)
    for (int64_t I = 0; I < nbr; ++I)
        for (int64_t J = 0; J < nbc; ++J) {
            double M[64];
            oracle_block_trace tr;
            int64_t b = I * nbc + J;
            load_block(A, lda, I, J, M);
            block(M, &tr);
            f[b] = tr.f;
            s[b] = tr.s;
            phi[b] = (uint8_t)tr.phi;
            memcpy(codes + b * NKEPT, tr.codes, NKEPT);
            if (psi)
                memcpy(psi + b * 64, tr.psi, 64);
            if (code_x)
                memcpy(code_x + b * NKEPT, tr.code_x, NKEPT * sizeof(double));
            if (phi_x)
                phi_x[b] = tr.phi_x;
        }
}

void oracle_compress(const double *A, int64_t rows, int64_t cols, int64_t lda,
                     double *f, double *s, uint8_t *phi, int8_t *codes,
                     uint8_t *psi, double *code_x, double *phi_x)
{
    compress_with(oracle_compress_block, A, rows, cols, lda, f, s, phi, codes, psi, code_x, phi_x);
}

/* Reading B (DCT of the predicted slopes), same outputs. */
void oracle_compress_predicted(const double *A, int64_t rows, int64_t cols, int64_t lda,
                               double *f, double *s, uint8_t *phi, int8_t *codes,
                               uint8_t *psi, double *code_x, double *phi_x)
{
    compress_with(oracle_compress_block_predicted, A, rows, cols, lda, f, s, phi, codes, psi, code_x, phi_x);
}

/* Compress only the listed blocks (flat indices), for sampled comparisons at
 * sizes where compressing everything on the CPU would take too long;
 * predicted != 0 selects reading B of the transform's input. */
void oracle_compress_blocks(const double *A, int64_t cols, int64_t lda,
                            const int64_t *blocks, int64_t count,
                            double *f, double *s, uint8_t *phi, int8_t *codes,
                            double *code_x, double *phi_x, int predicted)
{
    int64_t nbc = cols / NB;
    block_fn block = predicted ? oracle_compress_block_predicted : oracle_compress_block;
#pragma omp parallel for schedule(static)
    for (int64_t q = 0; q < count; ++q) {
        double M[64];
        oracle_block_trace tr;
        int64_t b = blocks[q];
        load_block(A, lda, b / nbc, b % nbc, M);
        block(M, &tr);
        f[q] = tr.f;
        s[q] = tr.s;
        phi[q] = (uint8_t)tr.phi;
        memcpy(codes + q * NKEPT, tr.codes, NKEPT);
        if (code_x)
            memcpy(code_x + q * NKEPT, tr.code_x, NKEPT * sizeof(double));
        if (phi_x)
            phi_x[q] = tr.phi_x;
    }
}

void oracle_decompress(const double *f, const double *s, const uint8_t *phi, const int8_t *codes,
                       int64_t rows, int64_t cols, double *A, int64_t lda)
{
    int64_t nbc = cols / NB, nbr = rows / NB;
#pragma omp parallel for schedule(static)
    for (int64_t I = 0; I < nbr; ++I)
        for (int64_t J = 0; J < nbc; ++J) {
            double B[64];
            int64_t b = I * nbc + J;
            oracle_decompress_block(f[b], s[b], phi[b], codes + b * NKEPT, B);
            for (int i = 0; i < NB; ++i)
                for (int j = 0; j < NB; ++j)
                    A[(I * NB + i) * lda + J * NB + j] = B[i * NB + j];
        }
}

/* Tunable rate: compression and decompression with L kept lines.  The
 * codes of block b start at byte b * cstride (cstride >= 16L - L^2; the
 * bytes after the codes are left as the caller set them). */
void oracle_compress_lines(const double *A, int64_t rows, int64_t cols, int64_t lda, int lines, int64_t cstride,
                           double *f, double *s, uint8_t *phi, int8_t *codes, double *code_x, double *phi_x)
{
    int64_t nbc = cols / NB, nbr = rows / NB;
    int n = oracle_kept_count(lines);
    double M[64], delta[64], dprime[64], D[64], m, px, cx[64];
    int K, p;
    int8_t c[64];
    for (int64_t I = 0; I < nbr; ++I)
        for (int64_t J = 0; J < nbc; ++J) {
            int64_t b = I * nbc + J;
            double sb;
            load_block(A, lda, I, J, M);
            oracle_normalize(M, delta);
            oracle_slope(delta, &K, &sb);
            oracle_divide_by_slope(delta, sb, dprime);
            oracle_dct(delta, sb, dprime, D);
            oracle_quantize_lines(D, lines, &m, &px, &p, cx, c);
            f[b] = M[0];
            s[b] = sb;
            phi[b] = (uint8_t)p;
            memcpy(codes + b * cstride, c, (size_t)n);
            if (code_x)
                memcpy(code_x + b * n, cx, (size_t)n * sizeof(double));
            if (phi_x)
                phi_x[b] = px;
        }
}

void oracle_decompress_lines(const double *f, const double *s, const uint8_t *phi, const int8_t *codes,
                             int64_t rows, int64_t cols, int lines, int64_t cstride, double *A, int64_t lda)
{
    int64_t nbc = cols / NB, nbr = rows / NB;
    double B[64];
    for (int64_t I = 0; I < nbr; ++I)
        for (int64_t J = 0; J < nbc; ++J) {
            int64_t b = I * nbc + J;
            oracle_decompress_block_lines(f[b], s[b], phi[b], lines, codes + b * cstride, B);
            for (int i = 0; i < NB; ++i)
                for (int j = 0; j < NB; ++j)
                    A[(I * NB + i) * lda + J * NB + j] = B[i * NB + j];
        }
}

/* Addition of compressed blocks, Algorithm 1, for nblk blocks.
 *   f = f1 + f2 ; s = s1 + s2
 *   phi = int8(phi1 phi2 / (phi1 + phi2))   (integer division, Eq. eq55)
 *   alpha_k = s_k / (s1 + s2) ; beta_k = alpha_k / phi_k * phi
 *   C[i] = int8(beta1 C1[i] + beta2 C2[i])
 * Readings: int8() truncates toward zero; codes saturate to [-127, 127]
 * (|alpha_k| can exceed 1 when the slopes have opposite signs); phi is kept
 * at least 1 so that the result can be decompressed; when s1 + s2 = 0 the
 * alphas are undefined and the codes are 0 (the block is the constant f). */
void oracle_add_codes(int64_t nblk, int ncodes, int64_t cstride,
                      const double *f1, const double *s1, const uint8_t *phi1, const int8_t *c1,
                      const double *f2, const double *s2, const uint8_t *phi2, const int8_t *c2,
                      double *f, double *s, uint8_t *phi, int8_t *codes);

void oracle_add(int64_t nblk,
                const double *f1, const double *s1, const uint8_t *phi1, const int8_t *c1,
                const double *f2, const double *s2, const uint8_t *phi2, const int8_t *c2,
                double *f, double *s, uint8_t *phi, int8_t *codes)
{
    oracle_add_codes(nblk, NKEPT, NKEPT, f1, s1, phi1, c1, f2, s2, phi2, c2, f, s, phi, codes);
}

/* Algorithm 1 on blocks of ncodes codes stored cstride bytes apart (the
 * tunable-rate records; Algorithm 1 treats every kept code the same way). */
void oracle_add_codes(int64_t nblk, int ncodes, int64_t cstride,
                      const double *f1, const double *s1, const uint8_t *phi1, const int8_t *c1,
                      const double *f2, const double *s2, const uint8_t *phi2, const int8_t *c2,
                      double *f, double *s, uint8_t *phi, int8_t *codes)
{
#pragma omp parallel for schedule(static)
    for (int64_t b = 0; b < nblk; ++b) {
        double fb = f1[b] + f2[b];
        double sb = s1[b] + s2[b];
        int p1 = phi1[b], p2 = phi2[b];
        int p = (p1 * p2) / (p1 + p2);
        if (p < 1)
            p = 1;
        int8_t out[64];
        if (sb == 0.0) {
            memset(out, 0, sizeof out);
        } else {
            double a1 = s1[b] / sb;
            double a2 = s2[b] / sb;
            double b1 = a1 / (double)p1 * (double)p;
            double b2 = a2 / (double)p2 * (double)p;
            for (int t = 0; t < ncodes; ++t) {
                double x = b1 * (double)c1[b * cstride + t] + b2 * (double)c2[b * cstride + t];
                double y = trunc(x);
                if (y > 127.0)
                    y = 127.0;
                if (y < -127.0)
                    y = -127.0;
                out[t] = (int8_t)y;
            }
        }
        f[b] = fb;
        s[b] = sb;
        phi[b] = (uint8_t)p;
        memcpy(codes + b * cstride, out, (size_t)ncodes);
    }
}

/* Multiplication by a constant, Algorithm 2: f and s are multiplied by c,
 * phi and the codes are copied. */
void oracle_scale_codes(int64_t nblk, int ncodes, int64_t cstride, const double *f1, const double *s1,
                        const uint8_t *phi1, const int8_t *c1, double c, double *f, double *s, uint8_t *phi,
                        int8_t *codes)
{
#pragma omp parallel for schedule(static)
    for (int64_t b = 0; b < nblk; ++b) {
        f[b] = f1[b] * c;
        s[b] = s1[b] * c;
        phi[b] = phi1[b];
        memcpy(codes + b * cstride, c1 + b * cstride, (size_t)ncodes);
    }
}

void oracle_scale(int64_t nblk, const double *f1, const double *s1, const uint8_t *phi1,
                  const int8_t *c1, double c, double *f, double *s, uint8_t *phi, int8_t *codes)
{
    oracle_scale_codes(nblk, NKEPT, NKEPT, f1, s1, phi1, c1, c, f, s, phi, codes);
}

/* Decompress the listed rows of a compressed matrix into out[count][cols]
 * (each row's blocks are decompressed whole; Eq. eqbbb gives the same row
 * values whether or not the later rows are computed). */
static void decompress_row(const double *f, const double *s, const uint8_t *phi, const int8_t *codes,
                           int64_t cols, int64_t i, double *row)
{
    int64_t nbc = cols / NB, I = i / NB;
    double B[64];
    for (int64_t J = 0; J < nbc; ++J) {
        int64_t b = I * nbc + J;
        oracle_decompress_block(f[b], s[b], phi[b], codes + b * NKEPT, B);
        for (int k = 0; k < NB; ++k)
            row[J * NB + k] = B[(i % NB) * NB + k];
    }
}

static void decompress_col(const double *f, const double *s, const uint8_t *phi, const int8_t *codes,
                           int64_t rows, int64_t cols, int64_t j, double *col)
{
    int64_t nbc = cols / NB, nbr = rows / NB, J = j / NB;
    double B[64];
    for (int64_t I = 0; I < nbr; ++I) {
        int64_t b = I * nbc + J;
        oracle_decompress_block(f[b], s[b], phi[b], codes + b * NKEPT, B);
        for (int k = 0; k < NB; ++k)
            col[I * NB + k] = B[k * NB + (j % NB)];
    }
}

/* Dot product, Algorithm 3 and Eq. eqbbb0 applied blockwise: line xrow[q] of
 * X with column ycol[q] of Y, X being rows_x x n and Y n x cols_y, on the
 * decompressed values, summed sequentially over k. */
void oracle_dot(const double *xf, const double *xs, const uint8_t *xphi, const int8_t *xc, int64_t n,
                const double *yf, const double *ys, const uint8_t *yphi, const int8_t *yc, int64_t cols_y,
                const int64_t *xrow, const int64_t *ycol, int64_t count, double *out)
{
#pragma omp parallel
    {
        double *r = (double *)malloc(sizeof(double) * (size_t)n);
        double *c = (double *)malloc(sizeof(double) * (size_t)n);
#pragma omp for schedule(static)
        for (int64_t q = 0; q < count; ++q) {
            decompress_row(xf, xs, xphi, xc, n, xrow[q], r);
            decompress_col(yf, ys, yphi, yc, n, cols_y, ycol[q], c);
            double acc = 0.0;
            for (int64_t k = 0; k < n; ++k)
                acc += r[k] * c[k];
            out[q] = acc;
        }
        free(r);
        free(c);
    }
}

/* Dot product of line xrow[q] of compressed X (n columns) with a dense
 * vector v_q = v + q*ldv (ldv = 0: one shared vector). */
void oracle_dot_dense(const double *xf, const double *xs, const uint8_t *xphi, const int8_t *xc, int64_t n,
                      const int64_t *xrow, const double *v, int64_t ldv, int64_t count, double *out)
{
#pragma omp parallel
    {
        double *r = (double *)malloc(sizeof(double) * (size_t)n);
#pragma omp for schedule(static)
        for (int64_t q = 0; q < count; ++q) {
            decompress_row(xf, xs, xphi, xc, n, xrow[q], r);
            const double *vq = v + q * ldv;
            double acc = 0.0;
            for (int64_t k = 0; k < n; ++k)
                acc += r[k] * vq[k];
            out[q] = acc;
        }
        free(r);
    }
}

/* Plain i-k-j product C = A B of dense row-major matrices, m x k times
 * k x n.  The matrix multiplication of the paper (last paragraph of Section
 * "Basic Linear Algebra Algorithms") decompresses each block once and then
 * multiplies; the tests feed this routine oracle-decompressed operands. */
void oracle_gemm(const double *A, int64_t lda, const double *B, int64_t ldb,
                 double *C, int64_t ldc, int64_t m, int64_t n, int64_t k)
{
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < m; ++i) {
        for (int64_t j = 0; j < n; ++j)
            C[i * ldc + j] = 0.0;
        for (int64_t p = 0; p < k; ++p) {
            double a = A[i * lda + p];
            for (int64_t j = 0; j < n; ++j)
                C[i * ldc + j] += a * B[p * ldb + j];
        }
    }
}
