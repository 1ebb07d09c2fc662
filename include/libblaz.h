/*
 * libblaz.h -- C ABI of the blaz compressed-matrix library for MI355X (gfx950).
 *
 * The method is M. Martel, "Compressed Matrix Computations" (arXiv
 * 2202.13007): a lossy, fixed-rate codec for 8x8 blocks of binary64 (block
 * splitting, normalization, prediction, DCT-II, quantization; Section
 * "Compression Scheme") and the operations that run on the compressed form
 * (addition, Algorithm 1; multiplication by a constant, Algorithm 2) or on
 * partly decompressed blocks (dot product, Algorithm 3 with Eqs. eqbbb0 and
 * eqbbb; matrix multiplication, last paragraph of Section "Basic Linear
 * Algebra Algorithms").
 *
 * Conventions for every entry point:
 *  - Data pointers (matrices, compressed arrays, index and output arrays,
 *    workspaces) are DEVICE pointers.  The blaz_matrix descriptor itself is
 *    host memory and is read during the call only.
 *  - A call validates its arguments synchronously and returns a non-zero
 *    blaz_status before anything is enqueued; on success the work is
 *    enqueued on `stream` (0 = the null stream) and the call returns without
 *    synchronizing.  No call allocates device memory, and none keeps a
 *    pointer after it returns.
 *  - A launch failure reported by the HIP runtime returns BLAZ_ERR_HIP.
 *  - Data conditions are not errors: saturated codes in an addition, phi
 *    clamps, constant blocks.  Non-finite inputs give unspecified contents
 *    in the affected blocks.  blaz_diagnose counts them in a compressed
 *    matrix.
 *  - Matrices are row-major binary64 with a leading dimension (elements)
 *    >= cols.  rows and cols must be multiples of 8 (the paper splits into
 *    8x8 blocks and gives no padding rule); 0 is allowed and gives an empty
 *    matrix on which every call is a successful no-op.
 */
#ifndef LIBBLAZ_H
#define LIBBLAZ_H

#include <stddef.h>
#include <stdint.h>

#include <hip/hip_runtime_api.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    BLAZ_OK = 0,
    BLAZ_ERR_NULL = -1,        /* a required pointer is NULL                          */
    BLAZ_ERR_SHAPE = -2,       /* rows/cols negative or not a multiple of 8, more than
                                  2^32 - 256 blocks, ld < cols, a dense operand whose
                                  last element lies 2^60 or more elements past its
                                  first, or a product whose launches would exceed one
                                  dispatch's 2^32 - 1 work-items                     */
    BLAZ_ERR_MISMATCH = -3,    /* operand shapes do not agree                         */
    BLAZ_ERR_ALIGN = -4,       /* a pointer is not aligned to its element type         */
    BLAZ_ERR_ARG = -5,         /* another invalid argument (count < 0 or a dot count
                                  above 2^27 - 8, bad enum, overlap, an array or
                                  operand whose extent passes the top of the address
                                  space)                                             */
    BLAZ_ERR_UNSUPPORTED = -6, /* a valid request the library does not implement       */
    BLAZ_ERR_WORKSPACE = -7,   /* workspace missing or smaller than required           */
    BLAZ_ERR_HIP = -8,         /* the HIP runtime reported an error                    */
    BLAZ_ERR_TOO_LARGE = -9    /* blaz_matmul_static: the product's workspace exceeds
                                  BLAZ_STATIC_SCRATCH_BYTES                           */
} blaz_status;

/* Arithmetic of the DCT stage in blaz_compress and of the contraction in
 * blaz_matmul.  BLAZ_PREC_FP64 is the plain method and the default. */
typedef enum {
    BLAZ_PREC_FP64 = 0,
    BLAZ_PREC_FP32 = 1,   /* FP32 operands on MFMA, FP32 accumulation               */
    BLAZ_PREC_BF16X3 = 2  /* operands split into BF16 hi + lo, three MFMA products,  */
                          /* FP32 accumulation                                       */
} blaz_precision;

/* A compressed rows x cols matrix: one record per 8x8 block, 45 bytes =
 * the paper's 360 bits (Section "Compression Scheme", last paragraph), kept
 * as four arrays.  Block (I, J) -- rows 8I..8I+7, columns 8J..8J+7 -- has
 * index b = I*(cols/8) + J.
 *   f[b]        first element M_00 of the block (binary64)
 *   s[b]        mean slope s, Eq. eqslope (binary64)
 *   phi[b]      re-scaling factor phi, Eq. eqphi (8-bit unsigned, >= 1)
 *   codes[28*b + t], t = 0..27
 *               the kept DCT coefficients trunc(phi * D_ij), int8, for the
 *               positions of the first two lines and first two columns in
 *               row-major order: (0,0..7), (1,0..7), (2,0), (2,1), ...,
 *               (7,0), (7,1).
 * lines: the tunable rate the paper's conclusion asks for, as the number L
 *   of kept lines (1..8): rows and columns 0..L-1 of the DCT, 16L - L^2
 *   codes in row-major scan order, stored blaz_code_stride(L) bytes apart
 *   (padded with zeros to whole 32-bit words).  0 means 2, the paper's
 *   scheme above, so a zero-initialized descriptor is the paper's format.
 *   Compression, decompression, add, sub, scale and matmul take any L (the
 *   operands of add, sub and scale share it, else BLAZ_ERR_MISMATCH; the two
 *   factors of a product may differ); the dot products, the low-precision
 *   transforms, the prediction side output and batching take L = 2 only
 *   (BLAZ_ERR_UNSUPPORTED otherwise).
 * The caller owns the four arrays (device memory): f and s 8-byte aligned,
 * codes 4-byte aligned. */
typedef struct blaz_matrix {
    int64_t rows;
    int64_t cols;
    double *f;
    double *s;
    uint8_t *phi;
    int8_t *codes;
    int64_t lines;
} blaz_matrix;

/* Number of 8x8 blocks of a rows x cols matrix, or a negative blaz_status
 * if the shape is invalid. */
int64_t blaz_block_count(int64_t rows, int64_t cols);

/* Bytes of the compressed form (45 per block), 0 for an invalid shape. */
size_t blaz_compressed_bytes(int64_t rows, int64_t cols);

/* Bytes of the codes of one block with L kept lines (0 = 2):
 * 4 * ceil((16L - L^2) / 4), i.e. 16, 28, 40, 48, 56, 60, 64, 64 for
 * L = 1..8; a negative blaz_status for L outside 0..8. */
int64_t blaz_code_stride(int64_t lines);

/* Bytes of the compressed form with L kept lines: (17 + code stride) per
 * block; 0 for an invalid shape or L. */
size_t blaz_compressed_bytes_lines(int64_t rows, int64_t cols, int64_t lines);

/* Compression (Section "Compression Scheme"): block splitting, normalization
 * (Eq. eqnorm), mean slope (Eqs. eqslope, eqslope2), prediction (Eq.
 * eqpredict), DCT-II (Eq. eqdct) and quantization (Eq. eqphi) of every
 * 8x8 block of A (out->rows x out->cols, leading dimension lda >= cols,
 * 8-byte aligned) into *out.
 * psi: optional ([nblk][64] uint8, row-major within the block) receives the
 *   prediction indexes Psi of Eq. eqpredict: for each element the first index
 *   of the grid point nearest to Delta'_ij = Delta_ij / s, as a search over
 *   all 256 points in increasing order finds it.  They are not part of the
 *   stored stream: the transform is applied to the normalized block (the
 *   reading under which Example 5 is reproduced), so Psi is a side output
 *   and the record does not depend on whether it is requested.  NULL skips
 *   it.
 * prec: BLAZ_PREC_FP64 runs every stage in binary64.  BLAZ_PREC_FP32 and
 *   BLAZ_PREC_BF16X3 run the 63 non-DC DCT coefficients in that arithmetic on
 *   MFMA; normalization, slope, DC term, phi and truncation stay binary64.
 * A and the output arrays must not overlap. */
blaz_status blaz_compress(const double *A, int64_t lda, const blaz_matrix *out, blaz_precision prec,
                          uint8_t *psi, hipStream_t stream);

/* Compression under the other reading of the transform's input (Section
 * "Compression Scheme", paragraph "Block Transform and Quantization": the
 * text names the normalized block, Eq. eqdct and Example 5 name Psi).  Here
 * the DCT-II takes the predicted slopes, the grid points
 * (s - s_max) + Psi_ij * (2 s_max / 256) of Eq. eqpredict that Psi selects,
 * with D_00 = 0.125 * (their sum in the pairwise order of the slope);
 * everything else, the record format and blaz_decompress are those of
 * blaz_compress (binary64).  On Example 5 this reading gives 62 of the 64
 * printed values (-52 for the printed -51 at (0,1) and (1,0)).
 * psi: optional side output as in blaz_compress.  out must hold two kept
 * lines (lines 0 or 2), else BLAZ_ERR_UNSUPPORTED; other arguments and
 * errors as blaz_compress with BLAZ_PREC_FP64. */
blaz_status blaz_compress_predicted(const double *A, int64_t lda, const blaz_matrix *out, uint8_t *psi,
                                    hipStream_t stream);

/* Decompression: dequantize (C/phi at the kept positions, zero elsewhere;
 * Section "Dot product"), inverse DCT, and the inverse of the normalization
 * (Eq. eqbbb read as the exact inverse of Eq. eqnorm) of every block of *in
 * into A (in->rows x in->cols, leading dimension lda >= cols, 8-byte
 * aligned).  A must not overlap the compressed arrays. */
blaz_status blaz_decompress(const blaz_matrix *in, double *A, int64_t lda, hipStream_t stream);

/* Addition of compressed matrices, Algorithm 1, blockwise: z = x + y.
 * f = f1 + f2; s = s1 + s2; phi = max(1, floor(phi1 phi2 / (phi1 + phi2)));
 * alpha_k = s_k / s; beta_k = (alpha_k / phi_k) * phi;
 * C = trunc(beta1 C1 + beta2 C2) saturated to [-127, 127]; C = 0 when s = 0.
 * All three descriptors must have the same shape and kept lines; z may be x
 * or y (in place), otherwise it must not overlap them. */
blaz_status blaz_add(const blaz_matrix *x, const blaz_matrix *y, const blaz_matrix *z, hipStream_t stream);

/* Subtraction z = x - y, which the paper says works like the addition:
 * Algorithm 1 applied to x and (-1) * y (Algorithm 2), fused in one pass.
 * Same shape and aliasing rules as blaz_add. */
blaz_status blaz_sub(const blaz_matrix *x, const blaz_matrix *y, const blaz_matrix *z, hipStream_t stream);

/* Multiplication by a constant, Algorithm 2, blockwise: z = c x.
 * f and s are multiplied by c; phi and the codes are copied (not touched
 * when z == x, the in-place form). */
blaz_status blaz_scale(const blaz_matrix *x, double c, const blaz_matrix *z, hipStream_t stream);

/* Dot products, Algorithm 3 with Eqs. eqbbb0 and eqbbb applied blockwise:
 * out[q] = sum_k X[xrow[q], k] * Y[k, ycol[q]] over the decompressed values,
 * for q = 0..count-1.  Only the lines 0..(xrow mod 8) of the blocks of X and
 * the columns 0..(ycol mod 8) of the blocks of Y that the product needs are
 * rebuilt.  x->cols must equal y->rows.  xrow and ycol are device arrays of
 * count int64; an index outside its matrix yields out[q] = NaN.  Queries are
 * taken 8 at a time: 8 consecutive queries on the lines 8I..8I+7 in order
 * (and the columns 8J..8J+7 of Y in order) rebuild each block once for the 8;
 * every query gets the same bits either way.  A call takes at most
 * 2^27 - 8 queries (32 lanes each in one dispatch of at most 2^32 - 1
 * work-items); more is BLAZ_ERR_ARG.  out (count doubles, 8-byte aligned;
 * xrow and ycol 8-byte aligned) must not overlap x, y, xrow or ycol
 * (BLAZ_ERR_ARG). */
blaz_status blaz_dot(const blaz_matrix *x, const int64_t *xrow, const blaz_matrix *y, const int64_t *ycol,
                     int64_t count, double *out, hipStream_t stream);

/* Dot products of lines of a compressed matrix with dense vectors:
 * out[q] = sum_k X[xrow[q], k] * v[q*ldv + k].  ldv = 0 uses one vector for
 * every q; otherwise ldv >= x->cols.  v is 16-byte aligned and, when
 * ldv != 0, ldv is even.  An index outside X yields NaN.  At most 2^27 - 8
 * queries, as for blaz_dot.  out must not overlap x, xrow or the vectors
 * (BLAZ_ERR_ARG). */
blaz_status blaz_dot_dense(const blaz_matrix *x, const int64_t *xrow, const double *v, int64_t ldv,
                           int64_t count, double *out, hipStream_t stream);

/* Bytes of workspace blaz_matmul needs for an m x k times k x n product
 * (b_compressed != 0: B is compressed too). */
size_t blaz_matmul_workspace_bytes(int64_t m, int64_t n, int64_t k, int b_compressed, blaz_precision prec);

/* Matrix multiplication on partly decompressed operands (last paragraph of
 * Section "Basic Linear Algebra Algorithms"): every block of A (and of B when
 * it is compressed) is decompressed once into the workspace, then the
 * product C = A B (m x n, leading dimension ldc >= n) is formed on the
 * matrix cores; m = a->rows, k = a->cols.  B is either compressed
 * (b != NULL with b->rows == k and b->cols == n, bdense == NULL) or dense
 * binary64 (b == NULL, bdense k x n with leading dimension ldb >= n, ldb
 * even, 16-byte aligned; it may be NULL only when k == 0).  Passing both
 * forms is BLAZ_ERR_ARG.  k == 0 writes zeros to C.
 * prec selects the contraction arithmetic (FP64, FP32, or BF16x3 with FP32
 * accumulation); the output is binary64 in every case.  workspace must hold
 * blaz_matmul_workspace_bytes() bytes, 256-byte aligned.  C must not overlap
 * the inputs or the workspace, and the workspace must not overlap the inputs
 * (BLAZ_ERR_ARG). */
blaz_status blaz_matmul(const blaz_matrix *a, const blaz_matrix *b, const double *bdense, int64_t n,
                        int64_t ldb, double *c, int64_t ldc, blaz_precision prec, void *workspace,
                        size_t ws_bytes, hipStream_t stream);

/* blaz_matmul with an explicit output tile for the contraction: 128 (a
 * 128 x 128 tile per workgroup) or 64; 0 lets the library choose, as
 * blaz_matmul does (128 when that still gives every compute unit a
 * workgroup, 64 below).  Results are the same for every tile: the K loop and
 * its summation order do not depend on it.  Any other value is BLAZ_ERR_ARG.
 * This is the knob the autotuner of the Python package sets per size class. */
blaz_status blaz_matmul_tiled(const blaz_matrix *a, const blaz_matrix *b, const double *bdense, int64_t n,
                              int64_t ldb, double *c, int64_t ldc, blaz_precision prec, void *workspace,
                              size_t ws_bytes, int32_t tile, hipStream_t stream);

/* Bytes of the library's static scratch array: device memory that every
 * device the library runs on holds from the library's load until the
 * process ends, used as the workspace of blaz_matmul_static. */
#define BLAZ_STATIC_SCRATCH_BYTES ((size_t)256 << 20)

/* blaz_matmul without a workspace argument, for callers that cannot allocate
 * device memory (code under HIP graph capture, serving loops and harnesses
 * that forbid allocation).  Same operands, results and errors as
 * blaz_matmul (bit for bit: the same kernels run), with the workspace taken
 * from the library's static scratch array of BLAZ_STATIC_SCRATCH_BYTES
 * bytes (256 MiB: every product up to 4096 x 4096 x 4096 in every operand
 * form and precision fits).  A product whose workspace
 * (blaz_matmul_workspace_bytes) exceeds it returns BLAZ_ERR_TOO_LARGE before
 * anything is enqueued.  The call allocates nothing: the first call on a
 * device looks up that device's address of the array (make it once before
 * capturing a graph).  Every call on a device shares that device's array,
 * which keeps the last call's contents (no call needs it cleared): calls
 * whose work may overlap on one device -- on different streams, or from
 * different host threads without ordering -- race on it and give undefined
 * results; calls on one stream are ordered and safe. */
blaz_status blaz_matmul_static(const blaz_matrix *a, const blaz_matrix *b, const double *bdense, int64_t n,
                               int64_t ldb, double *c, int64_t ldc, blaz_precision prec, hipStream_t stream);

/* Bytes of workspace blaz_matmul_compressed needs: the contraction's own
 * workspace plus an m x n binary64 staging area for the product. */
size_t blaz_matmul_compressed_workspace_bytes(int64_t m, int64_t n, int64_t k, int b_compressed,
                                              blaz_precision prec);

/* Matrix multiplication with a compressed result: C = A B as in
 * blaz_matmul_tiled (same operand forms, prec and tile), then C is
 * compressed blockwise into c (c->rows == a->rows, c->cols == n, else
 * BLAZ_ERR_MISMATCH) with the binary64 transform, so a product can stay
 * resident in the 45-byte form.  The paper leaves the output form of the
 * product open (last paragraph of Section "Basic Linear Algebra Algorithms");
 * this entry point gives the compressed one.  The result is bit for bit the
 * compression of blaz_matmul_tiled's output.  workspace holds
 * blaz_matmul_compressed_workspace_bytes() bytes, 256-byte aligned; c must
 * not overlap the inputs or the workspace. */
blaz_status blaz_matmul_compressed(const blaz_matrix *a, const blaz_matrix *b, const double *bdense, int64_t n,
                                   int64_t ldb, blaz_matrix *c, blaz_precision prec, void *workspace,
                                   size_t ws_bytes, int32_t tile, hipStream_t stream);

/* Counts of the data conditions in a compressed matrix, added (atomically,
 * so several calls may accumulate into the same array) to counters[0..3],
 * a device array of 4 uint64 the caller zeroes:
 *   [0] constant blocks: s == 0 (K = 0 in Eq. eqslope2; they decode to f)
 *   [1] phi clamps: blocks with s != 0 and phi == 255 (127/m >= 255, few
 *       non-zero slopes; reading of Eq. eqphi's 8-bit storage)
 *   [2] codes at +-127: the saturation bound of an addition (Algorithm 1),
 *       also reached without saturation when phi * m == 127 exactly
 *   [3] non-finite records: f or s is not finite
 * Reads the matrix only; the kept lines of any rate are counted.  counters
 * 8-byte aligned, not overlapping the matrix. */
blaz_status blaz_diagnose(const blaz_matrix *x, uint64_t *counters, hipStream_t stream);

/* ---------------------------------------------------------------------------
 * Batching: many operations, on matrices of any sizes, in one persistent
 * launch.  Every 8x8 block is independent (the paper's blockwise
 * generalisation, end of Section "Basic Linear Algebra Algorithms"), so the
 * work of a batch is a flat queue of chunks -- 64 consecutive blocks of one
 * compress / decompress / add / sub / scale, or one dot product -- that the
 * launched workgroups pop with an atomic counter until the queue is empty.
 * Each operation computes exactly what its standalone entry point computes
 * (the same per-block code runs), bit for bit.
 *
 * Usage: blaz_batch_plan() validates the items with the same rules as the
 * standalone calls and writes a plan image into caller-owned HOST memory;
 * the caller copies that image to device memory (any stream-ordered copy);
 * blaz_batch_run() then enqueues the launch.  The device plan can be run any
 * number of times, including from a captured HIP graph: a run is two kernel
 * launches (a one-thread counter reset, then the persistent kernel) and no
 * memset or copy.  The items of one batch run concurrently: no item may read
 * or write another item's output.  In a batch, the dense matrix of a
 * COMPRESS or DECOMPRESS item must be 16-byte aligned with an even ld.
 * ------------------------------------------------------------------------- */
typedef enum {
    BLAZ_OP_COMPRESS = 0,   /* x <- compress(dense, ld); binary64 transform      */
    BLAZ_OP_DECOMPRESS = 1, /* dense (ld) <- decompress(x)                       */
    BLAZ_OP_ADD = 2,        /* z <- x + y (Algorithm 1)                          */
    BLAZ_OP_SUB = 3,        /* z <- x - y                                        */
    BLAZ_OP_SCALE = 4,      /* z <- c x (Algorithm 2)                            */
    BLAZ_OP_DOT = 5,        /* out[q] <- <line xrow[q] of x, column ycol[q] of y> */
    BLAZ_OP_DOT_DENSE = 6   /* out[q] <- <line xrow[q] of x, dense + q*ld>       */
} blaz_op;

/* One operation of a batch (host memory; the pointers inside are device
 * pointers, with the layouts and alignment of the standalone calls). */
typedef struct blaz_batch_item {
    int32_t op;           /* a blaz_op                                            */
    int32_t reserved;     /* must be 0                                            */
    blaz_matrix x;        /* COMPRESS: output; others: first operand              */
    blaz_matrix y;        /* ADD, SUB: second operand; DOT: right operand         */
    blaz_matrix z;        /* ADD, SUB, SCALE: output                              */
    double *dense;        /* COMPRESS: input; DECOMPRESS: output; DOT_DENSE: vectors */
    int64_t ld;           /* leading dimension of dense (DOT_DENSE: ldv, 0 = shared) */
    double c;             /* SCALE: the constant                                  */
    const int64_t *xrow;  /* DOT, DOT_DENSE: line indices (count)                 */
    const int64_t *ycol;  /* DOT: column indices (count)                          */
    int64_t count;        /* DOT, DOT_DENSE: number of products                   */
    double *out;          /* DOT, DOT_DENSE: results (count)                      */
} blaz_batch_item;

/* Bytes of the plan image for n_items items (an upper bound: items with
 * nothing to do are dropped from the plan). */
size_t blaz_batch_plan_bytes(int64_t n_items);

/* Validate items[0..n_items) and write the plan image into plan (host,
 * plan_bytes >= blaz_batch_plan_bytes(n_items), 8-byte aligned).  On success
 * *n_plan is the number of planned items and *total_chunks the length of the
 * work queue.  On failure *n_plan holds the index of the first invalid item
 * and nothing is written to device memory (nothing is, in any case: this is
 * a host-only function).  Items that would read or write another item's
 * output are refused with BLAZ_ERR_ARG, *n_plan naming the later of the two;
 * items may share inputs. */
blaz_status blaz_batch_plan(const blaz_batch_item *items, int64_t n_items, void *plan, size_t plan_bytes,
                            int64_t *n_plan, int64_t *total_chunks);

/* Run a plan whose image has been copied to plan_dev (device, 8-byte
 * aligned).  counter: 8 bytes of device memory owned by the caller, reset
 * by the run itself; concurrent runs need distinct counters.  workgroups:
 * number of persistent workgroups (one wave each); 0 picks 8 per compute
 * unit of the current device.  chunks_per_claim: consecutive chunks a wave
 * takes per pop of the counter, 1..64 (0 means 1): fewer atomics against
 * coarser load balance; results do not depend on it.  n_plan and
 * total_chunks as returned by blaz_batch_plan. */
blaz_status blaz_batch_run(const void *plan_dev, int64_t n_plan, int64_t total_chunks, uint64_t *counter,
                           int64_t workgroups, int32_t chunks_per_claim, hipStream_t stream);

/* Run state of a resident plan buffer (device memory, 8-byte aligned). */
typedef struct blaz_batch_state {
    int64_t n_plan;        /* written by the caller: blaz_batch_plan's *n_plan         */
    int64_t total_chunks;  /* written by the caller: blaz_batch_plan's *total_chunks   */
    uint64_t counter;      /* work counter: 0 before a run, and 0 again after it       */
    int64_t status;        /* written by each run: BLAZ_OK, or BLAZ_ERR_ARG when the   */
                           /* counts are out of range (then the run does nothing else) */
} blaz_batch_state;

/* Run whatever plan was last copied into plan_dev, reading its counts from
 * *state when the launch executes rather than when it is enqueued, so that
 * one captured HIP graph of this call replays every later plan that is
 * copied into the same buffers (a serving loop's request steps).  plan_dev:
 * device buffer of `capacity` planned items (blaz_batch_plan_bytes(capacity)
 * bytes, 8-byte aligned), 1 <= capacity <= 2^30; the caller copies a plan
 * image and the whole state record (counter 0) stream-ordered before a
 * run.  The run is one kernel launch and no memset or copy: the wave that
 * makes its last claim resets the counter, so a plan can also be run again
 * without a new copy.  Counts with n_plan or total_chunks negative, n_plan
 * above capacity, or chunks without items are rejected on the device:
 * status becomes BLAZ_ERR_ARG and no item runs.  workgroups and
 * chunks_per_claim as blaz_batch_run (the grid is not trimmed to the chunk
 * count, which is unknown at enqueue time: waves with no chunk left exit at
 * once).  Concurrent runs need distinct states and plan buffers. */
blaz_status blaz_batch_run_resident(const void *plan_dev, int64_t capacity, blaz_batch_state *state,
                                    int64_t workgroups, int32_t chunks_per_claim, hipStream_t stream);

/* ---------------------------------------------------------------------------
 * Grouped products: many binary64 matrix multiplications (last paragraph of
 * Section "Basic Linear Algebra Algorithms": every block rebuilt once, then
 * the product) of any sizes in at most three launches -- one rebuild of
 * every compressed operand of every product, then one contraction over the
 * output tiles of every product on 128 x 128 tiles and one on 64 x 64 tiles.
 * Each product computes exactly what blaz_matmul_tiled computes for it with
 * BLAZ_PREC_FP64 (the same per-block rebuild and per-tile contraction run),
 * bit for bit.
 *
 * Usage mirrors batching: blaz_matmul_group_plan() validates the items with
 * blaz_matmul's rules, assigns each product's rebuilt operands a region of
 * the caller's workspace and writes a plan image into caller-owned HOST
 * memory; the caller copies the image to device memory; blaz_matmul_group_run()
 * enqueues the launches (no memset, copy or allocation, so a run can be
 * captured in a HIP graph; the plan and workspace may be reused by later
 * runs on the same stream).  The products of a group run concurrently: no
 * product may write another's operands or output (the plan call refuses such
 * a group with BLAZ_ERR_ARG; products may share operands).
 * ------------------------------------------------------------------------- */
typedef struct blaz_matmul_item {
    blaz_matrix a;          /* A, m x k, compressed (two kept lines)                */
    blaz_matrix b;          /* B, k x n, compressed (two kept lines), or an empty   */
                            /* descriptor (rows = cols = 0) when bdense is given    */
    const double *bdense;   /* dense binary64 B, k x n (ldb >= n, even, 16-byte     */
                            /* aligned), or NULL when b is compressed               */
    int64_t n;              /* columns of B and C                                   */
    int64_t ldb;            /* leading dimension of bdense                          */
    double *c;              /* C, m x n binary64, leading dimension ldc >= n        */
    int64_t ldc;
    int32_t tile;           /* output tile 64 or 128; 0 = blaz_matmul's choice     */
    int32_t reserved;       /* must be 0                                            */
} blaz_matmul_item;

/* Counts a plan was built with (host memory, filled by the plan call, read
 * by the run call). */
typedef struct blaz_matmul_group_info {
    int64_t rebuild_jobs;    /* compressed operands to rebuild                     */
    int64_t rebuild_waves;   /* waves of the rebuild launch                        */
    int64_t items128;        /* products on 128 x 128 tiles                        */
    int64_t workgroups128;   /* workgroups of their contraction launch             */
    int64_t items64;         /* products on 64 x 64 tiles                          */
    int64_t workgroups64;
    size_t plan_bytes;       /* bytes of the plan image                            */
    size_t workspace_bytes;  /* bytes of workspace the products need               */
} blaz_matmul_group_info;

/* Bytes of the plan image for n_items products (an upper bound). */
size_t blaz_matmul_group_plan_bytes(int64_t n_items);

/* Validate items[0..n_items) (BLAZ_PREC_FP64 contraction) and write the plan
 * image into plan (host, plan_bytes >= blaz_matmul_group_plan_bytes(n_items),
 * 8-byte aligned).  workspace: device memory of ws_bytes bytes, 256-byte
 * aligned, holding every product's rebuilt operands (8 m k bytes for A and
 * 8 k n for a compressed B, each rounded up to 256); info->workspace_bytes
 * returns the bytes needed, also when the call fails with BLAZ_ERR_WORKSPACE
 * (so a first call with workspace = NULL sizes it).  Products with m = 0 or
 * n = 0 are dropped; k = 0 writes zeros.  On an invalid product the status
 * of the first violated rule is returned and info->rebuild_jobs holds the
 * product's index.  Host-only: nothing is read or written on the device. */
blaz_status blaz_matmul_group_plan(const blaz_matmul_item *items, int64_t n_items, void *workspace,
                                   size_t ws_bytes, void *plan, size_t plan_bytes, blaz_matmul_group_info *info);

/* Run a plan whose image has been copied to plan_dev (device, 8-byte
 * aligned), with the counts the plan call returned in info. */
blaz_status blaz_matmul_group_run(const void *plan_dev, const blaz_matmul_group_info *info, hipStream_t stream);

/* A static description of a status code. */
const char *blaz_status_string(blaz_status status);

#ifdef __cplusplus
}
#endif

#endif /* LIBBLAZ_H */
