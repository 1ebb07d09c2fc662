"""Parity of the HIP library (through its C ABI) with the FP64 oracle.

Every case feeds the same seeded arrays to both sides.  Rules in parity.py.
"""
import numpy as np
import pytest
import torch

import oracle
import paper_2202_13007_amd as blaz
from synth import smooth_field, uniform_matrix, workload_inputs

from oracle.parity import (TIE_RATE_MAX, U32, assert_blocks_close, assert_dots_close, assert_same_compressed,
                           compare_compressed, low_precision_tol)

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    blaz._lib.lib()  # fails loudly if libblaz.so is missing
    yield


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def gpu_compress(A, psi=False, lda_pad=0, misalign=False):
    """Compress with the library; A is uploaded inside a wider buffer when
    lda_pad > 0 and at an 8-byte (not 16-byte) offset when misalign."""
    rows, cols = A.shape
    off = 1 if misalign else 0
    big = np.zeros((rows, cols + lda_pad + off))
    big[:, off:off + cols] = A
    t = dev(big)[:, off:off + cols]
    p = torch.empty((max(1, (rows // 8) * (cols // 8)), 64), dtype=torch.uint8, device="cuda") if psi else None
    m = blaz.compress(t, psi=p)
    torch.cuda.synchronize()
    return (m, p.cpu().numpy() if psi else None)


def host(m):
    return m.to_host()


def upload(c: oracle.Compressed):
    return blaz.BlazMatrix.from_host(c.rows, c.cols, c.f, c.s, c.phi, c.codes)


def oracle_tuple(c):
    return (c.f, c.s, c.phi, c.codes)


# --------------------------------------------------------------------------
# Compression
# --------------------------------------------------------------------------

def check_compress(A, what, max_ties=0, **kw):
    g, _ = gpu_compress(A, **kw)
    o, (_, code_x, phi_x) = oracle.compress(A, with_debug=True)
    ties = compare_compressed(host(g), oracle_tuple(o), code_x, phi_x, what)
    assert ties <= max_ties, f"{what}: {ties} boundary ties"
    return ties


def test_compress_plain_64_workload():
    """Two 64x64 smooth fields (4 sinusoids, <= 2 cycles/side, N(0, 1e-3))."""
    A, B = workload_inputs("plain-64")
    check_compress(A, "A")
    check_compress(B, "B")


@pytest.mark.parametrize("shape", [(8, 8), (8, 24), (24, 8), (64, 64), (264, 520), (1032, 528)])
def test_compress_shapes(shape):
    """Single block, one block row/column, and grids with ragged workgroup tails."""
    r, c = shape
    A = smooth_field(r, 8, 4.0, 1e-3, 1000 + r + c, cols=c) * 3.0 - 1.0
    check_compress(A, f"compress {shape}")


@pytest.mark.parametrize("lda_pad,misalign", [(8, False), (3, False), (0, True), (5, True)])
def test_compress_leading_dimension(lda_pad, misalign):
    A = smooth_field(72, 6, 3.0, 1e-3, 77, cols=136)
    check_compress(A, f"compress lda+{lda_pad} misalign={misalign}", lda_pad=lda_pad, misalign=misalign)


def special_blocks():
    """One block row of designed blocks."""
    u = np.arange(8.0)
    blocks = [
        np.full((8, 8), 2.5),                                   # constant: K = 0
        np.zeros((8, 8)),                                       # all zero
        0.01 * np.outer(u, u),                                  # Example 1
        np.outer(0.1 * u, 0.1 * u),                             # Example 1, other rounding
        1.25 + 0.3 * u[:, None] - 0.7 * u[None, :],             # affine
        np.cumsum(np.cumsum(np.full((8, 8), 0.37), 0), 1),      # sign-consistent (K = 63)
        np.where((u[:, None] + u[None, :]) % 2 == 0, 1.0, -1.0),  # checkerboard
        np.eye(8) * 1e-3,                                       # sparse
        np.pad(np.array([[1e-3]]), ((7, 0), (7, 0))),           # one non-zero Delta: phi clamps
        1e300 * np.sin(u[:, None] + 2 * u[None, :]),            # huge magnitudes
        1e-300 * np.cos(u[:, None] - u[None, :]),               # tiny magnitudes
        -np.exp(0.1 * (u[:, None] + u[None, :])),               # negative, smooth
    ]
    return np.hstack(blocks)


def test_compress_special_blocks():
    """Designed blocks.  Some are built to put a coefficient exactly on a
    truncation boundary (the sign-consistent block's DC term is 63/8 with
    phi = 16; the sparse diagonal block has rational coefficients); a code
    there may land on either side, so ties are allowed only up to the number
    of non-zero oracle values before truncation that sit within the tie
    distance of an integer (the DC term among them is pinned and must agree)."""
    from oracle.parity import near_integer
    A = special_blocks()
    g, _ = gpu_compress(A)
    o, (_, code_x, phi_x) = oracle.compress(A, with_debug=True)
    ties = compare_compressed(host(g), oracle_tuple(o), code_x, phi_x, "special blocks")
    with np.errstate(invalid="ignore"):
        boundary = int((near_integer(code_x) & (code_x != 0)).sum() + near_integer(phi_x).sum())
    print(f"special blocks: {ties} boundary ties of {boundary} values on a boundary")
    assert ties <= boundary
    np.testing.assert_array_equal(host(g)[3][:, 0], o.codes[:, 0])  # DC codes: pinned order


def test_compress_prediction_side_output():
    """Eq. eqpredict: Psi equals the oracle's brute-force argmin over the 256
    grid points exactly (half-way ties and huge or tiny slopes included), and
    requesting it leaves the record unchanged."""
    A = np.vstack([smooth_field(64, 4, 2.0, 1e-3, 5), special_blocks()[:, :64]])
    g, psi = gpu_compress(A, psi=True)
    o, (opsi, _, _) = oracle.compress(A, with_debug=True)
    np.testing.assert_array_equal(psi, opsi)
    plain, _ = gpu_compress(A)
    assert_same_compressed(host(g), host(plain), "record with and without psi")


def test_compress_full_size_8192_sampled():
    """8192x8192 field (16 sinusoids, <= 8 cycles/side): every block on the GPU,
    a sample of blocks on the oracle, properties on all blocks."""
    A, _ = workload_inputs("plain-8192")
    g, _ = gpu_compress(A)
    gf, gs, gphi, gcodes = host(g)
    nbc = A.shape[1] // 8
    rng = np.random.default_rng(0)
    # 38k blocks, over a million codes, so that the tie count bounds a rate of 1e-6
    sample = np.unique(np.concatenate([[0, 1, nbc - 1, nbc, len(gf) - 1],
                                       rng.integers(0, len(gf), 38000)]))
    of, os_, ophi, ocodes, code_x, phi_x = oracle.compress_blocks(A, sample)
    ties = compare_compressed((gf[sample], gs[sample], gphi[sample], gcodes[sample]),
                              (of, os_, ophi, ocodes), code_x, phi_x, "8192 sampled")
    ncodes = ocodes.size + len(sample)
    print(f"8192 sampled: {ties} boundary ties in {ncodes} codes and phi")
    assert ncodes >= 1_000_000 and ties <= TIE_RATE_MAX * ncodes
    # properties on every block
    np.testing.assert_array_equal(gf, A[::8, ::8].ravel())
    assert np.all(gs > 0) and np.all(gphi >= 1)
    assert np.all(np.abs(gcodes.astype(int)) <= 127)


# --------------------------------------------------------------------------
# Decompression
# --------------------------------------------------------------------------

@pytest.mark.parametrize("shape", [(64, 64), (8, 8), (24, 8), (264, 520)])
def test_decompress(shape):
    r, c = shape
    A = smooth_field(r, 6, 3.0, 1e-3, 300 + r, cols=c)
    o = oracle.compress(A)
    got = blaz.decompress(upload(o)).cpu().numpy()
    assert_blocks_close(got, oracle.decompress(o))


def test_decompress_special_blocks_and_leading_dimension():
    o = oracle.compress(special_blocks())
    want = oracle.decompress(o)
    x = upload(o)
    big = torch.zeros((8, want.shape[1] + 5), dtype=torch.float64, device="cuda")
    blaz.decompress(x, out=big[:, 1:1 + want.shape[1]])
    got = big.cpu().numpy()
    assert_blocks_close(got[:, 1:1 + want.shape[1]], want)
    assert np.all(got[:, 0] == 0) and np.all(got[:, 1 + want.shape[1]:] == 0)
    # a constant block comes back bit-exact
    np.testing.assert_array_equal(got[:, 1:9], np.full((8, 8), 2.5))


def test_decompress_random_records():
    """Any valid record (phi >= 1, codes in [-127, 127]) decodes like the oracle."""
    rng = np.random.default_rng(9)
    nb = 4 * 9
    c = oracle.Compressed(32, 72, rng.standard_normal(nb), rng.standard_normal(nb) * 0.1,
                          rng.integers(1, 256, nb).astype(np.uint8),
                          rng.integers(-127, 128, (nb, 28)).astype(np.int8))
    assert_blocks_close(blaz.decompress(upload(c)).cpu().numpy(), oracle.decompress(c))


def test_compress_then_decompress_full_size_sampled():
    """8192x8192: GPU round trip equals the oracle's decompression of the
    GPU's own codes (sampled blocks), and the method's error is a few percent."""
    A, _ = workload_inputs("plain-8192")
    g, _ = gpu_compress(A)
    back = blaz.decompress(g).cpu().numpy()
    gf, gs, gphi, gcodes = host(g)
    rng = np.random.default_rng(1)
    nbc = A.shape[1] // 8
    for b in np.unique(np.concatenate([[0, len(gf) - 1], rng.integers(0, len(gf), 400)])):
        I, J = divmod(int(b), nbc)
        want = oracle.decompress_block(gf[b], gs[b], gphi[b], gcodes[b])
        blk = back[8 * I:8 * I + 8, 8 * J:8 * J + 8]
        assert np.max(np.abs(blk - want)) <= 1e-12 * np.max(np.abs(want)), f"block {b}"
    rel = np.linalg.norm(back - A) / np.linalg.norm(A)
    assert rel < 0.05


# --------------------------------------------------------------------------
# Add, subtract, scale (Algorithms 1 and 2): bit-exact
# --------------------------------------------------------------------------

def random_records(rows, cols, seed, phi_lo=1):
    rng = np.random.default_rng(seed)
    nb = (rows // 8) * (cols // 8)
    return oracle.Compressed(rows, cols, rng.standard_normal(nb) * 10, rng.standard_normal(nb),
                             rng.integers(phi_lo, 256, nb).astype(np.uint8),
                             rng.integers(-127, 128, (nb, 28)).astype(np.int8))


def add_cases():
    A, B = workload_inputs("plain-64")
    x, y = oracle.compress(A), oracle.compress(B)
    yield "fields", x, y
    yield "self", x, x
    yield "opposite slopes cancel", x, oracle.scale(x, -1.0)
    yield "near cancellation saturates", x, oracle.scale(y, -0.97)
    r1, r2 = random_records(72, 520, 3), random_records(72, 520, 4)
    yield "random records", r1, r2
    r3 = random_records(72, 520, 5)
    r3.phi[:] = 1
    yield "phi = 1", r1, r3
    r4 = r2.copy()
    r4.s[::3] = 0.0
    yield "zero slopes", r1, r4


@pytest.mark.parametrize("case", range(7))
def test_add_bit_exact(case):
    name, x, y = list(add_cases())[case]
    got = host(blaz.add(upload(x), upload(y)))
    assert_same_compressed(got, oracle_tuple(oracle.add(x, y)), f"add {name}")


@pytest.mark.parametrize("case", range(7))
def test_sub_bit_exact(case):
    """Subtraction = Algorithm 1 on x and (-1) y."""
    name, x, y = list(add_cases())[case]
    got = host(blaz.sub(upload(x), upload(y)))
    assert_same_compressed(got, oracle_tuple(oracle.add(x, oracle.scale(y, -1.0))), f"sub {name}")


def test_add_in_place():
    x, y = random_records(16, 1032, 6), random_records(16, 1032, 7)
    gx, gy = upload(x), upload(y)
    blaz.add(gx, gy, out=gx)
    assert_same_compressed(host(gx), oracle_tuple(oracle.add(x, y)), "add in place (z = x)")
    gx2, gy2 = upload(x), upload(y)
    blaz.add(gx2, gy2, out=gy2)
    assert_same_compressed(host(gy2), oracle_tuple(oracle.add(x, y)), "add in place (z = y)")


@pytest.mark.parametrize("c", [1.7, -2.0, 0.0, 1e-300])
def test_scale_bit_exact(c):
    x = random_records(40, 264, 8)
    want = oracle_tuple(oracle.scale(x, c))
    assert_same_compressed(host(blaz.scale(upload(x), c)), want, f"scale {c}")
    gx = upload(x)
    blaz.scale(gx, c, out=gx)
    assert_same_compressed(host(gx), want, f"scale {c} in place")


def test_add_scale_full_size_8192_sampled():
    """8192x8192 compressed add and scale, sampled blocks against the oracle."""
    A, B = workload_inputs("plain-8192")
    gx, _ = gpu_compress(A)
    gy, _ = gpu_compress(B)
    gz = blaz.add(gx, gy)
    gw = blaz.scale(gz, 1.7)
    xh, yh, zh, wh = host(gx), host(gy), host(gz), host(gw)
    rng = np.random.default_rng(2)
    smp = np.unique(np.concatenate([[0, len(xh[0]) - 1], rng.integers(0, len(xh[0]), 5000)]))
    pick = lambda t: oracle.Compressed(8, 8 * len(smp), t[0][smp], t[1][smp], t[2][smp], t[3][smp])
    oz = oracle.add(pick(xh), pick(yh))
    assert_same_compressed(tuple(a[smp] for a in zh), oracle_tuple(oz), "add 8192 sampled")
    assert_same_compressed(tuple(a[smp] for a in wh), oracle_tuple(oracle.scale(oz, 1.7)), "scale 8192 sampled")


# --------------------------------------------------------------------------
# Dot products and matrix multiplication
# --------------------------------------------------------------------------

def test_dot_compressed():
    """Algorithm 3 blockwise: line i of X times column j of Y."""
    X = smooth_field(24, 4, 2.0, 1e-3, 400, cols=1040)
    Y = smooth_field(1040, 4, 2.0, 1e-3, 401, cols=40)
    ox, oy = oracle.compress(X), oracle.compress(Y)
    rng = np.random.default_rng(3)
    rows = np.concatenate([np.arange(24), rng.integers(0, 24, 40)])
    cols = np.concatenate([np.arange(24) % 40, rng.integers(0, 40, 40)])
    got = blaz.dot(upload(ox), dev(rows), upload(oy), dev(cols)).cpu().numpy()
    want = oracle.dot(ox, rows, oy, cols)
    Xd, Yd = oracle.decompress(ox), oracle.decompress(oy)
    mag = np.array([np.abs(Xd[i]) @ np.abs(Yd[:, j]) for i, j in zip(rows, cols)])
    assert_dots_close(got, want, mag, what="dot")


def test_dot_invalid_index_gives_nan():
    ox = oracle.compress(smooth_field(16, 2, 1.0, 0, 1))
    got = blaz.dot(upload(ox), dev(np.array([0, 16, -1, 3])), upload(ox), dev(np.array([0, 0, 1, 99]))).cpu().numpy()
    assert np.isfinite(got[0]) and np.isnan(got[1]) and np.isnan(got[2]) and np.isnan(got[3])


@pytest.mark.parametrize("shared", [False, True])
def test_dot_dense(shared):
    X = smooth_field(48, 4, 2.0, 1e-3, 410, cols=1096)
    ox = oracle.compress(X)
    rows = np.arange(48)[::-1].copy()
    V = uniform_matrix(1 if shared else 48, 1096, 411)
    v = V[0] if shared else V
    got = blaz.dot_dense(upload(ox), dev(rows), dev(v)).cpu().numpy()
    want = oracle.dot_dense(ox, rows, v, 0 if shared else 1096)
    Xd = oracle.decompress(ox)
    mag = np.array([np.abs(Xd[i]) @ np.abs(V[0 if shared else q]) for q, i in enumerate(rows)])
    assert_dots_close(got, want, mag, what="dot_dense")


def _bits(a):
    return np.asarray(a, dtype=np.float64).view(np.int64)


@pytest.mark.parametrize("kind", ["pairs", "own_vectors", "shared_vector"])
def test_dot_aligned_groups_equal_single_queries(kind):
    """Queries on the 8 lines of a block row, in order, rebuild each block
    once for the group; the same queries shifted off that alignment take the
    per-query path.  Both must give the same bits (2056 columns = 257 blocks
    per line, so the 256 slots wrap), and match the oracle."""
    X = smooth_field(64, 4, 2.0, 1e-3, 430, cols=2056)
    ox = oracle.compress(X)
    gx = upload(ox)
    rows = np.arange(64)
    shifted = np.concatenate([[5], rows])          # every group of 8 is now misaligned
    if kind == "pairs":
        oy = oracle.compress(smooth_field(2056, 4, 2.0, 1e-3, 431, cols=64))
        gy = upload(oy)
        got = blaz.dot(gx, dev(rows), gy, dev(rows)).cpu().numpy()
        alt = blaz.dot(gx, dev(shifted), gy, dev(np.concatenate([[3], rows]))).cpu().numpy()[1:]
        want = oracle.dot(ox, rows, oy, rows)
        Xd, Yd = oracle.decompress(ox), oracle.decompress(oy)
        mag = np.array([np.abs(Xd[i]) @ np.abs(Yd[:, i]) for i in rows])
    else:
        V = uniform_matrix(65, 2056, 432)
        if kind == "shared_vector":
            got = blaz.dot_dense(gx, dev(rows), dev(V[0])).cpu().numpy()
            alt = blaz.dot_dense(gx, dev(shifted), dev(V[0])).cpu().numpy()[1:]
            want = oracle.dot_dense(ox, rows, V[0], 0)
            Vq = np.repeat(V[:1], 64, axis=0)
        else:
            got = blaz.dot_dense(gx, dev(rows), dev(V[1:])).cpu().numpy()
            alt = blaz.dot_dense(gx, dev(shifted), dev(V)).cpu().numpy()[1:]
            want = oracle.dot_dense(ox, rows, V[1:], 2056)
            Vq = V[1:]
        Xd = oracle.decompress(ox)
        mag = np.array([np.abs(Xd[i]) @ np.abs(Vq[i]) for i in rows])
    assert np.array_equal(_bits(got), _bits(alt))
    assert_dots_close(got, want, mag, what=f"dot {kind} aligned")


def test_dot_ragged_group_and_invalid_in_aligned_position():
    """A last group of fewer than 8 queries, and an out-of-range index inside
    an otherwise aligned run, take the per-query path."""
    X = smooth_field(32, 4, 2.0, 1e-3, 433, cols=72)
    ox = oracle.compress(X)
    gx = upload(ox)
    V = uniform_matrix(1, 72, 434)[0]
    rows = np.concatenate([np.arange(8), [8, 9, 10, 99, 12, 13, 14, 15], np.arange(16, 27)])
    got = blaz.dot_dense(gx, dev(rows), dev(V)).cpu().numpy()
    ok = rows < 32
    assert np.isnan(got[~ok]).all() and np.isfinite(got[ok]).all()
    want = oracle.dot_dense(ox, rows[ok], V, 0)
    Xd = oracle.decompress(ox)
    assert_dots_close(got[ok], want, np.array([np.abs(Xd[i]) @ np.abs(V) for i in rows[ok]]), what="ragged")


def band_rows(og: oracle.Compressed, i: int) -> np.ndarray:
    """Line i of a compressed matrix, decompressed by the oracle (its block row only)."""
    nbc = og.cols // 8
    I = i // 8
    sl = slice(I * nbc, (I + 1) * nbc)
    band = oracle.Compressed(8, og.cols, og.f[sl], og.s[sl], og.phi[sl], og.codes[sl])
    return oracle.decompress(band)[i % 8]


def test_dot_dense_full_size_4096_sampled():
    """4096 dot products of compressed lines with their own dense vectors."""
    A, _, V = workload_inputs("linalg-4096")
    g, _ = gpu_compress(A)
    rows = np.arange(4096)
    got = blaz.dot_dense(g, dev(rows), dev(V)).cpu().numpy()
    og = oracle.Compressed(4096, 4096, *host(g))
    smp = np.array([0, 7, 8, 2047, 4095] + list(np.random.default_rng(4).integers(0, 4096, 15)))
    want = oracle.dot_dense(og, rows[smp], V[smp], 4096)
    mag = np.array([np.abs(band_rows(og, int(i))) @ np.abs(V[i]) for i in smp])
    assert_dots_close(got[smp], want, mag, what="dot_dense 4096")


def band_col(og: oracle.Compressed, j: int) -> np.ndarray:
    """Column j of a compressed matrix, decompressed by the oracle (its block column only)."""
    nbr, nbc = og.rows // 8, og.cols // 8
    idx = np.arange(nbr) * nbc + j // 8
    band = oracle.Compressed(og.rows, 8, og.f[idx], og.s[idx], og.phi[idx], og.codes[idx])
    return oracle.decompress(band)[:, j % 8]


def test_dot_compressed_and_shared_vector_full_size_4096_sampled():
    """The two other 4096 dot workloads as timed: row i of A with column i
    of a compressed B (aligned groups of 8 lines and 8 columns), and every
    row of A with one shared vector."""
    A, B, V = workload_inputs("linalg-4096")
    g, _ = gpu_compress(A)
    gb, _ = gpu_compress(B)
    rows = np.arange(4096)
    og = oracle.Compressed(4096, 4096, *host(g))
    ob = oracle.Compressed(4096, 4096, *host(gb))
    smp = np.array([0, 7, 8, 2047, 4095] + list(np.random.default_rng(5).integers(0, 4096, 15)))
    got = blaz.dot(g, dev(rows), gb, dev(rows)).cpu().numpy()
    want = oracle.dot(og, rows[smp], ob, rows[smp])
    mag = np.array([np.abs(band_rows(og, int(i))) @ np.abs(band_col(ob, int(i))) for i in smp])
    assert_dots_close(got[smp], want, mag, what="dot compressed pairs 4096")
    v0 = np.ascontiguousarray(V[0])
    got = blaz.dot_dense(g, dev(rows), dev(v0)).cpu().numpy()
    want = oracle.dot_dense(og, rows[smp], v0, 0)
    mag = np.array([np.abs(band_rows(og, int(i))) @ np.abs(v0) for i in smp])
    assert_dots_close(got[smp], want, mag, what="dot shared vector 4096")


def test_dot_equals_matmul_element():
    """Section "Accuracy Measurements": dot(i, j) is element (i, j) of the product."""
    X = smooth_field(64, 4, 2.0, 1e-3, 420)
    Y = smooth_field(64, 4, 2.0, 1e-3, 421)
    gx, gy = upload(oracle.compress(X)), upload(oracle.compress(Y))
    P = blaz.matmul(gx, gy).cpu().numpy()
    rows = np.repeat(np.arange(64), 64)
    cols = np.tile(np.arange(64), 64)
    d = blaz.dot(gx, dev(rows), gy, dev(cols)).cpu().numpy().reshape(64, 64)
    Xd, Yd = oracle.decompress(oracle.compress(X)), oracle.decompress(oracle.compress(Y))
    mag = np.abs(Xd) @ np.abs(Yd)
    assert np.all(np.abs(d - P) <= 2e-12 * mag)


# --------------------------------------------------------------------------
# Data-condition counts
# --------------------------------------------------------------------------

def condition_counts(c: oracle.Compressed):
    """The four counts of blaz_diagnose, from their definitions."""
    n = oracle.kept_count(c.lines)
    codes = c.codes[:, :n].astype(int)
    return np.array([(c.s == 0).sum(), ((c.s != 0) & (c.phi == 255)).sum(), (np.abs(codes) >= 127).sum(),
                     (~(np.isfinite(c.f) & np.isfinite(c.s))).sum()], dtype=np.int64)


def test_diagnose_counts_conditions():
    special = oracle.compress(special_blocks())         # constant, zero and clamping blocks
    x = random_records(64, 64, 7)
    y = random_records(64, 64, 8)
    y.s = -0.9 * x.s                                     # opposite slopes: |alpha| > 1, saturation
    summed = oracle.add(x, y)
    bad = random_records(16, 64, 9)
    bad.f[3] = np.nan
    bad.s[5] = np.inf
    three = oracle.compress_lines(special_blocks(), 3)
    for c in (special, summed, bad, three):
        want = condition_counts(c)
        got = blaz.diagnose(blaz.BlazMatrix.from_host(c.rows, c.cols, c.f, c.s, c.phi, c.codes, lines=c.lines))
        assert np.array_equal(got.cpu().numpy(), want), (got, want)
    assert condition_counts(special)[[0, 1]].min() >= 1 and condition_counts(summed)[2] > 0
    # counts accumulate into a caller's array
    acc = torch.zeros(4, dtype=torch.int64, device="cuda")
    g = upload(summed)
    blaz.diagnose(g, acc)
    blaz.diagnose(g, acc)
    assert np.array_equal(acc.cpu().numpy(), 2 * condition_counts(summed))


# --------------------------------------------------------------------------
# Matmul with a compressed result
# --------------------------------------------------------------------------

def blocks_max(M):
    r, c = M.shape
    return M.reshape(r // 8, 8, c // 8, 8).max(axis=(1, 3)).ravel()


def assert_compressed_product(got, Xd, Yd, what):
    """The GPU's compressed product against the oracle's compression of the
    oracle's product.  The two products differ by rounding only: each is a
    binary64 sum of k products, within k 2^-53 sum|x y| of the exact value,
    so per block e = max of 2 k 2^-53 sum|x y|.  Propagated through the
    compressor: |df| <= e, |ds| <= 128 e / K <= 128 e; the normalized block
    moves by sum|dD'| <= 256 e / s, so every coefficient by at most
    max|T_iu T_jv| * 256 e / s = 64 e / s, phi's argument 127/m by
    127 (64 e / s) / m^2, and a code's argument phi D by phi 64 e / s.  A code
    (or phi) may differ by exactly 1 where the oracle's argument lies that
    close to an integer; everything else must agree."""
    k = Xd.shape[1]
    P = oracle.gemm(Xd, Yd)
    o, (_, code_x, phi_x) = oracle.compress(P, with_debug=True)
    e = blocks_max(2.0 * k * 2.0 ** -53 * (np.abs(Xd) @ np.abs(Yd)))
    gf, gs, gphi, gcodes = host(got)
    slack = 2.0 ** -40
    assert np.all(o.s > 0), "test data must not hold constant product blocks"
    assert np.all(np.abs(gf - o.f) <= e + slack * np.abs(o.f)), f"{what}: f"
    assert np.all(np.abs(gs - o.s) <= 128 * e + slack * o.s), f"{what}: s"
    dD = 64.0 * e / o.s
    m = 127.0 / phi_x
    band_phi = 127.0 * dD / m ** 2 + slack * np.maximum(1.0, phi_x)
    dphi = gphi.astype(int) - o.phi.astype(int)
    near_phi = np.abs(phi_x - np.round(phi_x)) <= band_phi
    assert np.all((dphi == 0) | ((np.abs(dphi) == 1) & near_phi)), f"{what}: phi"
    same = dphi == 0
    band = (o.phi.astype(float) * dD)[:, None] + slack * np.maximum(1.0, np.abs(code_x))
    dc = gcodes.astype(int) - o.codes.astype(int)
    near = np.abs(code_x - np.round(code_x)) <= band
    ok = (dc == 0) | ((np.abs(dc) == 1) & near)
    assert np.all(ok[same]), f"{what}: {int((~ok[same]).sum())} codes differ off the perturbation band"
    return int((dc != 0)[same].sum()) + int((~same).sum())


@pytest.mark.parametrize("m,k,n,bform", [(128, 128, 128, "compressed"), (136, 200, 72, "dense"),
                                         (64, 8, 264, "compressed")])
def test_matmul_compressed_against_oracle(m, k, n, bform):
    X = smooth_field(m, 4, 2.0, 1e-3, 440, cols=k)
    Y = smooth_field(k, 4, 2.0, 1e-3, 441, cols=n) + 3.0
    ox = oracle.compress(X)
    Xd = oracle.decompress(ox)
    if bform == "compressed":
        oy = oracle.compress(Y)
        Yd = oracle.decompress(oy)
        got = blaz.matmul_compressed(upload(ox), upload(oy))
    else:
        Yd = Y
        got = blaz.matmul_compressed(upload(ox), dev(Y))
    torch.cuda.synchronize()
    flips = assert_compressed_product(got, Xd, Yd, f"matmul_compressed {m}x{k}x{n}")
    assert flips <= 1e-3 * (m // 8) * (n // 8) * 28


def test_matmul_compressed_full_size_4096_sampled():
    """The 4096^3 product of the compressed field and the compressed U[-1, 1]
    matrix, recompressed: a grid of sampled output blocks against the oracle's
    compression of the oracle's product of the decompressed block row and
    block column, under the perturbation band of the smaller cases."""
    A, B, _ = workload_inputs("linalg-4096")
    ga, gb = blaz.compress(dev(A)), blaz.compress(dev(B))
    got = host(blaz.matmul_compressed(ga, gb))
    oa, ob = oracle.Compressed(4096, 4096, *host(ga)), oracle.Compressed(4096, 4096, *host(gb))
    nbc = 512
    rng = np.random.default_rng(5)
    Is = np.unique(np.concatenate([[0, nbc - 1], rng.choice(nbc, 12, replace=False)]))
    Js = np.unique(np.concatenate([[0, nbc - 1], rng.choice(nbc, 12, replace=False)]))
    sample = np.array([I * nbc + J for I in Is for J in Js])
    rows = {}
    cols = {}
    Pb, mag = [], []
    for b in sample:
        I, J = divmod(int(b), nbc)
        if I not in rows:
            band = oracle.Compressed(8, 4096, oa.f[I * nbc:(I + 1) * nbc], oa.s[I * nbc:(I + 1) * nbc],
                                     oa.phi[I * nbc:(I + 1) * nbc], oa.codes[I * nbc:(I + 1) * nbc])
            rows[I] = oracle.decompress(band)
        if J not in cols:
            idx = np.arange(J, nbc * nbc, nbc)
            band = oracle.Compressed(4096, 8, ob.f[idx], ob.s[idx], ob.phi[idx], ob.codes[idx])
            cols[J] = oracle.decompress(band)
        Pb.append(oracle.gemm(rows[I], cols[J]))
        mag.append(np.abs(rows[I]) @ np.abs(cols[J]))
    P = np.hstack(Pb)
    M = np.hstack(mag)
    o, (_, code_x, phi_x) = oracle.compress(P, with_debug=True)
    e = blocks_max(2.0 * 4096 * 2.0 ** -53 * M)
    gf, gs, gphi, gcodes = (a[sample] for a in got)
    slack = 2.0 ** -40
    assert np.all(np.abs(gf - o.f) <= e + slack * np.abs(o.f))
    assert np.all(np.abs(gs - o.s) <= 128 * e + slack * np.abs(o.s))
    dD = 64.0 * e / np.where(o.s != 0, o.s, np.inf)
    dphi = gphi.astype(int) - o.phi.astype(int)
    near_phi = np.abs(phi_x - np.round(phi_x)) <= 127.0 * dD * (phi_x / 127.0) ** 2 + slack * np.maximum(1, phi_x)
    assert np.all((dphi == 0) | ((np.abs(dphi) == 1) & near_phi))
    same = dphi == 0
    band = (o.phi.astype(float) * dD)[:, None] + slack * np.maximum(1.0, np.abs(code_x))
    dc = gcodes.astype(int) - o.codes.astype(int)
    ok = (dc == 0) | ((np.abs(dc) == 1) & (np.abs(code_x - np.round(code_x)) <= band))
    assert np.all(ok[same])


@pytest.mark.parametrize("prec", ["fp64", "fp32", "bf16x3"])
@pytest.mark.parametrize("tile", [64, 128])
def test_matmul_compressed_is_compress_of_matmul(prec, tile):
    """Bit for bit the compression of the dense product, in every contraction
    arithmetic and tile, with dense and compressed B."""
    X = smooth_field(264, 4, 2.0, 1e-3, 442, cols=136)
    Y = smooth_field(136, 4, 2.0, 1e-3, 443, cols=200)
    gx, gy = blaz.compress(dev(X)), blaz.compress(dev(Y))
    for b in (gy, dev(Y)):
        got = blaz.matmul_compressed(gx, b, prec=prec, tile=tile)
        want = blaz.compress(blaz.matmul(gx, b, prec=prec, tile=tile))
        assert_same_compressed(host(got), host(want), f"matmul_compressed {prec} tile {tile}")


def test_matmul_compressed_k0_and_workspace_reuse():
    """k = 0 gives the compressed zero matrix; a second call with a smaller
    product reuses the same workspace and output buffers."""
    z = blaz.matmul_compressed(blaz.BlazMatrix.empty(16, 0), torch.empty((0, 24), dtype=torch.float64, device="cuda"))
    assert_same_compressed(host(z), oracle_tuple(oracle.compress(np.zeros((16, 24)))), "k = 0")
    X = smooth_field(128, 4, 2.0, 1e-3, 444)
    gx = blaz.compress(dev(X))
    ws = torch.empty(blaz.matmul_compressed_workspace_bytes(128, 128, 128, True), dtype=torch.uint8, device="cuda")
    first = blaz.matmul_compressed(gx, gx, workspace=ws)
    small = blaz.compress(dev(X[:64, :64]))
    second = blaz.matmul_compressed(small, small, workspace=ws)
    assert_same_compressed(host(second), host(blaz.compress(blaz.matmul(small, small))), "second call")
    assert_same_compressed(host(first), host(blaz.compress(blaz.matmul(gx, gx))), "first call")


def test_matmul_plain_64_workload():
    """64x64 partly-decompressed product of the two compressed fields."""
    A, B = workload_inputs("plain-64")
    ox, oy = oracle.compress(A), oracle.compress(B)
    got = blaz.matmul(upload(ox), upload(oy)).cpu().numpy()
    Xd, Yd = oracle.decompress(ox), oracle.decompress(oy)
    want = oracle.gemm(Xd, Yd)
    assert_dots_close(got, want, np.abs(Xd) @ np.abs(Yd), what="matmul 64")


@pytest.mark.parametrize("m,k,n", [(136, 200, 72), (8, 8, 8), (256, 64, 392), (392, 136, 264)])
def test_matmul_dense_b_ragged(m, k, n):
    A = smooth_field(m, 4, 2.0, 1e-3, 430 + m, cols=k)
    B = uniform_matrix(k, n, 431)
    ox = oracle.compress(A)
    got = blaz.matmul(upload(ox), dev(B)).cpu().numpy()
    Xd = oracle.decompress(ox)
    want = oracle.gemm(Xd, B)
    assert_dots_close(got, want, np.abs(Xd) @ np.abs(B), what=f"matmul {m}x{k}x{n}")


def test_matmul_leading_dimensions():
    A = smooth_field(64, 4, 2.0, 1e-3, 440, cols=128)
    B = uniform_matrix(128, 72, 441)
    ox = oracle.compress(A)
    Bbig = np.zeros((128, 80))
    Bbig[:, :72] = B
    Cbig = torch.full((64, 90), 7.0, dtype=torch.float64, device="cuda")
    blaz.matmul(upload(ox), dev(Bbig)[:, :72], out=Cbig[:, 4:76])
    got = Cbig.cpu().numpy()
    Xd = oracle.decompress(ox)
    assert_dots_close(got[:, 4:76], oracle.gemm(Xd, B), np.abs(Xd) @ np.abs(B), what="matmul ld")
    assert np.all(got[:, :4] == 7.0) and np.all(got[:, 76:] == 7.0)


def test_matmul_full_size_4096_sampled():
    """Compressed 4096x4096 field times dense U[-1, 1]: sampled entries, each
    computed by the oracle as a line of the decompressed A times a column of B."""
    A, B, _ = workload_inputs("linalg-4096")
    g, _ = gpu_compress(A)
    C = blaz.matmul(g, dev(B)).cpu().numpy()
    og = oracle.Compressed(4096, 4096, *host(g))
    rng = np.random.default_rng(5)
    ij = [(0, 0), (4095, 4095), (127, 128), (128, 127)] + [tuple(rng.integers(0, 4096, 2)) for _ in range(12)]
    for i, j in ij:
        bj = np.ascontiguousarray(B[:, j])
        want = oracle.dot_dense(og, [i], bj, 0)[0]
        mag = np.abs(band_rows(og, int(i))) @ np.abs(bj)
        assert abs(C[i, j] - want) <= 1e-12 * mag, (i, j, C[i, j], want)


# --------------------------------------------------------------------------
# Mixed-precision transform stage (FP32 / BF16x3 on MFMA), binary64 elsewhere
# --------------------------------------------------------------------------

# |D_mixed - D_64| <= eps * sum_e |Delta'_e| |K[e][c]| <= eps * K / 4 with
# K[e][c] = T(i, u) T(j, v), sum |Delta'| = K <= 63 and |K[e][c]| <= 1/4.
# The transform runs as two 8-point passes, R = Delta' T^T then D = T R,
# and |T| |R| <= |T| |Delta'| |T|^T, so the two passes' relative bounds add:
# FP32: operand rounding (Delta', T: 2 u32) and the 8-term FP32 sums of
# each pass, within 66 u32; BF16x3: each pass 3 * 2^-16 (the split of both
# operands, done in FP32, and the dropped lo * lo product), plus 2^-16 for
# the split of R into hi + lo between the passes, plus the FP32 roundings
# and sums.
MIXED_EPS = {"fp32": 66 * 2.0 ** -24, "bf16x3": 7 * 2.0 ** -16 + 66 * 2.0 ** -24}
D_ERR = {k: v * 63 / 4 for k, v in MIXED_EPS.items()}


def compare_mixed(gpu, orc, code_x, phi_x, prec):
    """f, s bit-exact; phi and codes equal except where the oracle's value
    before truncation is within the arithmetic's error bound of an integer.
    Returns (code mismatches, phi flips)."""
    gf, gs, gphi, gcodes = gpu
    of, os_, ophi, ocodes = orc
    assert np.array_equal(gf.view(np.uint64), of.view(np.uint64)), "f"
    assert np.array_equal(gs.view(np.uint64), os_.view(np.uint64)), "s"
    dD = D_ERR[prec]
    flips = np.flatnonzero(gphi != ophi)
    for b in flips:
        m = 127.0 / phi_x[b]
        # 127/m moves by at most (127/m) * dD / (m - dD)
        assert abs(int(gphi[b]) - int(ophi[b])) == 1, b
        assert abs(phi_x[b] - np.round(phi_x[b])) <= phi_x[b] * dD / (m - dD), (b, phi_x[b])
    D = code_x / ophi[:, None].astype(float)
    want_x = gphi[:, None].astype(float) * D  # the oracle's values at the GPU's phi
    want = np.trunc(want_x).astype(int)
    diff = gcodes.astype(int) - want
    bad = diff != 0
    tol = gphi[:, None].astype(float) * dD
    explained = (np.abs(diff) == 1) & (np.abs(want_x - np.round(want_x)) <= tol)
    assert np.all(explained | ~bad), (f"{prec}: {int((bad & ~explained).sum())} codes off by more than "
                                     f"the error bound")
    return int(bad.sum()), len(flips)


@pytest.mark.parametrize("prec", ["fp32", "bf16x3"])
@pytest.mark.parametrize("shape", [(64, 64), (1032, 528), (24, 8)])
def test_compress_mixed_precision(prec, shape):
    r, c = shape
    A = smooth_field(r, 32, 8.0, 1e-4, 460 + r, cols=c)
    t = dev(A)
    g = blaz.compress(t, prec=prec)
    o, (_, code_x, phi_x) = oracle.compress(A, with_debug=True)
    mism, flips = compare_mixed(host(g), oracle_tuple(o), code_x, phi_x, prec)
    n = o.codes.size
    print(f"{prec} {shape}: {mism} code mismatches of {n}, {flips} phi flips")
    # the binary64 codec is unaffected by the option
    g64 = blaz.compress(t)
    assert compare_compressed(host(g64), oracle_tuple(o), code_x, phi_x) == 0


@pytest.mark.parametrize("prec", ["fp32", "bf16x3"])
def test_compress_mixed_precision_special_blocks_and_psi(prec):
    A = np.vstack([special_blocks()[:, :64], smooth_field(8, 2, 0.5, 1e-3, 3, cols=64)])
    p = torch.empty((A.size // 64, 64), dtype=torch.uint8, device="cuda")
    g = blaz.compress(dev(A), prec=prec, psi=p)
    o, (opsi, code_x, phi_x) = oracle.compress(A, with_debug=True)
    compare_mixed(host(g), oracle_tuple(o), code_x, phi_x, prec)
    # Psi is computed in binary64 before the transform, as in the plain path
    p64 = torch.empty_like(p)
    blaz.compress(dev(A), psi=p64)
    assert torch.equal(p, p64)


@pytest.fixture(scope="module")
def field_16384():
    """The 16384x16384 field (32 sinusoids, <= 32 cycles/side, N(0, 1e-4)) on
    the host and on the device, shared by the tests at that size."""
    (A,) = workload_inputs("mixed-16384")
    t = dev(A)
    yield A, t
    del t
    torch.cuda.empty_cache()


def test_compress_full_size_16384_sampled(field_16384):
    """The binary64 path at 4.19 M blocks: every block on the GPU, 38k blocks
    (over a million codes) on the oracle, properties on all blocks."""
    A, t = field_16384
    gf, gs, gphi, gcodes = host(blaz.compress(t))
    rng = np.random.default_rng(8)
    nb = len(gf)
    smp = np.unique(np.concatenate([[0, nb - 1], rng.integers(0, nb, 38000)]))
    of, os_, ophi, ocodes, code_x, phi_x = oracle.compress_blocks(A, smp)
    ties = compare_compressed((gf[smp], gs[smp], gphi[smp], gcodes[smp]), (of, os_, ophi, ocodes),
                              code_x, phi_x, "16384 sampled")
    ncodes = ocodes.size + len(smp)
    print(f"16384 sampled: {ties} boundary ties in {ncodes} codes and phi")
    assert ncodes >= 1_000_000 and ties <= TIE_RATE_MAX * ncodes
    np.testing.assert_array_equal(gf, A[::8, ::8].ravel())
    assert np.all(gs > 0) and np.all(gphi >= 1)
    assert np.all(np.abs(gcodes.astype(int)) <= 127)


@pytest.mark.parametrize("prec", ["fp32", "bf16x3"])
def test_compress_mixed_precision_full_size_16384_sampled(prec, field_16384):
    """The 16384x16384 field in FP32 / BF16x3: all blocks on the GPU, a sample
    on the oracle; decompressed error next to the method's own error."""
    A, t = field_16384
    g = blaz.compress(t, prec=prec)
    gh = host(g)
    rng = np.random.default_rng(7)
    nb = len(gh[0])
    smp = np.unique(np.concatenate([[0, nb - 1], rng.integers(0, nb, 3000)]))
    of, os_, ophi, ocodes, code_x, phi_x = oracle.compress_blocks(A, smp)
    compare_mixed(tuple(a[smp] for a in gh), (of, os_, ophi, ocodes), code_x, phi_x, prec)
    g64 = blaz.compress(t)
    back = blaz.decompress(g)
    back64 = blaz.decompress(g64)
    own = (torch.linalg.norm(back64 - t) / torch.linalg.norm(t)).item()
    mixed = (torch.linalg.norm(back - t) / torch.linalg.norm(t)).item()
    delta = (torch.linalg.norm(back - back64) / torch.linalg.norm(t)).item()
    print(f"{prec}: method error {own:.4e}, with {prec} transform {mixed:.4e}, difference {delta:.3e}")
    assert mixed <= own * 1.01 + 1e-9


# Low-precision contractions (FP32, BF16 hi+lo with three products): the
# per-entry bound is low_precision_tol (oracle.parity).


def low_precision_fro(prec, k):
    """Expected-size bound on the relative Frobenius error: rounding errors of
    the K-term FP32 accumulation grow like sqrt(K) u32 with random signs."""
    return (2 + 4 * np.sqrt(k)) * U32 if prec == "fp32" else 1e-4


@pytest.mark.parametrize("prec", ["fp32", "bf16x3"])
@pytest.mark.parametrize("m,k,n", [(64, 64, 64), (136, 200, 72), (8, 8, 8), (392, 136, 264)])
def test_matmul_low_precision_dense_b(prec, m, k, n):
    A = smooth_field(m, 4, 2.0, 1e-3, 450 + m, cols=k)
    B = uniform_matrix(k, n, 451)
    ox = oracle.compress(A)
    got = blaz.matmul(upload(ox), dev(B), prec=prec).cpu().numpy()
    Xd = oracle.decompress(ox)
    want = oracle.gemm(Xd, B)
    mag = np.abs(Xd) @ np.abs(B)
    assert_dots_close(got, want, mag, rel=low_precision_tol(prec, k), what=f"matmul {prec}")
    rel = np.linalg.norm(got - want) / np.linalg.norm(want)
    assert rel < low_precision_fro(prec, k), rel


@pytest.mark.parametrize("prec", ["fp32", "bf16x3"])
def test_matmul_low_precision_compressed_b(prec):
    A, B = workload_inputs("plain-64")
    ox, oy = oracle.compress(A), oracle.compress(B)
    got = blaz.matmul(upload(ox), upload(oy), prec=prec).cpu().numpy()
    Xd, Yd = oracle.decompress(ox), oracle.decompress(oy)
    want = oracle.gemm(Xd, Yd)
    assert_dots_close(got, want, np.abs(Xd) @ np.abs(Yd), rel=low_precision_tol(prec, 64),
                      what=f"matmul {prec} compressed B")


@pytest.mark.parametrize("prec", ["fp32", "bf16x3"])
@pytest.mark.parametrize("tile", [64, 128])
@pytest.mark.parametrize("m,k,n", [(136, 200, 72), (392, 136, 264)])
def test_matmul_low_precision_compressed_b_is_dense_of_its_rebuild(prec, tile, m, k, n):
    """A compressed B is rebuilt straight into the operand precision and
    transposed; a dense B is converted from binary64.  Both must give the
    same operands, hence the same product bit for bit, when the dense B is
    the binary64 rebuild of the compressed one."""
    A = smooth_field(m, 4, 2.0, 1e-3, 480 + m, cols=k)
    B = smooth_field(k, 4, 2.0, 1e-3, 481 + k, cols=n)
    gx, gy = blaz.compress(dev(A)), blaz.compress(dev(B))
    got = blaz.matmul(gx, gy, prec=prec, tile=tile)
    want = blaz.matmul(gx, blaz.decompress(gy), prec=prec, tile=tile)
    assert torch.equal(got, want), (prec, tile, m, k, n, (got - want).abs().max().item())


def test_matmul_low_precision_k_beyond_a_grid_dimension():
    """k = 4,194,368: 65,537 tiles of 64 k-values, one more than a grid's y
    extent allows, so the B preparations must not put k on that axis.  A
    property check (the oracle would take minutes here): the FP32 and BF16x3
    products, with B dense and compressed, agree with the FP64 product (held
    to the oracle by the tests above) within the low-precision bounds."""
    m, k, n = 8, 4_194_368, 8
    A = smooth_field(m, 2, 1.0, 1e-3, 620, cols=k)
    B = uniform_matrix(k, n, 621)
    gx = blaz.compress(dev(A))
    dB = dev(B)
    gy = blaz.compress(dB)
    Bd = blaz.decompress(gy)
    Xd = blaz.decompress(gx)
    for b, bfull in ((dB, dB), (gy, Bd)):
        want = blaz.matmul(gx, b, prec="fp64").cpu().numpy()
        mag = (Xd.abs() @ bfull.abs()).cpu().numpy()
        for prec in ("fp32", "bf16x3"):
            got = blaz.matmul(gx, b, prec=prec).cpu().numpy()
            assert_dots_close(got, want, mag, rel=low_precision_tol(prec, k), what=f"matmul {prec} k={k}")
            # at this K the FP32 accumulation dominates both arithmetics: its
            # expected size, plus the BF16 split's own 3 * 2^-16
            rel = np.linalg.norm(got - want) / np.linalg.norm(want)
            fro = (2 + 4 * np.sqrt(k)) * U32 + (3 * 2.0 ** -16 if prec == "bf16x3" else 0.0)
            assert rel < fro, (prec, rel, fro)


@pytest.mark.parametrize("prec", ["fp32", "bf16x3"])
def test_matmul_low_precision_full_size_4096_sampled(prec):
    """Compressed 4096^2 field times dense U[-1, 1] in FP32 / BF16x3: sampled
    entries against the oracle, and the whole product against the FP64 path."""
    A, B, _ = workload_inputs("linalg-4096")
    g, _ = gpu_compress(A)
    dB = dev(B)
    C = blaz.matmul(g, dB, prec=prec)
    C64 = blaz.matmul(g, dB, prec="fp64")
    rel = (torch.linalg.norm(C - C64) / torch.linalg.norm(C64)).item()
    assert rel < low_precision_fro(prec, 4096), rel
    Ch = C.cpu().numpy()
    og = oracle.Compressed(4096, 4096, *host(g))
    rng = np.random.default_rng(6)
    for i, j in [(0, 0), (4095, 4095)] + [tuple(rng.integers(0, 4096, 2)) for _ in range(6)]:
        bj = np.ascontiguousarray(B[:, j])
        want = oracle.dot_dense(og, [i], bj, 0)[0]
        mag = np.abs(band_rows(og, int(i))) @ np.abs(bj)
        assert abs(Ch[i, j] - want) <= low_precision_tol(prec, 4096) * mag, (i, j, Ch[i, j], want)


@pytest.mark.parametrize("prec", ["fp64", "fp32", "bf16x3"])
@pytest.mark.parametrize("m,k,n", [(392, 136, 264), (64, 64, 64)])
def test_matmul_tiles_give_identical_results(prec, m, k, n):
    """The contraction tile (64 or 128) changes the grid, not the K order."""
    A = smooth_field(m, 4, 2.0, 1e-3, 470 + m, cols=k)
    B = uniform_matrix(k, n, 471)
    x, dB = upload(oracle.compress(A)), dev(B)
    c64 = blaz.matmul(x, dB, prec=prec, tile=64)
    c128 = blaz.matmul(x, dB, prec=prec, tile=128)
    assert torch.equal(c64.view(torch.int64), c128.view(torch.int64))
    with pytest.raises(blaz.BlazError):
        blaz.matmul(x, dB, prec=prec, tile=96)


def test_non_finite_input_is_contained_and_counted():
    """Non-finite inputs give unspecified contents in the affected blocks only:
    the kernels run, every other block is the oracle's, and blaz_diagnose
    counts the affected records."""
    A = smooth_field(32, 4, 2.0, 1e-3, 450, cols=48)
    A[3, 5] = np.nan      # block (0, 0): s becomes NaN
    A[17, 40] = np.inf    # block (2, 5)
    A[8, 8] = np.inf      # first element of block (1, 1): f is inf
    g = blaz.compress(dev(A))
    torch.cuda.synchronize()
    bad = {0, 2 * 6 + 5, 1 * 6 + 1}
    want, (_, cx, px) = oracle.compress(np.where(np.isfinite(A), A, 0.0), with_debug=True)
    got = host(g)
    keep = np.array([b not in bad for b in range(want.nblk)])
    sub = tuple(a[keep] for a in got)
    compare_compressed(sub, (want.f[keep], want.s[keep], want.phi[keep], want.codes[keep]), cx[keep], px[keep],
                       "finite blocks next to non-finite ones")
    counts = blaz.diagnose(g).cpu().numpy()
    assert counts[3] == 3
    D = blaz.decompress(g).cpu().numpy()  # runs; finite blocks decode as usual
    ok = np.isfinite(D).reshape(4, 8, 6, 8).all(axis=(1, 3)).ravel()
    assert all(ok[b] for b in range(want.nblk) if b not in bad)


def test_empty_and_k0():
    z = blaz.BlazMatrix.empty(0, 16)
    blaz.compress(torch.empty((0, 16), dtype=torch.float64, device="cuda"), out=z)
    a = blaz.BlazMatrix.empty(16, 0)
    C = blaz.matmul(a, torch.empty((0, 24), dtype=torch.float64, device="cuda"))
    assert C.shape == (16, 24) and torch.all(C == 0)
