"""Pins of the FP64 CPU oracle against what the paper and the mathematics fix.

Each test names the passage it checks.  Expected values are the paper's
printed worked examples (tests/golden), closed forms, textbook routines run as
libraries (scipy's orthonormal DCT-II), invariants and brute force; none comes
from the oracle itself or from the GPU library.
"""
import os

import numpy as np
import pytest
import scipy.fft

import oracle
from synth import smooth_field

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")

# Kept coefficients, restated from the paper: the first two lines and the first
# two columns of the 8x8 DCT, scanned row by row.
KEPT_MASK = np.zeros((8, 8), bool)
KEPT_MASK[:2, :] = True
KEPT_MASK[:, :2] = True


def load_golden(name):
    rows, meta = [], {}
    with open(os.path.join(GOLDEN, name)) as fh:
        for line in fh:
            line = line.strip()
            if line.startswith("#"):
                body = line[1:].strip()
                if "=" in body and len(body.split("=")) == 2 and " " not in body.split("=")[0].strip():
                    k, v = body.split("=")
                    meta[k.strip()] = float(v)
                continue
            if line:
                rows.append([float(x) for x in line.split()])
    return np.array(rows), meta


def example1():
    """Example 1: f(x, y) = x * y with x and y from 0 in steps of 0.1."""
    x = 0.1 * np.arange(8)
    return np.multiply.outer(x, x)


# --------------------------------------------------------------------------
# Worked examples 2-5 (Section "Compression Scheme")
# --------------------------------------------------------------------------

def test_example2_normalization():
    tr = oracle.compress_block(example1())
    want, _ = load_golden("ex2_delta.txt")
    assert np.max(np.abs(tr.arr("delta") - want)) < 5e-4
    assert tr.f == 0.0
    # closed form: border 0, interior 0.005 (i + j)
    i = np.arange(8)
    closed = 0.005 * np.add.outer(i, i)
    closed[0, :] = 0.0
    closed[:, 0] = 0.0
    assert np.max(np.abs(tr.arr("delta") - closed)) < 1e-15


def test_example3_slope():
    tr = oracle.compress_block(example1())
    want, meta = load_golden("ex3_dprime.txt")
    assert tr.K == 49
    assert abs(tr.s - meta["s"]) < 1e-15
    assert np.max(np.abs(tr.arr("dprime") - want)) < 5e-4


def test_example4_prediction():
    tr = oracle.compress_block(example1())
    want, _ = load_golden("ex4_psi.txt")
    np.testing.assert_array_equal(tr.arr("psi"), want.astype(np.uint8))


def test_example5_transform_and_quantization():
    tr = oracle.compress_block(example1())
    want, meta = load_golden("ex5_codes.txt")
    assert tr.phi == int(meta["phi"])
    D = tr.arr("D")
    np.testing.assert_array_equal(np.trunc(tr.phi * D).astype(int), want.astype(int))
    # the stored stream is exactly the kept positions of P', row-major
    np.testing.assert_array_equal(np.array(tr.codes), want[KEPT_MASK].astype(np.int8))


def test_example1_same_codes_either_way_the_input_is_rounded():
    """0.01*i*j and (0.1 i)(0.1 j) differ in the last bits; both give Example 5."""
    i = np.arange(8)
    a = oracle.compress_block(0.01 * np.multiply.outer(i, i))
    b = oracle.compress_block(example1())
    assert a.phi == b.phi == 20
    np.testing.assert_array_equal(np.array(a.codes), np.array(b.codes))


# --------------------------------------------------------------------------
# Stage-by-stage definitions
# --------------------------------------------------------------------------

def rand_block(seed, smooth=True):
    rng = np.random.default_rng(seed)
    if smooth:
        return smooth_field(8, 3, 0.7, 1e-3, seed) * rng.uniform(0.1, 10)
    return rng.standard_normal((8, 8))


def brute_normalize(M):
    """Eq. (1) as a 64x64 linear map applied to M (constructed column by column)."""
    L = np.zeros((64, 64))
    for e in range(64):
        E = np.zeros(64)
        E[e] = 1.0
        L[:, e] = oracle.compress_block(E.reshape(8, 8)).arr("delta").reshape(64)
    return L


def test_normalization_linear_map_matches_equation():
    """Eq. eqnorm: the map's matrix has exactly the printed stencil."""
    L = brute_normalize(None)
    for i in range(8):
        for j in range(8):
            row = L[i * 8 + j].reshape(8, 8)
            want = np.zeros((8, 8))
            if i == 0 and j == 0:
                pass
            elif i == 0:
                want[0, j], want[0, j - 1] = 1.0, -1.0
            elif j == 0:
                want[i, 0], want[i - 1, 0] = 1.0, -1.0
            else:
                want[i, j], want[i - 1, j], want[i, j - 1] = 1.0, -0.5, -0.5
            np.testing.assert_array_equal(row, want)


@pytest.mark.parametrize("seed", range(5))
def test_normalization_is_linear(seed):
    """Introduction: every stage but the quantization is a linear map."""
    M, N = rand_block(seed), rand_block(seed + 100)
    a, b = 1.7, -0.3
    d = oracle.compress_block(a * M + b * N).arr("delta")
    dm, dn = oracle.compress_block(M).arr("delta"), oracle.compress_block(N).arr("delta")
    assert np.max(np.abs(d - (a * dm + b * dn))) <= 1e-13 * max(1.0, np.max(np.abs(d)))


@pytest.mark.parametrize("seed", range(5))
def test_slope_definition(seed):
    """Eqs. eqslope/eqslope2: s = mean of |Delta| over its non-zero entries."""
    M = rand_block(seed, smooth=False)
    M[3, :] = M[2, :]  # forces some Delta to be exactly 0
    M[:, 5] = M[:, 4]
    tr = oracle.compress_block(M)
    delta = tr.arr("delta")
    nz = delta != 0
    assert tr.K == int(nz.sum())
    assert abs(tr.s - np.abs(delta[nz]).sum() / nz.sum()) <= 1e-15 * tr.s * 4
    np.testing.assert_allclose(tr.arr("dprime"), delta / tr.s, rtol=1e-15, atol=0)


def test_slope_uses_pairwise_order():
    """The summation order is fixed as a pairwise tree; on values whose plain
    left-to-right sum rounds differently the oracle must give the tree's sum."""
    # Delta row 0 = [0, x1..x7], all other rows built by the first column only.
    rng = np.random.default_rng(7)
    for _ in range(50):
        M = np.cumsum(np.cumsum(rng.standard_normal((8, 8)) * 10.0 ** rng.integers(-3, 3, (8, 8)),
                                axis=0), axis=1)
        tr = oracle.compress_block(M)
        a = np.abs(tr.arr("delta")).reshape(64)
        t = list(a)
        while len(t) > 1:
            t = [t[2 * k] + t[2 * k + 1] for k in range(len(t) // 2)]
        assert tr.s == t[0] / tr.K


@pytest.mark.parametrize("seed", range(8))
def test_dct_matches_scipy_orthonormal_dct2(seed):
    """Eq. eqdct with the alphas below Eq. eqdct2 is the orthonormal DCT-II."""
    tr = oracle.compress_block(rand_block(seed, smooth=seed % 2 == 0))
    ref = scipy.fft.dctn(tr.arr("dprime"), type=2, norm="ortho")
    D = tr.arr("D")
    assert np.max(np.abs(D - ref)) <= 1e-13 * np.max(np.abs(ref))


@pytest.mark.parametrize("seed", range(4))
def test_dct_parseval(seed):
    tr = oracle.compress_block(rand_block(seed, smooth=False))
    D, dp = tr.arr("D"), tr.arr("dprime")
    assert abs(np.sum(D * D) - np.sum(dp * dp)) <= 1e-13 * np.sum(dp * dp)


@pytest.mark.parametrize("seed", range(4))
def test_idct_matches_scipy(seed):
    D = np.random.default_rng(seed).standard_normal((8, 8))
    ref = scipy.fft.idctn(D, type=2, norm="ortho")
    assert np.max(np.abs(oracle.idct(D) - ref)) <= 1e-14 * 8


def test_dc_is_k_over_8_for_sign_consistent_blocks():
    """When every non-zero Delta has one sign, sum Delta' = K, so
    D_00 = alpha_0^2 K = K/8: Example 1 gives 49/8 (Example 5: m = 6.125)."""
    tr = oracle.compress_block(example1())
    assert abs(tr.D[0] - 49 / 8) <= 4e-15 * 8
    rng = np.random.default_rng(3)
    for _ in range(20):
        M = np.cumsum(np.cumsum(rng.uniform(0.1, 1.0, (8, 8)), 0), 1)  # increasing both ways
        tr = oracle.compress_block(M)
        assert tr.K == 63
        assert abs(tr.D[0] - 63 / 8) <= 4e-15 * 8


@pytest.mark.parametrize("seed", range(6))
def test_prediction_brute_force_equals_nearest_grid_point(seed):
    """Eq. eqpredict: Psi is the index of the nearest of 256 equidistant points
    of [s - s_max, s + s_max) spaced 2 s_max / 256 (closed form, away from ties)."""
    tr = oracle.compress_block(rand_block(seed, smooth=False))
    dp, s = tr.arr("dprime"), tr.s
    smax = np.max(np.abs(dp))
    q = (dp - (s - smax)) / (2 * smax / 256)
    k = np.clip(np.floor(q + 0.5), 0, 255)
    away = np.abs(q - np.floor(q) - 0.5) > 1e-9
    np.testing.assert_array_equal(tr.arr("psi")[away], k[away].astype(np.uint8))


@pytest.mark.parametrize("seed", range(6))
def test_quantization_definition(seed):
    """Eq. eqphi and Example 5: phi = trunc(127/m), m = max|D| over all 64;
    codes = trunc(phi D) at the kept positions, row-major."""
    tr = oracle.compress_block(rand_block(seed, smooth=seed % 2 == 1))
    ref = scipy.fft.dctn(tr.arr("dprime"), type=2, norm="ortho")
    m = np.max(np.abs(ref))
    assert abs(tr.m - m) <= 1e-13 * m
    assert tr.phi == min(255, int(np.trunc(127 / tr.m)))
    x = tr.phi * ref[KEPT_MASK]
    away = np.abs(x - np.round(x)) > 1e-9
    np.testing.assert_array_equal(np.array(tr.codes)[away], np.trunc(x[away]).astype(np.int8))
    assert np.all(np.abs(np.array(tr.codes)) <= 127)


def test_phi_clamped_for_sparse_delta():
    """Few non-zero Delta make 127/m exceed 8 bits: phi saturates at 255."""
    M = np.zeros((8, 8))
    M[7, 7] = 1e-3  # one non-zero interior Delta -> K = 1
    tr = oracle.compress_block(M)
    assert tr.K == 1 and 127 / tr.m > 255
    assert tr.phi == 255
    assert np.all(np.abs(np.array(tr.codes)) <= 127)


def test_constant_block():
    """A constant block has K = 0: s = 0, codes 0, and it decodes to f exactly."""
    M = np.full((8, 8), -3.25)
    tr = oracle.compress_block(M)
    assert tr.K == 0 and tr.s == 0.0 and tr.f == -3.25
    assert tr.phi == 255 and not np.any(np.array(tr.codes))
    np.testing.assert_array_equal(oracle.decompress_block(tr.f, tr.s, tr.phi, np.array(tr.codes)), M)


@pytest.mark.parametrize("b,c", [(0.3, 0.2), (-0.7, 0.1), (0.05, -0.5), (1.0, 0.0)])
def test_affine_block_closed_forms(b, c):
    """M_uv = a + b u + c v: Delta'_0v = c/s, Delta'_u0 = b/s,
    Delta'_uv = (b + c)/(2 s), s = (7|b| + 7|c| + 49|b + c|/2) / K."""
    a = 1.25
    u = np.arange(8)
    M = a + b * u[:, None] + c * u[None, :]
    tr = oracle.compress_block(M)
    K = 7 * (b != 0) + 7 * (c != 0) + 49 * (b + c != 0)
    assert tr.K == K
    s = (7 * abs(b) + 7 * abs(c) + 49 * abs(b + c) / 2) / K
    assert abs(tr.s - s) <= 1e-14 * s
    dp = tr.arr("dprime")
    np.testing.assert_allclose(dp[0, 1:], c / s, rtol=1e-13, atol=1e-15)
    np.testing.assert_allclose(dp[1:, 0], b / s, rtol=1e-13, atol=1e-15)
    np.testing.assert_allclose(dp[1:, 1:], (b + c) / (2 * s), rtol=1e-13, atol=1e-15)
    assert abs(tr.D[0] - dp.sum() / 8) <= 1e-13 * 8


def test_record_size_and_ratio():
    """29 8-bit integers + 2 binary64 = 360 bits per block; 4096/360 = 11.37."""
    c = oracle.compress(smooth_field(16, 2, 1.0, 0.0, 5))
    per_block = (c.f.nbytes + c.s.nbytes + c.phi.nbytes + c.codes.nbytes) / c.nblk
    assert per_block * 8 == 360
    assert abs(64 * 64 / 360 - 11.37) < 0.01


# --------------------------------------------------------------------------
# Decompression (Eq. eqbbb, read as the exact inverse of Eq. eqnorm)
# --------------------------------------------------------------------------

@pytest.mark.parametrize("seed", range(6))
def test_lossless_round_trip(seed):
    """Without quantization (all 64 real coefficients), IDCT and the inverse
    normalization undo the forward stages."""
    M = rand_block(seed, smooth=seed % 2 == 0) + 3.0
    tr = oracle.compress_block(M)
    B = oracle.inverse_normalize(tr.f, tr.s, oracle.idct(tr.arr("D")))
    assert np.max(np.abs(B - M)) <= 1e-13 * np.max(np.abs(M))


def test_inverse_normalization_inverts_equation1_exactly():
    """Inverse of Eq. eqnorm on integer-valued blocks is exact."""
    M = np.random.default_rng(1).integers(-1000, 1000, (8, 8)).astype(float)
    tr = oracle.compress_block(M)
    # s = 1 and P = Delta: halves of integers are exact, so the rebuild is exact
    B = oracle.inverse_normalize(M[0, 0], 1.0, tr.arr("delta"))
    np.testing.assert_array_equal(B, M)


def test_printed_subscripts_would_not_invert():
    """Eq. eqbbb indexes P one step behind; with that indexing even the exact
    Delta does not rebuild the block, which is why the inverse of Eq. eqnorm is used."""
    M = np.random.default_rng(2).standard_normal((8, 8))
    delta = oracle.compress_block(M).arr("delta")
    lit = np.zeros((8, 8))
    for i in range(8):
        for j in range(8):
            if i == 0 and j == 0:
                lit[i, j] = M[0, 0]
            elif i == 0:
                lit[i, j] = lit[0, j - 1] + delta[0, j - 1]
            elif j == 0:
                lit[i, j] = lit[i - 1, 0] + delta[i - 1, 0]
            else:
                lit[i, j] = (lit[i - 1, j] + lit[i, j - 1]) / 2 + delta[i - 1, j - 1]
    assert np.max(np.abs(lit - M)) > 1e-3
    B = oracle.inverse_normalize(M[0, 0], 1.0, delta)
    assert np.max(np.abs(B - M)) < 1e-13


def test_decompress_dequantizes_kept_codes_only():
    """Section "Dot product": discarded coefficients are zeros; kept ones C/phi."""
    rng = np.random.default_rng(4)
    codes = rng.integers(-127, 128, 28).astype(np.int8)
    phi, f, s = 37, 0.5, 0.02
    D = np.zeros((8, 8))
    D[KEPT_MASK] = codes / phi
    want = oracle.inverse_normalize(f, s, scipy.fft.idctn(D, type=2, norm="ortho"))
    got = oracle.decompress_block(f, s, phi, codes)
    assert np.max(np.abs(got - want)) <= 1e-14 * np.max(np.abs(want))


def test_example1_round_trip_error_is_small():
    """Example 1 only loses P'_44 to the quantization (Example 5)."""
    c = oracle.compress(example1())
    back = oracle.decompress(c)
    err = np.max(np.abs(back - example1()))
    assert err < 0.02 * np.max(np.abs(example1()))


@pytest.mark.parametrize("n", [64, 128])
def test_matrix_round_trip_small_relative_error(n):
    """The method's own error on smooth fields: a few percent of the range at most."""
    M = smooth_field(n, 4, 2.0, 1e-3, 11 + n)
    back = oracle.decompress(oracle.compress(M))
    assert np.linalg.norm(back - M) / np.linalg.norm(M) < 0.05


def test_blocks_are_independent_and_indexed_row_major():
    """Block (I, J) of the matrix is stored at I*(cols/8)+J and depends on that tile only."""
    M = smooth_field(24, 3, 1.5, 1e-3, 9, cols=40)
    c = oracle.compress(M)
    for I in range(3):
        for J in range(5):
            tr = oracle.compress_block(M[8 * I:8 * I + 8, 8 * J:8 * J + 8])
            b = I * 5 + J
            assert c.f[b] == tr.f and c.s[b] == tr.s and c.phi[b] == tr.phi
            np.testing.assert_array_equal(c.codes[b], np.array(tr.codes))
    f, s, phi, codes, _, _ = oracle.compress_blocks(M, [7, 0, 14])
    for q, b in enumerate([7, 0, 14]):
        assert f[q] == c.f[b] and s[q] == c.s[b] and phi[q] == c.phi[b]
        np.testing.assert_array_equal(codes[q], c.codes[b])


def test_debug_outputs_are_values_before_truncation():
    M = smooth_field(16, 3, 1.0, 1e-3, 21)
    c, (psi, code_x, phi_x) = oracle.compress(M, with_debug=True)
    np.testing.assert_array_equal(np.trunc(code_x).astype(np.int8), c.codes)
    np.testing.assert_array_equal(np.minimum(255, np.trunc(phi_x)).astype(np.uint8), c.phi)


# --------------------------------------------------------------------------
# Operations on compressed matrices (Section "Basic Linear Algebra Algorithms")
# --------------------------------------------------------------------------

def two_fields(n=32, seed=30):
    return (oracle.compress(smooth_field(n, 4, 2.0, 1e-3, seed)),
            oracle.compress(smooth_field(n, 4, 2.0, 1e-3, seed + 1)))


def test_add_header_fields():
    """Algorithm 1's sums and phi: f = f1 + f2, s = s1 + s2, phi = phi1 phi2 / (phi1 + phi2)."""
    x, y = two_fields()
    z = oracle.add(x, y)
    np.testing.assert_array_equal(z.f, x.f + y.f)
    np.testing.assert_array_equal(z.s, x.s + y.s)
    p1, p2 = x.phi.astype(int), y.phi.astype(int)
    np.testing.assert_array_equal(z.phi, np.maximum(1, (p1 * p2) // (p1 + p2)))


def test_add_is_commutative():
    x, y = two_fields()
    a, b = oracle.add(x, y), oracle.add(y, x)
    for k in ("f", "s", "phi", "codes"):
        np.testing.assert_array_equal(getattr(a, k), getattr(b, k))


def test_add_self_closed_form():
    """add(X, X): alpha = 1/2, phi = floor(phi1/2), beta = (0.5/phi1) phi,
    C = trunc(beta C1 + beta C1)."""
    x, _ = two_fields()
    z = oracle.add(x, x)
    p = np.maximum(1, x.phi.astype(int) // 2)
    np.testing.assert_array_equal(z.phi, p)
    beta = (0.5 / x.phi.astype(float)) * p
    c1 = x.codes.astype(float)
    want = np.trunc(beta[:, None] * c1 + beta[:, None] * c1).astype(np.int8)
    np.testing.assert_array_equal(z.codes, want)


def test_add_coefficients_follow_linearity():
    """Eq. eq55 and Eq. eqdct2: the decoded coefficient s C / phi of the sum is
    s1 C1/phi1 + s2 C2/phi2 up to one quantization step |s|/phi."""
    x, y = two_fields(48, 40)
    z = oracle.add(x, y)
    lhs = z.s[:, None] * z.codes / z.phi[:, None].astype(float)
    rhs = (x.s[:, None] * x.codes / x.phi[:, None].astype(float)
           + y.s[:, None] * y.codes / y.phi[:, None].astype(float))
    step = np.abs(z.s)[:, None] / z.phi[:, None].astype(float)
    assert np.all(np.abs(lhs - rhs) <= step * (1 + 1e-12))


def test_add_decompresses_close_to_the_sum():
    x, y = two_fields(64, 50)
    z = oracle.decompress(oracle.add(x, y))
    want = oracle.decompress(x) + oracle.decompress(y)
    assert np.linalg.norm(z - want) / np.linalg.norm(want) < 0.05


def test_add_opposite_slopes_saturate_and_cancel():
    """Readings for Algorithm 1: codes saturate at +-127; s1 + s2 = 0 gives 0 codes."""
    x, y = two_fields(16, 60)
    y_neg = oracle.scale(x, -1.0)
    z = oracle.add(x, y_neg)
    np.testing.assert_array_equal(z.s, np.zeros_like(z.s))
    assert not np.any(z.codes)
    np.testing.assert_array_equal(oracle.decompress(z), np.repeat(np.repeat(
        (x.f - x.f).reshape(2, 2), 8, 0), 8, 1))
    w = oracle.add(x, oracle.scale(y, -0.97))
    assert np.all(np.abs(w.codes.astype(int)) <= 127)


def test_scale_algorithm2():
    """Algorithm 2: f and s times c; phi and codes unchanged."""
    x, _ = two_fields()
    for c in (1.7, -2.0, 0.0):
        z = oracle.scale(x, c)
        np.testing.assert_array_equal(z.f, x.f * c)
        np.testing.assert_array_equal(z.s, x.s * c)
        np.testing.assert_array_equal(z.phi, x.phi)
        np.testing.assert_array_equal(z.codes, x.codes)


def test_scale_keeps_relative_error():
    """Section "Accuracy Measurements": changing the constant does not change
    the relative error; decompress(scale(X, c)) = c decompress(X)."""
    M = smooth_field(32, 4, 2.0, 1e-3, 70)
    x = oracle.compress(M)
    base = oracle.decompress(x)
    e0 = np.linalg.norm(base - M) / np.linalg.norm(M)
    for c in (2.0, 1.7, -0.3):
        sc = oracle.decompress(oracle.scale(x, c))
        assert np.max(np.abs(sc - c * base)) <= 8 * np.finfo(float).eps * np.max(np.abs(c * base)) * 8
        e = np.linalg.norm(sc - c * M) / np.linalg.norm(c * M)
        assert abs(e - e0) <= 1e-12


def test_dot_equals_matmul_element():
    """Section "Accuracy Measurements": dot(i, j) is element (i, j) of the product."""
    x = oracle.compress(smooth_field(24, 3, 1.0, 1e-3, 80, cols=16))
    y = oracle.compress(smooth_field(16, 3, 1.0, 1e-3, 81, cols=32))
    P = oracle.matmul(x, y)
    rows = np.array([0, 5, 23, 8, 15])
    cols = np.array([0, 31, 7, 16, 9])
    d = oracle.dot(x, rows, y, cols)
    np.testing.assert_allclose(d, P[rows, cols], rtol=1e-13, atol=1e-13)


def test_dot_and_gemm_match_numpy_on_decompressed():
    x = oracle.compress(smooth_field(16, 3, 1.0, 1e-3, 90))
    y = oracle.compress(smooth_field(16, 3, 1.0, 1e-3, 91))
    X, Y = oracle.decompress(x), oracle.decompress(y)
    np.testing.assert_allclose(oracle.matmul(x, y), X @ Y, rtol=1e-13, atol=1e-13)
    v = np.random.default_rng(0).uniform(-1, 1, (3, 16))
    d = oracle.dot_dense(x, [2, 9, 15], v, 16)
    np.testing.assert_allclose(d, [X[2] @ v[0], X[9] @ v[1], X[15] @ v[2]], rtol=1e-13)
    d0 = oracle.dot_dense(x, [2, 9], v[0], 0)
    np.testing.assert_allclose(d0, [X[2] @ v[0], X[9] @ v[0]], rtol=1e-13)
    B = np.random.default_rng(1).standard_normal((16, 8))
    np.testing.assert_allclose(oracle.gemm(X, B), X @ B, rtol=1e-13, atol=1e-13)


def test_gemm_catches_transpose():
    A = np.arange(6.0).reshape(2, 3)
    B = np.arange(12.0).reshape(3, 4)
    np.testing.assert_array_equal(oracle.gemm(A, B), A @ B)


def test_thread_count_does_not_change_results():
    """The whole-matrix loops split blocks, product rows and queries between
    threads; each is computed by the same sequential code, so one thread and
    several give the same bits."""
    A = smooth_field(64, 6, 3.0, 1e-3, 31, cols=136)
    B = smooth_field(136, 6, 3.0, 1e-3, 32, cols=72)
    rows = np.arange(0, 64, 3)
    V = np.random.default_rng(33).uniform(-1, 1, (len(rows), 136))
    outs = []
    try:
        for threads in (1, 4):
            oracle.set_threads(threads)
            x, (psi, cx, px) = oracle.compress(A, with_debug=True)
            y = oracle.compress(B)
            z = oracle.scale(oracle.add(x, x), -1.5)
            Xd, Yd = oracle.decompress(x), oracle.decompress(y)
            outs.append([x.f, x.s, x.phi, x.codes, psi, cx, px, z.f, z.s, z.phi, z.codes, Xd,
                         oracle.gemm(Xd, Yd), oracle.dot(x, rows, y, rows % 72),
                         oracle.dot_dense(x, rows, V, 136)])
    finally:
        oracle.set_threads(oracle_default_threads())
    for a, b in zip(*outs):
        assert np.array_equal(np.asarray(a).view(np.uint8), np.asarray(b).view(np.uint8))


def oracle_default_threads():
    import os
    return len(os.sched_getaffinity(0))
