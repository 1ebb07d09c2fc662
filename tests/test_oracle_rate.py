"""Pins of the oracle's tunable-rate form (L kept lines of DCT coefficients).

The conclusion asks for a tunable compression rate; it is read as the
number L of kept lines (rows and columns 0..L-1, 16L - L^2 codes), L = 2
being the paper's 28.  Nothing in the paper prints a rate-L example, so the
generalisation is pinned by what fixes it independently: the L = 2 case
equals the paper's functions bit for bit (and with them every pin of
test_oracle.py), the positions and order of the codes come from scipy's
orthonormal DCT-II, the decompression from scipy's inverse DCT and a numpy
inverse normalization, and Algorithm 1 / 2 keep their closed forms."""
import numpy as np
import pytest
import scipy.fft

import oracle
from synth import smooth_field


def field(n=64, seed=11):
    return smooth_field(n, 4, 2.0, 1e-3, seed)


def test_counts_strides_and_positions():
    assert [oracle.kept_count(L) for L in range(1, 9)] == [15, 28, 39, 48, 55, 60, 63, 64]
    assert [oracle.lib().oracle_kept_count(L) for L in range(1, 9)] == [15, 28, 39, 48, 55, 60, 63, 64]
    assert [oracle.code_stride(L) for L in range(1, 9)] == [16, 28, 40, 48, 56, 60, 64, 64]
    assert oracle.kept_positions(2) == oracle.KEPT
    assert oracle.kept_positions(8) == [(i, j) for i in range(8) for j in range(8)]


def test_two_lines_is_the_paper_scheme():
    A = field()
    a, (ax, ap) = oracle.compress_lines(A, 2, with_debug=True)
    b, (_, bx, bp) = oracle.compress(A, with_debug=True)
    for k in ("f", "s", "phi", "codes"):
        assert np.array_equal(getattr(a, k), getattr(b, k)), k
    assert np.array_equal(ax, bx) and np.array_equal(ap, bp)
    assert np.array_equal(oracle.decompress(a), oracle.decompress(b))


@pytest.mark.parametrize("lines", [1, 3, 5, 8])
def test_codes_are_scipy_dct_at_the_kept_positions(lines):
    """phi * D before truncation, D = orthonormal DCT-II of Delta' (the DC
    term to its pinned order), taken over the L-line mask in row-major order;
    phi and the codes are the same truncations as at L = 2."""
    A = field(seed=12)
    c, (cx, px) = oracle.compress_lines(A, lines, with_debug=True)
    pos = oracle.kept_positions(lines)
    for b in range(0, c.nblk, 7):
        I, J = divmod(b, A.shape[1] // 8)
        tr = oracle.compress_block(A[8 * I:8 * I + 8, 8 * J:8 * J + 8])
        D = scipy.fft.dctn(tr.arr("dprime"), type=2, norm="ortho")
        D[0, 0] = tr.arr("D")[0, 0]
        phi = c.phi[b]
        assert phi == tr.phi and px[b] == tr.phi_x
        want = np.array([phi * D[i, j] for i, j in pos])
        assert np.allclose(cx[b], want, rtol=1e-12, atol=1e-12)
        assert np.array_equal(c.codes[b, :len(pos)], np.trunc(cx[b]).astype(np.int8))
        assert not c.codes[b, len(pos):].any()  # word padding stays zero


@pytest.mark.parametrize("lines", [1, 3, 4, 8])
def test_decompression_is_scipy_idct_then_inverse_normalization(lines):
    A = field(seed=13)
    c = oracle.compress_lines(A, lines)
    got = oracle.decompress(c)
    pos = oracle.kept_positions(lines)
    nbc = A.shape[1] // 8
    for b in range(0, c.nblk, 5):
        I, J = divmod(b, nbc)
        D = np.zeros((8, 8))
        for t, (i, j) in enumerate(pos):
            D[i, j] = c.codes[b, t] / float(c.phi[b])
        P = c.s[b] * scipy.fft.idctn(D, type=2, norm="ortho")
        X = np.zeros((8, 8))
        for i in range(8):
            for j in range(8):
                if i == 0 and j == 0:
                    X[i, j] = c.f[b]
                elif i == 0:
                    X[i, j] = X[i, j - 1] + P[i, j]
                elif j == 0:
                    X[i, j] = X[i - 1, j] + P[i, j]
                else:
                    X[i, j] = (X[i - 1, j] + X[i, j - 1]) / 2 + P[i, j]
        blk = got[8 * I:8 * I + 8, 8 * J:8 * J + 8]
        assert np.allclose(blk, X, rtol=0, atol=1e-13 * max(1.0, np.abs(X).max()))


def test_coefficient_error_does_not_grow_with_more_lines():
    """The transform is orthonormal, so a block's error in the normalized
    domain is the error of its coefficients: kept ones lose |D - C/phi| <= |D|
    (phi is the same for every L, m being taken over all 64), dropped ones
    lose |D|.  Per block that error never grows with L.  (The decoded block's
    error can: the inverse normalization is not orthogonal.)  On smooth
    fields three lines decode clearly better than two."""
    A = field(64, 14)
    nbc = A.shape[1] // 8
    comp = {L: oracle.compress_lines(A, L) for L in range(1, 9)}
    for b in range(comp[2].nblk):
        I, J = divmod(b, nbc)
        tr = oracle.compress_block(A[8 * I:8 * I + 8, 8 * J:8 * J + 8])
        D = scipy.fft.dctn(tr.arr("dprime"), type=2, norm="ortho")
        D[0, 0] = tr.arr("D")[0, 0]
        errs = []
        for L in range(1, 9):
            c = comp[L]
            Dh = np.zeros((8, 8))
            for t, (i, j) in enumerate(oracle.kept_positions(L)):
                Dh[i, j] = c.codes[b, t] / float(c.phi[b])
            errs.append(float(np.sum((Dh - D) ** 2)))
        assert all(errs[k + 1] <= errs[k] * (1 + 1e-12) + 1e-30 for k in range(7)), (b, errs)
    for seed in (14, 15):
        A = field(128, seed)
        e2, e3 = (np.abs(oracle.decompress(oracle.compress_lines(A, L)) - A).mean() for L in (2, 3))
        assert e3 < 0.8 * e2


def test_add_and_scale_on_three_lines():
    """Algorithm 1's add(X, X): alpha = 1/2, phi = floor(phi1 / 2), and each
    code trunc(b C + b C) with b = (0.5 / phi1) phi; Algorithm 2 scales f and
    s and copies phi and every code."""
    A = field(seed=16)
    x = oracle.compress_lines(A, 3)
    z = oracle.add(x, x)
    n = oracle.kept_count(3)
    assert np.array_equal(z.f, x.f + x.f) and np.array_equal(z.s, x.s + x.s)
    p = np.maximum(1, x.phi.astype(int) // 2)
    assert np.array_equal(z.phi, p.astype(np.uint8))
    b = (0.5 / x.phi.astype(float)) * p
    y = b[:, None] * x.codes[:, :n] + b[:, None] * x.codes[:, :n]
    assert np.array_equal(z.codes[:, :n], np.clip(np.trunc(y), -127, 127).astype(np.int8))
    w = oracle.scale(x, -2.5)
    assert np.array_equal(w.f, x.f * -2.5) and np.array_equal(w.s, x.s * -2.5)
    assert np.array_equal(w.phi, x.phi) and np.array_equal(w.codes[:, :n], x.codes[:, :n])
