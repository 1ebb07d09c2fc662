"""Property tests on small random matrices (hypothesis): invariants of the
oracle's records and of Algorithms 1 and 2 on the CPU, and the GPU's
compress / add / scale, decompress, dots and products, the tunable rate and
the mixed-precision transform, a persistent batch and the predicted-slope
input against the oracle on the same random inputs, and the product's other
forms (compressed output, grouped, allocation-free) against the standalone
product.

Inputs are drawn per example from a structure (Gaussian, a single non-zero
per block, constant blocks, affine ramps, huge or tiny magnitudes, mixed
signs of slope) and a seed; hypothesis shrinks over those two choices."""
import os

import numpy as np
import pytest
from hypothesis import HealthCheck, example, given, settings
from hypothesis import strategies as st

import oracle
from oracle.parity import assert_same_compressed, compare_compressed, near_integer

STRUCTURES = ("normal", "sparse", "constant", "affine", "huge", "tiny", "sign_mixed")


def make_matrix(structure, seed, br, bc):
    rng = np.random.default_rng(seed)
    r, c = 8 * br, 8 * bc
    if structure == "normal":
        return rng.standard_normal((r, c))
    if structure == "sparse":  # one non-zero per block: sparse Delta
        A = np.zeros((r, c))
        for I in range(br):
            for J in range(bc):
                A[8 * I + rng.integers(8), 8 * J + rng.integers(8)] = rng.standard_normal() * 10.0 ** rng.integers(-3, 4)
        return A
    if structure == "constant":
        return np.kron(rng.standard_normal((br, bc)), np.ones((8, 8)))
    if structure == "affine":
        i, j = np.mgrid[0:r, 0:c]
        return rng.standard_normal() + rng.standard_normal() * i + rng.standard_normal() * j
    if structure == "huge":
        return rng.standard_normal((r, c)) * 1e150
    if structure == "tiny":
        return rng.standard_normal((r, c)) * 1e-150
    # alternating sign of the slope between neighbouring blocks
    return np.cumsum(rng.standard_normal((r, c)), axis=1) * np.where((np.arange(c) // 8) % 2, -1.0, 1.0)


# 1..9 blocks per side: up to 81 blocks, more than one 64-block wave with a
# ragged last one
matrices = st.tuples(st.sampled_from(STRUCTURES), st.integers(0, 2 ** 32 - 1), st.integers(1, 9), st.integers(1, 9))
# Derandomized (the same draws on every run) unless BLAZ_PROPERTY_EXPLORE is
# set, which draws afresh.
CPU = settings(max_examples=60, deadline=None, database=None, suppress_health_check=[HealthCheck.too_slow],
               derandomize=not os.environ.get("BLAZ_PROPERTY_EXPLORE"))


@CPU
@given(matrices)
def test_records_are_well_formed(m):
    A = make_matrix(*m)
    x = oracle.compress(A)
    blocks = A.reshape(A.shape[0] // 8, 8, A.shape[1] // 8, 8).transpose(0, 2, 1, 3).reshape(-1, 64)
    assert np.array_equal(x.f.view(np.uint64), blocks[:, 0].copy().view(np.uint64))  # f = X_00, exactly
    assert np.all(np.isfinite(x.s)) and np.all(x.s >= 0)
    assert np.all(x.phi >= 1)
    assert np.all(np.abs(x.codes.astype(int)) <= 127)
    flat = np.all(blocks == blocks[:, :1], axis=1)  # constant blocks: no slope, no codes
    assert np.all(x.s[flat] == 0) and not np.any(x.codes[flat])


@CPU
@given(matrices, matrices)
def test_add_commutes_and_a_block_minus_itself_is_zero(m1, m2):
    A = make_matrix(*m1)
    B = make_matrix(m2[0], m2[1], m1[2], m1[3])
    x, y = oracle.compress(A), oracle.compress(B)
    xy, yx = oracle.add(x, y), oracle.add(y, x)
    assert_same_compressed((xy.f, xy.s, xy.phi, xy.codes), (yx.f, yx.s, yx.phi, yx.codes), "x + y vs y + x")
    z = oracle.add(x, oracle.scale(x, -1.0))
    assert np.all(z.f == 0) and np.all(z.s == 0) and not np.any(z.codes)
    assert np.all(z.phi >= 1)


@CPU
@given(matrices, st.floats(-1e3, 1e3, allow_nan=False).filter(lambda c: c != 0))
def test_scale_keeps_codes_and_scales_the_block(m, c):
    A = make_matrix(*m)
    x = oracle.compress(A)
    z = oracle.scale(x, c)
    assert np.array_equal(z.codes, x.codes) and np.array_equal(z.phi, x.phi)
    assert np.array_equal(z.f, c * x.f) and np.array_equal(z.s, c * x.s)
    Dx, Dz = oracle.decompress(x), oracle.decompress(z)
    scale_ref = np.abs(c * Dx).max() + 1e-300
    assert np.abs(Dz - c * Dx).max() <= 1e-12 * scale_ref


@CPU
@given(matrices)
def test_phi_halves_towards_one_under_repeated_self_addition(m):
    x = oracle.compress(make_matrix(*m))
    for _ in range(9):
        z = oracle.add(x, x)
        assert np.array_equal(z.phi, np.maximum(1, x.phi.astype(int) * x.phi // (2 * x.phi.astype(int))).astype(np.uint8))
        assert np.all(np.abs(z.codes.astype(int)) <= 127)
        x = z
    assert np.all(x.phi == 1)


# --------------------------------------------------------------------------
# GPU against the oracle on the same random inputs
# --------------------------------------------------------------------------

def _boundary_values(code_x, phi_x):
    """Non-zero codes and phi whose value before truncation lies on (within
    2^-40 of) an integer: the mismatches the tie rule can explain."""
    with np.errstate(invalid="ignore"):
        return int((near_integer(code_x) & (code_x != 0)).sum() + near_integer(phi_x).sum())


# The GPU draws are derandomized too (the same 40 examples on every run).
GPU = settings(max_examples=40, deadline=None, database=None, derandomize=not os.environ.get("BLAZ_PROPERTY_EXPLORE"),
               suppress_health_check=[HealthCheck.too_slow])


@pytest.mark.gpu
@GPU
@given(matrices, st.floats(-1e3, 1e3, allow_nan=False))
@example(("sparse", 39078084, 1, 1), 0.0)  # a single non-zero: two codes on a boundary
def test_gpu_compress_add_scale_match_the_oracle(m, c):
    import torch
    import paper_2202_13007_amd as blaz
    A = make_matrix(*m)
    B = make_matrix(m[0], m[1] ^ 0x5A5A, m[2], m[3])
    o, (_, code_x, phi_x) = oracle.compress(A, with_debug=True)
    g = blaz.compress(torch.from_numpy(A).cuda())
    ties = compare_compressed(g.to_host(), (o.f, o.s, o.phi, o.codes), code_x, phi_x, f"compress {m}")
    # Structured blocks (one non-zero, affine ramps) have exact rational
    # coefficients that can sit on a truncation boundary, so ties are bounded
    # by the number of such values, as for the designed blocks of the parity
    # tests (compare_compressed has already checked each one is a boundary tie).
    boundary = _boundary_values(code_x, phi_x)
    assert ties <= boundary, (ties, boundary)
    ob = oracle.compress(B)
    x = blaz.BlazMatrix.from_host(o.rows, o.cols, o.f, o.s, o.phi, o.codes)
    y = blaz.BlazMatrix.from_host(ob.rows, ob.cols, ob.f, ob.s, ob.phi, ob.codes)
    s = oracle.add(o, ob)
    assert_same_compressed(blaz.add(x, y).to_host(), (s.f, s.s, s.phi, s.codes), f"add {m}")
    k = oracle.scale(o, c)
    assert_same_compressed(blaz.scale(x, c).to_host(), (k.f, k.s, k.phi, k.codes), f"scale {m} by {c}")


@pytest.mark.gpu
@GPU
@given(matrices, st.integers(1, 3))
def test_gpu_decompress_dot_matmul_match_the_oracle(m, bn):
    """The partly decompressed operations on the same structures: the GPU
    rebuilds, dots and products of the oracle's records (uploaded, so that
    no compression tie enters) against the oracle's, within the parity rules
    (1e-12 of each block's largest value, 1e-12 of sum |x_k y_k|)."""
    import torch
    import paper_2202_13007_amd as blaz
    from oracle.parity import assert_blocks_close, assert_dots_close
    A = make_matrix(*m)
    B = make_matrix(m[0], m[1] ^ 0x3C3C, m[3], bn)  # rows of B = columns of A
    o, ob = oracle.compress(A), oracle.compress(B)
    x = blaz.BlazMatrix.from_host(o.rows, o.cols, o.f, o.s, o.phi, o.codes)
    y = blaz.BlazMatrix.from_host(ob.rows, ob.cols, ob.f, ob.s, ob.phi, ob.codes)
    Xd, Yd = oracle.decompress(o), oracle.decompress(ob)
    assert_blocks_close(blaz.decompress(x).cpu().numpy(), Xd, what=f"decompress {m}")

    # every line of X against every column of Y
    rows, cols = np.meshgrid(np.arange(o.rows), np.arange(ob.cols), indexing="ij")
    xrow, ycol = rows.ravel().astype(np.int64), cols.ravel().astype(np.int64)
    mag = (np.abs(Xd)[xrow] * np.abs(Yd).T[ycol]).sum(axis=1)
    got = blaz.dot(x, torch.from_numpy(xrow).cuda(), y, torch.from_numpy(ycol).cuda()).cpu().numpy()
    assert_dots_close(got, oracle.dot(o, xrow, ob, ycol), mag, what=f"dot {m}")

    absprod = np.abs(Xd) @ np.abs(Yd)
    for b, ref, what in ((y, oracle.matmul(o, ob), "compressed B"),
                         (torch.from_numpy(Yd).cuda(), oracle.matmul(o, bdense=Yd), "dense B")):
        C = blaz.matmul(x, b).cpu().numpy()
        assert_dots_close(C.ravel(), ref.ravel(), absprod.ravel(), what=f"matmul {what} {m}")


@pytest.mark.gpu
@GPU
@given(matrices, st.integers(1, 8), st.floats(-1e3, 1e3, allow_nan=False))
def test_gpu_tunable_rate_matches_the_oracle(m, lines, c):
    """The tunable rate (L kept lines) on the same structures: compress (ties
    bounded by the boundary values), rebuild, add and scale of the oracle's
    records against the oracle."""
    import torch
    import paper_2202_13007_amd as blaz
    from oracle.parity import assert_blocks_close
    A = make_matrix(*m)
    B = make_matrix(m[0], m[1] ^ 0x0F0F, m[2], m[3])
    o, (code_x, phi_x) = oracle.compress_lines(A, lines, with_debug=True)
    g = blaz.compress(torch.from_numpy(A).cuda(), lines=lines)
    ties = compare_compressed(g.to_host(), (o.f, o.s, o.phi, o.codes), code_x, phi_x, f"compress L={lines} {m}")
    boundary = _boundary_values(code_x, phi_x)
    assert ties <= boundary, (ties, boundary)
    ob = oracle.compress_lines(B, lines)
    x = blaz.BlazMatrix.from_host(o.rows, o.cols, o.f, o.s, o.phi, o.codes, lines=lines)
    y = blaz.BlazMatrix.from_host(ob.rows, ob.cols, ob.f, ob.s, ob.phi, ob.codes, lines=lines)
    assert_blocks_close(blaz.decompress(x).cpu().numpy(), oracle.decompress(o), what=f"decompress L={lines} {m}")
    s = oracle.add(o, ob)
    assert_same_compressed(blaz.add(x, y).to_host(), (s.f, s.s, s.phi, s.codes), f"add L={lines} {m}")
    k = oracle.scale(o, c)
    assert_same_compressed(blaz.scale(x, c).to_host(), (k.f, k.s, k.phi, k.codes), f"scale L={lines} {m} by {c}")


@pytest.mark.gpu
@GPU
@given(matrices, st.sampled_from(["fp32", "bf16x3"]))
def test_gpu_mixed_precision_transform_matches_the_oracle(m, prec):
    """The transform on the matrix cores on the same structures: f and s
    bit-exact, phi and codes equal to the oracle's except where the oracle's
    value lies within the arithmetic's error bound of an integer."""
    import torch
    import paper_2202_13007_amd as blaz
    from test_gpu_parity import compare_mixed
    A = make_matrix(*m)
    o, (_, code_x, phi_x) = oracle.compress(A, with_debug=True)
    g = blaz.compress(torch.from_numpy(A).cuda(), prec=prec)
    compare_mixed(g.to_host(), (o.f, o.s, o.phi, o.codes), code_x, phi_x, prec)



@pytest.mark.gpu
@GPU
@given(matrices, st.floats(-1e3, 1e3, allow_nan=False))
def test_gpu_batch_and_predicted_input_match_the_oracle(m, c):
    """One persistent batch (compress, add, scale, decompress) and the
    predicted-slope transform input on the same structures, against the
    oracle under the parity rules."""
    import torch
    import paper_2202_13007_amd as blaz
    from oracle.parity import assert_blocks_close
    A = make_matrix(*m)
    B = make_matrix(m[0], m[1] ^ 0x7E7E, m[2], m[3])
    o, (_, code_x, phi_x) = oracle.compress(A, with_debug=True)
    ob = oracle.compress(B)
    x = blaz.BlazMatrix.from_host(o.rows, o.cols, o.f, o.s, o.phi, o.codes)
    y = blaz.BlazMatrix.from_host(ob.rows, ob.cols, ob.f, ob.s, ob.phi, ob.codes)
    dA = torch.from_numpy(A).cuda()
    cz, az, sz = (blaz.BlazMatrix.empty(o.rows, o.cols) for _ in range(3))
    D = torch.empty_like(dA)
    batch = blaz.Batch()
    batch.compress(dA, cz)
    batch.add(x, y, az)
    batch.scale(x, c, sz)
    batch.decompress(x, D)
    batch.plan().run()
    ties = compare_compressed(cz.to_host(), (o.f, o.s, o.phi, o.codes), code_x, phi_x, f"batch compress {m}")
    assert ties <= _boundary_values(code_x, phi_x), ties
    s = oracle.add(o, ob)
    assert_same_compressed(az.to_host(), (s.f, s.s, s.phi, s.codes), f"batch add {m}")
    k = oracle.scale(o, c)
    assert_same_compressed(sz.to_host(), (k.f, k.s, k.phi, k.codes), f"batch scale {m} by {c}")
    assert_blocks_close(D.cpu().numpy(), oracle.decompress(o), what=f"batch decompress {m}")

    p = torch.empty((o.nblk, 64), dtype=torch.uint8, device="cuda")
    g = blaz.compress_predicted(dA, psi=p)
    w, (wpsi, wx, wphi) = oracle.compress(A, with_debug=True, predicted=True)
    np.testing.assert_array_equal(p.cpu().numpy(), wpsi)
    ties = compare_compressed(g.to_host(), (w.f, w.s, w.phi, w.codes), wx, wphi, f"predicted {m}")
    assert ties <= _boundary_values(wx, wphi), ties


@pytest.mark.gpu
@GPU
@given(matrices, st.integers(1, 3), st.sampled_from(["fp64", "fp32", "bf16x3"]))
def test_gpu_product_forms_agree(m, bn, prec):
    """The product's other forms on the same structures, bit for bit: the
    compressed-output product is the compression of the dense product, and
    (binary64) a grouped launch and the allocation-free call equal the
    standalone product."""
    import torch
    import paper_2202_13007_amd as blaz
    A = make_matrix(*m)
    B = make_matrix(m[0], m[1] ^ 0x1D1D, m[3], bn)
    x, y = blaz.compress(torch.from_numpy(A).cuda()), blaz.compress(torch.from_numpy(B).cuda())
    Bd = torch.from_numpy(B).cuda()
    for b in (y, Bd):
        dense = blaz.matmul(x, b, prec=prec)
        got = blaz.matmul_compressed(x, b, prec=prec)
        assert_same_compressed(got.to_host(), blaz.compress(dense).to_host(), f"matmul_compressed {prec} {m}")
        if prec == "fp64":
            st_out = torch.empty_like(dense)
            blaz.matmul_static(x, b, out=st_out)
            assert torch.equal(st_out, dense), f"matmul_static {m}"
    if prec == "fp64":
        outs = [torch.empty((A.shape[0], B.shape[1]), dtype=torch.float64, device="cuda") for _ in range(2)]
        grp = blaz.MatmulGroup()
        grp.add(x, y, outs[0])
        grp.add(x, Bd, outs[1])
        grp.plan().run()
        assert torch.equal(outs[0], blaz.matmul(x, y)), f"group, compressed B {m}"
        assert torch.equal(outs[1], blaz.matmul(x, Bd)), f"group, dense B {m}"
