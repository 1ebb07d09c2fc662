"""GPU parity of the tunable rate (L kept lines of DCT coefficients) against
the oracle, under the rules of the paper's scheme: f, s, phi and codes
bit-exact except classified rounding-boundary ties, pad bytes zero;
decompression within 1e-12 of each block's magnitude; add, sub and scale
bit-exact; products within 1e-12 * sum |x y|."""
import numpy as np
import pytest
import torch

import oracle
import paper_2202_13007_amd as blaz
from oracle.parity import TIE_RATE_MAX, assert_blocks_close, assert_dots_close, assert_same_compressed, compare_compressed
from synth import smooth_field, workload_inputs

pytestmark = pytest.mark.gpu


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def upload(c: oracle.Compressed):
    return blaz.BlazMatrix.from_host(c.rows, c.cols, c.f, c.s, c.phi, c.codes, lines=c.lines)


def host(m):
    return m.to_host()


@pytest.mark.parametrize("lines", [1, 3, 4, 8])
@pytest.mark.parametrize("shape", [(64, 64), (264, 520), (1032, 528)])
def test_compress_lines(lines, shape):
    r, c = shape
    A = smooth_field(r, 6, 3.0, 1e-3, 500 + lines, cols=c)
    got = blaz.compress(dev(A), lines=lines)
    torch.cuda.synchronize()
    assert got.lines == lines and got.codes.shape == (got.nblk, oracle.code_stride(lines))
    want, (cx, px) = oracle.compress_lines(A, lines, with_debug=True)
    ties = compare_compressed(host(got), (want.f, want.s, want.phi, want.codes), cx, px, f"compress L={lines}")
    assert ties <= TIE_RATE_MAX * cx.size + 2


def test_compress_lines_workload_64_and_unaligned_input():
    A, _ = workload_inputs("plain-64")
    big = np.zeros((64, 66))
    big[:, 1:65] = A
    t = dev(big)[:, 1:65]  # 8-byte aligned only: the per-lane load path
    for lines in (1, 3, 5, 6, 7):
        got = blaz.compress(t, lines=lines)
        want, (cx, px) = oracle.compress_lines(A, lines, with_debug=True)
        compare_compressed(host(got), (want.f, want.s, want.phi, want.codes), cx, px, f"compress L={lines}")


@pytest.mark.parametrize("lines", [1, 3, 4, 5, 8])
def test_decompress_lines(lines):
    A = smooth_field(264, 6, 3.0, 1e-3, 510, cols=520)
    o = oracle.compress_lines(A, lines)
    got = blaz.decompress(upload(o)).cpu().numpy()
    assert_blocks_close(got, oracle.decompress(o), what=f"decompress L={lines}")


@pytest.mark.parametrize("lines", [1, 3, 8])
def test_add_sub_scale_lines_bit_exact(lines):
    A = smooth_field(136, 6, 3.0, 1e-3, 520, cols=264)
    B = smooth_field(136, 6, 3.0, 1e-3, 521, cols=264) * -0.7
    x, y = oracle.compress_lines(A, lines), oracle.compress_lines(B, lines)
    gx, gy = upload(x), upload(y)

    def tup(c):
        return (c.f, c.s, c.phi, c.codes)
    assert_same_compressed(host(blaz.add(gx, gy)), tup(oracle.add(x, y)), f"add L={lines}")
    assert_same_compressed(host(blaz.sub(gx, gy)), tup(oracle.add(x, oracle.scale(y, -1.0))), f"sub L={lines}")
    assert_same_compressed(host(blaz.scale(gx, -1.7)), tup(oracle.scale(x, -1.7)), f"scale L={lines}")
    gz = upload(x)
    blaz.scale(gz, 2.5, out=gz)  # in place
    assert_same_compressed(host(gz), tup(oracle.scale(x, 2.5)), f"scale in place L={lines}")


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_matmul_lines(prec):
    X = smooth_field(136, 4, 2.0, 1e-3, 530, cols=200)
    Y = smooth_field(200, 4, 2.0, 1e-3, 531, cols=72)
    ox, oy = oracle.compress_lines(X, 3), oracle.compress_lines(Y, 5)
    Xd, Yd = oracle.decompress(ox), oracle.decompress(oy)
    got = blaz.matmul(upload(ox), upload(oy), prec=prec).cpu().numpy()
    mag = np.abs(Xd) @ np.abs(Yd)
    if prec == "fp64":
        assert_dots_close(got, oracle.gemm(Xd, Yd), mag, what="matmul L=3 x L=5")
    else:
        assert np.all(np.abs(got - oracle.gemm(Xd, Yd)) <= (2 + 200 / 4 + 4) * 2.0 ** -24 * mag)


def test_matmul_compressed_output_at_another_rate():
    X = smooth_field(128, 4, 2.0, 1e-3, 532)
    gx = blaz.compress(dev(X))
    out = blaz.BlazMatrix.empty(128, 128, lines=4)
    got = blaz.matmul_compressed(gx, gx, out=out)
    want = blaz.compress(blaz.matmul(gx, gx), lines=4)
    assert_same_compressed(host(got), host(want), "compressed product, L = 4")


def test_dot_and_batch_refuse_other_rates():
    gx = blaz.compress(dev(smooth_field(16, 2, 1.0, 0.0, 533)), lines=3)
    idx = torch.zeros(1, dtype=torch.int64, device="cuda")
    with pytest.raises(blaz.BlazError) as e:
        blaz.dot(gx, idx, gx, idx)
    assert e.value.status == -6
    with pytest.raises(blaz.BlazError):
        blaz.Batch().scale(gx, 2.0, blaz.BlazMatrix.empty(16, 16, lines=3)).plan()


def strip_of_blocks(A, blocks):
    """The listed 8x8 blocks of A side by side in one 8-row strip (blocks are
    compressed independently, so the strip's records are theirs)."""
    nbc = A.shape[1] // 8
    return np.hstack([A[8 * (b // nbc):8 * (b // nbc) + 8, 8 * (b % nbc):8 * (b % nbc) + 8] for b in blocks])


@pytest.mark.parametrize("lines", [1, 3, 8])
def test_compress_lines_full_size_8192_sampled(lines):
    """The 8192^2 field at other rates: every block on the GPU, 1500 sampled
    blocks on the oracle."""
    A, _ = workload_inputs("plain-8192")
    g = blaz.compress(dev(A), lines=lines)
    gf, gs, gphi, gcodes = host(g)
    rng = np.random.default_rng(lines)
    sample = np.unique(np.concatenate([[0, 1023, 1024, len(gf) - 1], rng.integers(0, len(gf), 1500)]))
    want, (cx, px) = oracle.compress_lines(strip_of_blocks(A, sample), lines, with_debug=True)
    ties = compare_compressed((gf[sample], gs[sample], gphi[sample], gcodes[sample]),
                              (want.f, want.s, want.phi, want.codes), cx, px, f"8192 L={lines} sampled")
    assert ties <= 2


@pytest.mark.parametrize("seed", range(12))
def test_random_shapes_and_rates_sweep(seed):
    """Seeded sweep: random ragged shapes (multiples of 8 up to 520), random
    kept lines, random field parameters; compress against the oracle, the
    oracle's records decompressed within the tolerance, add bit-exact."""
    rng = np.random.default_rng(900 + seed)
    r, c = 8 * int(rng.integers(1, 66)), 8 * int(rng.integers(1, 66))
    lines = int(rng.integers(1, 9))
    A = smooth_field(r, int(rng.integers(1, 8)), float(rng.uniform(0.5, 6.0)), float(10 ** rng.uniform(-6, -1)),
                     1000 + seed, cols=c) * float(10 ** rng.uniform(-3, 3))
    got = blaz.compress(dev(A), lines=lines)
    want, (cx, px) = oracle.compress_lines(A, lines, with_debug=True)
    compare_compressed(host(got), (want.f, want.s, want.phi, want.codes), cx, px, f"sweep {r}x{c} L={lines}")
    back = blaz.decompress(upload(want)).cpu().numpy()
    assert_blocks_close(back, oracle.decompress(want), what=f"sweep decompress {r}x{c} L={lines}")
    B = oracle.compress_lines(smooth_field(r, 3, 2.0, 1e-3, 2000 + seed, cols=c), lines)
    assert_same_compressed(host(blaz.add(upload(want), upload(B))),
                           (lambda z: (z.f, z.s, z.phi, z.codes))(oracle.add(want, B)), f"sweep add L={lines}")
