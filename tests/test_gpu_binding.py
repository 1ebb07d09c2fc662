"""The Python binding refuses, before anything is enqueued, tensors the C ABI
cannot check itself: the library sees only pointers and the shapes in the
descriptors, so a short output, a dense operand of the wrong shape or a host
tensor would otherwise become an out-of-bounds device access."""
import pytest
import torch

import paper_2202_13007_amd as blaz

pytestmark = pytest.mark.gpu


def f64(*shape):
    return torch.zeros(shape, dtype=torch.float64, device="cuda")


def idx(n):
    return torch.zeros(n, dtype=torch.int64, device="cuda")


@pytest.fixture(scope="module")
def x():
    return blaz.compress(f64(16, 24))


def test_decompress_and_compress_shapes(x):
    with pytest.raises(ValueError):
        blaz.decompress(x, out=f64(16, 16))
    with pytest.raises(ValueError):
        blaz.decompress(x, out=f64(16, 24).t())  # not unit column stride
    with pytest.raises(ValueError):
        blaz.compress(f64(16, 16), out=blaz.BlazMatrix.empty(16, 24))
    with pytest.raises(ValueError):
        blaz.compress(f64(16, 24), psi=torch.empty((5, 64), dtype=torch.uint8, device="cuda"))


def test_short_descriptor_arrays(x):
    bad = blaz.BlazMatrix(16, 24, x.f, x.s, x.phi, x.codes[:5])
    with pytest.raises(ValueError):
        blaz.scale(bad, 2.0)
    bad = blaz.BlazMatrix(16, 24, x.f, x.s, x.phi.to(torch.int8), x.codes)
    with pytest.raises(ValueError):
        blaz.decompress(bad)


def test_dot_arguments(x):
    y = blaz.compress(f64(24, 8))
    with pytest.raises(ValueError):
        blaz.dot(x, idx(4), y, idx(4), out=f64(3))                    # short out
    with pytest.raises(ValueError):
        blaz.dot(x, idx(4).cpu(), y, idx(4))                          # host indices
    with pytest.raises(ValueError):
        blaz.dot(x, idx(4), y, idx(3))
    with pytest.raises(ValueError):
        blaz.dot_dense(x, idx(4), f64(4, 16))                         # vectors narrower than x
    with pytest.raises(ValueError):
        blaz.dot_dense(x, idx(4), f64(23))
    with pytest.raises(ValueError):
        blaz.dot_dense(x, idx(4), f64(3, 24))
    with pytest.raises(ValueError):
        blaz.diagnose(x, torch.zeros(4, dtype=torch.int64))


def test_matmul_arguments(x):
    with pytest.raises(ValueError):
        blaz.matmul(x, f64(16, 8))                                    # B rows != A cols
    with pytest.raises(ValueError):
        blaz.matmul(x, f64(24, 8), out=f64(8, 8))
    with pytest.raises(ValueError):
        blaz.matmul(x, f64(24, 8), workspace=torch.empty(10 ** 6, dtype=torch.float32, device="cuda"))
    with pytest.raises(ValueError):
        blaz.matmul_compressed(x, f64(8, 8))


def test_batch_arguments(x):
    y = blaz.compress(f64(24, 8))
    with pytest.raises(ValueError):
        blaz.Batch().dot(x, idx(4), y, idx(4), f64(2))
    with pytest.raises(ValueError):
        blaz.Batch().dot_dense(x, idx(4), f64(4, 8), f64(4))
    with pytest.raises(ValueError):
        blaz.Batch().compress(f64(16, 16), blaz.BlazMatrix.empty(16, 24))
    with pytest.raises(ValueError):
        blaz.Batch().decompress(x, f64(8, 24))


def test_valid_calls_still_run(x):
    y = blaz.compress(f64(24, 8))
    out = blaz.dot(x, idx(4), y, idx(4))
    C = blaz.matmul(x, y)
    torch.cuda.synchronize()
    assert out.shape == (4,) and C.shape == (16, 8)
