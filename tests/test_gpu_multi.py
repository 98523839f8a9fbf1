"""The several-vector product hmx_matvec_multi through the C ABI: every vector's result is
bit-identical to the one-vector product's (the kernels keep its summation order), for FP64 and
FP32 H-matrices, leaves of 64, 128 and 200 points (the leaf kernel's one-, two- and four-chunk
instances), an operator between different point sets and a dense operator, with 1 to 7 vectors
(groups of 4, 2, 1)."""
import numpy as np
import pytest

from paper_1804_00995_amd import inputs as I

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")

RULE = I.rule_3pt()


@pytest.fixture(scope="module")
def H():
    from paper_1804_00995_amd import hmx
    return hmx


def vectors(nr, n, seed, dtype):
    return torch.from_numpy(np.stack([I.complex_vector(n, seed + r) for r in range(nr)])).to(dtype).cuda()


def check(op, nr, seed):
    X = vectors(nr, op.cols, seed, op.cdtype)
    Y = op.matvec_multi(X)
    torch.cuda.synchronize()
    assert Y.shape == (nr, op.rows)
    for r in range(nr):
        assert torch.equal(Y[r], op.matvec(X[r].contiguous())), (nr, r)


@pytest.mark.parametrize("precision,leaf", [(0, 64), (1, 64), (0, 128), (1, 128), (0, 200)])
def test_hmatrix_bit_identical(H, precision, leaf):
    v, f = I.icosphere(4)
    op = H.build(torch.from_numpy(v).cuda(), torch.from_numpy(f).cuda(), *RULE, kern=H.HELMHOLTZ,
                 k=15.0, prm=H.params(tol=1e-6, leaf_size=leaf, precision=precision))
    assert op.info["n_far"] > 0
    for nr in (1, 2, 3, 4, 5, 7):
        check(op, nr, 10 * nr)


def test_rect_and_dense_bit_identical(H):
    v, f = I.icosphere(3)
    xyzw = H.quad_points(torch.from_numpy(v).cuda(), torch.from_numpy(f).cuda(), *RULE)
    T = np.random.default_rng(2).uniform(-2.0, 2.0, (3000, 3))
    rect = H.build_rect(torch.from_numpy(np.ascontiguousarray(T.T)).cuda(), xyzw, kern=H.HELMHOLTZ,
                        k=7.0, prm=H.params(tol=1e-6))
    assert rect.rows != rect.cols and rect.info["n_far"] > 0
    check(rect, 6, 1)
    dense = H.build_points(xyzw, kern=H.HELMHOLTZ, k=7.0, prm=H.params(tol=0.0))
    check(dense, 3, 2)


def test_shape_errors(H):
    v, f = I.icosphere(2)
    op = H.build(torch.from_numpy(v).cuda(), torch.from_numpy(f).cuda(), *RULE, k=3.0)
    with pytest.raises(ValueError):
        op.matvec_multi(torch.zeros((2, op.cols + 1), dtype=torch.complex128, device="cuda"))
    with pytest.raises(TypeError):
        op.matvec_multi(torch.zeros((2, op.cols), dtype=torch.complex64, device="cuda"))
