"""GPU parity of operators between different point sets (Section 5.1: the potential of a source
quadrature at a collection of other points) through the C ABI against the CPU oracle.

Bars: dense product to 1e-12 (FP64); H-matrix product within the ACA tolerance, on all rows at
small sizes and on sampled rows for 245 760 sources radiating onto a 256 x 256 grid; the block
partition covers the target x source rectangle exactly once with admissible far blocks; the
exterior sphere potential equals the oracle's quadrature sum; graph replays equal the eager
product bit for bit.
"""
import numpy as np
import pytest

import oracle
from paper_1804_00995_amd import inputs as I

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")

RULE = I.rule_3pt()


@pytest.fixture(scope="module")
def H():
    oracle.build(force=False)
    from paper_1804_00995_amd import hmx
    return hmx


def rel(a, b):
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


def sources(level):
    v, f = I.icosphere(level)
    P, W = oracle.quad_points(v, f, *RULE)
    xyzw = torch.from_numpy(np.vstack([P.T, W[None, :]]).copy()).cuda()
    return P, W, xyzw


def mixed_targets(n, P, seed=1):
    """Targets inside, near and outside the unit sphere, plus a few on source points."""
    rng = np.random.default_rng(seed)
    T = rng.uniform(-2.0, 2.0, (n, 3))
    T[:8] = P[rng.choice(P.shape[0], 8, replace=False)]
    return T


def grid_targets(nside, z=0.25, half=2.5):
    g = np.linspace(-half, half, nside)
    gx, gy = np.meshgrid(g, g, indexing="ij")
    return np.stack([gx.ravel(), gy.ravel(), np.full(gx.size, z)], 1)


def dev_targets(T):
    return torch.from_numpy(np.ascontiguousarray(T.T)).cuda()


def apply(op, x, dtype=torch.complex128):
    y = op.matvec(torch.from_numpy(x).to(dtype).cuda())
    torch.cuda.synchronize()
    return y.cpu().numpy().astype(np.complex128)


@pytest.mark.parametrize("kern,k", [(0, 0.0), (1, 7.0)])
def test_dense_equals_oracle(H, kern, k):
    P, W, xyzw = sources(3)
    T = mixed_targets(1500, P)
    op = H.build_rect(dev_targets(T), xyzw, kern=kern, k=k, prm=H.params(tol=0.0))
    assert op.rows == T.shape[0] and op.cols == P.shape[0] and op.info["is_dense"] == 1
    x = I.complex_vector(P.shape[0], 2)
    assert rel(apply(op, x), oracle.rect_matvec(T, P, W, kern, k, x)) <= 1e-12


@pytest.mark.parametrize("tol,bound", [(1e-3, 1e-3), (1e-6, 1e-5)])
def test_hmatrix_within_tolerance(H, tol, bound):
    P, W, xyzw = sources(4)
    T = np.vstack([mixed_targets(6000, P, seed=3), grid_targets(64)])
    op = H.build_rect(dev_targets(T), xyzw, kern=1, k=15.0, prm=H.params(tol=tol))
    assert op.info["n_far"] > 0 and op.info["n_near"] > 0
    x = I.complex_vector(P.shape[0], 5)
    assert rel(apply(op, x), oracle.rect_matvec(T, P, W, 1, 15.0, x)) <= bound


def test_block_partition_covers_rectangle(H):
    P, W, xyzw = sources(3)
    T = mixed_targets(2000, P, seed=4)
    Mt, Ms = T.shape[0], P.shape[0]
    op = H.build_rect(dev_targets(T), xyzw, kern=1, k=5.0)
    tree = op.export_tree()
    perm = tree["perm"]
    # targets keep the cluster positions [0, Mt), sources [Mt, Mt + Ms)
    assert np.array_equal(np.sort(perm[:Mt]), np.arange(Mt))
    assert np.array_equal(np.sort(perm[Mt:]), np.arange(Mt, Mt + Ms))
    nearR, farR, _ = op.export_blocks()
    cover = np.zeros((Mt, Ms), np.int32)
    for tb, te, sb, se in np.vstack([nearR, farR]):
        assert 0 <= tb < te <= Mt and Mt <= sb < se <= Mt + Ms
        cover[tb:te, sb - Mt:se - Mt] += 1
    assert (cover == 1).all()
    # far blocks are admissible: min(diam)^2 <= eta^2 dist^2 with the exported node boxes
    node_of = {(int(b), int(e)): i for i, (b, e) in enumerate(zip(tree["begin"], tree["end"]))}
    box = tree["box"]
    for tb, te, sb, se in farR:
        bt, bs = box[node_of[(tb, te)]], box[node_of[(sb, se)]]
        dt = ((bt[3:] - bt[:3]) ** 2).sum()
        ds = ((bs[3:] - bs[:3]) ** 2).sum()
        gap = np.maximum(0.0, np.maximum(bt[:3] - bs[3:], bs[:3] - bt[3:]))
        assert min(dt, ds) <= 1.5 ** 2 * (gap ** 2).sum() * (1 + 1e-12)


@pytest.mark.parametrize("kern,k", [(0, 0.0), (1, 5.0)])
def test_exterior_sphere_potential(H, kern, k):
    P, W, xyzw = sources(4)
    rng = np.random.default_rng(6)
    d = rng.standard_normal((500, 3))
    d /= np.linalg.norm(d, axis=1)[:, None]
    r = rng.uniform(1.3, 3.0, 500)
    T = d * r[:, None]
    op = H.build_rect(dev_targets(T), xyzw, kern=kern, k=k, prm=H.params(tol=1e-7))
    y = apply(op, np.ones(P.shape[0], np.complex128))
    ref = oracle.rect_matvec(T, P, W, kern, k, np.ones(P.shape[0], np.complex128))
    assert np.abs(y - ref).max() <= 1e-6 * np.abs(ref).max()
    exact = 1.0 / r if k == 0 else np.sin(k) / k * np.exp(1j * k * r) / r
    assert np.abs(y - exact).max() <= 2e-3 * np.abs(exact).max()


def test_fp32_mixed(H):
    P, W, xyzw = sources(4)
    T = grid_targets(80)
    op = H.build_rect(dev_targets(T), xyzw, kern=1, k=15.0, prm=H.params(precision=H.FP32_MIXED))
    x = I.complex_vector(P.shape[0], 7)
    assert rel(apply(op, x, torch.complex64), oracle.rect_matvec(T, P, W, 1, 15.0, x)) <= 1e-3


def test_graph_replays_equal_eager(H):
    P, W, xyzw = sources(3)
    T = mixed_targets(3000, P, seed=9)
    op = H.build_rect(dev_targets(T), xyzw, kern=1, k=9.0)
    x = torch.from_numpy(I.complex_vector(P.shape[0], 8)).cuda()
    ref = op.matvec(x)
    y = torch.zeros(T.shape[0], dtype=torch.complex128, device="cuda")
    g = op.graph(x, y)
    for _ in range(3):
        y.zero_()
        torch.cuda.synchronize()
        g.launch(2)
        torch.cuda.synchronize()
        assert torch.equal(y, ref)
    g.close()


def test_radiation_grid_sampled_rows(H):
    """245 760 sources (L6 sphere, k = 40) radiating onto a 256 x 256 grid crossing the sphere."""
    P, W, xyzw = sources(6)
    T = grid_targets(256, z=0.2, half=2.0)
    op = H.build_rect(dev_targets(T), xyzw, kern=1, k=40.0)
    x = I.complex_vector(P.shape[0], 0)
    y = apply(op, x)
    rows = np.sort(np.random.default_rng(11).choice(T.shape[0], 256, replace=False))
    assert rel(y[rows], oracle.rect_matvec(T, P, W, 1, 40.0, x, rows=rows)) <= 1e-3
