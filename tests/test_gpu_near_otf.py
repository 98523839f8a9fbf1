"""The near field computed in the product (near_mode = 1, the compute-on-the-fly policy of
Section 4): nothing stored, each near entry G(x_i, y_j) w_j evaluated again per product from
source tiles staged in LDS.  Checked against the oracle's dense product (an operator with every
block near equals the dense operator), against the stored near field (same entries, summation
order apart), in FP64 and FP32, for leaves of up to 64 and of more than 64 rows, between
different point sets, in HIP graph replays and in the several-vector product, and at the
245 760-point sphere on sampled rows."""
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


def sphere(level):
    v, f = I.icosphere(level)
    P, W = oracle.quad_points(v, f, *RULE)
    return v, f, torch.from_numpy(v).cuda(), torch.from_numpy(f).cuda(), P, W


def apply(op, x):
    y = op.matvec(torch.from_numpy(x).to(op.cdtype).cuda())
    torch.cuda.synchronize()
    return y.cpu().numpy().astype(np.complex128)


@pytest.mark.parametrize("leaf", [64, 200])
def test_all_near_equals_dense_oracle(H, leaf):
    # eta so small that no pair is admissible: every block is near, the product is the dense one
    v, f, vd, fd, P, W = sphere(3)
    op = H.build(vd, fd, *RULE, kern=H.HELMHOLTZ, k=5.0,
                 prm=H.params(tol=1e-3, eta=1e-9, leaf_size=leaf, near_mode=1))
    assert op.info["n_far"] == 0 and op.info["n_near"] > 0
    x = I.complex_vector(P.shape[0], 3)
    yr = oracle.dense_matvec(P, W, oracle.HELMHOLTZ, 5.0, x)
    assert rel(apply(op, x), yr) <= 1e-12
    op.close()


@pytest.mark.parametrize("precision,leaf", [(0, 64), (1, 64), (0, 128), (1, 128), (0, 200)])
def test_matches_stored_near_field(H, precision, leaf):
    v, f, vd, fd, P, W = sphere(4)
    kw = dict(tol=1e-6, leaf_size=leaf, precision=precision)
    st = H.build(vd, fd, *RULE, kern=H.HELMHOLTZ, k=15.0, prm=H.params(**kw))
    ot = H.build(vd, fd, *RULE, kern=H.HELMHOLTZ, k=15.0, prm=H.params(near_mode=1, **kw))
    assert ot.info["near_entries"] == st.info["near_entries"] > 0 and ot.info["n_far"] > 0
    # the build evaluates the near entries only when it stores them
    assert st.info["kernel_evals"] - ot.info["kernel_evals"] == st.info["near_entries"]
    es = 16 if precision == 0 else 8
    # no near-field storage: the operator is smaller by the near entries (the slot pools, whose
    # trimmed size depends on how the blocks fell to workgroups, are left out of the comparison)
    held = lambda op: op.info["bytes"] - op.info["factor_bytes"]
    assert held(st) - held(ot) >= 0.99 * es * st.info["near_entries"]
    x = I.complex_vector(P.shape[0], 4)
    ys, yo = apply(st, x), apply(ot, x)
    # the same factors (the build does not depend on the near mode) and the same near entries
    assert rel(yo, ys) <= (1e-13 if precision == 0 else 2e-6)
    yr = oracle.dense_matvec(P, W, oracle.HELMHOLTZ, 15.0, x)
    assert rel(yo, yr) <= (1e-5 if precision == 0 else 1e-4)
    st.close()
    ot.close()


def test_rect_graph_and_several_vectors(H):
    v, f, vd, fd, P, W = sphere(3)
    xyzw = H.quad_points(vd, fd, *RULE)
    T = np.random.default_rng(5).uniform(-1.5, 1.5, (2500, 3))
    Td = torch.from_numpy(np.ascontiguousarray(T.T)).cuda()
    kw = dict(tol=1e-6)
    st = H.build_rect(Td, xyzw, kern=H.HELMHOLTZ, k=6.0, prm=H.params(**kw))
    ot = H.build_rect(Td, xyzw, kern=H.HELMHOLTZ, k=6.0, prm=H.params(near_mode=1, **kw))
    x = I.complex_vector(P.shape[0], 5)
    assert st.info["n_near"] > 0
    assert rel(apply(ot, x), apply(st, x)) <= 1e-13
    # graph replays of the on-the-fly product equal its eager product
    op = H.build(vd, fd, *RULE, kern=H.HELMHOLTZ, k=6.0, prm=H.params(near_mode=1, **kw))
    xd = torch.from_numpy(x).cuda()
    y = op.matvec(xd)
    yg = torch.zeros_like(y)
    g = op.graph(xd, yg)
    for rep in range(5):
        yg.fill_(float("nan"))
        g.launch(1)
        torch.cuda.synchronize()
        assert torch.equal(yg, y), rep
    g.close()
    # several vectors: one product per vector, each equal to matvec's
    X = torch.from_numpy(np.stack([I.complex_vector(P.shape[0], 10 + r) for r in range(3)])).cuda()
    Y = op.matvec_multi(X)
    torch.cuda.synchronize()
    for r in range(3):
        assert torch.equal(Y[r], op.matvec(X[r].contiguous()))
    for o in (st, ot, op):
        o.close()


@pytest.mark.parametrize("precision", [0, 1])
def test_full_size_sampled_rows(H, precision):
    # the bench's sphere workload in both precisions, as it is timed
    v, f, vd, fd, P, W = sphere(6)
    op = H.build(vd, fd, *RULE, kern=H.HELMHOLTZ, k=40.0,
                 prm=H.params(near_mode=1, precision=precision))
    assert op.info["bytes"] < op.info["factor_bytes"] * 1.2
    x = I.complex_vector(P.shape[0], 0)
    y = apply(op, x)
    rows = np.sort(np.random.default_rng(123).choice(P.shape[0], 256, replace=False))
    yr = oracle.dense_rows(P, W, oracle.HELMHOLTZ, 40.0, x, rows)
    assert rel(y[rows], yr) <= 1e-3
    op.close()


def test_correction_needs_stored_blocks(H):
    v, f, vd, fd, P, W = sphere(2)
    with pytest.raises(H.HmxError) as e:
        H.build(vd, fd, *RULE, kern=H.HELMHOLTZ, k=3.0, prm=H.params(regularize=1, near_mode=1))
    assert e.value.code == H.EUNSUPPORTED
    with pytest.raises(H.HmxError) as e:
        H.build(vd, fd, *RULE, kern=H.HELMHOLTZ, k=3.0, prm=H.params(near_mode=2))
    assert e.value.code == H.EINVAL


@pytest.mark.parametrize("precision", [0, 1])
def test_batch_matches_stored_near_field(H, precision):
    # a batch of meshes with their own wavenumbers: each leaf takes its mesh's k
    descs = I.batch_ellipsoids(5, seed=7, t_min=300, t_max=2500)
    meshes = []
    for d in descs:
        v, f = I.batch_mesh(d)
        meshes.append((torch.from_numpy(v).cuda(), torch.from_numpy(f).cuda(), d["k"]))
    kw = dict(tol=1e-4, precision=precision)
    st = H.build_batch(meshes, *RULE, kern=H.HELMHOLTZ, prm=H.params(**kw))
    ot = H.build_batch(meshes, *RULE, kern=H.HELMHOLTZ, prm=H.params(near_mode=1, **kw))
    assert ot.info["near_entries"] == st.info["near_entries"] > 0
    M = int(st.mesh_offsets()[-1])
    x = I.complex_vector(M, 11)
    ys, yo = apply(st, x), apply(ot, x)
    assert rel(yo, ys) <= (1e-13 if precision == 0 else 2e-6)
    st.close()
    ot.close()
