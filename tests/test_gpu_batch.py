"""GPU tests of batched operators (independent meshes built and applied together) and of the
product captured in a HIP graph.

A batch operator is block-diagonal over its meshes, so each mesh's slice of the product must be
that mesh's own operator applied to its own slice: the tests compare slices with the CPU
oracle's dense product (within the ACA tolerance) and with single-mesh builds on the GPU (bit for
bit: the same tree, blocks, pivots and summation order)."""
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


def small_batch(n=6, seed=5):
    """A seeded batch of small ellipsoids (the large-batch recipe at 200..3000 triangles)."""
    return I.batch_ellipsoids(n, seed=seed, t_min=200, t_max=3000)


def device_meshes(descs):
    out = []
    for d in descs:
        v, f = I.batch_mesh(d)
        out.append((v, f, torch.from_numpy(v).cuda(), torch.from_numpy(f).cuda(), d["k"]))
    return out


def batch_vector(descs, meshes):
    return np.concatenate([I.complex_vector(3 * f.shape[0], d["seed"])
                           for d, (_, f, _, _, _) in zip(descs, meshes)])


@pytest.mark.parametrize("precision", [0, 1])
def test_batch_slices_match_single_builds_and_oracle(H, precision):
    descs = small_batch()
    ms = device_meshes(descs)
    prm = H.params(tol=1e-3, precision=precision)
    op = H.build_batch([(vd, fd, k) for _, _, vd, fd, k in ms], *RULE, kern=1, prm=prm)
    off = op.mesh_offsets()
    assert off[0] == 0 and np.array_equal(np.diff(off), [3 * f.shape[0] for _, f, _, _, _ in ms])
    cdt = torch.complex128 if precision == 0 else torch.complex64
    x = batch_vector(descs, ms)
    y = op.matvec(torch.from_numpy(x).to(cdt).cuda())
    ys = op.split(y)
    total_far = 0
    for i, (v, f, vd, fd, k) in enumerate(ms):
        single = H.build(vd, fd, *RULE, kern=1, k=k, prm=prm)
        xi = torch.from_numpy(x[off[i]:off[i + 1]]).to(cdt).cuda()
        yi = single.matvec(xi)
        torch.cuda.synchronize()
        assert torch.equal(ys[i], yi), f"mesh {i}"
        P, W = oracle.quad_points(v, f, *RULE)
        yr = oracle.dense_matvec(P, W, 1, k, x[off[i]:off[i + 1]])
        assert rel(ys[i].cpu().numpy().astype(np.complex128), yr) <= 1e-3, f"mesh {i}"
        total_far += single.info["n_far"]
        single.close()
    assert op.info["n_far"] == total_far


def test_batch_tree_stays_inside_meshes(H):
    descs = small_batch(5, seed=9)
    ms = device_meshes(descs)
    op = H.build_batch([(vd, fd, k) for _, _, vd, fd, k in ms], *RULE, kern=1)
    off = op.mesh_offsets()
    T = op.export_tree()
    mesh_of = np.searchsorted(off, np.arange(off[-1]), side="right") - 1
    # the permutation keeps every point inside its mesh's range
    assert np.array_equal(mesh_of[T["perm"]], mesh_of)
    # every node lies inside one mesh, and level 0 holds exactly one root per mesh
    assert np.all(mesh_of[T["begin"]] == mesh_of[T["end"] - 1])
    roots = T["level"] == 0
    assert np.array_equal(T["begin"][roots], off[:-1]) and np.array_equal(T["end"][roots], off[1:])
    nearR, farR, _ = op.export_blocks()
    for R in (nearR, farR):
        assert np.all(mesh_of[R[:, 0]] == mesh_of[R[:, 2]])
    # block areas cover each mesh's square exactly once
    area = np.zeros(len(off) - 1)
    for R in (nearR, farR):
        np.add.at(area, mesh_of[R[:, 0]], (R[:, 1] - R[:, 0]) * (R[:, 3] - R[:, 2]))
    assert np.array_equal(area, np.diff(off).astype(float) ** 2)


def test_batch_64_meshes_sampled_rows(H):
    """The 64-ellipsoid batch (triangles logU[2000, 40000], k U[2, 30], seed 0), built and
    applied as one operator; 24 seeded rows per mesh against the oracle's dense rows."""
    descs = I.batch_ellipsoids(64, seed=0)
    meshes, dev = [], []
    for d in descs:
        v, f = I.batch_mesh(d)
        meshes.append((v, f))
        dev.append((torch.from_numpy(v).cuda(), torch.from_numpy(f).cuda(), d["k"]))
    op = H.build_batch(dev, *RULE, kern=1, prm=H.params(tol=1e-3))
    off = op.mesh_offsets()
    x = np.concatenate([I.complex_vector(3 * f.shape[0], d["seed"]) for d, (_, f) in zip(descs, meshes)])
    y = op.matvec(torch.from_numpy(x).cuda())
    torch.cuda.synchronize()
    y = y.cpu().numpy()
    rng = np.random.default_rng(77)
    worst = 0.0
    for i, ((v, f), d) in enumerate(zip(meshes, descs)):
        P, W = oracle.quad_points(v, f, *RULE)
        rows = np.sort(rng.choice(P.shape[0], 24, replace=False))
        yr = oracle.dense_rows(P, W, 1, d["k"], x[off[i]:off[i + 1]], rows)
        e = rel(y[off[i] + rows], yr)
        worst = max(worst, e)
    print(f"64 meshes, {off[-1]} points: worst per-mesh sampled error {worst:.3e}, "
          f"build {op.info['t_total_ms']:.1f} ms")
    assert worst <= 1e-3


@pytest.mark.parametrize("batch", [False, True])
def test_graph_replays_equal_eager(H, batch):
    """A captured product replayed several times, with other device work and synchronisations
    between replays, equals the eager product each time (bit for bit)."""
    if batch:
        ms = device_meshes(small_batch(4, seed=2))
        op = H.build_batch([(vd, fd, k) for _, _, vd, fd, k in ms], *RULE, kern=1)
    else:
        v, f = I.icosphere(4)
        op = H.build(torch.from_numpy(v).cuda(), torch.from_numpy(f).cuda(), *RULE, kern=1, k=12.0)
    x = torch.from_numpy(I.complex_vector(op.M, 11)).cuda()
    ref = op.matvec(x)
    torch.cuda.synchronize()
    y = torch.zeros_like(x)
    g = op.graph(x, y)
    for rep in range(4):
        y.fill_(float("nan"))
        junk = torch.randn(1 << 20, device="cuda").sum()  # eager work between replays
        torch.cuda.synchronize()
        g.launch(1 + rep % 2)
        torch.cuda.synchronize()
        assert torch.equal(y, ref), f"replay {rep}"
        assert torch.isfinite(junk)
    g.close()


def test_dense_graph_replays_equal_eager(H):
    v, f = I.icosphere(2)
    op = H.build(torch.from_numpy(v).cuda(), torch.from_numpy(f).cuda(), *RULE, kern=1, k=5.0,
                 prm=H.params(tol=0.0))
    x = torch.from_numpy(I.complex_vector(op.M, 3)).cuda()
    ref = op.matvec(x)
    y = torch.zeros_like(x)
    g = op.graph(x, y)
    for rep in range(3):
        y.zero_()
        torch.cuda.synchronize()
        g.launch()
        torch.cuda.synchronize()
        assert torch.equal(y, ref), f"replay {rep}"
