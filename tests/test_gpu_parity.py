"""GPU parity: the HIP path through the C ABI against the CPU oracle on the same seeded inputs.

Bars: quadrature points bit-exact; cluster tree and block lists identical; dense product within
1e-12 relative; H-matrix product within the ACA tolerance of the dense product (1e-3 at tol 1e-3,
on all rows at small sizes and on seeded sampled rows at the 245 760-point size the bench times).
"""
import numpy as np
import pytest

import oracle
from paper_1804_00995_amd import inputs as I

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def H():
    oracle.build(force=False)
    from paper_1804_00995_amd import hmx
    return hmx


def mesh(level):
    v, f = I.icosphere(level)
    return v, f, torch.from_numpy(v).cuda(), torch.from_numpy(f).cuda()


def rel(a, b):
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


RULE = I.rule_3pt()


def build(H, level, kern=1, k=5.0, **kw):
    v, f, vd, fd = mesh(level)
    op = H.build(vd, fd, *RULE, kern=kern, k=k, prm=H.params(**kw))
    P, W = oracle.quad_points(v, f, *RULE)
    return op, P, W


def apply(op, x, dtype=torch.complex128):
    xd = torch.from_numpy(x).to(dtype).cuda()
    y = op.matvec(xd)
    torch.cuda.synchronize()
    return y.cpu().numpy().astype(np.complex128)


# ------------------------------------------------------------------------------ quadrature
@pytest.mark.parametrize("level", [0, 3])
def test_quad_points_bit_exact(H, level):
    v, f, vd, fd = mesh(level)
    g = H.quad_points(vd, fd, *RULE).cpu().numpy()
    P, W = oracle.quad_points(v, f, *RULE)
    for d in range(3):
        assert np.array_equal(g[d], P[:, d])
    assert np.abs(g[3] - W).max() <= 4e-16 * W.max()


def test_quad_points_rejects_bad_mesh(H):
    v, f, vd, fd = mesh(1)
    bad = fd.clone()
    bad[3, 1] = v.shape[0] + 5
    with pytest.raises(H.HmxError) as e:
        H.quad_points(vd, bad, *RULE)
    assert e.value.code == H.EINVAL
    vbad = vd.clone()
    vbad[2, 0] = float("nan")
    with pytest.raises(H.HmxError) as e:
        H.build(vbad, fd, *RULE, kern=1, k=1.0)
    assert e.value.code == H.EINVAL


# ------------------------------------------------------------------------------ dense (a0)
@pytest.mark.parametrize("kern,k", [(1, 5.0), (0, 0.0), (1, 40.0)])
def test_dense_matches_oracle(H, kern, k):
    op, P, W = build(H, 3, kern=kern, k=k, tol=0.0)
    assert op.info["is_dense"] == 1
    x = I.complex_vector(P.shape[0], 0)
    y = apply(op, x)
    yr = oracle.dense_matvec(P, W, kern, k, x)
    assert rel(y, yr) <= 1e-12


def test_dense_fp32_mixed(H):
    op, P, W = build(H, 3, kern=1, k=5.0, tol=0.0, precision=H.FP32_MIXED)
    x = I.complex_vector(P.shape[0], 0)
    y = apply(op, x, torch.complex64)
    yr = oracle.dense_matvec(P, W, 1, 5.0, x)
    assert rel(y, yr) <= 1e-5


# ------------------------------------------------------------------------------ tree, blocks
@pytest.mark.parametrize("level,leaf,max_mn", [(2, 7, 0), (3, 16, 0), (3, 64, 0), (4, 64, 0),
                                              (4, 128, 0), (3, 16, 96), (4, 64, 4096),
                                              (5, 64, 16384)])
def test_tree_and_blocks_identical(H, level, leaf, max_mn):
    op, P, W = build(H, level, leaf_size=leaf, tol=1e-3, max_far_mn=max_mn)
    Ho = oracle.HMatrix(P, W, 1, 5.0, leaf=leaf, tol=1e-3, max_mn=max_mn)
    T, To = op.export_tree(), Ho.tree()
    assert np.array_equal(T["perm"], To["perm"])
    g = {(b, e): (lv, tuple(bx)) for b, e, lv, bx in zip(T["begin"], T["end"], T["level"], T["box"])}
    o = {(b, e): (lv, tuple(bx)) for b, e, lv, bx in zip(To["begin"], To["end"], To["level"], To["box"])}
    assert g == o
    nearG, farG, _ = op.export_blocks()
    nearO, farO, _ = Ho.blocks()
    assert np.array_equal(nearG, nearO)
    assert np.array_equal(farG, farO)
    assert op.info["n_leaves"] == int((To["child0"] < 0).sum())


@pytest.mark.parametrize("cap", [1, 16, 300])
def test_block_recursion_with_small_buffers(H, cap):
    # buffers far below the lists' sizes: the recursion drops what does not fit, counts it, and
    # runs again with larger buffers until nothing is dropped; the lists equal the oracle's
    op, P, W = build(H, 4, leaf_size=32, tol=1e-3, force_block_cap=cap)
    Ho = oracle.HMatrix(P, W, 1, 5.0, leaf=32, tol=1e-3)
    nearG, farG, _ = op.export_blocks()
    nearO, farO, _ = Ho.blocks()
    assert np.array_equal(nearG, nearO) and np.array_equal(farG, farO)
    assert len(nearG) > 300 and len(farG) > 300


# ------------------------------------------------------------------------------ H product (a5-a7)
@pytest.mark.parametrize("level,kern,k", [(3, 1, 5.0), (3, 0, 0.0), (4, 1, 10.0), (4, 1, 25.0)])
def test_hmatvec_within_tolerance_of_dense(H, level, kern, k):
    op, P, W = build(H, level, kern=kern, k=k, tol=1e-3)
    x = I.complex_vector(P.shape[0], 0)
    y = apply(op, x)
    yr = oracle.dense_matvec(P, W, kern, k, x)
    assert rel(y, yr) <= 1e-3
    assert op.info["n_far"] > 0 and op.info["far_entries"] > 0


def test_hmatvec_tight_tolerance(H):
    op, P, W = build(H, 3, kern=1, k=8.0, tol=1e-9, leaf_size=32)
    x = I.complex_vector(P.shape[0], 3)
    assert rel(apply(op, x), oracle.dense_matvec(P, W, 1, 8.0, x)) <= 1e-7


def test_near_field_only_equals_dense(H):
    # 60 points in one leaf: the whole operator is one near block
    op, P, W = build(H, 0, kern=1, k=3.0, tol=1e-3)
    assert op.info["n_far"] == 0 and op.info["n_near"] == 1
    x = I.complex_vector(P.shape[0], 1)
    assert rel(apply(op, x), oracle.dense_matvec(P, W, 1, 3.0, x)) <= 1e-13


def test_poly2_exact_rank(H):
    op, P, W = build(H, 2, kern=H.TEST_POLY2, k=0.0, tol=1e-12, leaf_size=16)
    x = I.complex_vector(P.shape[0], 2)
    y = apply(op, x)
    yr = oracle.dense_matvec(P, W, oracle.POLY2, 0.0, x)
    assert rel(y, yr) <= 1e-11
    _, _, ranks = op.export_blocks()
    assert ranks.max() <= 12


@pytest.mark.parametrize("k", [5.0, 20.0])
def test_aca_blocks_error_bounds(H, k):
    op, P, W = build(H, 3, kern=1, k=k, tol=1e-3)
    perm = op.export_tree()["perm"]
    _, farR, ranks = op.export_blocks()
    sizes = (farR[:, 1] - farR[:, 0]) * (farR[:, 3] - farR[:, 2])
    for b in np.argsort(-sizes)[:10]:
        tb, te, sb, se = (int(v) for v in farR[b])
        m, n = te - tb, se - sb
        rows, cols = perm[tb:te], perm[sb:se]
        A = oracle.green(1, k, np.repeat(P[rows], n, 0), np.tile(P[cols], (m, 1))).reshape(m, n) * W[cols][None, :]
        U, V = op.export_far(int(b), m, n)
        assert V is not None
        r = U.shape[1]
        err = np.linalg.norm(A - U @ V.T)
        s = np.linalg.svd(A, compute_uv=False)
        assert err >= np.sqrt((s[r:] ** 2).sum()) * (1 - 1e-9)
        assert err <= 10 * 1e-3 * np.linalg.norm(A)


def test_ranks_close_to_oracle(H):
    op, P, W = build(H, 4, kern=1, k=15.0, tol=1e-3)
    Ho = oracle.HMatrix(P, W, 1, 15.0, leaf=64, tol=1e-3)
    _, _, rg = op.export_blocks()
    _, _, ro = Ho.blocks()
    assert rg.shape == ro.shape
    assert abs(int(rg.sum()) - int(ro.sum())) <= 0.02 * ro.sum()
    assert (np.abs(rg.astype(int) - ro.astype(int)) <= 2).mean() > 0.98


def test_deterministic(H):
    op1, P, W = build(H, 4, kern=1, k=12.0, tol=1e-3)
    op2, _, _ = build(H, 4, kern=1, k=12.0, tol=1e-3)
    x = I.complex_vector(P.shape[0], 5)
    y1, y1b, y2 = apply(op1, x), apply(op1, x), apply(op2, x)
    assert np.array_equal(y1, y1b)
    assert np.array_equal(y1, y2)


@pytest.mark.parametrize("precision", [0, 1])
def test_forced_dense_fallback(H, precision):
    # a rank cap of 2 forces ACA past its cap on most blocks: those are stored exactly, by the
    # assembly kernel in its FP64 or FP32 layout
    op, P, W = build(H, 3, kern=1, k=5.0, tol=1e-3, force_rank_cap=2, precision=precision)
    assert op.info["dense_far"] > 0
    x = I.complex_vector(P.shape[0], 0)
    y = apply(op, x, torch.complex128 if precision == 0 else torch.complex64)
    assert rel(y, oracle.dense_matvec(P, W, 1, 5.0, x)) <= 1e-3
    op.close()


def test_overflow_continuation_identical(H):
    # a first rank slot of 1 makes nearly every block continue in a larger slot; the factors
    # must be those of a single uninterrupted run
    opa, P, W = build(H, 3, kern=1, k=9.0, tol=1e-3, initial_rank=1, aca_arena=0)
    opb, _, _ = build(H, 3, kern=1, k=9.0, tol=1e-3, initial_rank=64, aca_arena=0)
    opc, _, _ = build(H, 3, kern=1, k=9.0, tol=1e-3)  # workgroup arenas, exact slots
    assert opa.info["overflow_blocks"] > 0
    x = I.complex_vector(P.shape[0], 4)
    ya = apply(opa, x)
    assert np.array_equal(ya, apply(opb, x))
    assert np.array_equal(ya, apply(opc, x))
    assert opc.info["factor_bytes"] < opb.info["factor_bytes"]


def test_schedule_classes_agree(H):
    # the same operator built with every far block in the middle class, and with the small-block
    # and 256-thread large-block kinds: each within the tolerance of the oracle's dense product,
    # and the per-class counts account for every far block
    ops = {}
    for name, kw in [("default", {}), ("mid_only", dict(aca_small_mn=0, aca_big_mn=1 << 30)),
                     ("big256", dict(aca_big_threads=256, aca_big_mn=512, aca_small_mn=256)),
                     ("wave", dict(aca_wave=1)), ("wave32", dict(aca_wave=1, precision=H.FP32_MIXED))]:
        ops[name], P, W = build(H, 4, kern=1, k=15.0, tol=1e-3, **kw)
    x = I.complex_vector(P.shape[0], 7)
    yr = oracle.dense_matvec(P, W, 1, 15.0, x)
    for name, op in ops.items():
        assert sum(op.info["aca_blocks"]) == op.info["n_far"], name
        dt = torch.complex64 if op.precision == H.FP32_MIXED else torch.complex128
        assert rel(apply(op, x, dt), yr) <= 1e-3, name
    assert ops["default"].info["aca_blocks"][3] > 0
    assert ops["mid_only"].info["aca_blocks"][3] == 0 and ops["mid_only"].info["aca_blocks"][0] == 0
    assert ops["big256"].info["aca_blocks"][0] > 0
    assert ops["default"].info["aca_blocks"][2] == 0
    assert ops["wave"].info["aca_blocks"][2] > 0 and ops["wave32"].info["aca_blocks"][2] > 0


def test_wavefront_overflow_continues_in_workgroups(H):
    # at tol 1e-8 wavefront blocks need more than the register capacity of 16 terms: they store
    # their state and continue in the workgroup kernel; the product stays within tolerance
    op, P, W = build(H, 4, kern=1, k=15.0, tol=1e-8, aca_wave=1)
    assert op.info["aca_blocks"][2] > 0 and op.info["overflow_blocks"] > 0
    x = I.complex_vector(P.shape[0], 8)
    assert rel(apply(op, x), oracle.dense_matvec(P, W, 1, 15.0, x)) <= 1e-7


def test_full_size_sampled_rows(H):
    """245 760 points (L6 sphere), k = 40, leaf 64, tol 1e-3: the configuration the bench times."""
    op, P, W = build(H, 6, kern=1, k=40.0, tol=1e-3)
    x = I.complex_vector(P.shape[0], 0)
    y = apply(op, x)
    rows = np.sort(np.random.default_rng(123).choice(P.shape[0], 384, replace=False))
    yr = oracle.dense_rows(P, W, 1, 40.0, x, rows)
    assert rel(y[rows], yr) <= 1e-3


# ------------------------------------------------------------------------------ FP32 mixed (a8)
@pytest.mark.parametrize("level,k,rows", [(4, 15.0, None), (6, 40.0, 256)])
def test_fp32_mixed_against_oracle_and_fp64(H, level, k, rows):
    """FP32 blocks and factors with FP64 distance, phase and ACA norms: error against the
    FP64 oracle's dense product and against the GPU FP64 H-matrix product."""
    op32, P, W = build(H, level, kern=1, k=k, tol=1e-3, precision=H.FP32_MIXED)
    op64, _, _ = build(H, level, kern=1, k=k, tol=1e-3)
    x = I.complex_vector(P.shape[0], 0)
    y32 = apply(op32, x, torch.complex64)
    y64 = apply(op64, x)
    if rows is None:
        idx = np.arange(P.shape[0])
        yr = oracle.dense_matvec(P, W, 1, k, x)
    else:
        idx = np.sort(np.random.default_rng(321).choice(P.shape[0], rows, replace=False))
        yr = oracle.dense_rows(P, W, 1, k, x, idx)
    e_oracle = rel(y32[idx], yr)
    e_fp64 = rel(y32, y64)
    print(f"fp32 vs oracle {e_oracle:.3e}, vs gpu fp64 {e_fp64:.3e}, fp64 vs oracle {rel(y64[idx], yr):.3e}")
    assert e_oracle <= 1e-3
    assert e_fp64 <= 1e-3
    assert op32.info["bytes"] < op64.info["bytes"]


# ------------------------------------------------------------------------------ row shares
@pytest.mark.parametrize("shares,near_mode", [(2, 0), (4, 0), (8, 0), (4, 1)])
def test_row_shares_sum_to_whole_product(H, shares, near_mode):
    """The operator split by rows into `shares` parts (one per device of a row-sharded build):
    each share's blocks are the whole operator's blocks whose row node lies in the share, and
    the shares' products add up to the whole product bit for bit (each row comes from exactly
    one share, computed with the same blocks in the same order), with the near field stored or
    computed in the product."""
    v, f, vd, fd = mesh(4)
    full = H.build(vd, fd, *RULE, kern=1, k=12.0, prm=H.params(near_mode=near_mode))
    x = torch.from_numpy(I.complex_vector(full.M, 8)).cuda()
    y_full = full.matvec(x)
    nearF, farF, rankF = full.export_blocks()
    acc = torch.zeros_like(y_full)
    covered = np.zeros(full.M, bool)
    perm = full.export_tree()["perm"]
    for r in range(shares):
        op = H.build(vd, fd, *RULE, kern=1, k=12.0,
                     prm=H.params(row_shares=shares, row_share=r, near_mode=near_mode))
        rb, re = op.info["row_begin"], op.info["row_end"]
        assert 0 <= rb < re <= full.M
        covered[rb:re] = True
        nearS, farS, rankS = op.export_blocks()
        inN = (nearF[:, 0] >= rb) & (nearF[:, 1] <= re)
        inF = (farF[:, 0] >= rb) & (farF[:, 1] <= re)
        assert np.array_equal(nearS, nearF[inN]) and np.array_equal(farS, farF[inF])
        y = op.matvec(x)
        rows = torch.from_numpy(perm[rb:re].astype(np.int64)).cuda()
        others = torch.ones(full.M, dtype=torch.bool, device="cuda")
        others[rows] = False
        assert torch.equal(y[rows], y_full[rows])
        assert bool((y[others] == 0).all())
        acc += y
        op.close()
    assert covered.all()
    assert torch.equal(acc, y_full)


def test_row_share_errors(H):
    v, f, vd, fd = mesh(1)  # 240 points: a tree of depth 2 at leaf 64
    with pytest.raises(H.HmxError) as e:
        H.build(vd, fd, *RULE, kern=1, k=3.0, prm=H.params(row_shares=1024, row_share=0))
    assert e.value.code == H.EUNSUPPORTED
    with pytest.raises(H.HmxError) as e:
        H.build(vd, fd, *RULE, kern=1, k=3.0, prm=H.params(row_shares=3))
    assert e.value.code == H.EINVAL


@pytest.mark.parametrize("precision", [0, 1])
def test_pool_exhaustion_rounds(H, precision):
    """A first slot pool of 1 MiB runs out almost at once: the blocks left over continue in later
    rounds with new pools (not-started blocks as fresh ones, the others from their saved state).
    The operator stays within the tolerance, with ranks close to a one-round build."""
    op, P, W = build(H, 4, kern=1, k=12.0, tol=1e-3, precision=precision, force_pool_bytes=1 << 20)
    ref, _, _ = build(H, 4, kern=1, k=12.0, tol=1e-3, precision=precision)
    assert op.info["aca_rounds"] > 1 and ref.info["aca_rounds"] == 1
    x = I.complex_vector(P.shape[0], 9)
    dt = torch.complex128 if precision == 0 else torch.complex64
    yr = oracle.dense_matvec(P, W, 1, 12.0, x)
    assert rel(apply(op, x, dt), yr) <= 1e-3
    _, _, r0 = ref.export_blocks()
    _, _, r1 = op.export_blocks()
    assert abs(int(r0.sum()) - int(r1.sum())) <= 0.01 * r0.sum()
    assert op.info["dense_far"] == ref.info["dense_far"]


# ------------------------------------------------------------------------------ apply only
@pytest.mark.parametrize("level,k", [(3, 5.0), (4, 12.0)])
def test_apply_only_with_oracle_factors(H, level, k):
    """The GPU product with the oracle's own far factors imported (same tree and blocks; near
    blocks assembled on the GPU) equals the oracle's H-matrix product to 1e-13: this checks
    gather, the block products, the per-leaf sums and the scatter apart from ACA."""
    op, P, W = build(H, level, kern=1, k=k, tol=1e-3)
    Ho = oracle.HMatrix(P, W, 1, k, leaf=64, tol=1e-3)
    nearG, farG, rG = op.export_blocks()
    nearO, farO, rO = Ho.blocks()
    assert np.array_equal(nearG, nearO) and np.array_equal(farG, farO)
    assert (rO >= 0).all() and (rG >= 0).all()  # no block stored dense at this tolerance
    Us, Vs = [], []
    for b, (tb, te, sb, se) in enumerate(farO):
        U, V = Ho.far_factors(b, int(te - tb), int(se - sb), int(rO[b]))
        Us.append(U)
        Vs.append(V)
    op.import_far(rO, Us, Vs)
    assert op.info["far_entries"] == Ho.info["s_far"]
    x = I.complex_vector(P.shape[0], 12)
    y = apply(op, x)
    yo = Ho.matvec(x)
    assert rel(y, yo) <= 1e-13
    # and once more through a captured graph
    xd = torch.from_numpy(x).cuda()
    yd = torch.zeros_like(xd)
    g = op.graph(xd, yd)
    g.launch(2)
    torch.cuda.synchronize()
    assert np.array_equal(yd.cpu().numpy(), y)


# ------------------------------------------------------------------------------ kernel values
@pytest.mark.parametrize("precision,bound", [(0, 1e-14), (1, 2e-6)])
def test_kernel_values_match_golden(H, precision, bound):
    """Two points at distance r with unit weights: the dense operator's entry K_01 = G(r) against
    the closed form written by tests/golden/make_golden.py (FP32 mode reduces k r in FP64)."""
    import os
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "green_kernel_values.txt")
    rows = [l.split() for l in open(path) if not l.startswith("#") and l.strip()]
    dt = torch.complex128 if precision == 0 else torch.complex64
    x = torch.tensor([0.0, 1.0], dtype=dt).cuda()
    for r, k, gre, gim in rows:
        r, k = float(r), float(k)
        g = complex(float(gre), float(gim))
        xyzw = torch.tensor([[0.0, r], [0.0, 0.0], [0.0, 0.0], [1.0, 1.0]], dtype=torch.float64).cuda()
        op = H.build_points(xyzw, kern=H.LAPLACE if k == 0 else H.HELMHOLTZ, k=k,
                            prm=H.params(tol=0.0, precision=precision))
        y = op.matvec(x).cpu().numpy()
        assert abs(complex(y[0]) - g) <= bound * abs(g), (r, k, y[0], g)
        assert y[1] == 0  # K_11 = 0 (r = 0) and K_10 x_0 = 0
        op.close()


@pytest.mark.parametrize("kern,k,lo,hi,bound", [(0, 0.0, -140.0, 140.0, 1e-15),
                                                (1, 40.0, -2.0, 1.0, 1e-12)])
def test_distance_and_reciprocal_over_wide_range(H, kern, k, lo, hi, bound):
    """Column 0 of the dense FP64 operator (a source of weight 1 at the origin) at targets whose
    distances span 10^lo to 10^hi, including the ranges that take the IEEE square root and
    division instead of the refined reciprocal square root, against numpy in FP64: 1 / (4 pi r)
    within a few ulp, and e^{ikr} / (4 pi r) within k r times the rounding of r."""
    rng = np.random.default_rng(5)
    n = 4000
    d = rng.standard_normal((n, 3))
    d /= np.linalg.norm(d, axis=1)[:, None]
    t = d * (10.0 ** rng.uniform(lo, hi, n))[:, None]
    pts = np.vstack([np.zeros((1, 3)), t])
    xyzw = torch.from_numpy(np.ascontiguousarray(
        np.vstack([pts.T, np.ones((1, n + 1))]))).cuda()
    op = H.build_points(xyzw, kern=kern, k=k, prm=H.params(tol=0.0))
    x = np.zeros(n + 1, np.complex128)
    x[0] = 1.0
    y = apply(op, x)
    op.close()
    r = np.sqrt((t * t).sum(axis=1))
    g = np.exp(1j * k * r) / (4.0 * np.pi * r)
    assert y[0] == 0
    err = np.abs(y[1:] - g) / np.abs(g)
    assert err.max() <= bound, (err.max(), r[err.argmax()])
