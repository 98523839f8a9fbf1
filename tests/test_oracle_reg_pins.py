"""Pins of the oracle's singular correction (Section 5.2, regularization of the kernels).

The correction replaces, for close pairs, the Gauss value of the 1/(4 pi r) part by its exact
y-integral over the source triangle.  Its pieces are pinned against facts the oracle does not use:
  * int_T 1/|x-y| at a vertex: the polar closed form H (asinh(t_b/H) - asinh(t_a/H));
  * int_T 1/|x-y| and int_T (y-x)/|x-y| at interior points of the plane: sums of polar closed
    forms over the three sub-triangles (x, v_i, v_i+1);
  * off-plane and outside points: brute force (Duffy-mapped Gauss-Legendre over the signed
    sub-triangles around the projection, numpy's leggauss as the library primitive);
  * the linear functions through the rule's points: partition of unity and exact reproduction of
    linear functions, and brute force of int L_q(y)/|x-y|;
  * the whole correction: on the unit sphere the corrected operator's Rayleigh quotients on zonal
    harmonics converge to the closed-form eigenvalues at second order in h (ratio 4 per mesh
    level), where the uncorrected operator converges at first order.
"""
import numpy as np
import pytest
from numpy.polynomial.legendre import leggauss
from scipy import special

import oracle
from paper_1804_00995_amd import inputs as I


@pytest.fixture(scope="module", autouse=True)
def _built():
    oracle.build(force=False)


def _rand_tri(rng):
    while True:
        tv = rng.standard_normal((3, 3))
        n = np.cross(tv[1] - tv[0], tv[2] - tv[0])
        # keep triangles whose smallest angle is not tiny (brute force converges on them)
        ang = []
        for i in range(3):
            a, b = tv[(i + 1) % 3] - tv[i], tv[(i + 2) % 3] - tv[i]
            ang.append(np.arccos(a @ b / np.linalg.norm(a) / np.linalg.norm(b)))
        if np.linalg.norm(n) > 0.5 and min(ang) > 0.35:
            return tv


def _polar_vertex(p, a, b):
    """int over triangle (p, a, b) of 1/|y-p| and of (y-p)/|y-p|, p a vertex (polar coordinates:
    rho(phi) = H / cos(phi) from p to the opposite edge)."""
    e = (b - a) / np.linalg.norm(b - a)
    F = a + ((p - a) @ e) * e  # foot of the perpendicular from p on the line ab
    H = np.linalg.norm(F - p)
    nh = (F - p) / H
    ta, tb = (a - F) @ e, (b - F) @ e
    i1 = H * (np.arcsinh(tb / H) - np.arcsinh(ta / H))
    ir = 0.5 * H * H * (nh * (np.arcsinh(tb / H) - np.arcsinh(ta / H))
                        + e * (np.hypot(H, tb) - np.hypot(H, ta)) / H)
    return i1, ir


def _duffy(p, a, b, f, ng):
    g, gw = leggauss(ng)
    g, gw = 0.5 * (g + 1), 0.5 * gw
    U, V = np.meshgrid(g, g, indexing="ij")
    WW = np.outer(gw, gw)
    Y = p + U[..., None] * (a - p) + (U * V)[..., None] * (b - a)
    J = U * np.linalg.norm(np.cross(a - p, b - a))
    val = f(Y)
    if val.ndim == 3:
        return (val * (J * WW)[..., None]).sum(axis=(0, 1))
    return (val * J * WW).sum()


def _brute(x, tv, f, ng=160):
    """int_T f(y) dy split at the projection rho of x into signed sub-triangles (rho, v_i, v_i+1),
    each Duffy-mapped at rho."""
    n = np.cross(tv[1] - tv[0], tv[2] - tv[0])
    n /= np.linalg.norm(n)
    rho = x - (n @ (x - tv[0])) * n
    tot = 0.0
    for i in range(3):
        a, b = tv[i], tv[(i + 1) % 3]
        sgn = np.sign(np.cross(a - rho, b - rho) @ n)
        if sgn != 0:
            tot = tot + sgn * _duffy(rho, a, b, f, ng)
    return tot, rho


def _bary(tv, Y):
    """Barycentric coordinates of points Y (..., 3) in the plane of tv."""
    n = np.cross(tv[1] - tv[0], tv[2] - tv[0])
    A2 = n @ n
    lam = [np.cross(tv[(i + 1) % 3] - Y, tv[(i + 2) % 3] - Y) @ n / A2 for i in range(3)]
    return np.stack(lam, -1)


def test_moments_at_vertex_closed_form():
    rng = np.random.default_rng(1)
    for _ in range(20):
        tv = _rand_tri(rng)
        for v in range(3):
            p, a, b = tv[v], tv[(v + 1) % 3], tv[(v + 2) % 3]
            i1, _ = oracle.tri_moments(p, tv)
            ref, _ = _polar_vertex(p, a, b)
            assert abs(i1 - ref) <= 1e-13 * abs(ref)


def test_moments_interior_points_polar_sums():
    rng = np.random.default_rng(2)
    for _ in range(20):
        tv = _rand_tri(rng)
        lam = rng.dirichlet([2.0, 2.0, 2.0])
        x = lam @ tv
        i1, ir = oracle.tri_moments(x, tv)
        r1, rr = 0.0, np.zeros(3)
        for i in range(3):
            a, b = tv[i], tv[(i + 1) % 3]
            s1, sr = _polar_vertex(x, a, b)
            r1 += s1
            rr += sr
        assert abs(i1 - r1) <= 1e-13 * abs(r1)
        assert np.linalg.norm(ir - rr) <= 1e-12 * (np.linalg.norm(rr) + np.sqrt(i1))


@pytest.mark.parametrize("where", ["above", "outside", "outside_above", "near_edge"])
def test_moments_brute_force(where):
    rng = np.random.default_rng({"above": 3, "outside": 4, "outside_above": 5, "near_edge": 6}[where])
    for _ in range(6):
        tv = _rand_tri(rng)
        c = tv.mean(0)
        n = np.cross(tv[1] - tv[0], tv[2] - tv[0])
        n /= np.linalg.norm(n)
        size = max(np.linalg.norm(tv[i] - tv[(i + 1) % 3]) for i in range(3))
        if where == "above":
            x = rng.dirichlet([2.0, 2.0, 2.0]) @ tv + 0.2 * size * n
        elif where == "outside":
            x = c + 1.7 * (tv[1] - c)
        elif where == "outside_above":
            x = c + 1.5 * (tv[2] - c) - 0.3 * size * n
        else:
            x = 0.5 * (tv[0] + tv[1]) + 0.25 * size * n + 0.1 * (c - tv[2])
        i1, ir = oracle.tri_moments(x, tv)
        b1, rho = _brute(x, tv, lambda Y: 1.0 / np.linalg.norm(x - Y, axis=-1))
        br, _ = _brute(x, tv, lambda Y: (Y - rho) / np.linalg.norm(x - Y, axis=-1)[..., None])
        assert abs(i1 - b1) <= 1e-11 * abs(b1), where
        assert np.linalg.norm(ir - br) <= 1e-10 * (np.linalg.norm(br) + abs(b1) * size), where


def test_lagrange_matrix_interpolates_rule_points():
    bary, _ = I.rule_3pt()
    lag = oracle.lagrange_matrix(bary)
    # L_q(point p) = sum_i lag[q, i] bary[p, i] = delta_qp
    assert np.allclose(lag @ np.asarray(bary).reshape(3, 3).T, np.eye(3), atol=1e-14)
    with pytest.raises(ValueError):
        oracle.lagrange_matrix(np.full((4, 3), 0.25))


def test_lagrange_partition_of_unity_and_linear_reproduction():
    bary, _ = I.rule_3pt()
    B = np.asarray(bary).reshape(3, 3)
    lag = oracle.lagrange_matrix(bary)
    rng = np.random.default_rng(7)
    for _ in range(10):
        tv = _rand_tri(rng)
        pts = B @ tv  # the rule's points on this triangle
        for x in (rng.dirichlet([2.0, 2.0, 2.0]) @ tv, tv.mean(0) + 0.4 * rng.standard_normal(3), pts[1]):
            J = oracle.tri_lagrange(x, tv, lag)
            i1, ir = oracle.tri_moments(x, tv)
            n = np.cross(tv[1] - tv[0], tv[2] - tv[0])
            n /= np.linalg.norm(n)
            rho = x - (n @ (x - tv[0])) * n
            # sum_q L_q = 1 and sum_q y_q L_q(y) = y on the triangle
            assert abs(J.sum() - i1) <= 1e-12 * abs(i1)
            assert np.linalg.norm(pts.T @ J - (rho * i1 + ir)) <= 1e-12 * np.linalg.norm(rho * i1 + ir) + 1e-13 * i1


def test_lagrange_brute_force():
    bary, _ = I.rule_3pt()
    lag = oracle.lagrange_matrix(bary)
    rng = np.random.default_rng(8)
    for _ in range(6):
        tv = _rand_tri(rng)
        n = np.cross(tv[1] - tv[0], tv[2] - tv[0])
        n /= np.linalg.norm(n)
        for x in (tv.mean(0) + 0.3 * n, tv.mean(0) + 1.6 * (tv[0] - tv.mean(0))):
            J = oracle.tri_lagrange(x, tv, lag)
            for q in range(3):
                f = lambda Y: (_bary(tv, Y) @ lag[q]) / np.linalg.norm(x - Y, axis=-1)
                ref, _ = _brute(x, tv, f)
                assert abs(J[q] - ref) <= 1e-11 * np.abs(J).max()


def test_correction_vanishes_beyond_radius_and_decays():
    """Pairs farther than alpha * d_T from the centroid get nothing; just inside, the exact integral
    and the Gauss rule nearly agree (the correction is local)."""
    v, f = I.icosphere(2)
    bary, wq = I.rule_3pt()
    P, W = oracle.quad_points(v, f, bary, wq)
    M = P.shape[0]
    rng = np.random.default_rng(9)
    x = I.complex_vector(M, 3)
    y1 = oracle.reg_apply(P, W, v, f, bary, 1.0, x)
    y2 = oracle.reg_apply(P, W, v, f, bary, 2.0, x)
    y0 = oracle.reg_apply(P, W, v, f, bary, 1e-9, x)
    assert np.abs(y0).max() == 0.0
    rows = np.array([5, 0, M - 1, 17])
    assert np.array_equal(oracle.reg_apply(P, W, v, f, bary, 2.0, x, rows=rows), y2[rows])
    # the ring between 1 and 2 diameters adds little next to the self and neighbour corrections
    assert np.linalg.norm(y2 - y1) < 0.05 * np.linalg.norm(y1)
    # single pairs: the gap between the exact integral and the 3-point rule shrinks with the
    # distance (smooth integrand, degree-2 rule) and is small at three diameters
    t = int(rng.integers(len(f)))
    tv = v[f[t]]
    lag = oracle.lagrange_matrix(bary)
    dT = max(np.linalg.norm(tv[i] - tv[(i + 1) % 3]) for i in range(3))
    out = rng.standard_normal(3)
    out /= np.linalg.norm(out)
    gaps = []
    for dist in (0.75, 1.5, 3.0):
        xt = tv.mean(0) + dist * dT * out
        J = oracle.tri_lagrange(xt, tv, lag)
        gauss = W[3 * t:3 * t + 3] / np.linalg.norm(xt - P[3 * t:3 * t + 3], axis=1)
        gaps.append(np.abs(J - gauss).max() / gauss.max())
    assert gaps[0] > gaps[1] > gaps[2] > 0
    assert gaps[2] < 1e-2


@pytest.mark.parametrize("ratio,close", [(1.97, True), (2.03, False)])
def test_closeness_radius_is_alpha_diameters(ratio, close):
    """A pair is close when the target lies within alpha * d_T of the source triangle's centroid
    (d_T its longest edge): a tiny second triangle placed at ratio * d_T from the first one's
    centroid receives a correction from it exactly when ratio <= alpha = 2."""
    bary, wq = I.rule_3pt()
    A = np.array([[0.0, 0.0, 0.0], [1.0, 0.0, 0.0], [0.3, 0.8, 0.0]])
    dA = max(np.linalg.norm(A[i] - A[(i + 1) % 3]) for i in range(3))
    u = np.array([0.6, -0.3, 0.74])
    u /= np.linalg.norm(u)
    B = A.mean(0) + ratio * dA * u + 1e-4 * np.array([[0.0, 0.0, 0.0], [1.0, 0.0, 0.0], [0.0, 1.0, 0.0]])
    v = np.vstack([A, B])
    f = np.array([[0, 1, 2], [3, 4, 5]], np.int32)
    P, W = oracle.quad_points(v, f, bary, wq)
    x = np.zeros(6, np.complex128)
    x[:3] = 1.0
    y = oracle.reg_apply(P, W, v, f, bary, 2.0, x)
    assert (np.abs(y[3:]) > 0).all() == close and (np.abs(y[3:]) == 0).all() == (not close)


def _eig(l, k):
    if k == 0:
        return 1.0 / (2 * l + 1)
    j, y = special.spherical_jn(l, k), special.spherical_yn(l, k)
    return 1j * k * j * (j + 1j * y)


def _rayleigh(level, kern, k, l, alpha):
    v, f = I.icosphere(level)
    bary, wq = I.rule_3pt()
    P, W = oracle.quad_points(v, f, bary, wq)
    d = np.random.default_rng(7).standard_normal(3)
    d /= np.linalg.norm(d)
    u = P @ d / np.linalg.norm(P, axis=1)
    fz = special.eval_legendre(l, u).astype(np.complex128)
    if alpha is None:
        Kf = oracle.dense_matvec(P, W, kern, k, fz)
    else:
        Kf = oracle.reg_dense_matvec(P, W, kern, k, v, f, bary, alpha, fz)
    return np.vdot(fz, W * Kf) / np.vdot(fz, W * fz)


@pytest.mark.parametrize("kern,k,l", [(oracle.LAPLACE, 0.0, 0), (oracle.LAPLACE, 0.0, 2),
                                      (oracle.HELMHOLTZ, 5.0, 0), (oracle.HELMHOLTZ, 5.0, 1),
                                      (oracle.HELMHOLTZ, 5.0, 3)])
def test_corrected_sphere_eigenvalues_second_order(kern, k, l):
    lam = _eig(l, k)
    err = [abs(_rayleigh(L, kern, k, l, 2.0) - lam) for L in (2, 3, 4)]
    # second order: halving h quarters the error (flat triangles and the smooth remainder of the
    # kernel are both O(h^2) once the singular part is integrated exactly)
    assert 3.6 <= err[0] / err[1] <= 4.4, err
    assert 3.6 <= err[1] / err[2] <= 4.4, err
    assert err[2] < 1e-3
    # the uncorrected operator at L4 is first order and several times worse
    assert abs(_rayleigh(4, kern, k, l, None) - lam) > 4 * err[2]


def test_hmatrix_correction_only_in_near_blocks():
    """With every block near (eta tiny), the oracle H-matrix with the correction equals the
    corrected dense product; with the default eta, its near blocks differ from the uncorrected
    H-matrix by exactly the close pairs inside them."""
    v, f = I.icosphere(2)
    bary, wq = I.rule_3pt()
    P, W = oracle.quad_points(v, f, bary, wq)
    x = I.complex_vector(P.shape[0], 4)
    H = oracle.HMatrix(P, W, oracle.HELMHOLTZ, 4.0, leaf=64, eta=1e-9, tol=1e-6, mesh=(v, f, bary),
                       reg_radius=2.0)
    assert H.info["n_far"] == 0
    ref = oracle.reg_dense_matvec(P, W, oracle.HELMHOLTZ, 4.0, v, f, bary, 2.0, x)
    y = H.matvec(x)
    assert np.linalg.norm(y - ref) <= 1e-13 * np.linalg.norm(ref)
    Hr = oracle.HMatrix(P, W, oracle.HELMHOLTZ, 4.0, leaf=32, tol=1e-6, mesh=(v, f, bary))
    Hp = oracle.HMatrix(P, W, oracle.HELMHOLTZ, 4.0, leaf=32, tol=1e-6)
    assert Hr.info["n_far"] > 0
    d = Hr.matvec(x) - Hp.matvec(x)
    # the difference is the correction restricted to near blocks: brute force over block ranges
    perm = Hp.tree()["perm"]
    nearR, _, _ = Hp.blocks()
    full = np.zeros(P.shape[0], np.complex128)
    C = _correction_matrix(P, W, v, f, bary, 2.0)
    for tb, te, sb, se in nearR:
        rows, cols = perm[tb:te], perm[sb:se]
        full[rows] += C[np.ix_(rows, cols)] @ x[cols]
    assert np.linalg.norm(d - full) <= 1e-12 * np.linalg.norm(full)
    assert np.linalg.norm(full) > 0


def _correction_matrix(P, W, v, f, bary, alpha):
    """The explicit correction matrix, column by column through the oracle's apply."""
    M = P.shape[0]
    C = np.zeros((M, M))
    for l in range(M):
        e = np.zeros(M, np.complex128)
        e[l] = 1.0
        C[:, l] = oracle.reg_apply(P, W, v, f, bary, alpha, e).real
    return C
