"""GPU parity of the Galerkin P1 operator A = Phi^T W K Phi and its GMRES solve (the paper's
acoustic example) through the C ABI, against the CPU oracle and the closed-form sound-soft sphere.

Bars: P1 interpolation and projection to 1e-14 of Phi and Phi^T W; the Galerkin product within
1e-6 of the oracle's matrix (H-matrix at tol 1e-8), with and without the singular correction;
GMRES solutions within 1e-6 of a dense solve of the oracle's system; the scattered field of the
sound-soft sphere within 3e-3 of the closed-form series at L4 (the oracle's own error there is
2.4e-3)."""
import numpy as np
import pytest
from scipy import special

import oracle
from paper_1804_00995_amd import inputs as I

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")

RULE = I.rule_3pt()
D = np.array([0.0, 0.0, 1.0])


@pytest.fixture(scope="module")
def H():
    oracle.build(force=False)
    from paper_1804_00995_amd import hmx
    return hmx


def rel(a, b):
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


def space(H, level, k, reg, tol=1e-8, precision=0):
    v, f = I.icosphere(level)
    vd, fd = torch.from_numpy(v).cuda(), torch.from_numpy(f).cuda()
    op = H.build(vd, fd, *RULE, kern=1, k=k, prm=H.params(tol=tol, regularize=int(reg), precision=precision))
    return v, f, op, H.P1(op, vd, fd, *RULE)


def host(t):
    torch.cuda.synchronize()
    return t.cpu().numpy().astype(np.complex128)


def dev(a, cdt=torch.complex128):
    return torch.from_numpy(np.ascontiguousarray(a)).to(cdt).cuda()


def test_interp_and_project_match_phi(H):
    v, f, op, p1 = space(H, 2, 3.0, False)
    P, W = oracle.quad_points(v, f, *RULE)
    Phi = oracle.p1_matrix(v, f, RULE[0])
    xv = I.complex_vector(v.shape[0], 1)
    zp = I.complex_vector(P.shape[0], 2)
    assert rel(host(p1.interp(dev(xv))), Phi @ xv) <= 1e-15
    assert rel(host(p1.project(dev(zp))), Phi.T @ (W * zp)) <= 1e-14


@pytest.mark.parametrize("reg", [False, True])
def test_galerkin_product_matches_oracle(H, reg):
    v, f, op, p1 = space(H, 3, 3.0, reg)
    A, Phi, P, W = oracle.galerkin_matrix(v, f, *RULE, oracle.HELMHOLTZ, 3.0, 2.0 if reg else None)
    xv = I.complex_vector(v.shape[0], 3)
    assert rel(host(p1.matvec(dev(xv))), A @ xv) <= 1e-6


def test_gmres_matches_dense_solve(H):
    v, f, op, p1 = space(H, 3, 3.0, True)
    A, Phi, P, W = oracle.galerkin_matrix(v, f, *RULE, oracle.HELMHOLTZ, 3.0, 2.0)
    pinc = np.exp(1j * 3.0 * P @ D)
    b = Phi.T @ (W * -pinc)
    bd = p1.project(dev(-pinc))
    assert rel(host(bd), b) <= 1e-14
    x, it, res = p1.gmres(bd, tol=1e-10, restart=80, max_iter=800)
    assert res <= 1e-9 and 0 < it < 800
    assert rel(host(x), np.linalg.solve(A, b)) <= 1e-6


def test_gmres_iteration_cap(H):
    v, f, op, p1 = space(H, 2, 3.0, True)
    P, W = oracle.quad_points(v, f, *RULE)
    b = p1.project(dev(-np.exp(1j * 3.0 * P @ D)))
    x, it, res = p1.gmres(b, tol=1e-12, restart=2, max_iter=3)
    assert it == 3 and res > 1e-6
    x0, it0, res0 = p1.gmres(torch.zeros_like(b), tol=1e-8)
    assert it0 == 0 and res0 == 0.0 and torch.count_nonzero(x0) == 0


def test_fp32_mixed_solve(H):
    v, f, op, p1 = space(H, 3, 3.0, True, precision=1)
    A, Phi, P, W = oracle.galerkin_matrix(v, f, *RULE, oracle.HELMHOLTZ, 3.0, 2.0)
    pinc = np.exp(1j * 3.0 * P @ D)
    b = p1.project(dev(-pinc, torch.complex64))
    x, it, res = p1.gmres(b, tol=1e-5, restart=80, max_iter=800)
    assert res <= 2e-5
    assert rel(host(x), np.linalg.solve(A, Phi.T @ (W * -pinc))) <= 1e-3


def mie_scattered(T, k, nmax=40):
    r = np.linalg.norm(T, axis=1)
    ct = T @ D / r
    s = np.zeros(len(r), np.complex128)
    for n in range(nmax):
        jn = special.spherical_jn(n, k)
        hn = jn + 1j * special.spherical_yn(n, k)
        hr = special.spherical_jn(n, k * r) + 1j * special.spherical_yn(n, k * r)
        s -= (1j ** n) * (2 * n + 1) * jn / hn * hr * special.eval_legendre(n, ct)
    return s


def test_sound_soft_sphere_end_to_end(H):
    """Galerkin single layer with the correction, GMRES, then the scattered field radiated to
    exterior points by the operator between point sets: all on the GPU."""
    k = 3.0
    v, f, op, p1 = space(H, 4, k, True, tol=1e-6)
    xyzw = H.quad_points(torch.from_numpy(v).cuda(), torch.from_numpy(f).cuda(), *RULE)
    P = xyzw[:3].T.cpu().numpy()
    b = p1.project(dev(-np.exp(1j * k * P @ D)))
    lam, it, res = p1.gmres(b, tol=1e-8, restart=100, max_iter=2000)
    assert res <= 1e-7
    rng = np.random.default_rng(3)
    u = rng.standard_normal((200, 3))
    u /= np.linalg.norm(u, axis=1)[:, None]
    T = u * rng.uniform(1.5, 3.0, 200)[:, None]
    rad = H.build_rect(dev(T.T, torch.float64), xyzw, kern=1, k=k, prm=H.params(tol=1e-6))
    ps = host(rad.matvec(p1.interp(lam)))
    ex = mie_scattered(T, k)
    assert np.abs(ps - ex).max() / np.abs(ex).max() <= 3e-3


def test_closed_operator_is_refused(H):
    v, f, op, p1 = space(H, 1, 2.0, False)
    x = torch.zeros(v.shape[0], dtype=torch.complex128, device="cuda")
    p1.matvec(x)
    op.close()
    with pytest.raises(RuntimeError):
        p1.matvec(x)
    p1.close()


def test_galerkin_on_dense_operator(H):
    """The P1 space also serves a dense operator (tol <= 0): A equals the oracle's matrix to 1e-12."""
    v, f, op, p1 = space(H, 2, 3.0, False, tol=0.0)
    assert op.info["is_dense"] == 1
    A, Phi, P, W = oracle.galerkin_matrix(v, f, *RULE, oracle.HELMHOLTZ, 3.0)
    xv = I.complex_vector(v.shape[0], 6)
    assert rel(host(p1.matvec(dev(xv))), A @ xv) <= 1e-12
