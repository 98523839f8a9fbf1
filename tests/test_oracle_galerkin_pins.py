"""Pins of the oracle's Galerkin P1 operator (eq. (BEM) with P1 test and trial functions) and of
the sound-soft sphere it solves (the paper's acoustic example), against facts the oracle does
not use:
  * the P1 basis at the quadrature points: partition of unity, and Phi^T W Phi equal to the P1
    mass matrix assembled from its closed form area/12 [[2,1,1],[1,2,1],[1,1,2]] (the rule is
    exact for quadratics);
  * the Galerkin matrix of the symmetric kernel is complex symmetric;
  * the correction matrix equals the correction applied column by column;
  * the scattered field of the sound-soft unit sphere, from the Galerkin solution of the
    single-layer equation with the singular correction, converges at second order in h to the
    closed-form series -sum_n i^n (2n+1) j_n(k)/h_n(k) h_n(k r) P_n(cos theta); without the
    correction it does not.
"""
import numpy as np
import pytest
from scipy import special

import oracle
from paper_1804_00995_amd import inputs as I

RULE = I.rule_3pt()


@pytest.fixture(scope="module", autouse=True)
def _built():
    oracle.build(force=False)


def mass_matrix_closed_form(v, f):
    nv = v.shape[0]
    Mm = np.zeros((nv, nv))
    loc = np.array([[2.0, 1.0, 1.0], [1.0, 2.0, 1.0], [1.0, 1.0, 2.0]]) / 12.0
    for t in f:
        area = 0.5 * np.linalg.norm(np.cross(v[t[1]] - v[t[0]], v[t[2]] - v[t[0]]))
        Mm[np.ix_(t, t)] += area * loc
    return Mm


def test_p1_basis_partition_and_mass_matrix():
    v, f = I.icosphere(2)
    P, W = oracle.quad_points(v, f, *RULE)
    Phi = oracle.p1_matrix(v, f, RULE[0])
    assert np.allclose(Phi.sum(1), 1.0, atol=1e-15)
    assert ((Phi != 0).sum(1) == 3).all()
    # interpolation: the basis reproduces the vertex coordinates at the points
    assert np.abs(Phi @ v - P).max() < 1e-14
    assert np.abs(Phi.T @ (W[:, None] * Phi) - mass_matrix_closed_form(v, f)).max() < 1e-15


def test_galerkin_matrix_symmetric_and_correction_matrix_consistent():
    v, f = I.icosphere(1)
    A, Phi, P, W = oracle.galerkin_matrix(v, f, RULE[0], RULE[1], oracle.HELMHOLTZ, 4.0)
    assert np.abs(A - A.T).max() <= 1e-15 * np.abs(A).max()
    C = oracle.reg_matrix(P, W, v, f, RULE[0], 2.0)
    for l in (0, 7, P.shape[0] - 1):
        e = np.zeros(P.shape[0], np.complex128)
        e[l] = 1.0
        assert np.array_equal(C[:, l], oracle.reg_apply(P, W, v, f, RULE[0], 2.0, e).real)


def mie_scattered(T, k, d, nmax=40):
    """Sound-soft unit sphere, incident e^{ik x.d}: the exterior scattered field."""
    r = np.linalg.norm(T, axis=1)
    ct = T @ d / r
    s = np.zeros(len(r), np.complex128)
    for n in range(nmax):
        jn = special.spherical_jn(n, k)
        hn = jn + 1j * special.spherical_yn(n, k)
        hr = special.spherical_jn(n, k * r) + 1j * special.spherical_yn(n, k * r)
        s -= (1j ** n) * (2 * n + 1) * jn / hn * hr * special.eval_legendre(n, ct)
    return s


def exterior_points(n=60, seed=3):
    rng = np.random.default_rng(seed)
    u = rng.standard_normal((n, 3))
    u /= np.linalg.norm(u, axis=1)[:, None]
    return u * rng.uniform(1.5, 3.0, n)[:, None]


def scattered_field(level, k, d, T, reg):
    v, f = I.icosphere(level)
    A, Phi, P, W = oracle.galerkin_matrix(v, f, RULE[0], RULE[1], oracle.HELMHOLTZ, k,
                                          2.0 if reg else None)
    lam = np.linalg.solve(A, -Phi.T @ (W * np.exp(1j * k * P @ d)))
    return oracle.rect_matvec(T, P, W, oracle.HELMHOLTZ, k, Phi @ lam)


def test_sound_soft_sphere_second_order():
    k, d = 3.0, np.array([0.0, 0.0, 1.0])
    T = exterior_points()
    ex = mie_scattered(T, k, d)
    err = [np.abs(scattered_field(L, k, d, T, True) - ex).max() / np.abs(ex).max() for L in (1, 2, 3)]
    assert 3.0 <= err[0] / err[1] <= 5.5, err
    assert 3.0 <= err[1] / err[2] <= 5.5, err
    assert err[2] < 1.5e-2
    plain = np.abs(scattered_field(3, k, d, T, False) - ex).max() / np.abs(ex).max()
    assert plain > 3 * err[2]
