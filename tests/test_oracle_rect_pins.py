"""Pins of the oracle's product at target points other than the sources (Section 5.1: integrals
with one integration and a collection of points).

  * brute force on a tiny mesh, entry by entry with mpmath;
  * the exterior potential of the unit density on the unit sphere, 1/|x| (Laplace) and
    sin(k)/k e^{ik|x|}/|x| (Helmholtz), approached at second order in h by the quadrature sums;
  * with the source points as targets, the square operator;
  * row sampling returns the same rows as the whole product.
"""
import math

import mpmath
import numpy as np
import pytest

import oracle
from paper_1804_00995_amd import inputs as I

RULE = I.rule_3pt()


@pytest.fixture(scope="module", autouse=True)
def _built():
    oracle.build(force=False)


def _exterior_targets(n, seed=5, rmin=1.3, rmax=3.0):
    rng = np.random.default_rng(seed)
    d = rng.standard_normal((n, 3))
    d /= np.linalg.norm(d, axis=1)[:, None]
    r = rng.uniform(rmin, rmax, n)
    return d * r[:, None], r


def test_brute_force_tiny():
    v, f = I.icosphere(1)
    P, W = oracle.quad_points(v, f, *RULE)
    T, _ = _exterior_targets(7, seed=2, rmin=0.2, rmax=2.0)  # inside, near and outside the mesh
    T = np.vstack([T, P[3]])  # one target on a source point
    k = 3.0
    x = I.complex_vector(P.shape[0], 9)
    y = oracle.rect_matvec(T, P, W, oracle.HELMHOLTZ, k, x)
    for i in range(T.shape[0]):
        acc = mpmath.mpc(0)
        for l in range(P.shape[0]):
            r = math.dist(T[i], P[l])
            if r > 0:
                acc += mpmath.exp(1j * k * r) / (4 * mpmath.pi * r) * W[l] * complex(x[l])
        assert abs(complex(acc) - y[i]) <= 1e-13 * abs(complex(acc))


@pytest.mark.parametrize("kern,k", [(oracle.LAPLACE, 0.0), (oracle.HELMHOLTZ, 5.0),
                                    (oracle.HELMHOLTZ, 15.0)])
def test_exterior_sphere_potential_second_order(kern, k):
    T, r = _exterior_targets(40)
    exact = 1.0 / r if k == 0 else np.sin(k) / k * np.exp(1j * k * r) / r
    errs = []
    for level in (3, 4, 5):
        v, f = I.icosphere(level)
        P, W = oracle.quad_points(v, f, *RULE)
        y = oracle.rect_matvec(T, P, W, kern, k, np.ones(P.shape[0], np.complex128))
        errs.append(np.abs(y - exact).max() / np.abs(exact).max())
    assert 3.5 <= errs[0] / errs[1] <= 4.5, errs
    assert 3.5 <= errs[1] / errs[2] <= 4.5, errs
    assert errs[2] < 4e-3


def test_sources_as_targets_is_the_square_operator():
    v, f = I.icosphere(2)
    P, W = oracle.quad_points(v, f, *RULE)
    x = I.complex_vector(P.shape[0], 3)
    assert np.array_equal(oracle.rect_matvec(P, P, W, oracle.HELMHOLTZ, 4.0, x),
                          oracle.dense_matvec(P, W, oracle.HELMHOLTZ, 4.0, x))


def test_rows_match_whole_product():
    v, f = I.icosphere(2)
    P, W = oracle.quad_points(v, f, *RULE)
    T, _ = _exterior_targets(50, seed=8)
    x = I.complex_vector(P.shape[0], 4)
    y = oracle.rect_matvec(T, P, W, oracle.HELMHOLTZ, 6.0, x)
    rows = np.array([7, 0, 49, 13])
    assert np.array_equal(oracle.rect_matvec(T, P, W, oracle.HELMHOLTZ, 6.0, x, rows=rows), y[rows])
