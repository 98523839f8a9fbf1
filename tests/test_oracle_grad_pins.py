"""Pins of the oracle's gradient kernels (Section 5.1: grady[exp(ikr)/r]j, the gradient of the
kernel in y): central differences of the plain kernel, and the double-layer identity on the unit
sphere, int_S dG/dn_y (x, y) dS_y = -1/2 for x on S (Laplace), which the quadrature sums
approach at first order in h (the integrand behaves like 1/r on the sphere)."""
import numpy as np
import pytest

import oracle
from paper_1804_00995_amd import inputs as I


@pytest.fixture(scope="module", autouse=True)
def _built():
    oracle.build(force=False)


@pytest.mark.parametrize("k", [0.0, 5.0, 40.0])
def test_gradient_matches_central_differences(k):
    rng = np.random.default_rng(int(k) + 1)
    x, y = rng.standard_normal((60, 3)), rng.standard_normal((60, 3))
    base = oracle.LAPLACE if k == 0 else oracle.HELMHOLTZ
    h = 1e-5 / max(1.0, k / 5.0)
    for j in range(3):
        e = np.zeros(3)
        e[j] = h
        fd = (oracle.green(base, k, x, y + e) - oracle.green(base, k, x, y - e)) / (2 * h)
        g = oracle.green(oracle.GRADY_X + j, k, x, y)
        assert np.abs(fd - g).max() <= 1e-7 * np.abs(g).max(), j
    assert oracle.green(oracle.GRADY_Y, k, x[:1], x[:1])[0] == 0.0  # r = 0


def test_double_layer_identity_first_order():
    bary, wq = I.rule_3pt()
    errs = []
    for level in (2, 3, 4):
        v, f = I.icosphere(level)
        P, W = oracle.quad_points(v, f, bary, wq)
        n = P / np.linalg.norm(P, axis=1)[:, None]
        rows = np.arange(0, P.shape[0], max(1, P.shape[0] // 300))
        D = sum(oracle.dense_rows(P, W, oracle.GRADY_X + j, 0.0, n[:, j].astype(np.complex128), rows)
                for j in range(3))
        errs.append(np.abs(D + 0.5).max())
    assert 1.6 <= errs[0] / errs[1] <= 2.4, errs
    assert 1.6 <= errs[1] / errs[2] <= 2.4, errs
    assert errs[2] < 1e-2
