"""Closed forms used to pin the oracle (test infrastructure only), evaluated with mpmath.

green_exact(r, k)
    G(r) = e^{ikr} / (4 pi r): the Helmholtz kernel (Section 5.2, eq. (Helmholtz)) with the
    1/(4 pi) factor of the acoustic example (Section 5.4); k = 0 gives the Laplace kernel.
sphere_eig_exact(l, k)
    eigenvalue of the single-layer operator of eq. (BEM) on the unit sphere for spherical
    harmonics of degree l: i k j_l(k) h_l^(1)(k) (spherical Bessel j_l, Hankel h_l^(1) = j_l + i
    y_l), and 1/(2l + 1) for k = 0.
"""
import mpmath

mpmath.mp.dps = 40


def green_exact(r, k):
    r = mpmath.mpf(r)
    return mpmath.exp(1j * mpmath.mpf(k) * r) / (4 * mpmath.pi * r)


def sphere_eig_exact(l, k):
    if k == 0:
        return mpmath.mpf(1) / (2 * l + 1)
    k = mpmath.mpf(k)
    half = mpmath.mpf(1) / 2
    j = mpmath.sqrt(mpmath.pi / (2 * k)) * mpmath.besselj(l + half, k)
    y = mpmath.sqrt(mpmath.pi / (2 * k)) * mpmath.bessely(l + half, k)
    return 1j * k * j * (j + 1j * y)
