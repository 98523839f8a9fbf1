"""Writes the closed-form reference values under tests/golden/ (run from the repository root:
python tests/golden/make_golden.py) from oracle/closed_forms.py (mpmath, 40 digits): values of
the formulas, independent of the C oracle and of the HIP library.

green_kernel_values.txt
    G(r) = e^{ikr} / (4 pi r) (the Helmholtz kernel of Section 5.2, eq. (Helmholtz), with the
    1/(4 pi) factor the acoustic example of Section 5.4 applies; k = 0 is the Laplace kernel).
sphere_single_layer_eigenvalues.txt
    eigenvalues of the single-layer operator of eq. (BEM) on the unit sphere for spherical
    harmonics of degree l: lambda_l(k) = i k j_l(k) h_l^(1)(k) (spherical Bessel and Hankel
    functions of the first kind), and 1 / (2l + 1) for the Laplace kernel.
"""
import os
import sys

import mpmath

sys.path.insert(0, os.path.join(os.path.dirname(os.path.abspath(__file__)), "..", ".."))
from oracle.closed_forms import green_exact as green, sphere_eig_exact as sphere_eig  # noqa: E402

HERE = os.path.dirname(os.path.abspath(__file__))


def main():
    with open(os.path.join(HERE, "green_kernel_values.txt"), "w") as fh:
        fh.write("# G(r) = exp(i k r) / (4 pi r): Section 5.2, eq. (Helmholtz), 1/(4 pi) as in Section 5.4\n")
        fh.write("# written by tests/golden/make_golden.py (mpmath, 40 digits)\n")
        fh.write("# r k re im\n")
        for r in ["0.001", "0.1", "1", "2.5", "10"]:
            for k in [0, 1, 5, 40, 120]:
                g = green(r, k)
                fh.write(f"{r} {k} {mpmath.nstr(mpmath.re(g), 25)} {mpmath.nstr(mpmath.im(g), 25)}\n")
    with open(os.path.join(HERE, "sphere_single_layer_eigenvalues.txt"), "w") as fh:
        fh.write("# single-layer eigenvalues on the unit sphere (operator of eq. (BEM), kernel of eq. (Helmholtz)):\n")
        fh.write("# lambda_l(k) = i k j_l(k) h_l^(1)(k); 1/(2l+1) for k = 0 (Laplace)\n")
        fh.write("# written by tests/golden/make_golden.py (mpmath, 40 digits)\n")
        fh.write("# k l re im\n")
        for k in [0, 5, 40]:
            for l in range(5):
                v = sphere_eig(l, k)
                fh.write(f"{k} {l} {mpmath.nstr(mpmath.re(v), 25)} {mpmath.nstr(mpmath.im(v), 25)}\n")


if __name__ == "__main__":
    main()
