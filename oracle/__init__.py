"""CPU FP64 oracle for the H-matrix BEM hot path -- test infrastructure only.

Only the tests, the package smoke check and the bench's CPU-baseline leg use this module.  It
loads ``liboracle_hmo.so`` built from ``hmo.c`` (plain C, libm, OpenMP, contraction off) and
shares no code with the HIP library.  ``mlp.py`` holds the numpy FP64 reference of the rank MLP.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "liboracle_hmo.so")

LAPLACE, HELMHOLTZ, POLY2 = 0, 1, 99
GRADY_X, GRADY_Y, GRADY_Z = 2, 3, 4


def build(force: bool = True) -> str:
    """Compile hmo.c with gcc (-O2, OpenMP, no FP contraction)."""
    src = os.path.join(_HERE, "hmo.c")
    if force or not os.path.exists(LIB_PATH) or os.path.getmtime(LIB_PATH) < os.path.getmtime(src):
        tmp = LIB_PATH + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-std=c99", "-fPIC", "-shared", "-fopenmp",
                               "-ffp-contract=off", "-fno-fast-math", "-Wall", "-o", tmp, src, "-lm"])
        os.replace(tmp, LIB_PATH)
    return LIB_PATH


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            build()
        L = C.CDLL(LIB_PATH)
        P = C.c_void_p
        i64, i32, f64 = C.c_int64, C.c_int32, C.c_double
        L.hmo_max_threads.restype = C.c_int
        L.hmo_quad_points.argtypes = [P, i64, P, i64, P, P, i32, P, P, P, P]
        L.hmo_quad_points.restype = C.c_int
        L.hmo_green.argtypes = [i32, f64, P, P, i64, P]
        L.hmo_dense_rows.argtypes = [P, P, P, P, i64, i32, f64, P, P, i64, P, i32]
        L.hmo_aca_dense.argtypes = [P, i64, i64, f64, i64, P, P, i64, P]
        L.hmo_aca_dense.restype = C.c_int
        L.hmo_hbuild.argtypes = [P, P, P, P, i64, i32, f64, i32, f64, f64, i32, i64, P, P, i32, P,
                                 f64]
        L.hmo_tri_moments.argtypes = [P, P, P]
        L.hmo_tri_lagrange.argtypes = [P, P, P, P]
        L.hmo_reg_apply.argtypes = [P, P, P, P, i64, P, P, i64, i32, P, f64, P, P, i64, P, i32]
        L.hmo_rect_rows.argtypes = [P, P, P, i64, P, P, P, P, i64, i32, f64, P, P, i64, P, i32]
        L.hmo_dense_matrix.argtypes = [P, P, P, P, i64, i32, f64, P]
        L.hmo_reg_matrix.argtypes = [P, P, P, P, i64, P, P, i64, i32, P, f64, P, i32]
        L.hmo_hbuild.restype = P
        L.hmo_hmatvec.argtypes = [P, P, P]
        L.hmo_hinfo.argtypes = [P, P]
        L.hmo_htree.argtypes = [P, P, P, P, P, P, P, P]
        L.hmo_hblocks.argtypes = [P, P, P, P]
        L.hmo_hfar_factors.argtypes = [P, i64, P, P]
        L.hmo_hfar_factors.restype = i64
        L.hmo_hfree.argtypes = [P]
        _lib = L
    return _lib


def _p(a):
    return a.ctypes.data_as(C.c_void_p)


def max_threads() -> int:
    return int(lib().hmo_max_threads())


def quad_points(vtx, tri, bary, what):
    """Quadrature points (M x 3) and weights (M), M = n_q * n_tri, point m = n_q * t + q."""
    vtx = np.ascontiguousarray(vtx, np.float64)
    tri = np.ascontiguousarray(tri, np.int32)
    bary = np.ascontiguousarray(bary, np.float64)
    what = np.ascontiguousarray(what, np.float64)
    nq = bary.shape[0]
    M = nq * tri.shape[0]
    X, Y, Z, W = (np.empty(M) for _ in range(4))
    rc = lib().hmo_quad_points(_p(vtx), vtx.shape[0], _p(tri), tri.shape[0], _p(bary), _p(what), nq,
                               _p(X), _p(Y), _p(Z), _p(W))
    if rc != 0:
        raise ValueError("triangle index out of range")
    return np.stack([X, Y, Z], 1), W


def green(kern, k, x, y):
    """G(x_i, y_i) for paired rows of x, y (n x 3)."""
    x = np.ascontiguousarray(x, np.float64).reshape(-1, 3)
    y = np.ascontiguousarray(y, np.float64).reshape(-1, 3)
    out = np.empty(x.shape[0], np.complex128)
    lib().hmo_green(kern, k, _p(x), _p(y), x.shape[0], _p(out))
    return out


def _soa(pts):
    pts = np.asarray(pts, np.float64)
    return [np.ascontiguousarray(pts[:, d]) for d in range(3)]


def dense_rows(pts, w, kern, k, x, rows=None, nthreads=0):
    """Rows of y = K x, K_il = G(x_i, x_l) w_l (r = 0 pairs give 0); all rows when rows is None."""
    X, Y, Z = _soa(pts)
    w = np.ascontiguousarray(w, np.float64)
    x = np.ascontiguousarray(x, np.complex128)
    M = X.shape[0]
    if rows is None:
        nr, rp = M, None
    else:
        rows = np.ascontiguousarray(rows, np.int64)
        nr, rp = rows.shape[0], _p(rows)
    y = np.empty(nr, np.complex128)
    lib().hmo_dense_rows(_p(X), _p(Y), _p(Z), _p(w), M, kern, k, _p(x), rp, nr, _p(y), nthreads)
    return y


def dense_matvec(pts, w, kern, k, x, nthreads=0):
    return dense_rows(pts, w, kern, k, x, None, nthreads)


def aca_dense(A, tol, rcap=None):
    """Reference ACA of a dense matrix: returns (U, V, converged) with A ~ U @ V.T."""
    A = np.ascontiguousarray(A, np.complex128)
    m, n = A.shape
    if rcap is None:
        rcap = (m * n) // (m + n)
    cap = max(1, min(m, n, rcap))
    U = np.zeros((cap, m), np.complex128)
    V = np.zeros((cap, n), np.complex128)
    r = C.c_int64(0)
    rc = lib().hmo_aca_dense(_p(A), m, n, tol, rcap, _p(U), _p(V), cap, C.byref(r))
    if rc < 0:
        raise RuntimeError("rank above capacity")
    k = r.value
    return U[:k].T.copy(), V[:k].T.copy(), bool(rc)


def rect_matvec(targets, pts, w, kern, k, x, rows=None, nthreads=0):
    """y = K x with K_il = G(t_i, x_l) w_l: the source quadrature's potential at other target
    points (Section 5.1); rows selects target rows (all when None)."""
    TX, TY, TZ = _soa(targets)
    X, Y, Z = _soa(pts)
    w = np.ascontiguousarray(w, np.float64)
    x = np.ascontiguousarray(x, np.complex128)
    if rows is None:
        rp, nr = None, TX.shape[0]
    else:
        rows = np.ascontiguousarray(np.atleast_1d(rows), np.int64)
        rp, nr = _p(rows), rows.shape[0]
    y = np.empty(nr, np.complex128)
    lib().hmo_rect_rows(_p(TX), _p(TY), _p(TZ), TX.shape[0], _p(X), _p(Y), _p(Z), _p(w), X.shape[0],
                        kern, k, _p(x), rp, nr, _p(y), nthreads)
    return y


# ------------------------------------------------------------------ Galerkin P1 (O9)
def p1_matrix(vtx, tri, bary):
    """Phi (M x nv): Phi[nq t + q, v] = lambda_v(point q of triangle t), the P1 hat function of
    vertex v at the quadrature points (eq. (BEM): the basis functions evaluated at the points)."""
    tri = np.asarray(tri)
    B = np.asarray(bary, np.float64).reshape(-1, 3)
    nq = B.shape[0]
    Phi = np.zeros((nq * tri.shape[0], np.asarray(vtx).shape[0]))
    for t in range(tri.shape[0]):
        for q in range(nq):
            for j in range(3):
                Phi[nq * t + q, tri[t, j]] += B[q, j]
    return Phi


def dense_matrix(pts, w, kern, k):
    """The point operator K = G W_y as an M x M matrix (G := 0 at r = 0)."""
    X, Y, Z = _soa(pts)
    w = np.ascontiguousarray(w, np.float64)
    M = X.shape[0]
    K = np.empty((M, M), np.complex128)
    lib().hmo_dense_matrix(_p(X), _p(Y), _p(Z), _p(w), M, kern, k, _p(K))
    return K


def reg_matrix(pts, w, vtx, tri, bary, alpha, nthreads=0):
    """The singular correction of every close pair as an M x M (real) matrix."""
    X, Y, Z = _soa(pts)
    w = np.ascontiguousarray(w, np.float64)
    vtx = np.ascontiguousarray(vtx, np.float64)
    tri = np.ascontiguousarray(tri, np.int32)
    lag = lagrange_matrix(bary)
    M = X.shape[0]
    C = np.empty((M, M))
    lib().hmo_reg_matrix(_p(X), _p(Y), _p(Z), _p(w), M, _p(vtx), _p(tri), tri.shape[0], 3, _p(lag),
                         alpha, _p(C), nthreads)
    return C


def galerkin_matrix(vtx, tri, bary, wq, kern, k, reg_radius=None):
    """A = Phi^T W_x K Phi (eq. (BEM) with P1 test and trial functions on the mesh), K the point
    operator, plus the singular correction when reg_radius is given."""
    P, W = quad_points(vtx, tri, bary, wq)
    K = dense_matrix(P, W, kern, k)
    if reg_radius is not None:
        K = K + reg_matrix(P, W, vtx, tri, bary, reg_radius)
    Phi = p1_matrix(vtx, tri, bary)
    return Phi.T @ (W[:, None] * K) @ Phi, Phi, P, W


# ------------------------------------------------------------------ singular correction (O7)
def lagrange_matrix(bary):
    """Coefficients of the linear functions through a 3-point rule (Section 5.2 reading): row q
    holds c_qi with L_q = sum_i c_qi lambda_i and L_q(point p) = delta_qp, i.e. (B^-1)^T for B the
    rule's barycentric coordinates (one point per row)."""
    B = np.asarray(bary, np.float64).reshape(-1, 3)
    if B.shape[0] != 3:
        raise ValueError("the correction needs a 3-point rule")
    return np.ascontiguousarray(np.linalg.inv(B).T)


def tri_moments(x, tv):
    """(I1, Irho): int_T 1/|x-y| dy and int_T (y - rho)/|x-y| dy, rho the projection of x on
    the plane of T = tv (3 x 3, one vertex per row)."""
    x = np.ascontiguousarray(x, np.float64)
    tv = np.ascontiguousarray(tv, np.float64)
    out = np.empty(4)
    lib().hmo_tri_moments(_p(x), _p(tv), _p(out))
    return out[0], out[1:].copy()


def tri_lagrange(x, tv, lag):
    """int_T L_q(y)/|x-y| dy for q = 0, 1, 2 (L_q = sum_i lag[q, i] lambda_i)."""
    x = np.ascontiguousarray(x, np.float64)
    tv = np.ascontiguousarray(tv, np.float64)
    lag = np.ascontiguousarray(lag, np.float64)
    out = np.empty(3)
    lib().hmo_tri_lagrange(_p(x), _p(tv), _p(lag), _p(out))
    return out


def reg_apply(pts, w, vtx, tri, bary, alpha, x, rows=None, nthreads=0):
    """(C x)[rows]: the singular correction of every close pair applied to x (points of the
    3-point rule bary on mesh (vtx, tri), triangle-major); all rows when rows is None."""
    X, Y, Z = _soa(pts)
    w = np.ascontiguousarray(w, np.float64)
    vtx = np.ascontiguousarray(vtx, np.float64)
    tri = np.ascontiguousarray(tri, np.int32)
    lag = lagrange_matrix(bary)
    x = np.ascontiguousarray(x, np.complex128)
    if rows is None:
        rp, nr = None, X.shape[0]
    else:
        rows = np.ascontiguousarray(rows, np.int64)
        rp, nr = _p(rows), rows.shape[0]
    y = np.empty(nr, np.complex128)
    lib().hmo_reg_apply(_p(X), _p(Y), _p(Z), _p(w), X.shape[0], _p(vtx), _p(tri), tri.shape[0], 3,
                        _p(lag), alpha, _p(x), rp, nr, _p(y), nthreads)
    return y


def reg_dense_matvec(pts, w, kern, k, vtx, tri, bary, alpha, x, nthreads=0):
    """The regularized dense product: K x plus the correction of every close pair."""
    return dense_matvec(pts, w, kern, k, x, nthreads) + reg_apply(pts, w, vtx, tri, bary, alpha, x,
                                                                  nthreads=nthreads)


class HMatrix:
    """Oracle H-matrix: cluster tree, block tree, dense near blocks, reference ACA far blocks.

    mesh = (vtx, tri, bary) and reg_radius = alpha add the singular correction to the close
    pairs of the near blocks."""

    def __init__(self, pts, w, kern, k, leaf=64, eta=1.5, tol=1e-3, nthreads=0, max_mn=0, mesh=None,
                 reg_radius=2.0):
        X, Y, Z = _soa(pts)
        w = np.ascontiguousarray(w, np.float64)
        self.M = X.shape[0]
        vtx = tri = lag = None
        if mesh is not None:
            vtx = np.ascontiguousarray(mesh[0], np.float64)
            tri = np.ascontiguousarray(mesh[1], np.int32)
            lag = lagrange_matrix(mesh[2])
        self._h = lib().hmo_hbuild(_p(X), _p(Y), _p(Z), _p(w), self.M, kern, k, leaf, eta, tol, nthreads,
                                   max_mn, None if vtx is None else _p(vtx),
                                   None if tri is None else _p(tri), 3,
                                   None if lag is None else _p(lag), float(reg_radius))
        info = np.zeros(9, np.int64)
        lib().hmo_hinfo(self._h, _p(info))
        keys = ["n_nodes", "n_near", "n_far", "s_near", "s_far", "n_dense_far", "s_dense_far",
                "max_rank", "sum_rank"]
        self.info = {kk: int(v) for kk, v in zip(keys, info)}

    def matvec(self, x):
        x = np.ascontiguousarray(x, np.complex128)
        y = np.empty(self.M, np.complex128)
        lib().hmo_hmatvec(self._h, _p(x), _p(y))
        return y

    def tree(self):
        n = self.info["n_nodes"]
        perm = np.empty(self.M, np.int32)
        b, e = np.empty(n, np.int64), np.empty(n, np.int64)
        lev, c0, c1 = (np.empty(n, np.int32) for _ in range(3))
        box = np.empty((n, 6))
        lib().hmo_htree(self._h, _p(perm), _p(b), _p(e), _p(lev), _p(c0), _p(c1), _p(box))
        return {"perm": perm, "begin": b, "end": e, "level": lev, "child0": c0, "child1": c1, "box": box}

    def blocks(self):
        nn, nf = self.info["n_near"], self.info["n_far"]
        nearR = np.empty((nn, 4), np.int64)
        farR = np.empty((nf, 4), np.int64)
        ranks = np.empty(nf, np.int64)
        lib().hmo_hblocks(self._h, _p(nearR), _p(farR), _p(ranks))
        return nearR, farR, ranks

    def far_factors(self, b, m, n, rank):
        U = np.empty((max(rank, 1), m), np.complex128)
        V = np.empty((max(rank, 1), n), np.complex128)
        r = lib().hmo_hfar_factors(self._h, b, _p(U), _p(V))
        if r < 0:
            return None
        return U[:r].T.copy(), V[:r].T.copy()

    def close(self):
        if self._h:
            lib().hmo_hfree(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
