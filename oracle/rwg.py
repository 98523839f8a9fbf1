"""CPU FP64 oracle of the electromagnetic boundary integral equations (Section 5.5: EFIE, MFIE and
CFIE on lowest-order Raviart-Thomas / RWG elements, Section 4) -- test infrastructure only.

Only the tests and the bench's CPU-baseline leg use this module.  Dense matrices throughout: the
point operators come from the oracle's C kernels (``dense_matrix``, ``reg_matrix``), the RWG
functions from their definition, evaluated at the quadrature points.

Conventions (readings of Section 5.5, each written out here):
  * one unknown per edge of a closed, consistently oriented triangle mesh; edges numbered in
    increasing (a, b), a < b their vertex numbers;
  * on triangle t the edge opposite local vertex j carries psi(y) = s l / (2 A) (y - p_j), l the
    edge length, A the area, p_j the opposite vertex, s = +1 on the triangle whose own vertex
    order runs a -> b along the edge and -1 on the other; div psi = s l / A;
  * n the unit normal (v1 - v0) x (v2 - v0) / |.| of each triangle (outward for an outward
    oriented mesh);
  * EFIE matrix T = i k sum_d Psi_d^T W K Psi_d - (i / k) D^T W K D, K = G W the single-layer
    point operator (G = e^{ikr} / (4 pi r)) with the singular correction when asked;
  * MFIE matrix (1/2) Id - NxK with NxK_ij = int int (n x psi_i)(x) . (grad_y G(x, y) x psi_j(y)),
    Id the RWG mass matrix;
  * CFIE matrix -beta T + (1 - beta) ((1/2) Id - NxK), right-hand side
    beta <psi_i, E_inc> - (1 - beta) <n x psi_i, H_inc>;
  * the surface current J = sum_e x_e psi_e radiates the far field
    F(u) = i k / (4 pi) (I - u u^T) int J(y) e^{-i k u.y} dy (E_s ~ F e^{ikR} / R).
"""
from __future__ import annotations

import numpy as np

from . import GRADY_X, HELMHOLTZ, dense_matrix, quad_points, reg_matrix


def rwg_edges(tri):
    """(edges E x 2 with a < b, tedge nt x 3 = edge opposite local vertex j, tsign nt x 3 = +-1).
    Raises ValueError unless every edge is shared by exactly two triangles that run along it in
    opposite directions (a closed, consistently oriented mesh)."""
    tri = np.asarray(tri, np.int64)
    nt = tri.shape[0]
    a = np.stack([tri[:, (j + 1) % 3] for j in range(3)], 1)  # edge opposite j runs a -> b
    b = np.stack([tri[:, (j + 2) % 3] for j in range(3)], 1)
    lo, hi = np.minimum(a, b), np.maximum(a, b)
    keys = np.stack([lo.ravel(), hi.ravel()], 1)
    edges, inv, counts = np.unique(keys, axis=0, return_inverse=True, return_counts=True)
    inv = inv.ravel()
    if (counts != 2).any():
        raise ValueError("every edge must belong to exactly two triangles")
    sign = np.where(a < b, 1, -1).ravel()
    tot = np.zeros(edges.shape[0], np.int64)
    np.add.at(tot, inv, sign)
    if (tot != 0).any():
        raise ValueError("the two triangles of an edge must run along it in opposite directions")
    return edges, inv.reshape(nt, 3), sign.reshape(nt, 3)


def rwg_matrices(vtx, tri, bary):
    """(Psi 3 x M x E, Div M x E, NxPsi 3 x M x E): the RWG functions, their surface divergence
    and n x psi at the quadrature points (point nq t + q of triangle t)."""
    vtx = np.asarray(vtx, np.float64)
    tri = np.asarray(tri, np.int64)
    B = np.asarray(bary, np.float64).reshape(-1, 3)
    nq, nt = B.shape[0], tri.shape[0]
    edges, tedge, tsign = rwg_edges(tri)
    E, M = edges.shape[0], nq * nt
    Psi = np.zeros((3, M, E))
    Div = np.zeros((M, E))
    NxPsi = np.zeros((3, M, E))
    for t in range(nt):
        V = vtx[tri[t]]
        cr = np.cross(V[1] - V[0], V[2] - V[0])
        area = 0.5 * np.linalg.norm(cr)
        n = cr / np.linalg.norm(cr)
        for q in range(nq):
            y = B[q] @ V
            row = nq * t + q
            for j in range(3):
                e = tedge[t, j]
                ln = np.linalg.norm(V[(j + 2) % 3] - V[(j + 1) % 3])
                c = tsign[t, j] * ln / (2.0 * area)
                psi = c * (y - V[j])
                Psi[:, row, e] += psi
                Div[row, e] += 2.0 * c
                NxPsi[:, row, e] += np.cross(n, psi)
    return Psi, Div, NxPsi


def _sandwich(A, W, K, B):
    return A.T @ (W[:, None] * (K @ B))


def em_matrices(vtx, tri, bary, wq, k, reg_radius=None, parts=("T", "NxK", "Id")):
    """Dense EFIE matrix T, MFIE double-layer part NxK and RWG mass matrix Id (E x E each) of the
    mesh, plus the RWG matrices and the points: (dict, Psi, Div, NxPsi, P, W)."""
    P, W = quad_points(vtx, tri, bary, wq)
    Psi, Div, NxPsi = rwg_matrices(vtx, tri, bary)
    out = {}
    if "T" in parts:
        K = dense_matrix(P, W, HELMHOLTZ, k)
        if reg_radius is not None:
            K = K + reg_matrix(P, W, vtx, tri, bary, reg_radius)
        out["T"] = 1j * k * sum(_sandwich(Psi[d], W, K, Psi[d]) for d in range(3)) \
            - (1j / k) * _sandwich(Div, W, K, Div)
        del K
    if "NxK" in parts:
        G = [dense_matrix(P, W, GRADY_X + d, k) for d in range(3)]
        NxK = 0
        for e in range(3):
            c = G[(e + 1) % 3] @ Psi[(e + 2) % 3] - G[(e + 2) % 3] @ Psi[(e + 1) % 3]
            NxK = NxK + NxPsi[e].T @ (W[:, None] * c)
        out["NxK"] = NxK
    if "Id" in parts:
        out["Id"] = sum(Psi[d].T @ (W[:, None] * Psi[d]) for d in range(3))
    return out, Psi, Div, NxPsi, P, W


def cfie_matrix(mats, beta):
    """-beta T + (1 - beta) ((1/2) Id - NxK); beta = 1 gives -T (the EFIE), beta = 0 the MFIE."""
    A = 0
    if beta != 0:
        A = A - beta * mats["T"]
    if beta != 1:
        A = A + (1 - beta) * (0.5 * mats["Id"] - mats["NxK"])
    return A


def plane_wave(P, k, d, pol):
    """E = pol e^{ik d.x} and H = (d x pol) e^{ik d.x} at the points (3 x M complex each)."""
    ph = np.exp(1j * k * (P @ np.asarray(d, np.float64)))
    Ei = np.asarray(pol, np.float64)[:, None] * ph[None, :]
    Hi = np.cross(d, pol)[:, None] * ph[None, :]
    return Ei, Hi


def cfie_rhs(Psi, NxPsi, W, Ei, Hi, beta):
    """beta <psi_i, E_inc> - (1 - beta) <n x psi_i, H_inc> with the point quadrature."""
    b = beta * sum(Psi[d].T @ (W * Ei[d]) for d in range(3))
    b = b - (1 - beta) * sum(NxPsi[d].T @ (W * Hi[d]) for d in range(3))
    return b


def far_field(Psi, P, W, x, k, dirs):
    """F(u) (n_dirs x 3) of the current J = sum_e x_e psi_e, u the unit directions."""
    J = np.stack([Psi[d] @ x for d in range(3)], 1)  # M x 3
    u = np.asarray(dirs, np.float64)
    ph = np.exp(-1j * k * (u @ P.T)) * W[None, :]  # n_dirs x M
    Jh = ph @ J
    Jh = Jh - u * (u * Jh).sum(1, keepdims=True)
    return 1j * k / (4 * np.pi) * Jh
