"""Seeded synthetic inputs shared by the GPU path's tests, the oracle's tests and the bench.

This module holds input generation only: triangulated spheres and ellipsoids (the paper's BEM
workloads are generated sphere meshes, Section 5.4), the reference quadrature rule handed to
both implementations, and seeded complex vectors.  None of the method's arithmetic (quadrature
points, Green kernel, clustering, compression, products) lives here.

Readings of the paper used here:
  * sphere mesh: icosahedral refinement, each new edge midpoint projected to the unit sphere
    (the paper calls its mesher without stating the algorithm, Section 5.4);
  * arbitrary triangle counts: frequency-m geodesic icosphere with 20*m^2 triangles;
  * ellipsoids: the unit mesh scaled by the semi-axes (a, b, c), axis aligned, centred at 0;
  * 3-point rule: the interior degree-2 rule with barycentrics (2/3,1/6,1/6) and permutations,
    weight 1/3 each on the reference triangle (the paper uses 3 points per triangle, Section 5.3
    footnote and the acoustic example of Section 5.4, without naming the rule).
"""
from __future__ import annotations

import math

import numpy as np

__all__ = [
    "icosahedron", "icosphere", "geodesic_sphere", "ellipsoid", "rule_3pt", "rule_1pt",
    "complex_vector", "batch_ellipsoids", "mesh_stats",
]


def icosahedron():
    """Regular icosahedron on the unit sphere: 12 golden-ratio vertices, 20 outward faces."""
    t = (1.0 + math.sqrt(5.0)) / 2.0
    v = np.array([
        [-1, t, 0], [1, t, 0], [-1, -t, 0], [1, -t, 0],
        [0, -1, t], [0, 1, t], [0, -1, -t], [0, 1, -t],
        [t, 0, -1], [t, 0, 1], [-t, 0, -1], [-t, 0, 1],
    ], dtype=np.float64)
    v /= np.linalg.norm(v, axis=1, keepdims=True)
    f = np.array([
        [0, 11, 5], [0, 5, 1], [0, 1, 7], [0, 7, 10], [0, 10, 11],
        [1, 5, 9], [5, 11, 4], [11, 10, 2], [10, 7, 6], [7, 1, 8],
        [3, 9, 4], [3, 4, 2], [3, 2, 6], [3, 6, 8], [3, 8, 9],
        [4, 9, 5], [2, 4, 11], [6, 2, 10], [8, 6, 7], [9, 8, 1],
    ], dtype=np.int32)
    return v, _orient_outward(v, f)


def _orient_outward(v, f):
    a, b, c = v[f[:, 0]], v[f[:, 1]], v[f[:, 2]]
    n = np.cross(b - a, c - a)
    flip = np.einsum("ij,ij->i", n, a + b + c) < 0
    f = f.copy()
    f[flip] = f[flip][:, [0, 2, 1]]
    return f


def icosphere(level: int):
    """Unit icosphere after `level` recursive 4-splits (nt = 20*4^level, nv = 10*4^level + 2).

    Each split inserts the midpoint of every edge, projected to the unit sphere, and replaces a
    triangle (a, b, c) by (a, ab, ca), (ab, b, bc), (ca, bc, c), (ab, bc, ca).
    """
    v, f = icosahedron()
    for _ in range(level):
        e = np.concatenate([f[:, [0, 1]], f[:, [1, 2]], f[:, [2, 0]]], axis=0)
        e.sort(axis=1)
        uniq, inv = np.unique(e, axis=0, return_inverse=True)
        inv = inv.reshape(-1)
        mid = 0.5 * (v[uniq[:, 0]] + v[uniq[:, 1]])
        mid /= np.linalg.norm(mid, axis=1, keepdims=True)
        nt = f.shape[0]
        base = v.shape[0]
        ab = base + inv[0:nt]
        bc = base + inv[nt:2 * nt]
        ca = base + inv[2 * nt:3 * nt]
        a, b, c = f[:, 0], f[:, 1], f[:, 2]
        f = np.concatenate([
            np.stack([a, ab, ca], 1), np.stack([ab, b, bc], 1),
            np.stack([ca, bc, c], 1), np.stack([ab, bc, ca], 1),
        ], axis=0).astype(np.int32)
        v = np.concatenate([v, mid], axis=0)
    return np.ascontiguousarray(v), np.ascontiguousarray(f, dtype=np.int32)


def geodesic_sphere(m: int):
    """Frequency-m geodesic icosphere: every icosahedron face cut into an m-grid (20*m^2
    triangles, 10*m^2 + 2 vertices), grid points projected to the unit sphere.

    Grid points shared between faces are identified through a canonical key (the face corner
    ids with their integer barycentric weights), so shared vertices are computed once.
    """
    if m < 1:
        raise ValueError("m must be >= 1")
    v0, f0 = icosahedron()
    key_to_id = {}
    pts = []
    tris = []

    def vid(corners, weights):
        key = tuple(sorted((c, w) for c, w in zip(corners, weights) if w != 0))
        idx = key_to_id.get(key)
        if idx is None:
            p = np.zeros(3)
            for c, w in key:
                p = p + (w / m) * v0[c]
            idx = len(pts)
            key_to_id[key] = idx
            pts.append(p)
        return idx

    for a, b, c in f0:
        grid = {}
        for i in range(m + 1):
            for j in range(m + 1 - i):
                grid[i, j] = vid((a, b, c), (m - i - j, i, j))
        for i in range(m):
            for j in range(m - i):
                tris.append((grid[i, j], grid[i + 1, j], grid[i, j + 1]))
                if i + j < m - 1:
                    tris.append((grid[i + 1, j], grid[i + 1, j + 1], grid[i, j + 1]))
    v = np.array(pts, dtype=np.float64)
    v /= np.linalg.norm(v, axis=1, keepdims=True)
    f = _orient_outward(v, np.array(tris, dtype=np.int32))
    return np.ascontiguousarray(v), np.ascontiguousarray(f, dtype=np.int32)


def ellipsoid(vtx, axes):
    """Scale a unit-sphere mesh to the axis-aligned ellipsoid with semi-axes `axes`."""
    return np.ascontiguousarray(vtx * np.asarray(axes, dtype=np.float64)[None, :])


def rule_3pt():
    """Interior degree-2 rule on the reference triangle: barycentrics (n_q x 3), weights (n_q).

    The weights sum to 1, so a physical weight is the triangle area times the listed weight.
    """
    bary = np.array([[2 / 3, 1 / 6, 1 / 6], [1 / 6, 2 / 3, 1 / 6], [1 / 6, 1 / 6, 2 / 3]],
                    dtype=np.float64)
    w = np.full(3, 1.0 / 3.0)
    return bary, w


def rule_1pt():
    """Centroid rule (the default single point per simplex)."""
    return np.array([[1 / 3, 1 / 3, 1 / 3]], dtype=np.float64), np.ones(1)


def complex_vector(n: int, seed: int):
    """Seeded complex vector with N(0,1) real and imaginary parts (real part drawn first)."""
    rng = np.random.default_rng(seed)
    re = rng.standard_normal(n)
    im = rng.standard_normal(n)
    return re + 1j * im


def batch_ellipsoids(n_meshes: int = 64, seed: int = 0, t_min: int = 2000, t_max: int = 40000,
                     k_range=(2.0, 30.0), axis_range=(0.5, 2.0)):
    """Seeded batch of ellipsoid meshes: semi-axes ~ U[axis_range] independently, triangle
    count T ~ logU[t_min, t_max] realised as a frequency-m geodesic sphere with
    m = round(sqrt(T/20)), wavenumber k ~ U[k_range], vector seed 1000 + i.

    Returns a list of dicts {vtx, tri, k, axes, seed, m}.
    """
    rng = np.random.default_rng(seed)
    out = []
    for i in range(n_meshes):
        axes = rng.uniform(axis_range[0], axis_range[1], size=3)
        t = math.exp(rng.uniform(math.log(t_min), math.log(t_max)))
        k = rng.uniform(k_range[0], k_range[1])
        m = max(1, int(round(math.sqrt(t / 20.0))))
        out.append({"axes": axes, "m": m, "k": float(k), "seed": 1000 + i})
    return out


def batch_mesh(desc):
    """Materialise one mesh of `batch_ellipsoids`."""
    v, f = geodesic_sphere(desc["m"])
    return ellipsoid(v, desc["axes"]), f


def mesh_stats(vtx, tri):
    """Edge lengths (min, mean, max) and the polyhedral surface area."""
    a, b, c = vtx[tri[:, 0]], vtx[tri[:, 1]], vtx[tri[:, 2]]
    e = np.concatenate([np.linalg.norm(b - a, axis=1), np.linalg.norm(c - b, axis=1),
                        np.linalg.norm(a - c, axis=1)])
    area = 0.5 * np.linalg.norm(np.cross(b - a, c - a), axis=1).sum()
    return float(e.min()), float(e.mean()), float(e.max()), float(area)
