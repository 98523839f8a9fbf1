"""Thin ctypes binding of libhmx (include/hmx.h): argument marshalling only.

Device memory and streams come from PyTorch (ROCm); every step of the operator runs in the
HIP kernels of libhmx.so.  Importing this module loads the library and raises ImportError when
it has not been built (``python -m paper_1804_00995_amd.build``): there is no fallback path.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np
# torch ships the HIP runtime it was built with; loading it first makes libhmx.so resolve its
# libamdhip64.so.7 dependency to that same runtime, so device pointers and streams are shared.
import torch  # noqa: F401

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libhmx.so")

LAPLACE, HELMHOLTZ, TEST_POLY2 = 0, 1, 99
GRADY_X, GRADY_Y, GRADY_Z = 2, 3, 4
FP64, FP32_MIXED = 0, 1
RANK_ADAPTIVE, RANK_LEARNED = 0, 1

OK, EINVAL, ENOMEM, EDEVICE, EUNSUPPORTED, EINTERNAL = 0, -1, -2, -3, -4, -5
STATIC_WORK_BYTES = 64 << 20  # HMX_STATIC_WORK_BYTES: scratch of hmx_matvec_multi_static

if not os.path.exists(LIB_PATH):
    raise ImportError(f"{LIB_PATH} is missing: build it with `python -m paper_1804_00995_amd.build`")
_lib = C.CDLL(LIB_PATH)


class Params(C.Structure):
    _fields_ = [
        ("struct_size", C.c_int32),
        ("tol", C.c_double),
        ("leaf_size", C.c_int32),
        ("eta", C.c_double),
        ("precision", C.c_int32),
        ("rank_model", C.c_int32),
        ("initial_rank", C.c_int32),
        ("force_pred_scale", C.c_double),
        ("force_rank_cap", C.c_int32),
        ("pool_limit_bytes", C.c_int64),
        ("aca_big_mn", C.c_int32),
        ("aca_gram_min_mn", C.c_int32),
        ("aca_serial", C.c_int32),
        ("aca_mid_threads", C.c_int32),
        ("aca_arena", C.c_int32),
        ("row_shares", C.c_int32),
        ("row_share", C.c_int32),
        ("force_pool_bytes", C.c_int64),
        ("max_far_mn", C.c_int32),
        ("aca_big_threads", C.c_int32),
        ("aca_small_mn", C.c_int32),
        ("aca_wave", C.c_int32),
        ("regularize", C.c_int32),
        ("reg_radius", C.c_double),
        ("near_mode", C.c_int32),
        ("force_block_cap", C.c_int64),
    ]


class Info(C.Structure):
    _fields_ = [(n, C.c_int64) for n in (
        "n_points", "n_nodes", "n_leaves", "n_near", "n_far", "near_entries", "far_entries",
        "dense_far", "dense_far_entries", "max_rank", "sum_rank", "overflow_blocks", "bytes")] + [
        ("precision", C.c_int32), ("is_dense", C.c_int32)] + [
        (n, C.c_double) for n in ("t_tree_ms", "t_blocks_ms", "t_near_ms", "t_aca_ms", "t_total_ms")] + [
        ("kernel_evals", C.c_int64), ("factor_bytes", C.c_int64), ("predicted_entries", C.c_int64),
        ("aca_blocks", C.c_int64 * 4), ("aca_ms", C.c_double * 4), ("aca_bytes", C.c_int64 * 4),
        ("aca_rounds", C.c_int32), ("row_begin", C.c_int64), ("row_end", C.c_int64),
        ("n_rows", C.c_int64), ("n_cols", C.c_int64), ("pool_reserved_bytes", C.c_int64)]

    def as_dict(self):
        d = {}
        for name, _ in self._fields_:
            v = getattr(self, name)
            d[name] = list(v) if isinstance(v, C.Array) else v
        return d


_P, _i64, _i32, _f64 = C.c_void_p, C.c_int64, C.c_int32, C.c_double
_sig = {
    "hmx_params_default": [C.POINTER(Params)],
    "hmx_quad_points": [_P, _i64, _P, _i64, _P, _P, _i32, _P, _P],
    "hmx_build": [_P, _i64, _P, _i64, _P, _P, _i32, _i32, _f64, C.POINTER(Params), _P, C.POINTER(_P)],
    "hmx_build_points": [_P, _i64, _i32, _f64, C.POINTER(Params), _P, C.POINTER(_P)],
    "hmx_build_rect": [_P, _i64, _P, _i64, _i32, _f64, C.POINTER(Params), _P, C.POINTER(_P)],
    "hmx_p1_create": [_P, _P, _i64, _P, _i64, _P, _P, _i32, _P, C.POINTER(_P)],
    "hmx_p1_interp": [_P, _P, _P, _P],
    "hmx_p1_project": [_P, _P, _P, _P],
    "hmx_galerkin_matvec": [_P, _P, _P, _P],
    "hmx_gmres": [_P, _P, _P, _i32, _i32, _f64, _P, C.POINTER(_i32), C.POINTER(_f64)],
    "hmx_rwg_create": [_P, _P, _P, _P, _P, _i64, _P, _i64, _P, _P, _i32, _P, C.POINTER(_P)],
    "hmx_rwg_n_edges": [_P, C.POINTER(_i64)],
    "hmx_rwg_edges": [_P, _P, _P],
    "hmx_rwg_interp": [_P, _P, _P, _P],
    "hmx_rwg_rhs": [_P, _f64, _P, _P, _P, _P],
    "hmx_cfie_matvec": [_P, _f64, _P, _P, _P],
    "hmx_cfie_gmres": [_P, _f64, _P, _P, _i32, _i32, _f64, _P, C.POINTER(_i32), C.POINTER(_f64)],
    "hmx_matvec": [_P, _P, _P, _P],
    "hmx_matvec_multi_work_bytes": [_P, C.POINTER(C.c_size_t)],
    "hmx_matvec_multi": [_P, _i32, C.POINTER(_P), C.POINTER(_P), _P, _P],
    "hmx_matvec_multi_static": [_P, _i32, C.POINTER(_P), C.POINTER(_P), _P],
    "hmx_info": [_P, C.POINTER(Info)],
    "hmx_export_tree": [_P, _P, _P, _P, _P, _P, _P, _P],
    "hmx_export_blocks": [_P, _P, _P, _P],
    "hmx_export_far": [_P, _i64, _P, _P, _P],
    "hmx_far_features": [_P, _P],
    "hmx_mlp_predict": [_P, _P, _P, _i64, _P, _P],
    "hmx_mlp_loss_grad": [_P, _P, _P, _i64, _P, _P, _P],
    "hmx_mlp_train": [_P, _P, _P, _i64, _i32, _i32, C.c_float, _P, _P],
    "hmx_set_rank_model": [_P, _P, C.c_float, C.c_float],
    "hmx_build_batch": [_P, _i32, _P, _P, _i32, _i32, C.POINTER(Params), _P, C.POINTER(_P)],
    "hmx_mesh_offsets": [_P, _P, _i32, C.POINTER(_i32)],
    "hmx_graph_create": [_P, _P, _P, C.POINTER(_P)],
    "hmx_graph_launch": [_P, _i32, _P],
    "hmx_import_far": [_P, _P, _P, _P],
    "hmx_autotune": [_P, _i64, _i32, _f64, C.POINTER(Params), C.c_char_p, _P, C.POINTER(Params),
                     C.POINTER(_f64)],
    "hmx_autotune_batch": [_P, _i32, _P, _P, _i32, _i32, C.POINTER(Params), C.c_char_p, _P,
                           C.POINTER(Params), C.POINTER(_f64)],
}
MLP_NPARAMS = 4545
for _name, _args in _sig.items():
    _f = getattr(_lib, _name)
    _f.argtypes = _args
    _f.restype = C.c_int
_lib.hmx_destroy.argtypes = [_P]
_lib.hmx_destroy.restype = None
_lib.hmx_last_error.argtypes = []
_lib.hmx_last_error.restype = C.c_char_p
_lib.hmx_release_cache.argtypes = []
_lib.hmx_release_cache.restype = None
_lib.hmx_graph_destroy.argtypes = [_P]
_lib.hmx_graph_destroy.restype = None
_lib.hmx_p1_destroy.argtypes = [_P]
_lib.hmx_p1_destroy.restype = None
_lib.hmx_rwg_destroy.argtypes = [_P]
_lib.hmx_rwg_destroy.restype = None

EXPORTED = sorted(list(_sig) + ["hmx_destroy", "hmx_last_error", "hmx_release_cache",
                                "hmx_graph_destroy", "hmx_p1_destroy", "hmx_rwg_destroy"])


class Mesh(C.Structure):
    _fields_ = [("vtx", _P), ("n_vtx", _i64), ("tri", _P), ("n_tri", _i64), ("k", _f64)]


def release_cache():
    """Return the library's cached free device blocks to the HIP runtime."""
    _lib.hmx_release_cache()


class HmxError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"hmx error {code}: {msg}")
        self.code = code


def _check(rc):
    if rc != OK:
        raise HmxError(rc, _lib.hmx_last_error().decode())


def params(**kw) -> Params:
    """Default parameters with keyword overrides (tol, leaf_size, eta, precision, ...)."""
    p = Params()
    _check(_lib.hmx_params_default(C.byref(p)))
    for k, v in kw.items():
        if not hasattr(p, k):
            raise TypeError(f"unknown parameter {k}")
        setattr(p, k, v)
    return p


def _stream_ptr(stream):
    if stream is None:
        import torch
        return C.c_void_p(torch.cuda.current_stream().cuda_stream)
    if isinstance(stream, int):
        return C.c_void_p(stream)
    return C.c_void_p(stream.cuda_stream)


def _dev(t, dtype, name):
    import torch
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise TypeError(f"{name} must be a device tensor")
    if t.dtype != dtype:
        raise TypeError(f"{name} must be {dtype}, got {t.dtype}")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    return C.c_void_p(t.data_ptr())


def _host_rule(bary, w):
    bary = np.ascontiguousarray(bary, np.float64).reshape(-1, 3)
    w = np.ascontiguousarray(w, np.float64).reshape(-1)
    if bary.shape[0] != w.shape[0]:
        raise ValueError("rule barycentrics and weights differ in length")
    return bary, w


def quad_points(vtx, tri, bary, w, stream=None):
    """Quadrature points and weights on the device: returns a (4, M) float64 tensor X, Y, Z, W."""
    import torch
    bary, w = _host_rule(bary, w)
    nq = bary.shape[0]
    M = tri.shape[0] * nq
    out = torch.empty((4, M), dtype=torch.float64, device=vtx.device)
    _check(_lib.hmx_quad_points(_dev(vtx, torch.float64, "vtx"), vtx.shape[0],
                                _dev(tri, torch.int32, "tri"), tri.shape[0],
                                bary.ctypes.data_as(_P), w.ctypes.data_as(_P), nq,
                                C.c_void_p(out.data_ptr()), _stream_ptr(stream)))
    return out


class Operator:
    """A built operator K = G W_y (dense or H-matrix), applied with `matvec` or `@`."""

    def __init__(self, handle, precision):
        self._h = handle
        self.precision = precision
        self.info = self._info()
        self.M = self.info["n_points"]
        self.rows, self.cols = self.info["n_rows"], self.info["n_cols"]

    @property
    def cdtype(self):
        import torch
        return torch.complex128 if self.precision == FP64 else torch.complex64

    def _info(self):
        i = Info()
        _check(_lib.hmx_info(self._h, C.byref(i)))
        return i.as_dict()

    def matvec(self, x, y=None, stream=None):
        import torch
        if x.shape != (self.cols,):
            raise ValueError(f"x must have shape ({self.cols},)")
        if y is None:
            y = torch.empty(self.rows, dtype=x.dtype, device=x.device)
        elif y.shape != (self.rows,):
            raise ValueError(f"y must have shape ({self.rows},)")
        _check(_lib.hmx_matvec(self._h, _dev(x, self.cdtype, "x"), _dev(y, self.cdtype, "y"),
                               _stream_ptr(stream)))
        return y

    def matvec_multi(self, X, Y=None, stream=None):
        """Y[r] = K X[r] for the nr rows of X (nr, cols): the operator's entries read once per
        group of up to four vectors; each row bit-identical to matvec's."""
        import torch
        if X.dim() != 2 or X.shape[1] != self.cols:
            raise ValueError(f"X must have shape (nr, {self.cols})")
        nr = X.shape[0]
        if Y is None:
            Y = torch.empty((nr, self.rows), dtype=X.dtype, device=X.device)
        elif Y.shape != (nr, self.rows):
            raise ValueError(f"Y must have shape ({nr}, {self.rows})")
        _dev(X, self.cdtype, "X")
        _dev(Y, self.cdtype, "Y")
        nb = C.c_size_t(0)
        _check(_lib.hmx_matvec_multi_work_bytes(self._h, C.byref(nb)))
        work = torch.empty(max(nb.value, 1), dtype=torch.uint8, device=X.device)
        xs = (_P * nr)(*[X[r].data_ptr() for r in range(nr)])
        ys = (_P * nr)(*[Y[r].data_ptr() for r in range(nr)])
        _check(_lib.hmx_matvec_multi(self._h, nr, xs, ys, C.c_void_p(work.data_ptr()),
                                     _stream_ptr(stream)))
        self._work = work  # kept until the next call so that the queued kernels can use it
        return Y

    def matvec_multi_static(self, X, Y=None, stream=None):
        """matvec_multi on the library's static scratch (no work buffer is allocated; products on
        one device must not overlap in time).  Y may be given to keep the call allocation-free."""
        import torch
        if X.dim() != 2 or X.shape[1] != self.cols:
            raise ValueError(f"X must have shape (nr, {self.cols})")
        nr = X.shape[0]
        if Y is None:
            Y = torch.empty((nr, self.rows), dtype=X.dtype, device=X.device)
        elif Y.shape != (nr, self.rows):
            raise ValueError(f"Y must have shape ({nr}, {self.rows})")
        _dev(X, self.cdtype, "X")
        _dev(Y, self.cdtype, "Y")
        xs = (_P * nr)(*[X[r].data_ptr() for r in range(nr)])
        ys = (_P * nr)(*[Y[r].data_ptr() for r in range(nr)])
        _check(_lib.hmx_matvec_multi_static(self._h, nr, xs, ys, _stream_ptr(stream)))
        return Y

    def __matmul__(self, x):
        return self.matvec(x)

    def mesh_offsets(self):
        """Point offsets of the operator's meshes (n_meshes + 1 entries)."""
        n = C.c_int32(0)
        _check(_lib.hmx_mesh_offsets(self._h, None, 0, C.byref(n)))
        off = np.empty(n.value + 1, np.int64)
        _check(_lib.hmx_mesh_offsets(self._h, off.ctypes.data_as(_P), off.size, C.byref(n)))
        return off

    def split(self, v):
        """Per-mesh views of a concatenated vector."""
        off = self.mesh_offsets()
        return [v[off[i]:off[i + 1]] for i in range(off.size - 1)]

    def graph(self, x, y):
        """The product y = K x captured once in a HIP graph (replay with Graph.launch)."""
        return Graph(self, x, y)

    def export_tree(self):
        n = self.info["n_nodes"]
        perm = np.empty(self.M, np.int32)
        b, e = np.empty(n, np.int64), np.empty(n, np.int64)
        lev, c0, c1 = (np.empty(n, np.int32) for _ in range(3))
        box = np.empty((n, 6))
        _check(_lib.hmx_export_tree(self._h, *(a.ctypes.data_as(_P) for a in (perm, b, e, lev, c0, c1, box))))
        return {"perm": perm, "begin": b, "end": e, "level": lev, "child0": c0, "child1": c1, "box": box}

    def export_blocks(self):
        nn, nf = self.info["n_near"], self.info["n_far"]
        nearR = np.empty((max(nn, 1), 4), np.int64)
        farR = np.empty((max(nf, 1), 4), np.int64)
        ranks = np.empty(max(nf, 1), np.int32)
        _check(_lib.hmx_export_blocks(self._h, nearR.ctypes.data_as(_P), farR.ctypes.data_as(_P),
                                      ranks.ctypes.data_as(_P)))
        return nearR[:nn], farR[:nf], ranks[:nf]

    def export_far(self, b, m, n):
        cdt = np.complex128 if self.precision == FP64 else np.complex64
        # a rank never exceeds min(m, n); a dense far block fills U with m x n entries
        U = np.empty(max(m * n, 1), cdt)
        V = np.empty(max(m * n, 1), cdt)
        r = C.c_int32(0)
        _check(_lib.hmx_export_far(self._h, b, U.ctypes.data_as(_P), V.ctypes.data_as(_P), C.byref(r)))
        if r.value < 0:
            return U[:m * n].reshape(n, m).T.copy(), None
        k = r.value
        return U[:m * k].reshape(k, m).T.copy(), V[:n * k].reshape(k, n).T.copy()

    def import_far(self, ranks, Us, Vs):
        """Replace the low-rank far factors (test support): ranks (n_far,) with -1 for blocks
        stored dense; Us, Vs lists of (m x r) and (n x r) arrays for the low-rank blocks in order."""
        cdt = np.complex128 if self.precision == FP64 else np.complex64
        ranks = np.ascontiguousarray(ranks, np.int32)
        U = np.concatenate([np.asarray(u, cdt).T.ravel() for u in Us]) if Us else np.zeros(1, cdt)
        V = np.concatenate([np.asarray(v, cdt).T.ravel() for v in Vs]) if Vs else np.zeros(1, cdt)
        U, V = np.ascontiguousarray(U), np.ascontiguousarray(V)
        _check(_lib.hmx_import_far(self._h, ranks.ctypes.data_as(_P), U.ctypes.data_as(_P),
                                   V.ctypes.data_as(_P)))
        self.info = self._info()

    def far_features(self):
        """Raw features (n_far x 4 float32) of the far blocks, in export_blocks order."""
        nf = self.info["n_far"]
        f = np.empty((max(nf, 1), 4), np.float32)
        _check(_lib.hmx_far_features(self._h, f.ctypes.data_as(_P)))
        return f[:nf]

    def close(self):
        if self._h:
            _lib.hmx_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def build(vtx, tri, bary, w, kern=HELMHOLTZ, k=0.0, prm: Params | None = None, stream=None) -> Operator:
    """Operator of a triangle mesh (vtx float64 (nv,3), tri int32 (nt,3) device tensors)."""
    import torch
    bary, w = _host_rule(bary, w)
    prm = prm or params()
    h = C.c_void_p()
    _check(_lib.hmx_build(_dev(vtx, torch.float64, "vtx"), vtx.shape[0], _dev(tri, torch.int32, "tri"),
                          tri.shape[0], bary.ctypes.data_as(_P), w.ctypes.data_as(_P), bary.shape[0],
                          kern, float(k), C.byref(prm), _stream_ptr(stream), C.byref(h)))
    return Operator(h, prm.precision)


def build_points(xyzw, kern=HELMHOLTZ, k=0.0, prm: Params | None = None, stream=None) -> Operator:
    """Operator from points and weights: xyzw float64 (4, M) device tensor (X, Y, Z, W)."""
    import torch
    prm = prm or params()
    h = C.c_void_p()
    _check(_lib.hmx_build_points(_dev(xyzw, torch.float64, "xyzw"), xyzw.shape[1], kern, float(k),
                                 C.byref(prm), _stream_ptr(stream), C.byref(h)))
    return Operator(h, prm.precision)


def build_rect(targets, xyzw, kern=HELMHOLTZ, k=0.0, prm: Params | None = None,
               stream=None) -> Operator:
    """Potential of a source quadrature at other points: targets float64 (3, Mt) device tensor
    (X, Y, Z), sources xyzw float64 (4, Ms) device tensor (X, Y, Z, W).  The operator maps
    vectors of Ms entries to vectors of Mt entries."""
    import torch
    prm = prm or params()
    h = C.c_void_p()
    _check(_lib.hmx_build_rect(_dev(targets, torch.float64, "targets"), targets.shape[1],
                               _dev(xyzw, torch.float64, "xyzw"), xyzw.shape[1], kern, float(k),
                               C.byref(prm), _stream_ptr(stream), C.byref(h)))
    return Operator(h, prm.precision)


class P1:
    """The P1 space of the mesh an operator was built on: the Galerkin product
    A = Phi^T W K Phi and its GMRES solve (vectors of n_vtx entries, the operator's type)."""

    def __init__(self, op, vtx, tri, bary, w, stream=None):
        import torch
        bary, w = _host_rule(bary, w)
        self._op = op  # the space uses the operator
        self.nv = vtx.shape[0]
        self.M = op.M
        self._h = C.c_void_p()
        _check(_lib.hmx_p1_create(op._h, _dev(vtx, torch.float64, "vtx"), vtx.shape[0],
                                  _dev(tri, torch.int32, "tri"), tri.shape[0], bary.ctypes.data_as(_P),
                                  w.ctypes.data_as(_P), bary.shape[0], _stream_ptr(stream),
                                  C.byref(self._h)))

    def _vec(self, n, like):
        import torch
        if not self._op._h or not self._h:
            raise RuntimeError("the P1 space or its operator has been closed")
        return torch.empty(n, dtype=self._op.cdtype, device=like.device)

    def interp(self, xv, stream=None):
        xp = self._vec(self.M, xv)
        _check(_lib.hmx_p1_interp(self._h, _dev(xv, self._op.cdtype, "xv"), _dev(xp, self._op.cdtype, "xp"),
                                  _stream_ptr(stream)))
        return xp

    def project(self, zp, stream=None):
        yv = self._vec(self.nv, zp)
        _check(_lib.hmx_p1_project(self._h, _dev(zp, self._op.cdtype, "zp"), _dev(yv, self._op.cdtype, "yv"),
                                   _stream_ptr(stream)))
        return yv

    def matvec(self, xv, stream=None):
        yv = self._vec(self.nv, xv)
        _check(_lib.hmx_galerkin_matvec(self._h, _dev(xv, self._op.cdtype, "xv"),
                                        _dev(yv, self._op.cdtype, "yv"), _stream_ptr(stream)))
        return yv

    def gmres(self, b, tol=1e-8, restart=100, max_iter=1000, stream=None):
        """x, iterations, true relative residual."""
        x = self._vec(self.nv, b)
        it, res = C.c_int32(0), C.c_double(0.0)
        _check(_lib.hmx_gmres(self._h, _dev(b, self._op.cdtype, "b"), _dev(x, self._op.cdtype, "x"),
                              restart, max_iter, float(tol), _stream_ptr(stream), C.byref(it),
                              C.byref(res)))
        return x, it.value, res.value

    def close(self):
        if self._h:
            _lib.hmx_p1_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class RWG:
    """The RWG space of a closed, outward-oriented mesh (one unknown per edge, edges in increasing
    vertex pairs) for the electromagnetic equations: the CFIE product
    A = -beta T + (1 - beta) (Id / 2 - NxK) (beta = 1 the EFIE, 0 the MFIE), its right-hand side
    and its GMRES solve.  `single` is the Helmholtz single layer of the mesh (needed for
    beta > 0), `grads` its three y-gradient operators (needed for beta < 1)."""

    def __init__(self, single, grads, vtx, tri, bary, w, stream=None):
        import torch
        bary, w = _host_rule(bary, w)
        grads = list(grads) if grads is not None else [None, None, None]
        self._ops = [o for o in [single] + grads if o is not None]  # the space uses them
        if not self._ops:
            raise ValueError("no operator given")
        self._op = self._ops[0]
        self.M = self._op.M
        self._h = C.c_void_p()
        hs = [o._h if o is not None else None for o in [single] + grads]
        _check(_lib.hmx_rwg_create(hs[0], hs[1], hs[2], hs[3], _dev(vtx, torch.float64, "vtx"),
                                   vtx.shape[0], _dev(tri, torch.int32, "tri"), tri.shape[0],
                                   bary.ctypes.data_as(_P), w.ctypes.data_as(_P), bary.shape[0],
                                   _stream_ptr(stream), C.byref(self._h)))
        n = C.c_int64(0)
        _check(_lib.hmx_rwg_n_edges(self._h, C.byref(n)))
        self.n_edges = n.value

    def _vec(self, n, like):
        import torch
        if not self._h or any(not o._h for o in self._ops):
            raise RuntimeError("the RWG space or one of its operators has been closed")
        return torch.empty(n, dtype=self._op.cdtype, device=like.device)

    @staticmethod
    def _size(t, n, name):
        if t.numel() != n:
            raise ValueError(f"{name} must have {n} entries, got {t.numel()}")

    def edges(self, device="cuda", stream=None):
        import torch
        if not self._h:
            raise RuntimeError("the RWG space has been closed")
        e = torch.empty((self.n_edges, 2), dtype=torch.int32, device=device)
        _check(_lib.hmx_rwg_edges(self._h, _dev(e, torch.int32, "edges"), _stream_ptr(stream)))
        return e

    def interp(self, x, stream=None):
        """(4, M): J_x, J_y, J_z and div J at the quadrature points."""
        self._size(x, self.n_edges, "x")
        u = self._vec(4 * self.M, x)
        _check(_lib.hmx_rwg_interp(self._h, _dev(x, self._op.cdtype, "x"), _dev(u, self._op.cdtype, "u"),
                                   _stream_ptr(stream)))
        return u.view(4, self.M)

    def rhs(self, beta, e_inc=None, h_inc=None, stream=None):
        """beta <psi, E_inc> - (1 - beta) <n x psi, H_inc>; fields (3, M) at the points."""
        ref = e_inc if e_inc is not None else h_inc
        if ref is None:
            raise ValueError("no incident field given")
        for t, name in ((e_inc, "e_inc"), (h_inc, "h_inc")):
            if t is not None:
                self._size(t, 3 * self.M, name)
        b = self._vec(self.n_edges, ref)
        ep = _dev(e_inc, self._op.cdtype, "e_inc") if e_inc is not None else None
        hp = _dev(h_inc, self._op.cdtype, "h_inc") if h_inc is not None else None
        _check(_lib.hmx_rwg_rhs(self._h, float(beta), ep, hp, _dev(b, self._op.cdtype, "b"),
                                _stream_ptr(stream)))
        return b

    def matvec(self, beta, x, stream=None):
        self._size(x, self.n_edges, "x")
        y = self._vec(self.n_edges, x)
        _check(_lib.hmx_cfie_matvec(self._h, float(beta), _dev(x, self._op.cdtype, "x"),
                                    _dev(y, self._op.cdtype, "y"), _stream_ptr(stream)))
        return y

    def gmres(self, beta, b, tol=1e-8, restart=100, max_iter=1000, stream=None):
        """x, iterations, true relative residual."""
        self._size(b, self.n_edges, "b")
        x = self._vec(self.n_edges, b)
        it, res = C.c_int32(0), C.c_double(0.0)
        _check(_lib.hmx_cfie_gmres(self._h, float(beta), _dev(b, self._op.cdtype, "b"),
                                   _dev(x, self._op.cdtype, "x"), restart, max_iter, float(tol),
                                   _stream_ptr(stream), C.byref(it), C.byref(res)))
        return x, it.value, res.value

    def close(self):
        if self._h:
            _lib.hmx_rwg_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def build_batch(meshes, bary, w, kern=HELMHOLTZ, prm: Params | None = None, stream=None) -> Operator:
    """One block-diagonal operator for independent meshes: `meshes` is a list of
    (vtx float64 (nv,3), tri int32 (nt,3) device tensors, k).  Vectors are the per-mesh vectors
    concatenated in mesh order (Operator.split gives the per-mesh views)."""
    import torch
    bary, w = _host_rule(bary, w)
    prm = prm or params()
    arr = (Mesh * len(meshes))()
    for i, (vtx, tri, k) in enumerate(meshes):
        arr[i] = Mesh(_dev(vtx, torch.float64, "vtx").value, vtx.shape[0],
                      _dev(tri, torch.int32, "tri").value, tri.shape[0], float(k))
    h = C.c_void_p()
    _check(_lib.hmx_build_batch(arr, len(meshes), bary.ctypes.data_as(_P), w.ctypes.data_as(_P),
                                bary.shape[0], kern, C.byref(prm), _stream_ptr(stream), C.byref(h)))
    return Operator(h, prm.precision)


class Graph:
    """A product captured in a HIP graph (fixed operator, x and y); `launch(reps)` replays it."""

    def __init__(self, op, x, y):
        if x.shape != (op.cols,) or y.shape != (op.rows,):
            raise ValueError(f"x must have shape ({op.cols},) and y ({op.rows},)")
        self._op, self._x, self._y = op, x, y  # keep the captured buffers alive
        self._g = C.c_void_p()
        _check(_lib.hmx_graph_create(op._h, _dev(x, op.cdtype, "x"), _dev(y, op.cdtype, "y"),
                                     C.byref(self._g)))

    def launch(self, reps=1, stream=None):
        if not self._op._h or not self._g:
            raise RuntimeError("the graph or its operator has been closed")
        _check(_lib.hmx_graph_launch(self._g, reps, _stream_ptr(stream)))

    def close(self):
        if self._g:
            _lib.hmx_graph_destroy(self._g)
            self._g = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def autotune(xyzw, kern=HELMHOLTZ, k=0.0, prm: Params | None = None, cache_path=None, stream=None):
    """Fastest ACA schedule for building from these points (xyzw float64 (4, M) device tensor):
    returns (params with the chosen schedule, build ms).  A cache file, when given, is read and
    updated."""
    import torch
    prm = prm or params()
    out = Params()
    ms = C.c_double(0)
    path = None if cache_path is None else os.fsencode(cache_path)
    _check(_lib.hmx_autotune(_dev(xyzw, torch.float64, "xyzw"), xyzw.shape[1], kern, float(k),
                             C.byref(prm), path, _stream_ptr(stream), C.byref(out), C.byref(ms)))
    return out, ms.value


def autotune_batch(meshes, bary, w, kern=HELMHOLTZ, prm: Params | None = None, cache_path=None,
                   stream=None):
    """Fastest ACA schedule for build_batch(meshes, bary, w, kern, prm): returns (params with the
    chosen schedule, build ms)."""
    import torch
    bary, w = _host_rule(bary, w)
    prm = prm or params()
    arr = (Mesh * len(meshes))()
    for i, (vtx, tri, k) in enumerate(meshes):
        arr[i] = Mesh(_dev(vtx, torch.float64, "vtx").value, vtx.shape[0],
                      _dev(tri, torch.int32, "tri").value, tri.shape[0], float(k))
    out = Params()
    ms = C.c_double(0)
    path = None if cache_path is None else os.fsencode(cache_path)
    _check(_lib.hmx_autotune_batch(arr, len(meshes), bary.ctypes.data_as(_P), w.ctypes.data_as(_P),
                                   bary.shape[0], kern, C.byref(prm), path, _stream_ptr(stream),
                                   C.byref(out), C.byref(ms)))
    return out, ms.value


# ------------------------------------------------------------------------ learned block ranks
def _f32(a, n=None):
    a = np.ascontiguousarray(a, np.float32).reshape(-1)
    if n is not None and a.size != n:
        raise ValueError(f"expected {n} floats, got {a.size}")
    return a


def mlp_predict(theta, norm, feat, stream=None):
    """Predicted ln(1 + rank) of blocks with raw features `feat` (device float32 (n, 4))."""
    import torch
    theta, norm = _f32(theta, MLP_NPARAMS), _f32(norm, 8)
    n = feat.shape[0]
    out = torch.empty(n, dtype=torch.float32, device=feat.device)
    _check(_lib.hmx_mlp_predict(theta.ctypes.data_as(_P), norm.ctypes.data_as(_P),
                                _dev(feat, torch.float32, "feat"), n, C.c_void_p(out.data_ptr()),
                                _stream_ptr(stream)))
    return out


def mlp_loss_grad(theta, X, y, stream=None):
    """(loss, gradient) of the mean squared error on standardized features X, targets y (device)."""
    import torch
    theta = _f32(theta, MLP_NPARAMS)
    g = np.empty(MLP_NPARAMS, np.float32)
    loss = C.c_float(0)
    _check(_lib.hmx_mlp_loss_grad(theta.ctypes.data_as(_P), _dev(X, torch.float32, "X"),
                                  _dev(y, torch.float32, "y"), X.shape[0], g.ctypes.data_as(_P),
                                  C.byref(loss), _stream_ptr(stream)))
    return float(loss.value), g


def mlp_train(theta, X, y, epochs=40, batch=4096, lr=1e-3, stream=None):
    """Adam training on the device; returns (trained theta, mean batch loss per epoch)."""
    import torch
    th = _f32(theta, MLP_NPARAMS).copy()
    hist = np.empty(epochs, np.float32)
    _check(_lib.hmx_mlp_train(th.ctypes.data_as(_P), _dev(X, torch.float32, "X"),
                              _dev(y, torch.float32, "y"), X.shape[0], epochs, batch, lr,
                              hist.ctypes.data_as(_P), _stream_ptr(stream)))
    return th, hist


def set_rank_model(theta=None, norm=None, alpha=1.0, beta=0.0):
    """Process-wide model for builds with rank_model=RANK_LEARNED (None clears it)."""
    if theta is None:
        _check(_lib.hmx_set_rank_model(None, None, 1.0, 0.0))
        return
    theta, norm = _f32(theta, MLP_NPARAMS), _f32(norm, 8)
    _check(_lib.hmx_set_rank_model(theta.ctypes.data_as(_P), norm.ctypes.data_as(_P), alpha, beta))
