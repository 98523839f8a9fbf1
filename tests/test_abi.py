"""The C ABI: libhmx.so loads, exports every entry point declared in include/hmx.h, and rejects
invalid arguments on the host before any device work (no GPU needed for these calls)."""
import ctypes as C
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "hmx.h")


def _declared():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(hmx_[a-z_0-9]+)\s*\(", text)))


@pytest.fixture(scope="module")
def hmx():
    from paper_1804_00995_amd import hmx as H
    return H


def test_header_declares_expected_entry_points():
    names = _declared()
    for n in ["hmx_build", "hmx_build_points", "hmx_matvec", "hmx_quad_points", "hmx_info",
              "hmx_destroy", "hmx_last_error", "hmx_params_default"]:
        assert n in names


def test_library_exports_every_declared_symbol(hmx):
    lib = C.CDLL(hmx.LIB_PATH)
    for name in _declared():
        assert hasattr(lib, name), name
    assert sorted(hmx.EXPORTED) == sorted(n for n in _declared())


def test_params_default(hmx):
    p = hmx.params()
    assert p.struct_size == C.sizeof(hmx.Params)
    assert p.tol == 1e-3 and p.leaf_size == 64 and p.eta == 1.5
    assert p.precision == hmx.FP64 and p.rank_model == hmx.RANK_ADAPTIVE
    assert p.initial_rank >= 1 and p.force_pred_scale == 1.0
    assert p.aca_arena == 1 and p.aca_big_threads == 0 and p.aca_small_mn == 1024
    assert p.regularize == 0 and p.reg_radius == 2.0


def test_null_arguments_rejected_on_host(hmx):
    lib = hmx._lib
    h = C.c_void_p()
    p = hmx.params()
    rc = lib.hmx_build(None, 3, None, 1, None, None, 3, 1, 5.0, C.byref(p), None, C.byref(h))
    assert rc == hmx.EINVAL and b"null" in lib.hmx_last_error()
    assert lib.hmx_matvec(None, None, None, None) == hmx.EINVAL
    assert lib.hmx_info(None, None) == hmx.EINVAL
    assert lib.hmx_params_default(None) == hmx.EINVAL
    lib.hmx_destroy(None)  # NULL-safe


def test_bad_params_rejected_on_host(hmx):
    lib = hmx._lib
    h = C.c_void_p()
    fake = C.c_void_p(16)  # never dereferenced: parameters are checked first
    bary = (C.c_double * 9)(2 / 3, 1 / 6, 1 / 6, 1 / 6, 2 / 3, 1 / 6, 1 / 6, 1 / 6, 2 / 3)
    w = (C.c_double * 3)(1 / 3, 1 / 3, 1 / 3)
    for kw, code in [({"leaf_size": 0}, hmx.EINVAL), ({"eta": -1.0}, hmx.EINVAL),
                     ({"precision": 7}, hmx.EINVAL), ({"leaf_size": 300}, hmx.EUNSUPPORTED),
                     ({"struct_size": 8}, hmx.EINVAL), ({"aca_big_threads": 128}, hmx.EINVAL),
                     ({"aca_mid_threads": 512}, hmx.EINVAL), ({"aca_small_mn": -1}, hmx.EINVAL),
                     ({"aca_arena": 2}, hmx.EINVAL), ({"aca_wave": 3}, hmx.EINVAL),
                     ({"regularize": 2}, hmx.EINVAL), ({"regularize": 1, "reg_radius": 0.0}, hmx.EINVAL),
                     ({"regularize": 1, "reg_radius": float("nan")}, hmx.EINVAL),
                     ({"regularize": 1, "tol": 0.0}, hmx.EUNSUPPORTED),
                     ({"force_block_cap": -1}, hmx.EINVAL)]:
        p = hmx.params(**kw)
        rc = lib.hmx_build(fake, 3, fake, 1, bary, w, 3, 1, 5.0, C.byref(p), None, C.byref(h))
        assert rc == code, (kw, rc, lib.hmx_last_error())
    p = hmx.params()
    assert lib.hmx_build(fake, 3, fake, 1, bary, w, 3, 1, -1.0, C.byref(p), None, C.byref(h)) == hmx.EINVAL
    assert lib.hmx_build(fake, 3, fake, 1, bary, w, 3, 42, 1.0, C.byref(p), None, C.byref(h)) == hmx.EINVAL
    assert lib.hmx_build(fake, 3, fake, 1, bary, w, 3, 5, 1.0, C.byref(p), None, C.byref(h)) == hmx.EINVAL
    reg = hmx.params(regularize=1)  # the correction is for the kernel itself, not its gradient
    assert lib.hmx_build(fake, 3, fake, 1, bary, w, 3, hmx.GRADY_X, 1.0, C.byref(reg), None,
                         C.byref(h)) == hmx.EINVAL
    badw = (C.c_double * 3)(0.3, 0.3, 0.3)
    assert lib.hmx_build(fake, 3, fake, 1, bary, badw, 3, 1, 1.0, C.byref(p), None, C.byref(h)) == hmx.EINVAL
    badb = (C.c_double * 9)(1.2, -0.1, -0.1, 1 / 6, 2 / 3, 1 / 6, 1 / 6, 1 / 6, 2 / 3)
    assert lib.hmx_build(fake, 3, fake, 1, badb, w, 3, 1, 1.0, C.byref(p), None, C.byref(h)) == hmx.EINVAL
    assert lib.hmx_build(fake, 3, fake, 1, bary, w, 0, 1, 1.0, C.byref(p), None, C.byref(h)) == hmx.EINVAL
    assert lib.hmx_build(fake, 0, fake, 1, bary, w, 3, 1, 1.0, C.byref(p), None, C.byref(h)) == hmx.EINVAL


def test_singular_correction_arguments_rejected_on_host(hmx):
    """The correction needs the mesh, a 3-point rule with non-collinear points and the Laplace or
    Helmholtz kernel; every case is rejected before any device work."""
    lib = hmx._lib
    h = C.c_void_p()
    fake = C.c_void_p(16)
    p = hmx.params(regularize=1)
    w3 = (C.c_double * 3)(1 / 3, 1 / 3, 1 / 3)
    bary = (C.c_double * 9)(2 / 3, 1 / 6, 1 / 6, 1 / 6, 2 / 3, 1 / 6, 1 / 6, 1 / 6, 2 / 3)
    one = (C.c_double * 3)(1 / 3, 1 / 3, 1 / 3)
    w1 = (C.c_double * 1)(1.0)
    assert lib.hmx_build(fake, 3, fake, 1, one, w1, 1, 1, 1.0, C.byref(p), None, C.byref(h)) == hmx.EINVAL
    assert b"3-point" in lib.hmx_last_error()
    # three points on one line of the triangle
    line = (C.c_double * 9)(0.5, 0.5, 0.0, 0.25, 0.75, 0.0, 0.75, 0.25, 0.0)
    assert lib.hmx_build(fake, 3, fake, 1, line, w3, 3, 1, 1.0, C.byref(p), None, C.byref(h)) == hmx.EINVAL
    assert b"collinear" in lib.hmx_last_error()
    assert lib.hmx_build(fake, 3, fake, 1, bary, w3, 3, hmx.TEST_POLY2, 1.0, C.byref(p), None,
                         C.byref(h)) == hmx.EINVAL
    assert lib.hmx_build_points(fake, 10, 1, 1.0, C.byref(p), None, C.byref(h)) == hmx.EINVAL
    assert b"mesh" in lib.hmx_last_error()
    meshes = (hmx.Mesh * 1)(hmx.Mesh(fake, 3, fake, 1, 5.0))
    assert lib.hmx_build_batch(meshes, 1, one, w1, 1, 1, C.byref(p), None, C.byref(h)) == hmx.EINVAL


def test_rect_argument_errors_without_gpu(hmx):
    lib = hmx._lib
    h = C.c_void_p()
    fake = C.c_void_p(4096)
    p = hmx.params()
    assert lib.hmx_build_rect(None, 5, fake, 7, 1, 1.0, C.byref(p), None, C.byref(h)) == hmx.EINVAL
    assert lib.hmx_build_rect(fake, 0, fake, 7, 1, 1.0, C.byref(p), None, C.byref(h)) == hmx.EINVAL
    assert lib.hmx_build_rect(fake, 5, fake, 0, 1, 1.0, C.byref(p), None, C.byref(h)) == hmx.EINVAL
    assert lib.hmx_build_rect(fake, 5, fake, 7, 1, -2.0, C.byref(p), None, C.byref(h)) == hmx.EINVAL
    reg = hmx.params(regularize=1)
    assert lib.hmx_build_rect(fake, 5, fake, 7, 1, 1.0, C.byref(reg), None, C.byref(h)) == hmx.EINVAL
    shares = hmx.params(row_shares=2)
    assert lib.hmx_build_rect(fake, 5, fake, 7, 1, 1.0, C.byref(shares), None,
                              C.byref(h)) == hmx.EUNSUPPORTED


def test_galerkin_argument_errors_without_gpu(hmx):
    lib = hmx._lib
    h = C.c_void_p()
    fake = C.c_void_p(4096)
    bary = (C.c_double * 9)(2 / 3, 1 / 6, 1 / 6, 1 / 6, 2 / 3, 1 / 6, 1 / 6, 1 / 6, 2 / 3)
    w = (C.c_double * 3)(1 / 3, 1 / 3, 1 / 3)
    assert lib.hmx_p1_create(None, fake, 3, fake, 1, bary, w, 3, None, C.byref(h)) == hmx.EINVAL
    assert lib.hmx_p1_interp(None, fake, fake, None) == hmx.EINVAL
    assert lib.hmx_p1_project(None, fake, fake, None) == hmx.EINVAL
    assert lib.hmx_galerkin_matvec(None, fake, fake, None) == hmx.EINVAL
    it, res = C.c_int32(0), C.c_double(0)
    assert lib.hmx_gmres(None, fake, fake, 10, 10, 1e-6, None, C.byref(it), C.byref(res)) == hmx.EINVAL
    lib.hmx_p1_destroy(None)  # NULL-safe


def test_matvec_multi_argument_errors_without_gpu(hmx):
    lib = hmx._lib
    fake = C.c_void_p(4096)
    ptrs = (C.c_void_p * 2)(4096, 8192)
    nb = C.c_size_t(0)
    assert lib.hmx_matvec_multi_work_bytes(None, C.byref(nb)) == hmx.EINVAL
    assert lib.hmx_matvec_multi(None, 2, ptrs, ptrs, fake, None) == hmx.EINVAL
    assert lib.hmx_matvec_multi(fake, 0, ptrs, ptrs, fake, None) == hmx.EINVAL  # nr < 1
    assert lib.hmx_matvec_multi(fake, 2, None, ptrs, fake, None) == hmx.EINVAL
    # aliasing is refused before the operator is read (the fake operator is never touched):
    # an output equal to an input of a later group, and an output listed twice
    xs = (C.c_void_p * 3)(4096, 8192, 12288)
    ys = (C.c_void_p * 3)(16384, 20480, 4096)
    assert lib.hmx_matvec_multi(fake, 3, xs, ys, fake, None) == hmx.EINVAL
    assert b"aliases" in lib.hmx_last_error()
    ys2 = (C.c_void_p * 3)(16384, 20480, 16384)
    assert lib.hmx_matvec_multi(fake, 3, xs, ys2, fake, None) == hmx.EINVAL
    assert b"twice" in lib.hmx_last_error()


def test_rwg_argument_errors_without_gpu(hmx):
    lib = hmx._lib
    h = C.c_void_p()
    fake = C.c_void_p(4096)
    bary = (C.c_double * 9)(2 / 3, 1 / 6, 1 / 6, 1 / 6, 2 / 3, 1 / 6, 1 / 6, 1 / 6, 2 / 3)
    w = (C.c_double * 3)(1 / 3, 1 / 3, 1 / 3)
    # no operator, or one or two of the three gradient operators
    assert lib.hmx_rwg_create(None, None, None, None, fake, 4, fake, 4, bary, w, 3, None, C.byref(h)) == hmx.EINVAL
    assert lib.hmx_rwg_create(None, fake, None, None, fake, 4, fake, 4, bary, w, 3, None, C.byref(h)) == hmx.EINVAL
    assert lib.hmx_rwg_create(fake, fake, fake, None, fake, 4, fake, 4, bary, w, 3, None, C.byref(h)) == hmx.EINVAL
    n = C.c_int64(0)
    assert lib.hmx_rwg_n_edges(None, C.byref(n)) == hmx.EINVAL
    assert lib.hmx_rwg_edges(None, fake, None) == hmx.EINVAL
    assert lib.hmx_rwg_interp(None, fake, fake, None) == hmx.EINVAL
    assert lib.hmx_rwg_rhs(None, 0.5, fake, fake, fake, None) == hmx.EINVAL
    assert lib.hmx_cfie_matvec(None, 0.5, fake, fake, None) == hmx.EINVAL
    it, res = C.c_int32(0), C.c_double(0)
    assert lib.hmx_cfie_gmres(None, 0.5, fake, fake, 10, 10, 1e-6, None, C.byref(it), C.byref(res)) == hmx.EINVAL
    lib.hmx_rwg_destroy(None)  # NULL-safe


def test_batch_argument_errors_without_gpu():
    import ctypes as C
    from paper_1804_00995_amd import hmx
    lib = hmx._lib
    p = hmx.params()
    h = C.c_void_p()
    bary = (C.c_double * 9)(2 / 3, 1 / 6, 1 / 6, 1 / 6, 2 / 3, 1 / 6, 1 / 6, 1 / 6, 2 / 3)
    w = (C.c_double * 3)(1 / 3, 1 / 3, 1 / 3)
    fake = C.c_void_p(4096)
    meshes = (hmx.Mesh * 2)(hmx.Mesh(fake, 3, fake, 1, 5.0), hmx.Mesh(fake, 3, fake, 1, 7.0))
    assert lib.hmx_build_batch(None, 2, bary, w, 3, 1, C.byref(p), None, C.byref(h)) == hmx.EINVAL
    assert lib.hmx_build_batch(meshes, 0, bary, w, 3, 1, C.byref(p), None, C.byref(h)) == hmx.EINVAL
    dense = hmx.params(tol=0.0)
    assert lib.hmx_build_batch(meshes, 2, bary, w, 3, 1, C.byref(dense), None, C.byref(h)) == hmx.EINVAL
    assert b"tol" in lib.hmx_last_error()
    meshes[1].k = -1.0
    assert lib.hmx_build_batch(meshes, 2, bary, w, 3, 1, C.byref(p), None, C.byref(h)) == hmx.EINVAL
    meshes[1].k = 7.0
    meshes[1].n_tri = 0
    assert lib.hmx_build_batch(meshes, 2, bary, w, 3, 1, C.byref(p), None, C.byref(h)) == hmx.EINVAL
    n = C.c_int32(0)
    assert lib.hmx_mesh_offsets(None, None, 0, C.byref(n)) == hmx.EINVAL
    assert lib.hmx_graph_create(None, None, None, C.byref(h)) == hmx.EINVAL
    assert lib.hmx_graph_launch(None, 1, None) == hmx.EINVAL
    lib.hmx_graph_destroy(None)  # NULL-safe


def test_autotune_argument_errors_without_gpu():
    import ctypes as C
    from paper_1804_00995_amd import hmx
    lib = hmx._lib
    out = hmx.Params()
    ms = C.c_double(0)
    fake = C.c_void_p(4096)
    assert lib.hmx_autotune(None, 10, 1, 1.0, None, None, None, C.byref(out), C.byref(ms)) == hmx.EINVAL
    assert lib.hmx_autotune(fake, 0, 1, 1.0, None, None, None, C.byref(out), C.byref(ms)) == hmx.EINVAL
    dense = hmx.params(tol=0.0)
    assert lib.hmx_autotune(fake, 10, 1, 1.0, C.byref(dense), None, None, C.byref(out),
                            C.byref(ms)) == hmx.EINVAL
    bad = hmx.params(aca_serial=2)
    h = C.c_void_p()
    assert lib.hmx_build_points(fake, 10, 1, 1.0, C.byref(bad), None, C.byref(h)) == hmx.EINVAL
    bad = hmx.params(aca_big_mn=1)
    assert lib.hmx_build_points(fake, 10, 1, 1.0, C.byref(bad), None, C.byref(h)) == hmx.EINVAL


def test_import_far_argument_errors_without_gpu():
    from paper_1804_00995_amd import hmx
    lib = hmx._lib
    assert lib.hmx_import_far(None, None, None, None) == hmx.EINVAL
