"""GPU tests of the ACA schedule settings and their autotuner: every schedule gives an operator
within the tolerance of the dense product, and the tuner's choice is cached by problem class."""
import json
import time

import numpy as np
import pytest

import oracle
from paper_1804_00995_amd import inputs as I

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")
RULE = I.rule_3pt()


@pytest.fixture(scope="module")
def H():
    oracle.build(force=False)
    from paper_1804_00995_amd import hmx
    return hmx


@pytest.fixture(scope="module")
def sphere4():
    v, f = I.icosphere(4)
    P, W = oracle.quad_points(v, f, *RULE)
    xyzw = torch.from_numpy(np.ascontiguousarray(np.vstack([P.T, W[None, :]]))).cuda()
    x = I.complex_vector(P.shape[0], 6)
    return P, W, xyzw, x, oracle.dense_matvec(P, W, 1, 14.0, x)


def rel(a, b):
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


@pytest.mark.parametrize("big,gram,serial,mid", [(2, 0, 0, 256), (2, 1 << 30, 1, 128),
                                                 (1 << 30, 0, 0, 64), (4096, 1024, 1, 64),
                                                 (1 << 30, 1 << 30, 0, 256)])
def test_schedules_within_tolerance(H, sphere4, big, gram, serial, mid):
    P, W, xyzw, x, yr = sphere4
    op = H.build_points(xyzw, kern=1, k=14.0,
                        prm=H.params(aca_big_mn=big, aca_gram_min_mn=gram, aca_serial=serial,
                                     aca_mid_threads=mid))
    y = op.matvec(torch.from_numpy(x).cuda()).cpu().numpy()
    assert rel(y, yr) <= 1e-3
    ref = H.build_points(xyzw, kern=1, k=14.0)
    # the schedule changes rounding, not the method: ranks agree closely
    _, _, r0 = ref.export_blocks()
    _, _, r1 = op.export_blocks()
    assert abs(int(r0.sum()) - int(r1.sum())) <= 0.01 * r0.sum()


def test_autotune_choice_and_cache(H, sphere4, tmp_path):
    P, W, xyzw, x, yr = sphere4
    cache = tmp_path / "tune.json"
    t0 = time.perf_counter()
    prm, ms = H.autotune(xyzw, kern=1, k=14.0, cache_path=str(cache))
    t1 = time.perf_counter()
    assert prm.aca_big_mn in (2048, 4096, 8192, 1 << 30)
    assert prm.aca_gram_min_mn in (0, 1024, 4096, 1 << 30)
    assert prm.aca_serial in (0, 1) and ms > 0
    assert prm.max_far_mn in (0, 32768, 16384, 12288, 8192)
    assert prm.aca_mid_threads in (256, 128, 64)
    assert prm.aca_big_threads in (0, 512, 256)
    assert prm.aca_small_mn in (1024, 512, 2048, 0)
    assert prm.aca_wave in (0, 1)
    entries = json.loads(cache.read_text())
    assert len(entries) == 1
    (key, val), = entries.items()
    assert key.startswith("gfx") and f"|helmholtz|M2^{int(np.log2(P.shape[0]))}|tol1e-3|leaf64|" in key
    assert val["aca_big_mn"] == prm.aca_big_mn and val["aca_serial"] == prm.aca_serial
    assert val["max_far_mn"] == prm.max_far_mn
    assert val["aca_big_threads"] == prm.aca_big_threads
    assert val["aca_small_mn"] == prm.aca_small_mn
    assert val["aca_wave"] == prm.aca_wave
    # a second call for the same class is answered from the cache, without builds
    t2 = time.perf_counter()
    prm2, ms2 = H.autotune(xyzw, kern=1, k=14.0, cache_path=str(cache))
    t3 = time.perf_counter()
    assert (prm2.aca_big_mn, prm2.aca_gram_min_mn, prm2.aca_serial) == \
        (prm.aca_big_mn, prm.aca_gram_min_mn, prm.aca_serial)
    assert t3 - t2 < 0.2 * (t1 - t0)
    op = H.build_points(xyzw, kern=1, k=14.0, prm=prm)
    y = op.matvec(torch.from_numpy(x).cuda()).cpu().numpy()
    assert rel(y, yr) <= 1e-3
