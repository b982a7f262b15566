"""C-ABI checks that need no GPU: the library loads, exports every function
include/lipfit.h declares, and its host-side validation rejects bad arguments
before any device work (status codes of include/lipfit.h)."""
import ctypes
import os
import subprocess

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
LIB = os.path.join(ROOT, "paper_2606_04670_amd", "liblipfit.so")

pytestmark = pytest.mark.skipif(not os.path.exists(LIB),
                                reason="liblipfit.so not built (run __graft_entry__.build())")


@pytest.fixture(scope="module")
def L():
    from paper_2606_04670_amd import _lib
    _lib.load()
    return _lib


def test_exports_every_declared_symbol(L):
    names = L.header_symbols()
    assert len(names) >= 13
    out = subprocess.run(["nm", "-D", "--defined-only", LIB], capture_output=True, text=True,
                         check=True).stdout
    exported = {line.split()[-1] for line in out.splitlines() if line.strip()}
    missing = [n for n in names if n not in exported]
    assert not missing, missing
    lib = L.load()
    for n in names:
        assert getattr(lib, n) is not None


def test_status_strings(L):
    lib = L.load()
    for st in range(8):
        assert lib.lip_status_string(st)
    assert lib.lip_status_string(0) == b"ok"


def test_workspace_size_monotone(L):
    lib = L.load()
    a = lib.lip_workspace_size(1000, 1000, 4, 0)
    b = lib.lip_workspace_size(100000, 1000000, 4, 0)
    assert 0 < a < b
    assert lib.lip_workspace_size(0, 0, 0, 0) > 0


FAKE = ctypes.c_void_p(0x1000)  # never dereferenced: validation fails first


def _metric(L, d=3, norm=2, w=None, mon=None):
    keep = []
    wp = monp = None
    if w is not None:
        wa = np.asarray(w, np.float32)
        keep.append(wa)
        wp = wa.ctypes.data_as(ctypes.c_void_p)
    if mon is not None:
        ma = np.asarray(mon, np.int8)
        keep.append(ma)
        monp = ma.ctypes.data_as(ctypes.c_void_p)
    m = L.LipMetric(d, norm, wp, monp)
    return m, keep


def _eval(L, m, n=10, q=5, M=1.0, Mk=None, ws=FAKE, ws_bytes=1 << 30, flags=0, x=FAKE):
    lib = L.load()
    return lib.lip_fit_eval(ctypes.byref(m), x, FAKE, n, M, Mk, FAKE, q, FAKE, None, None, None,
                            None, ws, ws_bytes, flags, None)


def test_fit_eval_validation(L):
    m, keep = _metric(L)
    assert _eval(L, m, n=0) == L.LIP_E_SHAPE
    assert _eval(L, m, q=-1) == L.LIP_E_SHAPE
    assert _eval(L, m, M=-1.0) == L.LIP_E_VALUE
    assert _eval(L, m, M=float("nan")) == L.LIP_E_VALUE
    assert _eval(L, m, M=float("inf")) == L.LIP_E_VALUE
    assert _eval(L, m, x=None) == L.LIP_E_ARG
    assert _eval(L, m, ws=None) == L.LIP_E_WORKSPACE
    assert _eval(L, m, flags=1 << 7) == L.LIP_E_ARG
    assert _eval(L, m, q=0) == L.LIP_OK  # no-op, no device work
    bad_d, k1 = _metric(L, d=0)
    assert _eval(L, bad_d) == L.LIP_E_SHAPE
    big_d, k2 = _metric(L, d=17)
    assert _eval(L, big_d) == L.LIP_E_SHAPE
    bad_norm, k3 = _metric(L, norm=4)
    assert _eval(L, bad_norm) == L.LIP_E_ARG
    bad_w, k4 = _metric(L, w=[1.0, 0.0, 1.0])
    assert _eval(L, bad_w) == L.LIP_E_VALUE
    bad_mon, k5 = _metric(L, mon=[0, 7, 0])
    assert _eval(L, bad_mon) == L.LIP_E_VALUE
    case_no_ab, k5b = _metric(L, mon=[0, 2, 0])  # a case of Sec. 4.2 needs a and b
    assert _eval(L, case_no_ab) == L.LIP_E_ARG
    # BF16 path: l2 without monotone coordinates only
    l1, k6 = _metric(L, norm=1)
    assert _eval(L, l1, flags=L.LIP_FLAG_BF16) == L.LIP_E_UNSUPPORTED
    monm, k7 = _metric(L, mon=[1, 0, 0])
    assert _eval(L, monm, flags=L.LIP_FLAG_BF16) == L.LIP_E_UNSUPPORTED
    assert L.load().lip_fit_eval(None, FAKE, FAKE, 10, 1.0, None, FAKE, 5, FAKE, None, None,
                                 None, None, FAKE, 1 << 30, 0, None) == L.LIP_E_ARG


def test_other_entry_points_validation(L):
    lib = L.load()
    m, keep = _metric(L)
    # backward
    assert lib.lip_fit_backward(ctypes.byref(m), FAKE, FAKE, 0, 1.0, None, FAKE, 5, FAKE, FAKE,
                                FAKE, None, None, FAKE, FAKE, FAKE, None, 0, 0, None) \
        == L.LIP_E_SHAPE
    assert lib.lip_fit_backward(ctypes.byref(m), FAKE, FAKE, 10, 1.0, None, FAKE, 5, None, FAKE,
                                FAKE, None, None, FAKE, FAKE, FAKE, None, 0, 0, None) \
        == L.LIP_E_ARG
    assert lib.lip_fit_backward(ctypes.byref(m), FAKE, FAKE, 10, 1.0, None, FAKE, 5, FAKE, FAKE,
                                FAKE, None, None, FAKE, FAKE, FAKE, None, 0,
                                L.LIP_FLAG_DETERMINISTIC, None) == L.LIP_E_WORKSPACE
    assert lib.lip_fit_backward(ctypes.byref(m), FAKE, FAKE, 10, 1.0, None, FAKE, 0, FAKE, FAKE,
                                FAKE, None, None, FAKE, FAKE, FAKE, None, 0, 0, None) == L.LIP_OK
    # consistency
    assert lib.lip_consistency(ctypes.byref(m), FAKE, FAKE, 10, 1.0, None, -1.0, FAKE, None, None, None, None,
                               None, None, FAKE, 1 << 30, 0, None) == L.LIP_E_VALUE
    assert lib.lip_consistency(ctypes.byref(m), FAKE, FAKE, 10, 1.0, None, 0.0, None, None, None, None, None,
                               None, None, FAKE, 1 << 30, 0, None) == L.LIP_E_ARG
    assert lib.lip_consistency(ctypes.byref(m), FAKE, FAKE, 10, 1.0, None, 0.0, FAKE, None, None, None, None,
                               None, None, FAKE, 16, 0, None) == L.LIP_E_WORKSPACE
    # estimate_M
    assert lib.lip_estimate_M(ctypes.byref(m), FAKE, FAKE, 10, 7, 16, None, None, None, FAKE,
                              1 << 30, 0, None) == L.LIP_E_ARG
    assert lib.lip_estimate_M(ctypes.byref(m), FAKE, FAKE, 10, L.LIP_M_LOCAL_KNN, 0, None, None,
                              None, FAKE, 1 << 30, 0, None) == L.LIP_E_VALUE
    assert lib.lip_estimate_M(ctypes.byref(m), FAKE, FAKE, 10, L.LIP_M_LOCAL_KNN, 33, None, None,
                              None, FAKE, 1 << 30, 0, None) == L.LIP_E_VALUE
    assert lib.lip_estimate_M(ctypes.byref(m), FAKE, FAKE, 0, L.LIP_M_GLOBAL, 16, None, None,
                              None, FAKE, 1 << 30, 0, None) == L.LIP_E_SHAPE


def test_tuning_table(L):
    lib = L.load()
    lib.lip_tune_clear()
    cfg = L.LipTileCfg()
    assert lib.lip_tune_get(4, 2, 1, 100000, 1000000, ctypes.byref(cfg)) == L.LIP_OK
    default = (cfg.tile, cfg.split, cfg.waves)
    assert cfg.tile % 8 == 0 and cfg.split >= 1 and cfg.waves >= 1
    bad = L.LipTileCfg(12, 1, 4, 0)
    assert lib.lip_tune_set(4, 2, 1, 0, 0, ctypes.byref(bad)) == L.LIP_E_VALUE
    bad_flags = L.LipTileCfg(32, 1, 4, 4)
    assert lib.lip_tune_set(4, 2, 1, 0, 0, ctypes.byref(bad_flags)) == L.LIP_E_VALUE
    bad_waves = L.LipTileCfg(32, 1, 9, 0)
    assert lib.lip_tune_set(4, 2, 1, 0, 0, ctypes.byref(bad_waves)) == L.LIP_E_VALUE
    eight = L.LipTileCfg(32, 8, 8, L.LIP_TILE_L2_FILTER)
    assert lib.lip_tune_set(4, 2, 1, 0, 0, ctypes.byref(eight)) == L.LIP_OK
    assert lib.lip_tune_set(4, 2, 1, 0, 0, None) == L.LIP_OK
    # the default turns the l2 filter on with monotone coordinates
    for d, m, norm, want in ((4, 2, 2, 1), (4, 0, 2, 0), (8, 4, 2, 1), (4, 2, 1, 0), (2, 1, 2, 1),
                             (16, 0, 2, 0), (16, 1, 2, 1)):
        lib.lip_tune_get(d, m, norm, 1000, 1000, ctypes.byref(cfg))
        assert cfg.flags == want, (d, m, norm)
    lib.lip_tune_get(4, 2, 2, 100000, 1000000, ctypes.byref(cfg))
    assert (cfg.split, cfg.waves, cfg.flags) == (8, 4,
                                                 L.LIP_TILE_L2_FILTER | L.LIP_TILE_QUERY_ORDER)
    assert lib.lip_tune_set(4, 2, 1, 10, 0, ctypes.byref(bad)) == L.LIP_E_SHAPE
    # an entry for every size
    good = L.LipTileCfg(128, 2, 2, 0)
    assert lib.lip_tune_set(4, 2, 1, 0, 0, ctypes.byref(good)) == L.LIP_OK
    got = L.LipTileCfg()
    lib.lip_tune_get(4, 2, 1, 10, 10, ctypes.byref(got))
    assert (got.tile, got.split, got.waves) == (128, 2, 2)
    # an entry for one size class (factor-4 buckets of n and q) wins over it
    sized = L.LipTileCfg(16, 8, 4, 0)
    assert lib.lip_tune_set(4, 2, 1, 100000, 1000000, ctypes.byref(sized)) == L.LIP_OK
    for n, q in ((100000, 1000000), (70000, 1048575), (131071, 800000)):
        lib.lip_tune_get(4, 2, 1, n, q, ctypes.byref(got))
        assert (got.tile, got.split, got.waves) == (16, 8, 4), (n, q)
    for n, q in ((100000, 4000), (1000, 1000000), (300000, 1000000)):
        lib.lip_tune_get(4, 2, 1, n, q, ctypes.byref(got))
        assert (got.tile, got.split, got.waves) == (128, 2, 2), (n, q)
    # removing both entries restores the default
    assert lib.lip_tune_set(4, 2, 1, 100000, 1000000, None) == L.LIP_OK
    assert lib.lip_tune_set(4, 2, 1, 0, 0, None) == L.LIP_OK
    lib.lip_tune_get(4, 2, 1, 100000, 1000000, ctypes.byref(got))
    assert (got.tile, got.split, got.waves) == default
    assert lib.lip_tune_get(4, 5, 1, 10, 10, ctypes.byref(got)) == L.LIP_E_SHAPE


def test_tune_cache_file(L, tmp_path):
    """lip_tune_save / lip_tune_load: round trip, architecture filter,
    malformed files change nothing."""
    lib = L.load()
    lib.lip_tune_clear()
    a = L.LipTileCfg(64, 4, 2, 1)
    b = L.LipTileCfg(32, 1, 4, 0)
    assert lib.lip_tune_set(3, 1, 2, 5000, 20000, ctypes.byref(a)) == L.LIP_OK
    assert lib.lip_tune_set(7, 0, 3, 0, 0, ctypes.byref(b)) == L.LIP_OK
    path = str(tmp_path / "tune.json")
    assert lib.lip_tune_save(path.encode(), b"gfx950") == L.LIP_OK
    import json
    doc = json.load(open(path))
    assert doc["format"] == "lipfit-tune-1"
    assert sorted((e["d"], e["n_class"], e["tile"]) for e in doc["entries"]) == [(3, 6, 64),
                                                                                (7, -1, 32)]
    lib.lip_tune_clear()
    got = L.LipTileCfg()
    # another architecture's entries are not loaded
    assert lib.lip_tune_load(path.encode(), b"gfx942") == L.LIP_OK
    lib.lip_tune_get(3, 1, 2, 5000, 20000, ctypes.byref(got))
    assert got.tile != 64 or got.split != 4
    assert lib.lip_tune_load(path.encode(), b"gfx950") == L.LIP_OK
    lib.lip_tune_get(3, 1, 2, 5000, 20000, ctypes.byref(got))
    assert (got.tile, got.split, got.waves, got.flags) == (64, 4, 2, 1)
    lib.lip_tune_get(7, 0, 3, 123, 456, ctypes.byref(got))
    assert (got.tile, got.split, got.waves) == (32, 1, 4)
    # malformed or invalid files: LIP_E_VALUE and no change
    lib.lip_tune_clear()
    for text in ('{"format": "other", "entries": []}',
                 '{"format": "lipfit-tune-1", "entries": [{"arch": "gfx950", "d": 3}]}',
                 doc_text_bad_tile(),
                 '{"format": "lipfit-tune-1", "entries": [',
                 'not json'):
        bad = tmp_path / "bad.json"
        bad.write_text(text)
        assert lib.lip_tune_load(str(bad).encode(), b"gfx950") == L.LIP_E_VALUE, text
    lib.lip_tune_get(3, 1, 2, 5000, 20000, ctypes.byref(got))
    assert (got.tile, got.split) != (64, 4)
    assert lib.lip_tune_load(str(tmp_path / "missing.json").encode(), b"gfx950") == L.LIP_E_ARG
    lib.lip_tune_clear()


def doc_text_bad_tile():
    return ('{"format": "lipfit-tune-1", "entries": [{"arch": "gfx950", "d": 3, "n_mon": 1, '
            '"norm": 2, "n_class": 6, "q_class": 7, "tile": 12, "split": 1, "waves": 4}]}')


def test_python_binding_refuses_cpu_tensors():
    import torch
    import paper_2606_04670_amd as lf
    x = torch.zeros(4, 2)
    with pytest.raises(ValueError):
        lf.fit_eval(x, torch.zeros(4), torch.zeros(3, 2), lf.Metric(2, "l2"), M=1.0)


def test_step_entry_points_validation(L):
    lib = L.load()
    m, keep = _metric(L)
    P = ctypes.c_void_p
    pairs = np.array([[0, 1], [2, 3]], np.int64)
    bad_pairs = np.array([[0, 1], [2, 10]], np.int64)
    probs = np.array([0.25, 0.75])
    bad_probs = np.array([0.75, 0.25])
    zero_prob = np.array([0.0, 0.5])
    pp = lambda a: a.ctypes.data_as(P)

    def knots(n=10, prs=pairs, pb=probs, K=2, ws=FAKE, ws_bytes=1 << 30, out=FAKE):
        return lib.lip_local_knots(ctypes.byref(m), FAKE, n, pp(prs), prs.shape[0], pp(pb), K,
                                   out, ws, ws_bytes, 0, None)
    assert knots(n=0) == L.LIP_E_SHAPE
    assert knots(K=9) == L.LIP_E_SHAPE
    assert knots(prs=bad_pairs) == L.LIP_E_VALUE
    assert knots(pb=bad_probs) == L.LIP_E_VALUE
    assert knots(pb=zero_prob) == L.LIP_E_VALUE
    assert knots(out=None) == L.LIP_E_ARG
    assert knots(ws=None) == L.LIP_E_WORKSPACE
    assert knots(ws_bytes=64) == L.LIP_E_WORKSPACE
    assert knots(K=0) == L.LIP_OK  # nothing to compute, no device work

    kn = np.array([0.5, 1.0])
    kn_bad = np.array([1.0, 0.5])
    kn_neg = np.array([-1.0, 0.5])

    def steps(n=10, k=kn, K=2, d1=FAKE, ws=FAKE, ws_bytes=1 << 30):
        return lib.lip_local_steps(ctypes.byref(m), FAKE, FAKE, n, pp(k), K, d1, None, None, ws,
                                   ws_bytes, 0, None)
    assert steps(n=0) == L.LIP_E_SHAPE
    assert steps(K=9) == L.LIP_E_SHAPE
    assert steps(k=kn_bad) == L.LIP_E_VALUE
    assert steps(k=kn_neg) == L.LIP_E_VALUE
    assert steps(d1=None) == L.LIP_E_ARG
    assert steps(ws_bytes=16) == L.LIP_E_WORKSPACE

    def ev(n=10, q=5, k=kn, K=2, V=FAKE, flags=0):
        st = L.LipSteps(K, pp(k), FAKE, V)
        return lib.lip_fit_eval_steps(ctypes.byref(m), FAKE, FAKE, n, ctypes.byref(st), FAKE, q,
                                      FAKE, None, None, None, None, FAKE, 1 << 30, flags, None)
    assert ev(n=0) == L.LIP_E_SHAPE
    assert ev(K=-1) == L.LIP_E_SHAPE
    assert ev(k=kn_bad) == L.LIP_E_VALUE
    assert ev(V=None) == L.LIP_E_ARG
    assert ev(flags=L.LIP_FLAG_BF16) == L.LIP_E_UNSUPPORTED
    assert ev(q=0) == L.LIP_OK
    assert lib.lip_fit_eval_steps(ctypes.byref(m), FAKE, FAKE, 10, None, FAKE, 5, FAKE, None,
                                  None, None, None, FAKE, 1 << 30, 0, None) == L.LIP_E_ARG


def test_smooth_entry_point_validation(L):
    lib = L.load()
    m, keep = _metric(L)

    def sm(n=10, M=1.0, eps=FAKE, p=1.0, prune=0.0, ws=FAKE, ws_bytes=1 << 30, flags=0):
        return lib.lip_smooth_objective(ctypes.byref(m), FAKE, FAKE, n, M, None, eps, p, prune,
                                        FAKE, FAKE, ws, ws_bytes, flags, None)
    assert sm(n=0) == L.LIP_E_SHAPE
    assert sm(M=-1.0) == L.LIP_E_VALUE
    assert sm(p=0.0) == L.LIP_E_VALUE
    assert sm(p=float("inf")) == L.LIP_E_VALUE
    assert sm(prune=-0.5) == L.LIP_E_VALUE
    assert sm(prune=float("nan")) == L.LIP_E_VALUE
    assert sm(prune=float("inf")) == L.LIP_E_VALUE
    assert sm(eps=None) == L.LIP_E_ARG
    assert sm(ws_bytes=16) == L.LIP_E_WORKSPACE
    assert sm(flags=L.LIP_FLAG_BF16) == L.LIP_E_ARG


def test_fit_eval_k_validation(L):
    lib = L.load()
    m, keep = _metric(L)
    wk = np.array([0.5, 0.5], np.float32)
    neg = np.array([0.5, -0.5], np.float32)
    pp = lambda a: a.ctypes.data_as(ctypes.c_void_p)

    def ev(n=10, k=2, w=wk, q=5, flags=0, ws_bytes=1 << 30):
        return lib.lip_fit_eval_k(ctypes.byref(m), FAKE, FAKE, n, 1.0, None, k, pp(w), FAKE, q,
                                  FAKE, None, None, FAKE, ws_bytes, flags, None)
    assert ev(k=0) == L.LIP_E_SHAPE
    assert ev(k=L.LIP_MAX_K + 1, n=100) == L.LIP_E_SHAPE
    assert ev(n=1, k=2) == L.LIP_E_SHAPE
    assert ev(w=neg) == L.LIP_E_VALUE
    assert ev(flags=L.LIP_FLAG_BF16) == L.LIP_E_UNSUPPORTED
    assert ev(ws_bytes=16) == L.LIP_E_WORKSPACE
    assert ev(q=0) == L.LIP_OK


def test_regional_metric_validation(L):
    lib = L.load()
    kind = np.array([2, 0, 5], np.int8)
    a = np.array([0.1, 0.0, 0.2], np.float32)
    b = np.array([0.5, 0.0, 0.1], np.float32)   # b < a in coordinate 2
    good_b = np.array([0.5, 0.0, 0.3], np.float32)
    pp = lambda v: v.ctypes.data_as(ctypes.c_void_p)
    m_bad = L.LipMetric(3, 2, None, pp(kind), pp(a), pp(b))
    m_noab = L.LipMetric(3, 2, None, pp(kind), None, None)
    m_ok = L.LipMetric(3, 2, None, pp(kind), pp(a), pp(good_b))

    def ev(m, q=0):
        return lib.lip_fit_eval(ctypes.byref(m), FAKE, FAKE, 10, 1.0, None, FAKE, q, FAKE, None,
                                None, None, None, FAKE, 1 << 30, 0, None)
    assert ev(m_bad) == L.LIP_E_VALUE
    assert ev(m_noab) == L.LIP_E_ARG
    assert ev(m_ok) == L.LIP_OK  # q = 0: validated, no device work
    bad_kind = np.array([6, 0, 0], np.int8)
    assert ev(L.LipMetric(3, 2, None, pp(bad_kind), pp(a), pp(good_b))) == L.LIP_E_VALUE
    # the other entry points do not take the regional kinds
    assert lib.lip_consistency(ctypes.byref(m_ok), FAKE, FAKE, 10, 1.0, None, 0.0, FAKE, None, None, None,
                               None, None, None, FAKE, 1 << 30, 0, None) == L.LIP_E_UNSUPPORTED
