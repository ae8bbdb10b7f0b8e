"""Host-side checks of libte that need no GPU: exported symbols and plan validation."""
import ctypes
import os
import re

import numpy as np
import pytest

import synth

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "te.h")


def _lib_or_build():
    from paper_1401_4068_amd import _lib
    if not os.path.exists(_lib.LIB_PATH):
        from paper_1401_4068_amd import build
        build.build()
    return _lib


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(te_[a-z_0-9]+)\s*\(", text)))


def test_library_exports_every_declared_function():
    _lib = _lib_or_build()
    L = ctypes.CDLL(_lib.LIB_PATH)
    names = declared_functions()
    assert "te_plan_create" in names and "te_knn_counts" in names
    for n in names:
        assert hasattr(L, n), n
    assert set(names) <= set(_lib.SIGNATURES), set(names) - set(_lib.SIGNATURES)


def _plan(**kw):
    from paper_1401_4068_amd import Plan
    args = dict(n_pairs=1, n_trials=20, n_samples=50, d_y=2, d_x=2, tau=1, u=1, k=4, window_start=[10],
                window_len=[10], trials=None, n_surrogates=0)
    args.update(kw)
    return Plan(**args)


def test_plan_sizes_without_gpu():
    _lib_or_build()
    p = _plan(n_surrogates=5, window_start=[10, 20, 30], window_len=[10, 5, 8], trials=[20, 10, 15])
    full, mn, plain = p.workspace_bytes()
    assert full >= mn > 0 and plain > 0
    # coordinate storage alone: per window (1 + d_y) N + (S + 1) d_x N floats
    N = np.array([200, 50, 120])
    assert full >= 4 * np.sum(N * 3 + 6 * N * 2)


@pytest.mark.parametrize("bad,msg", [
    (dict(d_y=0), "d_y and d_x"),
    (dict(d_x=5), "d_y and d_x"),
    (dict(k=0), "k must be"),
    (dict(k=16), "k must be"),
    (dict(tau=0), "tau and u"),
    (dict(u=0), "tau and u"),
    (dict(window_start=[1]), "history"),                       # needs 2 samples of history
    (dict(window_start=[45], window_len=[10]), "past n_samples"),
    (dict(window_len=[0]), "length"),
    (dict(trials=[21]), "trials"),
    (dict(trials=[1], window_len=[4]), "need more than k"),     # N = 4 <= k
    (dict(n_trials=1 << 14, n_samples=(1 << 14) + 10, window_len=[1 << 14]), "more than 134217728"),  # N = 2^28
    (dict(n_surrogates=-1), "n_surrogates"),
    (dict(window_start=[], window_len=None), "n_points"),        # no analysis window at all
])
def test_plan_rejects_invalid_geometry(bad, msg):
    from paper_1401_4068_amd import TEError
    _lib_or_build()
    with pytest.raises(TEError) as ei:
        _plan(**bad)
    assert ei.value.status == 1 and msg in str(ei.value)


def test_plan_accepts_the_largest_window():
    _lib_or_build()
    p = _plan(n_trials=1 << 13, n_samples=(1 << 14) + 10, window_len=[1 << 14], n_surrogates=1)   # N = 2^27
    assert p.workspace_bytes()[0] > 4 * 3 * (1 << 27)


def test_history_rule_matches_embedding():
    # d_y = 4, d_x = 4, tau = 2, u = 5: history = max(1 + 3*2, 5 + 3*2) = 11
    assert synth.history(4, 4, 2, 5) == 11
    _lib_or_build()
    _plan(d_y=4, d_x=4, tau=2, u=5, window_start=[11])
    from paper_1401_4068_amd import TEError
    with pytest.raises(TEError):
        _plan(d_y=4, d_x=4, tau=2, u=5, window_start=[10])


def test_tuning_table_roundtrip(tmp_path):
    import paper_1401_4068_amd as te
    _lib_or_build()
    src = tmp_path / "tune.txt"
    src.write_text("3 3 4 12 16 2 3 1.5\n2 2 4 11 4 1 6 0.25\n9 9 4 11 4 1 6 0.25\n3 3 4 13 5 2 3 1.0\n")
    te.tune_clear()
    te.tune_load(src)                                 # invalid rows (d = 9, slots = 5) are skipped
    out = tmp_path / "out.txt"
    te.tune_save(out)
    rows = sorted(out.read_text().split("\n"))
    rows = [r for r in rows if r]
    assert [r.split()[:7] for r in rows] == [["2", "2", "4", "11", "4", "1", "6"], ["3", "3", "4", "12", "16", "2", "3"]]
    te.tune_clear()
    empty = tmp_path / "empty.txt"
    empty.write_text("garbage\n")
    with pytest.raises(te.TEError):
        te.tune_load(empty)


def test_delay_scan_sizes_and_validation_without_gpu():
    import paper_1401_4068_amd as te
    _lib_or_build()
    wl = synth.generic((31, 7), n_pairs=2, R=120, T=80, d_y=2, d_x=2, u=3, starts=(20, 35, 50),
                       windows=(10, 7, 15), trials=(120, 80, 100), n_surrogates=5)
    p = te.Plan.from_workload(wl)
    full, minimum = p.delay_scan_workspace_bytes([1, 2, 3])
    assert full > minimum > 0
    # more delays need more room: one source block per delay
    assert p.delay_scan_workspace_bytes(list(range(1, 10)))[0] > full
    for bad, msg in (([20], "start at sample >= 21"), ([0], ">= 1"), ([], "n_u")):
        with pytest.raises(te.TEError) as ei:
            p.delay_scan_workspace_bytes(bad)
        assert ei.value.status == 1 and msg in str(ei.value)


def test_conditioning_needs_room_in_the_target_past():
    import paper_1401_4068_amd as te
    _lib_or_build()
    _plan(d_y=3, cond_source=1)
    with pytest.raises(te.TEError) as ei:
        _plan(d_y=4, cond_source=1)
    assert "d_y <= 3" in str(ei.value)
    with pytest.raises(te.TEError):
        _plan(cond_source=2)


def test_async_rejects_missing_arguments_without_gpu():
    """te_surrogates_async checks its arguments before it touches the device."""
    from paper_1401_4068_amd import _lib
    _lib_or_build()
    L = _lib.lib()
    p = _plan(n_surrogates=3)
    dummy = ctypes.c_void_p(1 << 20)                 # never dereferenced: the calls fail first
    null = ctypes.c_void_p(0)
    cases = [
        (null, dummy, dummy, dummy, dummy, dummy),   # no plan
        (p._h, null, dummy, dummy, dummy, dummy),    # no x
        (p._h, dummy, dummy, dummy, dummy, null),    # no out
    ]
    for plan, x, y, perms, ws, out in cases:
        st = L.te_surrogates_async(plan, x, y, perms, ws, 1 << 20, null, out)
        assert st == 1, st
        assert L.te_last_error() is not None


def test_drawn_permutation_sizes_and_checks_without_gpu():
    """Surrogates without caller permutations are drawn from the plan's seed; the
    permutation export sizes its workspace and checks its arguments on the host."""
    from paper_1401_4068_amd import _lib
    _lib_or_build()
    L = _lib.lib()
    p = _plan(n_surrogates=3, window_start=[10, 20], window_len=[10, 5], trials=[20, 12], seed=7)
    nb = L.te_plan_permutations_workspace_bytes(p._h)
    assert nb >= 6 * 40                               # one 40-byte row descriptor per surrogate chunk
    assert L.te_plan_permutations_workspace_bytes(ctypes.c_void_p(0)) == 0
    null = ctypes.c_void_p(0)
    assert L.te_plan_permutations(p._h, null, nb, null, ctypes.c_void_p(1 << 20)) == 1
    assert L.te_plan_permutations(p._h, ctypes.c_void_p(1 << 20), nb - 1, null, ctypes.c_void_p(1 << 20)) == 2
    q = _plan(n_surrogates=0)
    assert L.te_plan_permutations(q._h, ctypes.c_void_p(1 << 20), 256, null, ctypes.c_void_p(1 << 20)) == 0


@pytest.mark.parametrize("dims,taus,k,w,W,msg", [
    ([9], [1], 4, 20, 10, "candidate 0"),            # d above 8
    ([2], [0], 4, 20, 10, "candidate 0"),            # tau below 1
    ([3], [4], 4, 8, 10, "history"),                 # needs 1 + 2 * 4 = 9 samples before the window
    ([1], [1], 0, 20, 10, "k must be"),
    ([1], [1], 17, 20, 10, "k must be"),
    ([1], [1], 4, 45, 10, "runs past"),
    ([1], [1], 4, 20, 1, "points"),                  # N = 2 trials x 1 <= k
    ([], [], 4, 20, 10, "n_cand"),
])
def test_ragwitz_rejects_invalid_geometry_without_gpu(dims, taus, k, w, W, msg):
    """Validation happens before any device call (fake device pointers are never used)."""
    from paper_1401_4068_amd import TEError
    from paper_1401_4068_amd._lib import check
    L = _lib_or_build().lib()
    i32p = ctypes.POINTER(ctypes.c_int32)
    d = np.array(dims + [1], np.int32)
    t = np.array(taus + [1], np.int32)
    score = np.zeros(4)
    with pytest.raises(TEError) as ei:
        check(L.te_ragwitz(ctypes.c_void_p(16), 2, 50, w, W, d.ctypes.data_as(i32p), t.ctypes.data_as(i32p),
                           len(dims), k, ctypes.c_void_p(256), 1 << 20, None, None,
                           score.ctypes.data_as(ctypes.POINTER(ctypes.c_double))))
    assert ei.value.status == 1 and msg in str(ei.value)
