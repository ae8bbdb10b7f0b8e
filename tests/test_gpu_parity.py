"""GPU parity: libte (through its C interface) against the CPU oracle.

Bars: radii and the three neighbour counts bit-exact for every point; TE within
1e-6 nats of the oracle (the required tolerance).  With identical counts the only
difference left is float64 summation order (about 1e-13), so TE is also checked
at 1e-9, a level a single differing count (>= 1/N^2, about 4e-8 at N = 5000)
would exceed.
"""
import math
import sys
import zlib

import numpy as np
import pytest

import synth
from oracle import oracle
from synth.rng import derive_key, normal64, uniform01

pytestmark = pytest.mark.gpu

TOL = 1e-6
TIGHT = 1e-9


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def te():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1401_4068_amd as te
    te.lib()
    return te


def dev(wl):
    import torch
    x = torch.from_numpy(np.ascontiguousarray(wl.x)).cuda()
    y = torch.from_numpy(np.ascontiguousarray(wl.y)).cuda()
    perms = None if wl.perms is None or wl.n_surrogates == 0 else torch.from_numpy(np.ascontiguousarray(wl.perms)).cuda()
    return x, y, perms


# ------------------------------------------------------------ kernel level

def _points(key, N, D, kind):
    if kind == "gauss":
        return normal64(key, N * D).reshape(N, D).astype(np.float32)
    if kind == "grid":
        return np.floor(uniform01(key, N * D) * 5).reshape(N, D).astype(np.float32)
    if kind == "dups":
        base = np.floor(uniform01(key, (N // 4 + 1) * D) * 3).reshape(-1, D)
        idx = np.floor(uniform01(derive_key(key, 3), N) * base.shape[0]).astype(int)
        return base[idx].astype(np.float32)
    if kind == "subnormal":       # differences land in the binary32 subnormal range
        return (normal64(key, N * D).reshape(N, D) * 2.0 ** -130).astype(np.float32)
    if kind == "fine":
        return (1.0 + uniform01(key, N * D).reshape(N, D) * 2.0 ** -18).astype(np.float32)
    raise ValueError(kind)


def _knn_case(te, sizes, d_y, d_x, k, kind, seed=0):
    import torch
    D = 1 + d_y + d_x
    chunks = [_points(derive_key(seed, n, D, k, zlib.crc32(kind.encode()) & 0xFFFF), n, D, kind) for n in sizes]
    off = np.zeros(len(sizes) + 1, np.int64)
    off[1:] = np.cumsum(sizes)
    stride = int(off[-1]) + 37            # coordinate stride larger than the point count
    soa = np.zeros((D, stride), np.float32)
    soa[:, :off[-1]] = np.concatenate(chunks).T
    say("knn case", dict(sizes=sizes, d_y=d_y, d_x=d_x, k=k, kind=kind))
    eps, cnt, tev = te.knn_counts(torch.from_numpy(soa).cuda(), off, d_y, d_x, k)
    torch.cuda.synchronize()
    eps = eps.cpu().numpy()
    cnt = cnt.cpu().numpy()
    ref = oracle.counts_batch(chunks, d_y, d_x, k)
    for c, (re, rc) in enumerate(ref):
        sl = slice(off[c], off[c + 1])
        np.testing.assert_array_equal(eps[sl], re.astype(np.float32), err_msg="eps chunk %d" % c)
        assert np.all(re.astype(np.float32).astype(np.float64) == re)
        np.testing.assert_array_equal(cnt[:, sl], rc, err_msg="counts chunk %d" % c)
        t_ref = oracle.te_from_counts(rc, k)
        assert abs(tev[c] - t_ref) <= TIGHT, (c, tev[c], t_ref)


@pytest.mark.parametrize("d_y,d_x", [(1, 1), (2, 2), (3, 3), (4, 4), (1, 4), (3, 2)])
@pytest.mark.parametrize("kind", ["gauss", "grid", "dups"])
def test_knn_counts_bit_exact(te, d_y, d_x, kind):
    _knn_case(te, [5, 64, 65, 127, 300, 1031], d_y, d_x, 4, kind)


@pytest.mark.parametrize("k", [1, 2, 7, 15])
def test_knn_counts_other_k(te, k):
    _knn_case(te, [k + 1, 70, 513], 2, 3, k, "gauss")
    _knn_case(te, [k + 1, 200], 3, 3, k, "grid")


@pytest.mark.parametrize("kind", ["subnormal", "fine"])
def test_knn_counts_rounding_edge_values(te, kind):
    _knn_case(te, [130, 700], 3, 3, 4, kind)


def test_knn_counts_large_chunk_multi_tile(te):
    _knn_case(te, [4100, 2500, 33], 3, 3, 4, "gauss", seed=5)


@pytest.mark.parametrize("kind", ["grid", "dups"])
def test_knn_counts_tiled_walk_with_ties(te, kind):
    """Chunks of at least 8 192 points (pass 1 walks outward in tiles) on grid and
    duplicated points, where distances tie everywhere."""
    _knn_case(te, [8192, 9001], 3, 3, 4, kind, seed=7)


# ------------------------------------------------------------ full estimates

def _compare(wl, te_orig, te_surr=None, pv=None, points=None):
    ref = oracle.te_workload(wl, points=points)
    for (p, c, s), r in ref.items():
        got = te_orig[p, c] if s == 0 else te_surr[p, c, s - 1]
        assert abs(got - r) <= TOL, ((p, c, s), got, r)
        assert abs(got - r) <= TIGHT, ((p, c, s), got, r)
    if pv is not None and wl.n_surrogates:
        for p in range(wl.n_pairs):
            for c in (range(wl.n_points) if points is None else points):
                rs = [ref[(p, c, s)] for s in range(1, wl.n_surrogates + 1)]
                assert pv[p, c] == oracle.p_value(ref[(p, c, 0)], rs)


def test_linear_pair_single_estimate_full_size(te):
    """Linear Gaussian AR(1) pair, 100 trials x 20-sample window -> N = 2000, D = 5, k = 4."""
    wl = synth.linear_pair()
    say("linear pair", wl.chunk_sizes())
    x, y, _ = dev(wl)
    plan = te.Plan.from_workload(wl)
    out = plan.estimate(x, y)
    _compare(wl, out)
    t0, _, pv = plan.surrogates(x, y)
    assert t0[0, 0] == out[0, 0]
    assert math.isnan(pv[0, 0])


def test_uneven_chunks_with_surrogates(te):
    wl = synth.uneven_surrogates(R=300, T=60, n_points=6, n_surrogates=7, n_lo=100, n_hi=2600)
    say("uneven", wl.chunk_sizes(), wl.trials, wl.window_len)
    x, y, perms = dev(wl)
    plan = te.Plan.from_workload(wl)
    t0, ts, pv = plan.surrogates(x, y, perms)
    _compare(wl, t0, ts, pv)


def test_meg_like_pairs_tau2(te):
    wl = synth.meg_like(n_pairs=3, R=20, T=160, n_points=4, n_surrogates=3, on=60, off=120)
    say("meg-like", wl.chunk_sizes())
    x, y, perms = dev(wl)
    plan = te.Plan.from_workload(wl)
    t0, ts, pv = plan.surrogates(x, y, perms)
    _compare(wl, t0, ts, pv)
    plain = plan.estimate(x, y)
    np.testing.assert_array_equal(plain, t0)


def test_nonlinear_full_size_sampled(te):
    """500 trials x 300 samples, 100 windows of 10 samples (N = 5000, D = 7): all windows on the
    GPU, both paths; the oracle checks a seeded sample of windows."""
    wl = synth.nonlinear_ensemble()
    say("nonlinear full", wl.n_points, wl.chunk_sizes()[0])
    x, y, _ = dev(wl)
    plan = te.Plan.from_workload(wl)
    t0, _, _ = plan.surrogates(x, y)
    plain = plan.estimate(x, y)
    np.testing.assert_array_equal(plain, t0)
    pts = sorted(set(np.floor(uniform01(derive_key(99), 6) * wl.n_points).astype(int).tolist()) | {0, 99})
    _compare(wl, t0, points=pts)


def test_split_workspace_gives_identical_results(te):
    import torch
    wl = synth.uneven_surrogates(R=200, T=60, n_points=5, n_surrogates=4, n_lo=100, n_hi=1500)
    x, y, perms = dev(wl)
    plan = te.Plan.from_workload(wl)
    full, mn, _ = plan.workspace_bytes()
    a = plan.surrogates(x, y, perms)
    ws_small = torch.empty(mn, dtype=torch.uint8, device="cuda")
    say("split", full, mn)
    b = plan.surrogates(x, y, perms, ws=ws_small)
    for u, v in zip(a, b):
        np.testing.assert_array_equal(u, v)


def test_graph_replay_matches_eager(te):
    import torch
    wl = synth.uneven_surrogates(R=120, T=60, n_points=3, n_surrogates=5, n_lo=100, n_hi=1200)
    x, y, perms = dev(wl)
    plan = te.Plan.from_workload(wl)
    eager = plan.surrogates(x, y, perms)
    s = torch.cuda.Stream()
    for rep in range(4):
        say("graph replay", rep)
        g = plan.surrogates(x, y, perms, stream=s, use_graph=True)
        for u, v in zip(eager, g):
            np.testing.assert_array_equal(u, v)
        # unrelated eager work between replays
        z = torch.randn(1 << 16, device="cuda").sum()
        torch.cuda.synchronize()
        assert torch.isfinite(z)


def _async_split(plan, a):
    G, S = plan.n_pairs * plan.n_points, plan.n_surrogates
    est = a[:G * (S + 1)].reshape(plan.n_pairs, plan.n_points, S + 1)
    return est[..., 0], est[..., 1:], a[G * (S + 1):].reshape(plan.n_pairs, plan.n_points)


def test_async_matches_batched(te):
    import torch
    wl = synth.uneven_surrogates(R=150, T=60, n_points=4, n_surrogates=3, n_lo=300, n_hi=1500)
    x, y, perms = dev(wl)
    plan = te.Plan.from_workload(wl)
    t0, ts, pv = plan.surrogates(x, y, perms)
    G, S = plan.n_pairs * plan.n_points, plan.n_surrogates
    s = torch.cuda.Stream()
    ws = plan.workspace()
    say("async: three calls back to back on one workspace, then one into pinned host memory")
    outs = [plan.surrogates_async(x, y, perms, ws=ws, stream=s) for _ in range(3)]
    host = torch.empty(G * (S + 1) + G, dtype=torch.float64).pin_memory()
    plan.surrogates_async(x, y, perms, ws=ws, stream=s, out=host)
    s.synchronize()
    for o in outs + [host]:
        a0, a1, a2 = _async_split(plan, o.cpu().numpy())
        np.testing.assert_array_equal(a0, t0)
        np.testing.assert_array_equal(a1, ts)
        np.testing.assert_array_equal(a2, pv)
    full, mn, _ = plan.workspace_bytes()
    assert mn < full
    with pytest.raises(te.TEError) as ei:
        plan.surrogates_async(x, y, perms, ws=torch.empty(mn, dtype=torch.uint8, device="cuda"))
    assert ei.value.status == 2


def test_async_two_streams_share_a_plan(te):
    import torch
    wl = synth.uneven_surrogates(R=120, T=60, n_points=3, n_surrogates=4, n_lo=200, n_hi=1500)
    x, y, perms = dev(wl)
    plan = te.Plan.from_workload(wl)
    t0, ts, pv = plan.surrogates(x, y, perms)
    streams = [torch.cuda.Stream(), torch.cuda.Stream()]
    wss = [plan.workspace(), plan.workspace()]
    G, S = plan.n_pairs * plan.n_points, plan.n_surrogates
    outs = [torch.empty(G * (S + 1) + G, dtype=torch.float64, device="cuda") for _ in range(2)]
    say("async: 10 calls alternating over two streams and workspaces")
    for i in range(10):
        plan.surrogates_async(x, y, perms, ws=wss[i % 2], stream=streams[i % 2], out=outs[i % 2])
    torch.cuda.synchronize()
    for o in outs:
        a0, a1, a2 = _async_split(plan, o.cpu().numpy())
        np.testing.assert_array_equal(a0, t0)
        np.testing.assert_array_equal(a1, ts)
        np.testing.assert_array_equal(a2, pv)


def test_large_batch_pvalues_in_their_own_kernel(te):
    """Over 1 024 chunks the p-values (and the error word) come from a kernel of their own."""
    import torch
    wl = synth.uneven_surrogates(R=100, T=60, n_points=6, n_surrogates=200, n_lo=100, n_hi=600)
    assert wl.n_pairs * wl.n_points * (wl.n_surrogates + 1) > 1024
    x, y, perms = dev(wl)
    plan = te.Plan.from_workload(wl)
    t0, ts, pv = plan.surrogates(x, y, perms)
    say("large batch", wl.chunk_sizes().min(), wl.chunk_sizes().max())
    _compare(wl, t0, ts, pv)
    out = plan.surrogates_async(x, y, perms)
    torch.cuda.synchronize()
    a0, a1, a2 = _async_split(plan, out.cpu().numpy())
    np.testing.assert_array_equal(a0, t0)
    np.testing.assert_array_equal(a1, ts)
    np.testing.assert_array_equal(a2, pv)
    # invalid input: an error on the synchronous path, all NaN on the queued one
    wl.y[0, 3, int(wl.window_start[0]) + 1] = np.nan
    x, y, perms = dev(wl)
    with pytest.raises(te.TEError):
        plan.surrogates(x, y, perms)
    out = plan.surrogates_async(x, y, perms)
    torch.cuda.synchronize()
    assert np.isnan(out.cpu().numpy()).all()


def test_async_without_surrogates_and_invalid_input(te):
    import torch
    wl = synth.generic((15,), R=30, T=40, starts=(20,), windows=(10,))
    x, y, _ = dev(wl)
    plan = te.Plan.from_workload(wl)
    t0, _, _ = plan.surrogates(x, y)
    out = plan.surrogates_async(x, y)
    torch.cuda.synchronize()
    a0, a1, a2 = _async_split(plan, out.cpu().numpy())
    np.testing.assert_array_equal(a0, t0)
    assert a1.size == 0 and np.isnan(a2).all()
    wl.y[0, 3, 25] = np.nan                                 # target future of point (3, 25)
    x, y, _ = dev(wl)
    out = plan.surrogates_async(x, y)
    torch.cuda.synchronize()
    assert np.isnan(out.cpu().numpy()).all()


def test_runs_are_bitwise_reproducible(te):
    wl = synth.uneven_surrogates(R=150, T=60, n_points=4, n_surrogates=3, n_lo=300, n_hi=1500)
    x, y, perms = dev(wl)
    plan = te.Plan.from_workload(wl)
    a = plan.surrogates(x, y, perms)
    b = plan.surrogates(x, y, perms)
    for u, v in zip(a, b):
        np.testing.assert_array_equal(u, v)


def test_identity_surrogates_equal_original(te):
    import torch
    wl = synth.generic((12,), R=30, T=40, starts=(20,), windows=(10,), n_surrogates=3)
    wl.perms[:] = np.arange(wl.n_trials, dtype=np.int32)
    x, y, perms = dev(wl)
    plan = te.Plan.from_workload(wl)
    t0, ts, pv = plan.surrogates(x, y, perms)
    assert np.all(ts[0, 0] == t0[0, 0])
    assert pv[0, 0] == 1.0


def test_nonfinite_input_is_rejected(te):
    import torch
    wl = synth.generic((13,), R=30, T=40, starts=(20,), windows=(10,))
    # window [20, 30) with d_y = d_x = 2, tau = 1, u = 1 reads samples 18..29 only
    wl.y[0, 3, 17] = np.nan
    wl.x[0, 5, 3] = np.inf
    x, y, _ = dev(wl)
    plan = te.Plan.from_workload(wl)
    assert np.isfinite(plan.estimate(x, y)).all()          # values outside the windows are never read
    wl.y[0, 3, 25] = np.nan                                 # target future of point (3, 25)
    x, y, _ = dev(wl)
    with pytest.raises(te.TEError) as ei:
        plan.estimate(x, y)
    assert ei.value.status == 1
    with pytest.raises(te.TEError):
        plan.surrogates(x, y)
    wl.y[0, 3, 25] = 1.0
    wl.x[0, 7, 18] = -np.inf                                # source past of point (7, 19)
    x, y, _ = dev(wl)
    with pytest.raises(te.TEError):
        plan.surrogates(x, y)


def test_invalid_permutation_is_rejected(te):
    import torch
    wl = synth.generic((14,), R=30, T=40, starts=(20,), windows=(10,), n_surrogates=2)
    wl.perms[0, 0, 1, 4] = wl.perms[0, 0, 1, 5]      # duplicate entry
    x, y, perms = dev(wl)
    plan = te.Plan.from_workload(wl)
    with pytest.raises(te.TEError) as ei:
        plan.surrogates(x, y, perms)
    assert ei.value.status == 1
    wl.perms[0, 0, 1, 4] = 30                        # out of range
    x, y, perms = dev(wl)
    with pytest.raises(te.TEError):
        plan.surrogates(x, y, perms)


@pytest.mark.parametrize("slots,wpg,wg", [(4, 1, 3), (16, 2, 1), (8, 1, 7), (16, 4, 0)])
def test_results_do_not_depend_on_launch_shape(te, monkeypatch, slots, wpg, wg):
    wl = synth.uneven_surrogates(R=150, T=60, n_points=3, n_surrogates=3, n_lo=300, n_hi=3000)
    x, y, perms = dev(wl)
    ref = te.Plan.from_workload(wl).surrogates(x, y, perms)
    monkeypatch.setenv("TE_SLOTS", str(slots))
    monkeypatch.setenv("TE_WAVES_PER_WG", str(wpg))
    if wg:
        monkeypatch.setenv("TE_WG_PER_CU", str(wg))
    say("shape", slots, wpg, wg)
    got = te.Plan.from_workload(wl).surrogates(x, y, perms)
    for u, v in zip(ref, got):
        np.testing.assert_array_equal(u, v)


def test_autotune_records_a_valid_shape(te, tmp_path):
    r = te.autotune(3, 3, 4, 2000, n_chunks=40)
    say("tuned", r)
    assert r["slots"] in (4, 8, 16) and 1 <= r["waves_per_wg"] <= 4 and r["wg_per_cu"] >= 1 and r["ms"] > 0
    path = tmp_path / "tune.txt"
    te.tune_save(path)
    row = path.read_text().split()
    assert row[:7] == ["3", "3", "4", "10", str(r["slots"]), str(r["waves_per_wg"]), str(r["wg_per_cu"])]
    # a plan created now uses the tuned shape; its estimates are unchanged
    wl = synth.generic((31,), R=100, T=40, d_y=3, d_x=3, starts=(20,), windows=(20,))
    x, y, _ = dev(wl)
    a = te.Plan.from_workload(wl).estimate(x, y)
    te.tune_clear()
    b = te.Plan.from_workload(wl).estimate(x, y)
    np.testing.assert_array_equal(a, b)


def test_knn_counts_chunk_larger_than_lds_sort(te):
    """N = 17 000 pads to 32 768 keys: the sort runs in global scratch with LDS tiles."""
    _knn_case(te, [17000, 700], 2, 2, 4, "gauss", seed=11)


def test_work_counters_and_pruning(te):
    """Sorted search spaces evaluate fewer pairs than N(N-1) per pass; counters report them."""
    wl = synth.nonlinear_ensemble(R=300, T=60, n_points=4, window=10)
    x, y, _ = dev(wl)
    plan = te.Plan.from_workload(wl)
    te.profile_enable(True, work=True)
    te.profile_work(reset=True)
    plan.surrogates(x, y)
    w1, w2 = te.profile_work(reset=True)
    te.profile_enable(False)
    n = wl.chunk_sizes()
    method = int(np.sum(n * (n - 1)))
    say("evaluated", w1, w2, "method", method)
    assert 0 < w1 <= method + int(np.sum(n)) and 0 < w2 <= method + int(np.sum(n))


@pytest.mark.parametrize("no_sort", [False, True])
def test_local_te_per_point(te, monkeypatch, no_sort):
    """Per-point local TE (eq. 17 on the pooled points) against the oracle, point by point in
    window order; its window means are the estimates (eq. 18)."""
    if no_sort:
        monkeypatch.setenv("TE_NO_SORT", "1")
    wl = synth.uneven_surrogates(R=220, T=60, n_points=4, n_surrogates=0, n_lo=90, n_hi=2100)
    say("local", no_sort, wl.chunk_sizes())
    x, y, _ = dev(wl)
    plan = te.Plan.from_workload(wl)
    parts, te_out = plan.local(x, y)
    t0, _, _ = plan.surrogates(x, y)
    np.testing.assert_array_equal(te_out, t0)
    for p in range(wl.n_pairs):
        for c in range(wl.n_points):
            got = parts[p * wl.n_points + c].cpu().numpy()
            pts = oracle.embed(wl.x[p], wl.y[p], wl.d_y, wl.d_x, wl.tau, wl.u, int(wl.window_start[c]),
                               int(wl.window_len[c]), int(wl.trials[c]))
            ref = oracle.local_te(pts, wl.d_y, wl.d_x, wl.k)
            assert got.shape == ref.shape
            np.testing.assert_allclose(got, ref, rtol=0, atol=1e-12)
            assert abs(got.mean() - te_out[p, c]) <= 1e-12


def _scan_workload(n_surrogates=5):
    return synth.generic((31, 7), n_pairs=2, R=120, T=80, d_y=2, d_x=2, u=3, starts=(20, 35, 50),
                         windows=(10, 7, 15), trials=(120, 80, 100), n_surrogates=n_surrogates, coupling=0.6)


def _check_scan(wl, u_values, got):
    te_scan, u_best, te_surr, pv = got
    ref_scan, ref_best, ref_surr, ref_pv = oracle.delay_scan(wl, u_values)
    for (p, c), r in ref_scan.items():
        assert np.max(np.abs(te_scan[p, c] - r)) <= TIGHT, (p, c)
        top = np.sort(r)[::-1]
        if len(top) > 1 and top[0] - top[1] < 1e-9:       # a near tie: either delay is a maximum
            assert r[u_values.index(int(u_best[p, c]))] >= top[0] - 1e-9
            continue
        assert u_best[p, c] == ref_best[(p, c)], (p, c)
        if wl.n_surrogates:
            assert np.max(np.abs(te_surr[p, c] - ref_surr[(p, c)])) <= TIGHT, (p, c)
            assert pv[p, c] == ref_pv[(p, c)]
        else:
            assert math.isnan(pv[p, c])


def test_delay_scan_matches_oracle(te):
    """eq. 5: originals at every delay, the device-side argmax, surrogates at the chosen delay."""
    wl = _scan_workload()
    u_values = [1, 2, 3, 4, 5, 6, 7, 8, 3]
    x, y, perms = dev(wl)
    plan = te.Plan.from_workload(wl)
    got = plan.delay_scan(x, y, u_values, perms)
    say("scan", got[1].tolist())
    _check_scan(wl, u_values, got)
    np.testing.assert_array_equal(got[0][:, :, 2], got[0][:, :, 8])      # repeated delay, same estimate
    # the scan at the plan's own delay equals te_surrogates
    t0, ts, pv = plan.surrogates(x, y, perms)
    np.testing.assert_array_equal(got[0][:, :, 2], t0)


def test_delay_scan_split_workspace_and_no_surrogates(te):
    import torch
    wl = _scan_workload()
    u_values = [2, 4, 6, 1, 3]
    x, y, perms = dev(wl)
    plan = te.Plan.from_workload(wl)
    full, minimum = plan.delay_scan_workspace_bytes(u_values)
    assert full > minimum > 0
    a = plan.delay_scan(x, y, u_values, perms)
    ws = torch.empty(minimum, dtype=torch.uint8, device="cuda")
    b = plan.delay_scan(x, y, u_values, perms, ws=ws)
    for u, v in zip(a, b):
        np.testing.assert_array_equal(u, v)
    wl0 = _scan_workload(n_surrogates=0)
    plan0 = te.Plan.from_workload(wl0)
    got = plan0.delay_scan(x, y, u_values)
    assert got[2] is None
    _check_scan(wl0, u_values, got)


def test_delay_scan_rejects_delays_without_history(te):
    wl = _scan_workload()
    x, y, perms = dev(wl)
    plan = te.Plan.from_workload(wl)
    for bad in ([20], [0], []):
        with pytest.raises(te.TEError) as ei:
            plan.delay_scan(x, y, bad, perms)
        assert ei.value.status == 1


def test_plan_autotune_on_own_data(te):
    """Tuning on the plan's data picks a valid shape; the estimates do not change."""
    wl = synth.uneven_surrogates(R=150, T=60, n_points=3, n_surrogates=3, n_lo=300, n_hi=3000)
    x, y, perms = dev(wl)
    plan = te.Plan.from_workload(wl)
    ref = plan.surrogates(x, y, perms)
    r = plan.autotune(x, y, perms)
    say("plan tuned", r)
    assert r["slots"] in (4, 8, 16) and 1 <= r["waves_per_wg"] <= 4 and r["wg_per_cu"] >= 1 and r["ms"] > 0
    got = plan.surrogates(x, y, perms)
    for u, v in zip(ref, got):
        np.testing.assert_array_equal(u, v)
    te.tune_clear()


def test_conditioning_on_current_source(te):
    """x_t in the conditioning set (stored as row 0 of each source block, so it follows the
    trial shuffle): batched, plain and served paths against the oracle."""
    wl = synth.generic((88,), n_pairs=2, R=150, T=70, d_y=2, d_x=2, u=2, starts=(20, 35, 50),
                       windows=(10, 7, 15), trials=(150, 90, 120), n_surrogates=4, coupling=0.6)
    wl.cond_source = 1
    x, y, perms = dev(wl)
    plan = te.Plan.from_workload(wl)
    t0, ts, pv = plan.surrogates(x, y, perms)
    _compare(wl, t0, ts, pv)
    np.testing.assert_array_equal(plan.estimate(x, y), t0)
    # without the conditioning the estimates differ (the flag reaches the kernels)
    wl0 = synth.generic((88,), n_pairs=2, R=150, T=70, d_y=2, d_x=2, u=2, starts=(20, 35, 50),
                        windows=(10, 7, 15), trials=(150, 90, 120), n_surrogates=4, coupling=0.6)
    u0 = te.Plan.from_workload(wl0).surrogates(x, y, perms)[0]
    assert np.max(np.abs(u0 - t0)) > 1e-3
    srv = te.Server(arena_bytes=256 << 20, max_slots=2)
    got = srv.wait(srv.submit(wl), timeout_s=60)
    srv.close()
    for u, v in zip((t0, ts, pv), got):
        np.testing.assert_array_equal(u, v)


def _sampled_compare(wl, got, picks):
    """Oracle on selected (pair, point, s) chunks of a full-size workload."""
    t0, ts, pv = got
    jobs, keys = [], []
    for (p, c, s) in picks:
        row = -1 if s == 0 else (p * wl.n_points + c) * wl.n_surrogates + (s - 1)
        jobs.append((p, int(wl.window_start[c]), int(wl.window_len[c]), int(wl.trials[c]), row))
        keys.append((p, c, s))
    ref = oracle.te_jobs(wl.x, wl.y, wl.d_y, wl.d_x, wl.tau, wl.u, wl.k, jobs, wl.perms)
    for (p, c, s), r in zip(keys, ref):
        g = t0[p, c] if s == 0 else ts[p, c, s - 1]
        assert abs(g - r) <= TIGHT, ((p, c, s), g, r)


def test_uneven_surrogates_full_size_sampled(te):
    """The uneven-surrogate batch at full size (5000 trials, 60 windows of 1 000-49 400 points, 200
    surrogates each: 12 060 chunks, 3.7 GB of workspace) in the launch shape the benchmark uses;
    the oracle checks originals and surrogates of the windows it can finish in seconds."""
    wl = synth.uneven_surrogates()
    n = wl.chunk_sizes()
    x, y, perms = dev(wl)
    plan = te.Plan.from_workload(wl)
    got = plan.surrogates(x, y, perms)
    small = [int(c) for c in np.argsort(n)[:3]]
    mid = int(np.argsort(np.abs(n - 10000))[0])
    say("uneven full: checking windows", [(c, int(n[c])) for c in small + [mid]])
    picks = [(0, c, s) for c in small for s in (0, 1, 200)] + [(0, mid, 0), (0, mid, 117)]
    _sampled_compare(wl, got, picks)
    # p-values follow from the estimates exactly
    for c in small:
        assert got[2][0, c] == oracle.p_value(got[0][0, c], got[1][0, c])


def test_meg_like_full_size_sampled(te):
    """The MEG-shaped batch at full size (16 pairs x 40 windows x 101 chunks of 2 400 points, D = 9)."""
    wl = synth.meg_like()
    x, y, perms = dev(wl)
    got = te.Plan.from_workload(wl).surrogates(x, y, perms)
    rng_picks = np.floor(uniform01(derive_key(4242), 24) * np.array([16, 40, 101] * 8)).astype(int).reshape(8, 3)
    picks = [tuple(int(v) for v in r) for r in rng_picks] + [(0, 0, 0), (15, 39, 100)]
    _sampled_compare(wl, got, picks)


@pytest.mark.parametrize("cond", [0, 1])
def test_plain_per_chunk_path_equals_batched(te, cond):
    """te_estimate_each (every chunk on its own: embed, search, reduce) gives the batched
    path's estimates and p-values bit for bit, with given and with drawn permutations."""
    wl = synth.uneven_surrogates(R=200, T=60, n_points=4, n_surrogates=6, n_lo=100, n_hi=2500)
    wl.cond_source = cond
    x, y, perms = dev(wl)
    plan = te.Plan.from_workload(wl)
    ref = plan.surrogates(x, y, perms)
    say("plain per chunk, cond", cond, wl.chunk_sizes())
    for got in (plan.estimate_each(x, y, perms), plan.estimate_each(x, y, None)):
        for u, v in zip(ref, got):
            np.testing.assert_array_equal(u, v)
    np.testing.assert_array_equal(plan.estimate(x, y), ref[0])


# ------------------------------------------------------------ chunk sets

def _both_ways(te, monkeypatch, wl, run):
    """run(plan) with the window's chunks searched in sets (the default) and one chunk
    at a time (TE_NO_SETS=1): the results must be identical bit for bit."""
    monkeypatch.setenv("TE_NO_SETS", "1")
    single = run(te.Plan.from_workload(wl))
    monkeypatch.delenv("TE_NO_SETS")
    sets = run(te.Plan.from_workload(wl))
    for u, v in zip(single, sets):
        if u is None:
            assert v is None
        else:
            np.testing.assert_array_equal(u, v)
    return sets


@pytest.mark.parametrize("d_y,d_x,S", [(1, 1, 2), (2, 4, 3), (4, 4, 4), (4, 1, 7), (3, 3, 5), (2, 2, 1)])
def test_chunk_sets_equal_single_chunk_search(te, monkeypatch, d_y, d_x, S):
    """Sets of up to four chunks of a window (original + surrogates, full and partial sets)
    against the single-chunk search, on uneven windows with ragged 64-point blocks; the set
    path is also checked against the oracle."""
    wl = synth.generic((6061, d_y, d_x, S), R=60, T=70, d_y=d_y, d_x=d_x, starts=(30, 41, 55),
                       windows=(13, 7, 10), trials=(60, 47, 33), n_surrogates=S)
    say("sets case", dict(d_y=d_y, d_x=d_x, S=S, sizes=wl.chunk_sizes().tolist()))
    x, y, perms = dev(wl)
    got = _both_ways(te, monkeypatch, wl, lambda plan: plan.surrogates(x, y, perms))
    _compare(wl, *got)


@pytest.mark.parametrize("step", [0.25, 0.5])
def test_chunk_sets_tiled_walk_with_ties(te, monkeypatch, step):
    """Windows of 8 400 and 9 600 points (the tiled pass 1 of sorted chunks, the wide set
    kernel at d_y = d_x = 3) on series rounded to a grid of the given step, so that
    coordinate differences and distances tie: sets against the single-chunk search bit
    for bit, and against the oracle."""
    wl = synth.generic((6071, int(step * 4)), R=400, T=70, d_y=3, d_x=3, starts=(30, 40), windows=(21, 24),
                       trials=(400, 400), n_surrogates=3)
    wl.x = (np.round(wl.x / step) * step).astype(np.float32)
    wl.y = (np.round(wl.y / step) * step).astype(np.float32)
    say("tied sets case", dict(step=step, sizes=wl.chunk_sizes().tolist()))
    x, y, perms = dev(wl)
    got = _both_ways(te, monkeypatch, wl, lambda plan: plan.surrogates(x, y, perms))
    _compare(wl, *got)


def test_chunk_sets_async_split_and_counters(te, monkeypatch):
    import torch
    wl = synth.uneven_surrogates(R=150, T=60, n_points=3, n_surrogates=6, n_lo=300, n_hi=3000)
    x, y, perms = dev(wl)
    G, S = wl.n_pairs * wl.n_points, wl.n_surrogates

    def run(plan):
        full, minimum, _ = plan.workspace_bytes()
        out = torch.empty(G * (S + 1) + G, dtype=torch.float64, device="cuda")
        plan.surrogates_async(x, y, perms, out=out)
        torch.cuda.synchronize()
        ws = torch.empty(minimum, dtype=torch.uint8, device="cuda")
        split = plan.surrogates(x, y, perms, ws=ws)
        return [out.cpu().numpy()] + list(split)
    _both_ways(te, monkeypatch, wl, run)
    # work counters: a set evaluates its target comparisons once for all its chunks
    plan = te.Plan.from_workload(wl)
    te.profile_enable(False, work=True)
    te.profile_work_all(reset=True)
    plan.surrogates(x, y, perms)
    w = te.profile_work_all(reset=True)
    te.profile_enable(False)
    say("counters", w)
    assert 0 < w[2] < w[0] and 0 < w[3] < w[1]
    assert w[0] <= 4 * w[2] and w[1] <= 4 * w[3]


def test_chunk_sets_in_delay_scan(te, monkeypatch):
    wl = _scan_workload()
    u_values = [1, 2, 3, 4, 5, 6, 7, 8, 3]
    x, y, perms = dev(wl)
    got = _both_ways(te, monkeypatch, wl, lambda plan: plan.delay_scan(x, y, u_values, perms))
    _check_scan(wl, u_values, got)
