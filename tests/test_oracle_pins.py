"""Pins for the CPU oracle: it must agree with things other than itself.

Every check here runs on the CPU.  Sources of truth:
  * a hand-worked example of eq. 9 (tests/golden/hand_example_ksg.json);
  * an exhaustive pure-Python search with full sorting (oracle/tiny.py);
  * exact rational harmonic numbers for the digamma function;
  * hand-written embedding vectors for eq. 6-7;
  * the closed-form TE of a Gaussian VAR(1) pair (TE equals linear Granger
    causality for Gaussian data) and the closed-form MI of a bivariate normal;
  * exact invariances of the max-norm statistics.
"""
import json
import math
import os
import zlib

import numpy as np
import pytest

import synth
from closed_form import gaussian_mi, gaussian_te, gaussian_te_delay
from oracle import oracle, tiny
from synth.rng import derive_key, normal64, permutation, uniform01

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")
EULER_GAMMA = 0.57721566490153286060651209008240243


# ---------------------------------------------------------------- hand example

def test_hand_example_counts_and_te():
    g = json.load(open(os.path.join(GOLDEN, "hand_example_ksg.json")))
    pts = np.array(g["points"], np.float32)
    for case in g["cases"]:
        k = case["k"]
        eps, cnt = oracle.counts(pts, g["d_y"], g["d_x"], k)
        assert eps.tolist() == case["eps"]
        assert cnt.T.tolist() == case["counts_P_TP_PS"]
        assert oracle.te_from_counts(cnt, k) == pytest.approx(case["te_nats"], abs=1e-15)
        # the exhaustive search agrees and its exact rational TE is the printed value
        e2, c2, _ = tiny.neighbours(pts, g["d_y"], g["d_x"], k)
        assert e2.tolist() == case["eps"]
        assert c2.T.tolist() == case["counts_P_TP_PS"]
        assert tiny.te_exact_minus_gamma_free(c2, k) == case["te_nats"]
        # per-point local values (eq. 17 on the pooled points) and their mean (eq. 18)
        lte = oracle.local_te(pts, g["d_y"], g["d_x"], k)
        assert lte.tolist() == pytest.approx(case["local_te_nats"], abs=1e-15)
        assert lte.mean() == pytest.approx(case["te_nats"], abs=1e-15)


# ------------------------------------------------------- exhaustive brute force

def _random_points(key, N, D, kind):
    if kind == "gauss":
        return normal64(key, N * D).reshape(N, D).astype(np.float32)
    if kind == "grid":   # integer grid: many exact ties in distances and at the radius
        return np.floor(uniform01(key, N * D) * 4).reshape(N, D).astype(np.float32)
    if kind == "dups":   # repeated points: zero radii when k duplicates exist
        base = np.floor(uniform01(key, (N // 3 + 1) * D) * 3).reshape(-1, D)
        idx = np.floor(uniform01(derive_key(key, 9), N) * base.shape[0]).astype(int)
        return base[idx].astype(np.float32)
    if kind == "fine":   # values whose differences round in binary32
        u = uniform01(key, N * D).reshape(N, D)
        return (1.0 + u * 2.0 ** -20).astype(np.float32) * np.float32(3.0)
    raise ValueError(kind)


@pytest.mark.parametrize("kind", ["gauss", "grid", "dups", "fine"])
@pytest.mark.parametrize("d_y,d_x", [(1, 1), (2, 2), (3, 3), (4, 4), (1, 3), (3, 2)])
def test_oracle_matches_exhaustive_search(kind, d_y, d_x):
    D = 1 + d_y + d_x
    for N, k in ((6, 1), (17, 3), (40, 4), (64, 2)):
        pts = _random_points(derive_key(31, N, D, zlib.crc32(kind.encode()) & 0xFFFF), N, D, kind)
        eps, cnt = oracle.counts(pts, d_y, d_x, k)
        e2, c2, knn = tiny.neighbours(pts, d_y, d_x, k)
        np.testing.assert_array_equal(eps, e2)
        np.testing.assert_array_equal(cnt, c2)
        # radius property: at least k other points at distance <= eps, fewer than k strictly inside
        for i in range(N):
            assert len(knn[i]) >= k
        # every count covers the points strictly inside the joint ball
        assert np.all(cnt[1] <= cnt[0]) and np.all(cnt[2] <= cnt[0])
        te = oracle.te_from_counts(cnt, k)
        assert te == pytest.approx(float(tiny.te_exact_minus_gamma_free(c2, k)), abs=1e-13)


@pytest.mark.parametrize("kind", ["gauss", "grid", "dups"])
def test_counts_split_over_threads_equal_the_single_thread_call(kind):
    """ksg_counts_split (reference points cut into contiguous ranges, one per thread) gives
    the single-thread result bit for bit, for thread counts that do and do not divide N,
    and for more threads than points."""
    for N, D, d_y, d_x, k in ((9, 3, 1, 1, 2), (301, 7, 3, 3, 4), (1000, 9, 4, 4, 4)):
        pts = _random_points(derive_key(53, N, zlib.crc32(kind.encode()) & 0xFFFF), N, D, kind)
        e1, c1 = oracle.counts(pts, d_y, d_x, k)
        for threads in (2, 3, 7, 16, N + 5):
            e2, c2 = oracle.counts(pts, d_y, d_x, k, n_threads=threads)
            np.testing.assert_array_equal(e1, e2)
            np.testing.assert_array_equal(c1, c2)


def test_counts_of_listed_points_equal_the_whole_chunk_and_brute_force():
    pts = _random_points(derive_key(54), 60, 5, "grid")
    e1, c1 = oracle.counts(pts, 2, 2, 3)
    idx = np.array([0, 59, 17, 17, 3], np.int64)
    e2, c2 = oracle.counts_points(pts, 2, 2, 3, idx)
    np.testing.assert_array_equal(e2, e1[idx])
    np.testing.assert_array_equal(c2, c1[:, idx])
    e3, c3, _ = tiny.neighbours(pts, 2, 2, 3)            # exhaustive pure-Python search
    np.testing.assert_array_equal(e2, e3[idx])
    np.testing.assert_array_equal(c2, c3[:, idx])
    with pytest.raises(ValueError):
        oracle.counts_points(pts, 2, 2, 3, np.array([60], np.int64))


def test_counts_batch_offsets_and_strides():
    """ksg_counts_batch (chunks of mixed sizes in one concatenated array, threaded over chunks)
    gives every chunk's single-chunk result, and the exhaustive search's on the small ones."""
    sizes = [5, 64, 1, 33, 700, 2]
    kinds = ["gauss", "grid", "dups", "fine", "gauss", "grid"]
    chunks = [_random_points(derive_key(55, i), n + 4, 6, kind) for i, (n, kind) in enumerate(zip(sizes, kinds))]
    for threads in (1, 3, 0):
        got = oracle.counts_batch(chunks, 2, 3, 4, n_threads=threads)
        assert len(got) == len(chunks)
        for ch, (e, c) in zip(chunks, got):
            e1, c1 = oracle.counts(ch, 2, 3, 4)
            np.testing.assert_array_equal(e, e1)
            np.testing.assert_array_equal(c, c1)
            if ch.shape[0] <= 70:
                e2, c2, _ = tiny.neighbours(ch, 2, 3, 4)
                np.testing.assert_array_equal(e, e2)
                np.testing.assert_array_equal(c, c2)


def test_strict_inside_joint_ball_is_counted_everywhere():
    pts = _random_points(derive_key(7), 50, 7, "gauss")
    eps, cnt = oracle.counts(pts, 3, 3, 4)
    _, _, knn = tiny.neighbours(pts, 3, 3, 4)
    for i in range(50):
        inside = 0
        for j in range(50):
            if j != i:
                d = max(abs(float(np.float32(pts[i, m]) - np.float32(pts[j, m]))) for m in range(7))
                inside += d < eps[i]
        assert inside <= 3                        # fewer than k strictly inside
        assert min(cnt[:, i]) >= inside           # marginal distances never exceed the joint one


# ----------------------------------------------------------------- digamma

def test_digamma_against_exact_harmonic_numbers():
    assert oracle.digamma_int(1) == pytest.approx(-EULER_GAMMA, abs=1e-16)
    for n in range(1, 51):
        exact = float(tiny.harmonic(n - 1)) - EULER_GAMMA
        assert oracle.digamma_int(n) == pytest.approx(exact, abs=2e-15)
    for n in range(1, 200):
        assert oracle.digamma_int(n + 1) - oracle.digamma_int(n) == pytest.approx(1.0 / n, abs=1e-14)
    for n in (1000, 20000, 100000):     # asymptotic series ln n - 1/2n - 1/12n^2 + 1/120n^4
        asym = math.log(n) - 1 / (2 * n) - 1 / (12 * n * n) + 1 / (120 * n ** 4)
        assert oracle.digamma_int(n) == pytest.approx(asym, abs=1e-12)


def test_te_from_counts_exact_rational():
    key = derive_key(11)
    N, k = 37, 4
    c = np.floor(uniform01(key, 3 * N) * 30).reshape(3, N).astype(np.int32)
    c[1] = np.minimum(c[1], c[0])
    c[2] = np.minimum(c[2], c[0])
    assert oracle.te_from_counts(c, k) == pytest.approx(float(tiny.te_exact_minus_gamma_free(c, k)), abs=1e-13)


def test_local_te_exact_rational_and_mean():
    key = derive_key(12)
    N, k = 41, 3
    c = np.floor(uniform01(key, 3 * N) * 25).reshape(3, N).astype(np.int32)
    c[1] = np.minimum(c[1], c[0])
    c[2] = np.minimum(c[2], c[0])
    lte = oracle.local_from_counts(c, k)
    for i in range(N):
        exact = tiny.harmonic(k - 1) + tiny.harmonic(int(c[0, i])) - tiny.harmonic(int(c[1, i])) \
            - tiny.harmonic(int(c[2, i]))
        assert lte[i] == pytest.approx(float(exact), abs=1e-14)
    # eq. 18: the average of the local values is the estimate of eq. 9
    assert lte.mean() == pytest.approx(oracle.te_from_counts(c, k), abs=1e-13)


def test_local_te_follows_point_permutation():
    key = derive_key(13)
    pts = normal64(key, 60 * 5).reshape(60, 5).astype(np.float32)
    perm = permutation(derive_key(key, 1), 60)
    a = oracle.local_te(pts, 2, 2, 4)
    b = oracle.local_te(pts[perm], 2, 2, 4)
    assert np.array_equal(a[perm], b)


def test_p_value_convention():
    assert oracle.p_value(0.5, [0.1, 0.5, 0.7, 0.2]) == 0.5      # ties count as "equal or larger"
    assert oracle.p_value(1.0, [0.1, 0.2]) == 0.0
    assert math.isnan(oracle.p_value(1.0, []))


# ---------------------------------------------------------------- embedding

def test_embedding_indices_by_hand():
    R, T = 3, 12
    y = np.array([[1000.0 * r + t for t in range(T)] for r in range(R)], np.float32)
    x = -y
    # d_y = 2, d_x = 2, tau = 2, u = 3, window [7, 9), all 3 repetitions
    pts = oracle.embed(x, y, 2, 2, 2, 3, 7, 2)
    assert pts.shape == (6, 5)
    # point order is repetition-major: q = r * W + (t' - w)
    assert pts[0].tolist() == [7, 6, 4, -4, -2]          # r = 0, t' = 7
    assert pts[1].tolist() == [8, 7, 5, -5, -3]          # r = 0, t' = 8
    assert pts[3].tolist() == [1008, 1007, 1005, -1005, -1003]
    assert pts[4].tolist() == [2007, 2006, 2004, -2004, -2002]
    # a source permutation moves only the source block, for every t' of the window
    perm = np.array([2, 0, 1], np.int32)
    sp = oracle.embed(x, y, 2, 2, 2, 3, 7, 2, src_perm=perm)
    assert sp[0].tolist() == [7, 6, 4, -2004, -2002]
    assert sp[5].tolist() == [2008, 2007, 2005, -1005, -1003]
    # fewer pooled repetitions
    assert oracle.embed(x, y, 2, 2, 2, 3, 7, 2, Rc=2).shape == (4, 5)
    # windows without enough history are rejected (t' - u - (d_x - 1) tau < 0)
    with pytest.raises(ValueError):
        oracle.embed(x, y, 2, 2, 2, 3, 4, 2)
    with pytest.raises(ValueError):
        oracle.embed(x, y, 2, 2, 2, 3, 11, 2)        # window runs past the end


# ------------------------------------------------ statistical pins (closed forms)

def _c1_like(coupling, seeds, d=2):
    vals = []
    for s in seeds:
        w = synth.linear_pair(seed_offset=1000 + s, coupling=coupling, d=d)
        vals.append(oracle.te_workload(w)[(0, 0, 0)])
    return np.array(vals)


BIAS_BUDGET = 0.02   # KSG bias allowance at N = 2000, k = 4, D = 5 (measured about -0.005)


def test_gaussian_ar_closed_form():
    truth = gaussian_te(c=0.4, d_y=2, d_x=2)
    assert truth == pytest.approx(0.0920092, abs=5e-8)
    v = _c1_like(0.4, range(20))
    se = v.std(ddof=1) / math.sqrt(len(v))
    assert abs(v.mean() - truth) < 3 * se + BIAS_BUDGET


def test_independent_processes_give_zero():
    v = _c1_like(0.0, range(20))
    se = v.std(ddof=1) / math.sqrt(len(v))
    assert gaussian_te(c=0.0) == pytest.approx(0.0, abs=1e-15)
    assert abs(v.mean()) < 3 * se + BIAS_BUDGET


def test_coupling_sweep_tracks_closed_form():
    cs = [0.0, 0.2, 0.4, 0.8]
    truth = [gaussian_te(c=c) for c in cs]
    means = [_c1_like(c, range(6)).mean() for c in cs]
    assert np.all(np.diff(truth) > 0)
    assert np.all(np.diff(means) > 0)
    for m, t in zip(means, truth):
        assert abs(m - t) < 0.03 + 0.1 * t


@pytest.mark.parametrize("rho", [0.0, 0.6, 0.9])
def test_no_target_past_reduces_to_ksg_mutual_information(rho):
    """d_y = 0: the estimator becomes KSG MI estimator 1, psi(k) + psi(N) - <psi(n_x+1) + psi(n_y+1)>."""
    vals = []
    N, k = 1500, 4
    for s in range(8):
        g = normal64(derive_key(5, s, int(rho * 100)), 2 * N).reshape(2, N)
        a = g[0]
        b = rho * g[0] + math.sqrt(1 - rho * rho) * g[1]
        pts = np.stack([b, a], axis=1).astype(np.float32)       # (target, source)
        eps, cnt = oracle.counts(pts, 0, 1, k)
        assert np.all(cnt[0][eps > 0] == N - 1)
        vals.append(oracle.te_from_counts(cnt, k))
    v = np.array(vals)
    assert abs(v.mean() - gaussian_mi(rho)) < 3 * v.std(ddof=1) / math.sqrt(len(v)) + 0.01


# ------------------------------------------------------------- exact invariants

def _chunk(seed=3, d=3, R=60, W=10):
    w = synth.generic((seed,), R=R, T=40, d_y=d, d_x=d, starts=(20,), windows=(W,))
    return w, oracle.embed(w.x[0], w.y[0], d, d, 1, 1, 20, W)


def test_point_order_invariance():
    w, pts = _chunk()
    eps, cnt = oracle.counts(pts, 3, 3, 4)
    perm = permutation(derive_key(8), pts.shape[0])
    e2, c2 = oracle.counts(pts[perm], 3, 3, 4)
    np.testing.assert_array_equal(e2, eps[perm])
    np.testing.assert_array_equal(c2, cnt[:, perm])
    assert oracle.te_from_counts(c2, 4) == pytest.approx(oracle.te_from_counts(cnt, 4), abs=1e-12)


@pytest.mark.parametrize("m", [-20, -3, 5, 20])
def test_power_of_two_scaling_is_exact(m):
    _, pts = _chunk()
    eps, cnt = oracle.counts(pts, 3, 3, 4)
    e2, c2 = oracle.counts(pts * np.float32(2.0 ** m), 3, 3, 4)
    np.testing.assert_array_equal(c2, cnt)
    np.testing.assert_array_equal(e2, eps * 2.0 ** m)


def test_coordinate_negation_is_exact():
    _, pts = _chunk()
    eps, cnt = oracle.counts(pts, 3, 3, 4)
    for col in range(pts.shape[1]):
        q = pts.copy()
        q[:, col] = -q[:, col]
        e2, c2 = oracle.counts(q, 3, 3, 4)
        np.testing.assert_array_equal(c2, cnt)
        np.testing.assert_array_equal(e2, eps)


def test_identity_surrogate_equals_original():
    w, pts = _chunk()
    ident = np.arange(w.n_trials, dtype=np.int32)
    sp = oracle.embed(w.x[0], w.y[0], 3, 3, 1, 1, 20, 10, src_perm=ident)
    np.testing.assert_array_equal(sp, pts)


def test_source_shuffle_equals_target_shuffle_with_inverse():
    """{(y(r), x(phi(r)))} and {(y(phi^-1(r)), x(r))} are the same point set."""
    w, _ = _chunk()
    R = w.n_trials
    phi = permutation(derive_key(19), R)
    inv = np.empty_like(phi)
    inv[phi] = np.arange(R, dtype=np.int32)
    a = oracle.embed(w.x[0], w.y[0], 3, 3, 1, 1, 20, 10, src_perm=phi)
    b = oracle.embed(w.x[0], w.y[0], 3, 3, 1, 1, 20, 10, tgt_perm=inv)
    assert sorted(map(tuple, a.tolist())) == sorted(map(tuple, b.tolist()))
    ea, ca = oracle.counts(a, 3, 3, 4)
    eb, cb = oracle.counts(b, 3, 3, 4)
    assert oracle.te_from_counts(ca, 4) == pytest.approx(oracle.te_from_counts(cb, 4), abs=1e-12)
    assert sorted(zip(ea, *ca)) == sorted(zip(eb, *cb))


def test_trial_relabelling_is_a_point_permutation():
    w, pts = _chunk()
    R = w.n_trials
    phi = permutation(derive_key(23), R)
    x2, y2 = w.x[0][phi], w.y[0][phi]
    q = oracle.embed(x2, y2, 3, 3, 1, 1, 20, 10)
    e1, c1 = oracle.counts(pts, 3, 3, 4)
    e2, c2 = oracle.counts(q, 3, 3, 4)
    assert oracle.te_from_counts(c2, 4) == pytest.approx(oracle.te_from_counts(c1, 4), abs=1e-12)


def test_double_difference_diagnostic_runs():
    _, pts = _chunk()
    _, c0 = oracle.counts(pts, 3, 3, 4, mode=0)
    _, c1 = oracle.counts(pts, 3, 3, 4, mode=1)
    # the rounding reading changes at most a handful of counts on Gaussian data
    assert np.count_nonzero(c0 != c1) <= 0.01 * c0.size


def test_batched_oracle_equals_single_chunk_calls():
    w = synth.generic((41,), R=30, T=40, d_y=2, d_x=2, starts=(10, 20, 25), windows=(10, 8, 12),
                      trials=(30, 25, 12), n_surrogates=3)
    te = oracle.te_workload(w)
    for (p, c, s), v in te.items():
        perm = None if s == 0 else w.perms[p, c, s - 1]
        pts = oracle.embed(w.x[p], w.y[p], 2, 2, 1, 1, int(w.window_start[c]), int(w.window_len[c]),
                           Rc=int(w.trials[c]), src_perm=perm)
        _, cnt = oracle.counts(pts, 2, 2, 4)
        assert v == oracle.te_from_counts(cnt, 4)


# ------------------------------------------------------------ delay scan (eq. 5)

def _delayed_pair(delay, coupling, R=200, T=60, start=30, window=10, d_y=2, d_x=1, n_surrogates=0, seed=77):
    from synth.processes import coupled_ar
    x, y = coupled_ar(synth.configs.BASE_SEED + seed, R, T, coupling=coupling, delay=delay)
    wl = synth.configs.Workload(name="delayed", x=x[None], y=y[None], d_y=d_y, d_x=d_x, tau=1, u=1, k=4,
                                window_start=np.array([start], np.int32), window_len=np.array([window], np.int32),
                                trials=np.array([R], np.int32), n_surrogates=n_surrogates)
    if n_surrogates:
        wl.perms = synth.configs.make_perms(synth.configs.BASE_SEED + seed, 1, wl.trials, n_surrogates, R)
    return wl


def test_closed_form_delay_generalizes_the_var1_pin():
    for c in (0.0, 0.4, 0.8):
        assert gaussian_te_delay(c=c, delay=1, d_y=2, d_x=2) == pytest.approx(gaussian_te(c=c, d_y=2, d_x=2), abs=1e-14)
    curve = [gaussian_te_delay(c=0.8, delay=4, d_y=2, d_x=1, u=u) for u in range(1, 9)]
    assert int(np.argmax(curve)) + 1 == 4
    # a source embedding of d_x samples sees x_{t-delay} for every u in [delay - d_x + 1, delay]
    flat = [gaussian_te_delay(c=0.8, delay=4, d_y=2, d_x=2, u=u) for u in (3, 4)]
    assert flat[0] == pytest.approx(flat[1], rel=1e-9)


def test_delay_scan_recovers_the_coupling_delay():
    """eq. 5: the scan's maximum sits at the true delay, and the curve follows the closed form."""
    wl = _delayed_pair(delay=4, coupling=0.8)
    u_values = list(range(1, 9))
    te_scan, u_best, _, pv = oracle.delay_scan(wl, u_values)
    assert u_best[(0, 0)] == 4
    truth = np.array([gaussian_te_delay(c=0.8, delay=4, d_y=2, d_x=1, u=u) for u in u_values])
    assert np.max(np.abs(te_scan[(0, 0)] - truth)) < 0.04
    assert math.isnan(pv[(0, 0)])


def test_delay_scan_ties_and_surrogates_at_the_chosen_delay():
    wl = _delayed_pair(delay=3, coupling=0.8, n_surrogates=9, seed=78)
    te_scan, u_best, te_surr, pv = oracle.delay_scan(wl, [5, 3, 3, 2])
    assert u_best[(0, 0)] == 3                       # first maximum in table order
    assert te_scan[(0, 0)][1] == te_scan[(0, 0)][2]
    # the surrogates are those of eq. 10 at u = 3, and the p-value counts them
    direct = oracle.te_jobs(wl.x, wl.y, wl.d_y, wl.d_x, wl.tau, 3, wl.k,
                            [(0, 30, 10, 200, s) for s in range(9)], wl.perms)
    np.testing.assert_array_equal(te_surr[(0, 0)], direct)
    assert pv[(0, 0)] == 0.0


# ------------------------------------------- conditioning on the current source sample

def test_conditioned_embedding_by_hand():
    x = np.arange(3 * 12, dtype=np.float32).reshape(3, 12) * -1.0
    y = np.arange(3 * 12, dtype=np.float32).reshape(3, 12)
    pts = oracle.embed(x, y, 2, 1, 1, 2, 5, 2, cond=True)
    assert pts.shape == (6, 5)
    # (y_t, y_{t-1}, y_{t-2}, x_t, x_{t-u}) with t = 5, u = 2, repetition 0
    assert pts[0].tolist() == [5, 4, 3, -5, -3]
    perm = np.array([2, 0, 1], np.int32)
    sp = oracle.embed(x, y, 2, 1, 1, 2, 5, 2, src_perm=perm, cond=True)
    assert sp[1].tolist() == [6, 5, 4, -30, -28]            # repetition 0 takes its source from repetition 2


def test_conditioning_on_current_source_closed_form():
    """With x strongly autocorrelated, x_t carries most of what X_past says about y_t: the
    conditioned TE is the Gaussian closed form with x_t added to the conditioning set."""
    from synth.processes import coupled_ar
    cond_truth = gaussian_te_delay(a_x=0.9, c=0.4, delay=1, d_y=2, d_x=2, cond=True)
    plain_truth = gaussian_te_delay(a_x=0.9, c=0.4, delay=1, d_y=2, d_x=2)
    assert cond_truth == pytest.approx(0.0616720, abs=5e-7) and plain_truth > 2 * cond_truth
    vc, vp = [], []
    for s in range(10):
        x, y = coupled_ar(synth.configs.BASE_SEED + 500 + s, 100, 100, a_x=0.9, coupling=0.4, delay=1)
        wl = synth.configs.Workload(name="cond", x=x[None], y=y[None], d_y=2, d_x=2, tau=1, u=1, k=4,
                                    window_start=np.array([80], np.int32), window_len=np.array([20], np.int32),
                                    trials=np.array([100], np.int32), cond_source=1)
        vc.append(oracle.te_workload(wl)[(0, 0, 0)])
        wl.cond_source = 0
        vp.append(oracle.te_workload(wl)[(0, 0, 0)])
    vc, vp = np.array(vc), np.array(vp)
    assert abs(vc.mean() - cond_truth) < 3 * vc.std(ddof=1) / math.sqrt(len(vc)) + BIAS_BUDGET
    assert abs(vp.mean() - plain_truth) < 3 * vp.std(ddof=1) / math.sqrt(len(vp)) + BIAS_BUDGET
    assert vp.mean() - vc.mean() > 0.05
