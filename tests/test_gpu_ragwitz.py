"""GPU parity of te_ragwitz (local-predictor scores of target embeddings) against the
oracle in oracle/ragwitz.py: per-point predictions bit for bit (same binary32 distances,
same rank order, same fp64 sums), scores within 1e-12 relative (only the order of the
final fp64 sums differs)."""
import sys

import numpy as np
import pytest

import synth
from oracle import ragwitz as rg
from synth.rng import derive_key, normal64

pytestmark = pytest.mark.gpu

REL = 1e-12


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


def _ar_series(seed, R, T, grid=None):
    e = normal64(derive_key(seed, R, T), R * T).reshape(R, T)
    y = np.zeros((R, T))
    for t in range(2, T):
        y[:, t] = 0.6 * y[:, t - 1] - 0.5 * y[:, t - 2] + e[:, t]
    if grid:
        y = np.round(y / grid) * grid
    return y.astype(np.float32)


def _check(te, y, w, W, cands, k, full=True, sample=None):
    import torch
    say("ragwitz case", dict(shape=y.shape, w=w, W=W, cands=cands, k=k))
    scores, pred = te.ragwitz(torch.from_numpy(y).cuda(), w, W, cands, k, want_pred=True)
    pred = pred.cpu().numpy()
    for c, (d, tau) in enumerate(cands):
        S, tgt = rg.states(y, d, tau, w, W)
        # the score is the stated function of the library's own predictions
        assert scores[c] == pytest.approx(rg.nmse(tgt, pred[c]), rel=REL)
        if full:
            ref = rg.predictions(S, tgt, k)
            np.testing.assert_array_equal(pred[c], ref, err_msg="candidate %d" % c)
            assert scores[c] == pytest.approx(rg.nmse(tgt, ref), rel=REL)
        if sample is not None:
            np.testing.assert_array_equal(pred[c][sample], rg.predictions_points(S, tgt, k, sample))
    return scores


@pytest.mark.parametrize("k", [1, 4, 7, 16])
def test_small_windows_bit_exact(te, k):
    y = _ar_series(1, 30, 60)
    _check(te, y, 17, 40, [(1, 1), (2, 1), (2, 2), (3, 1), (4, 2), (8, 2)], k)


@pytest.mark.parametrize("grid", [0.25, 1.0])
def test_ties_ranked_by_index(te, grid):
    """Series rounded to a grid: distances tie everywhere, so the rank order decides."""
    y = _ar_series(2, 25, 50, grid=grid)
    _check(te, y, 9, 37, [(1, 1), (2, 1), (3, 3)], 4)


def test_ragged_pool_and_tail(te):
    """N = 47 x 113 = 5 311 points: a partial last wave and a tail below eight candidates."""
    y = _ar_series(3, 47, 130)
    _check(te, y, 12, 113, [(2, 1), (5, 2)], 4)


def test_minimal_pool_and_constant_target(te):
    import torch
    y = _ar_series(4, 1, 12)
    _check(te, y, 3, 5, [(1, 1), (3, 1)], 4)                  # N = k + 1
    flat = np.ones((4, 20), np.float32)
    scores, _ = te.ragwitz(torch.from_numpy(flat).cuda(), 2, 10, [(1, 1)], 3)
    assert np.isnan(scores[0])


def test_ar_scenario_window_full_size(te):
    """A window of the AR scenarios (50 trials x 300 samples, N = 15 000): sampled points
    against the oracle, the score against the library's own predictions; the AR(2)
    process prefers two past samples to one."""
    y = _ar_series(5, 50, 560)
    cands = [(1, 1), (2, 1), (3, 1), (2, 2), (4, 1)]
    sample = np.unique(np.round(np.linspace(0, 14999, 97)).astype(int))
    scores = _check(te, y, 200, 300, cands, 4, full=False, sample=sample)
    assert int(np.argmin(scores)) in (1, 2, 4) and scores[1] < 0.9 * scores[0]


def test_nonfinite_and_bad_geometry_are_rejected(te):
    import torch
    y = _ar_series(6, 10, 40)
    y[3, 5] = np.nan                                          # in the history of t = 7 for tau = 1
    with pytest.raises(te.TEError) as ei:
        te.ragwitz(torch.from_numpy(y).cuda(), 6, 20, [(2, 1)], 4)
    assert ei.value.status == 1 and "non-finite" in str(ei.value)
    y[3, 5] = 0.0
    with pytest.raises(te.TEError):
        te.ragwitz(torch.from_numpy(y).cuda(), 2, 20, [(3, 1)], 4)   # no history for d = 3
