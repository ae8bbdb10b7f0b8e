"""Pins for the local-predictor (Ragwitz) oracle, oracle/ragwitz.py, on the CPU.

Sources of truth: a hand-worked five-point example (tests/golden/hand_example_ragwitz.json);
the closed form for k = N - 1 (the prediction is the mean of all other targets, so the
error is N/(N-1) times the deviation and the score N^2/(N-1)^2 for any data); a periodic
series whose state determines the next sample (neighbours at distance 0 share it: score
exactly 0, which a prediction from the neighbours' states or from the wrong points breaks);
i.i.d. noise (score near 1 + 1/k: the neighbours carry no information, and a state that
leaked the target would score near 0); an AR(2) process (two past samples beat one);
exact invariance under power-of-two scaling and dyadic shifts.
"""
import json
import os
from fractions import Fraction

import numpy as np
import pytest

from oracle import ragwitz as rg
from synth.rng import derive_key, normal64

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def test_hand_example():
    g = json.load(open(os.path.join(GOLDEN, "hand_example_ragwitz.json")))
    y = np.array([g["y"]], np.float32)
    S, tgt = rg.states(y, g["d"], g["tau"], g["w"], g["W"])
    assert S[:, 0].tolist() == g["states"] and tgt.tolist() == g["targets"]
    for case in g["cases"]:
        k = case["k"]
        assert rg.neighbours(S, k).tolist() == case["neighbours"]
        pred = rg.predictions(S, tgt, k)
        assert pred.tolist() == case["predictions"]
        assert float(np.sum((tgt - pred) ** 2)) == case["sum_sq_error"]
        assert rg.nmse(tgt, pred) == pytest.approx(float(Fraction(case["nmse_num"], case["nmse_den"])), rel=1e-15)
        assert rg.predictions_points(S, tgt, k, [0, 3, 4]).tolist() == [case["predictions"][i] for i in (0, 3, 4)]


@pytest.mark.parametrize("N", [7, 40])
def test_all_other_points_closed_form(N):
    y = normal64(derive_key(11, N), N + 3).reshape(1, -1).astype(np.float32)
    S, tgt = rg.states(y, 2, 1, 3, N)
    score = rg.nmse(tgt, rg.predictions(S, tgt, N - 1))
    assert score == pytest.approx(N * N / (N - 1) ** 2, rel=1e-12)


@pytest.mark.parametrize("d,tau", [(1, 1), (2, 1), (2, 3), (3, 2)])
def test_periodic_series_is_predicted_exactly(d, tau):
    pattern = np.array([0.0, 1.0, 3.0, 2.0, 5.0], np.float32)     # distinct values: y_{t-1} fixes y_t
    R, T = 8, 40
    y = np.stack([np.roll(np.tile(pattern, T // 5), -r) for r in range(R)]).astype(np.float32)
    S, tgt = rg.states(y, d, tau, 10, 25)
    pred = rg.predictions(S, tgt, 4)
    assert np.array_equal(pred, tgt.astype(np.float64))
    assert rg.nmse(tgt, pred) == 0.0


def test_iid_noise_scores_near_one_plus_one_over_k():
    k = 4
    y = normal64(derive_key(12), 60 * 60).reshape(60, 60).astype(np.float32)
    S, tgt = rg.states(y, 2, 1, 5, 50)
    score = rg.nmse(tgt, rg.predictions(S, tgt, k))
    assert abs(score - (1 + 1 / k)) < 0.1


def test_invariant_under_scaling_and_dyadic_shifts():
    y = np.round(normal64(derive_key(13), 6 * 50).reshape(6, 50) * 64) / 64
    y = y.astype(np.float32)
    base, _ = rg.ragwitz(y, [(1, 1), (2, 1), (2, 2)], 3, 5, 40)
    scaled, _ = rg.ragwitz(y * np.float32(4), [(1, 1), (2, 1), (2, 2)], 3, 5, 40)
    shifted, _ = rg.ragwitz(y + np.float32(2), [(1, 1), (2, 1), (2, 2)], 3, 5, 40)
    assert np.array_equal(base, scaled)
    np.testing.assert_allclose(shifted, base, rtol=1e-12)


def test_ar2_process_prefers_two_past_samples():
    """y_t = 0.6 y_{t-1} - 0.5 y_{t-2} + noise: two past samples predict better than one."""
    R, T = 40, 120
    e = normal64(derive_key(14), R * T).reshape(R, T)
    y = np.zeros((R, T))
    for t in range(2, T):
        y[:, t] = 0.6 * y[:, t - 1] - 0.5 * y[:, t - 2] + e[:, t]
    scores, best = rg.ragwitz(y.astype(np.float32), [(1, 1), (2, 1)], 4, 20, 100)
    assert best == 1 and scores[1] < 0.9 * scores[0]


def test_rejects_windows_without_history():
    with pytest.raises(ValueError):
        rg.states(np.zeros((2, 20), np.float32), 3, 2, 4, 5)
