"""Local-predictor error of delay embeddings of the target (the Ragwitz criterion).

TEST INFRASTRUCTURE ONLY: used by the tests and the benchmark's CPU-baseline leg,
never by the library; it shares no code with the GPU path.

The embedding section of Wollstadt et al. 2014 chooses the embedding dimension d
and delay tau of the target's past state Y_{t-1} = (y_{t-1}, y_{t-1-tau}, ...,
y_{t-1-(d-1)tau}) as the pair that best predicts the next sample with a local
predictor (Ragwitz and Kantz).  The paper gives no formula; the reading used here:

* points: every trial r and every analysis time t in [w, w + W) of the window,
  pooled into one ensemble (trial-major order, point r * W + (t - w));
* distance: the maximum norm of the binary32 coordinate differences, as in the
  KSG search;
* predictor: the mean of y_t' over the k nearest other points (self excluded;
  equal distances ranked by point index), summed in fp64 in that rank order;
* score: the normalised mean squared error sum_i (y_i - yhat_i)^2 / sum_i (y_i -
  mean y)^2, in fp64; the chosen embedding is the candidate with the smallest score.

Parity pins (tests/test_ragwitz_oracle.py): with k = N - 1 the score is N^2/(N-1)^2
for any data; a periodic series whose state determines the next sample scores 0;
a hand-worked five-point example; invariance under shifts and power-of-two scales.
"""
from __future__ import annotations

import numpy as np


def states(y, d: int, tau: int, w: int, W: int, trials=None):
    """Pooled states [N, d] (binary32) and targets [N] of the window [w, w + W)."""
    y = np.asarray(y, np.float32)
    R = y.shape[0] if trials is None else int(trials)
    if w < 1 + (d - 1) * tau:
        raise ValueError("window starts before the embedding's history")
    S = np.empty((R * W, d), np.float32)
    tgt = np.empty(R * W, np.float32)
    for r in range(R):
        for t in range(w, w + W):
            i = r * W + (t - w)
            tgt[i] = y[r, t]
            for m in range(d):
                S[i, m] = y[r, t - 1 - m * tau]
    return S, tgt


def neighbours(S, k: int):
    """[N, k] indices of each point's k nearest other points, ranked by (distance, index)."""
    S = np.asarray(S, np.float32)
    N = S.shape[0]
    if not 1 <= k < N:
        raise ValueError("need 1 <= k < N")
    out = np.empty((N, k), np.int64)
    for i in range(N):
        dist = np.max(np.abs(S - S[i]), axis=1)      # binary32 differences, exact max
        dist[i] = np.inf
        order = np.argsort(dist, kind="stable")      # ties keep index order
        out[i] = order[:k]
    return out


def predictions(S, tgt, k: int):
    """Per-point local predictions yhat_i (fp64, neighbour targets summed in rank order)."""
    nb = neighbours(S, k)
    pred = np.empty(len(tgt), np.float64)
    for i in range(len(tgt)):
        s = 0.0
        for j in nb[i]:
            s += float(tgt[j])
        pred[i] = s / k
    return pred


def nmse(tgt, pred) -> float:
    """Normalised mean squared prediction error."""
    t = np.asarray(tgt, np.float64)
    e = float(np.sum((t - pred) ** 2))
    v = float(np.sum((t - t.mean()) ** 2))
    return e / v


def ragwitz(y, candidates, k: int, w: int, W: int, trials=None):
    """Scores of the (d, tau) candidates and the chosen one (smallest score, first on ties)."""
    scores = []
    for d, tau in candidates:
        S, tgt = states(y, d, tau, w, W, trials)
        scores.append(nmse(tgt, predictions(S, tgt, k)))
    best = int(np.argmin(scores))
    return np.array(scores), best


def predictions_points(S, tgt, k: int, idx):
    """Predictions of the listed points only (each O(N)), for sampled checks at full size."""
    S = np.asarray(S, np.float32)
    out = np.empty(len(idx), np.float64)
    for n, i in enumerate(idx):
        dist = np.max(np.abs(S - S[i]), axis=1)
        dist[i] = np.inf
        nb = np.argsort(dist, kind="stable")[:k]
        s = 0.0
        for j in nb:
            s += float(tgt[j])
        out[n] = s / k
    return out
