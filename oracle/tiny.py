"""Exhaustive pure-Python KSG statistics for tiny chunks (N of a few dozen).

TEST INFRASTRUCTURE ONLY.  A second, independent statement of the neighbour
search of the KSG type-1 estimator (text before eq. 9 of Wollstadt et al.
2014): for every point, sort all distances to the other points and take the
k-th; then count points strictly inside that radius in each marginal space.
It uses numpy float32 scalars for the binary32 coordinate differences and a
full sort instead of the C oracle's running selection, so the two only agree
if both are right.
"""
from __future__ import annotations

from fractions import Fraction

import numpy as np


def _absdiff32(a, b) -> float:
    return abs(float(np.float32(a) - np.float32(b)))


def _dist(p, q, dims) -> float:
    return max((_absdiff32(p[m], q[m]) for m in dims), default=0.0)


def neighbours(pts, d_y: int, d_x: int, k: int):
    """Returns (eps, counts[3][N], knn lists): knn[i] = indices with distance <= eps_i."""
    pts = np.asarray(pts, np.float32)
    N, D = pts.shape
    assert D == 1 + d_y + d_x
    joint = list(range(D))
    sp = {"P": list(range(1, 1 + d_y)), "TP": list(range(0, 1 + d_y)), "PS": list(range(1, D))}
    eps, cnt, knn = [], [[], [], []], []
    for i in range(N):
        ds = sorted((_dist(pts[i], pts[j], joint), j) for j in range(N) if j != i)
        e = ds[k - 1][0]
        eps.append(e)
        knn.append(sorted(j for d, j in ds if d <= e))
        for s, name in enumerate(("P", "TP", "PS")):
            cnt[s].append(sum(1 for j in range(N) if j != i and _dist(pts[i], pts[j], sp[name]) < e))
    return np.array(eps), np.array(cnt, dtype=np.int64), knn


def harmonic(n: int) -> Fraction:
    """H_n = sum_{m=1}^n 1/m exactly."""
    return sum((Fraction(1, m) for m in range(1, n + 1)), Fraction(0))


def te_exact_minus_gamma_free(counts, k: int) -> Fraction:
    """Exact rational value of the estimator (eq. 9) for integer counts.

    With psi(n+1) = H_n - gamma, the Euler constant cancels:
    TE = H_{k-1} + (1/N) sum_i (H_{nP} - H_{nTP} - H_{nPS}).
    """
    cnt = np.asarray(counts)
    N = cnt.shape[1]
    acc = Fraction(0)
    for i in range(N):
        acc += harmonic(int(cnt[0, i])) - harmonic(int(cnt[1, i])) - harmonic(int(cnt[2, i]))
    return harmonic(k - 1) + acc / N
