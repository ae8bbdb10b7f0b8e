"""Closed-form transfer entropy of a stationary Gaussian VAR(1) pair.

For jointly Gaussian variables TE equals linear Granger causality (the
"Relation ... to other measures of connectivity" section):
TE = 1/2 ln( Var(y_t | Y_past) / Var(y_t | Y_past, X_past) ), in nats.

The process is s_t = (x_t, y_t) = A s_{t-1} + e_t with Cov(e) = I and
A = [[a_x, 0], [c, a_y]].  Its stationary covariance P solves P = A P A^T + I and
Cov(s_{t+h}, s_t) = A^h P.  Used only as a pin for the oracle.
"""
from __future__ import annotations

import numpy as np


def var1_lag_cov(a_x: float, a_y: float, c: float, max_lag: int):
    A = np.array([[a_x, 0.0], [c, a_y]])
    n = 2
    vecP = np.linalg.solve(np.eye(n * n) - np.kron(A, A), np.eye(n).reshape(-1))
    P = vecP.reshape(n, n)
    G = [P]
    for _ in range(max_lag):
        G.append(A @ G[-1])
    return G


def gaussian_te(a_x=0.5, a_y=0.5, c=0.4, d_y=2, d_x=2, tau=1, u=1) -> float:
    """TE(X -> Y) with the embedding of eq. 6-7 (target past at t-1, source past at t-u)."""
    X, Y = 0, 1
    past_y = [(Y, 1 + m * tau) for m in range(d_y)]
    past_x = [(X, u + m * tau) for m in range(d_x)]
    allv = [(Y, 0)] + past_y + past_x
    G = var1_lag_cov(a_x, a_y, c, max(l for _, l in allv) + 1)

    def cov(v, w):
        (a, la), (b, lb) = v, w
        if la <= lb:
            return G[lb - la][a, b]
        return G[la - lb][b, a]

    def cond_var(target, given):
        if not given:
            return cov(target, target)
        S = np.array([[cov(p, q) for q in given] for p in given])
        s = np.array([cov(target, q) for q in given])
        return cov(target, target) - s @ np.linalg.solve(S, s)

    return 0.5 * np.log(cond_var((Y, 0), past_y) / cond_var((Y, 0), past_y + past_x))


def delayed_lag_cov(a_x: float, a_y: float, c: float, delay: int, max_lag: int):
    """Autocovariances of x_t = a_x x_{t-1} + e, y_t = a_y y_{t-1} + c x_{t-delay} + e'.

    Companion state z_t = (x_t, x_{t-1}, ..., x_{t-delay+1}, y_t) follows a VAR(1)
    z_t = A z_{t-1} + B e_t; returns G[h] = Cov(z_{t+h}, z_t) and the indices of x_t, y_t.
    """
    n = delay + 1
    A = np.zeros((n, n))
    A[0, 0] = a_x
    for i in range(1, delay):
        A[i, i - 1] = 1.0
    A[delay, delay - 1] = c
    A[delay, delay] = a_y
    Q = np.zeros((n, n))
    Q[0, 0] = 1.0
    Q[delay, delay] = 1.0
    vecP = np.linalg.solve(np.eye(n * n) - np.kron(A, A), Q.reshape(-1))
    P = vecP.reshape(n, n)
    G = [P]
    for _ in range(max_lag):
        G.append(A @ G[-1])
    return G, 0, delay


def gaussian_te_delay(a_x=0.5, a_y=0.5, c=0.4, delay=1, d_y=2, d_x=2, tau=1, u=1, cond=False) -> float:
    """TE(X -> Y) at assumed delay u for a pair coupled with delay `delay` (eq. 6-7 embedding).

    cond: the current source sample x_t joins the conditioning set."""
    past_y = [("y", 1 + m * tau) for m in range(d_y)] + ([("x", 0)] if cond else [])
    past_x = [("x", u + m * tau) for m in range(d_x)]
    allv = [("y", 0)] + past_y + past_x
    G, ix, iy = delayed_lag_cov(a_x, a_y, c, delay, max(l for _, l in allv) + 1)
    idx = {"x": ix, "y": iy}

    def cov(v, w):
        (a, la), (b, lb) = v, w
        if la <= lb:
            return G[lb - la][idx[a], idx[b]]
        return G[la - lb][idx[b], idx[a]]

    def cond_var(target, given):
        S = np.array([[cov(p, q) for q in given] for p in given])
        s = np.array([cov(target, q) for q in given])
        return cov(target, target) - s @ np.linalg.solve(S, s)

    return 0.5 * np.log(cond_var(("y", 0), past_y) / cond_var(("y", 0), past_y + past_x))


def gaussian_mi(rho: float) -> float:
    """I(X; Y) of a bivariate normal with correlation rho."""
    return -0.5 * np.log(1.0 - rho * rho)
