"""The synthetic workloads: series, analysis geometry and surrogate permutations.

A workload bundles everything both sides need to run the same job:

* ``x``, ``y``: float32 [pairs, R, T] source and target ensembles;
* embedding parameters d_y, d_x, tau, u and the neighbour count k;
* per analysis time point c: the first sample w_c of its window, the window
  length W_c in samples and the number R_c of repetitions pooled (the first R_c);
* ``perms``: int32 [pairs, points, S, R] trial permutations for the S
  surrogates of every (pair, point); row entries past R_c are the identity.

Named builders give the five workloads at full size; keyword arguments shrink
them for tests.  Seeds are 14014068 + 1000 * workload + pair.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

from .processes import ar_scenario, coupled_ar, switched_pink_pair
from .rng import derive_key, permutations, uniform01

BASE_SEED = 14014068


@dataclass
class Workload:
    name: str
    x: np.ndarray                 # float32 [P, R, T]
    y: np.ndarray                 # float32 [P, R, T]
    d_y: int
    d_x: int
    tau: int
    u: int
    k: int
    window_start: np.ndarray      # int32 [C]
    window_len: np.ndarray        # int32 [C]
    trials: np.ndarray            # int32 [C]
    n_surrogates: int = 0
    perms: np.ndarray | None = None   # int32 [P, C, S, R] or None when S == 0
    meta: dict = field(default_factory=dict)
    cond_source: int = 0          # 1: condition on the current source sample x_t as well
    perm_seed: int = 0            # seed of make_perms that drew ``perms`` (the library draws the same)

    @property
    def n_pairs(self) -> int:
        return int(self.x.shape[0])

    @property
    def n_trials(self) -> int:
        return int(self.x.shape[1])

    @property
    def n_samples(self) -> int:
        return int(self.x.shape[2])

    @property
    def n_points(self) -> int:
        return int(self.window_start.shape[0])

    @property
    def dim(self) -> int:
        return 1 + self.d_y + self.d_x

    def chunk_sizes(self) -> np.ndarray:
        """Points pooled per analysis time point: R_c * W_c."""
        return (self.trials.astype(np.int64) * self.window_len.astype(np.int64))

    def n_estimates(self) -> int:
        return self.n_pairs * self.n_points * (1 + self.n_surrogates)

    def directed_pairs(self) -> int:
        """Sum over all chunks (originals and surrogates) of N_c (N_c - 1)."""
        n = self.chunk_sizes()
        return int(self.n_pairs * (1 + self.n_surrogates) * np.sum(n * (n - 1)))


def make_perms(seed: int, n_pairs: int, trials: np.ndarray, n_surr: int, R: int) -> np.ndarray:
    """Independent uniform permutations per (pair, point, surrogate)."""
    C = len(trials)
    out = np.tile(np.arange(R, dtype=np.int32), (n_pairs, C, max(n_surr, 0), 1))
    if n_surr <= 0:
        return out
    for p in range(n_pairs):
        for c in range(C):
            rc = int(trials[c])
            keys = [derive_key(seed, 77, p, c, s) for s in range(n_surr)]
            out[p, c, :, :rc] = permutations(keys, rc)
    return out


def _stack(pairs):
    xs, ys = zip(*pairs)
    return np.ascontiguousarray(np.stack(xs)), np.ascontiguousarray(np.stack(ys))


def linear_pair(R=100, T=100, d=2, window=20, start=80, coupling=0.4, seed_offset=0, k=4,
                n_surrogates=0, name="linear_ar"):
    """Coupled linear Gaussian AR(1) pair, one window (the CPU-sized single estimate).

    x_t = 0.5 x_{t-1} + e;  y_t = 0.5 y_{t-1} + c x_{t-1} + e;  u = 1, tau = 1.
    """
    seed = BASE_SEED + 1000 * 1 + seed_offset
    x, y = coupled_ar(seed, R, T, coupling=coupling, delay=1)
    w = Workload(name=name, x=x[None], y=y[None], d_y=d, d_x=d, tau=1, u=1, k=k,
                 window_start=np.array([start], np.int32), window_len=np.array([window], np.int32),
                 trials=np.array([R], np.int32), n_surrogates=n_surrogates,
                 meta=dict(seed=seed, coupling=coupling))
    if n_surrogates:
        w.perm_seed = int(seed)
        w.perms = make_perms(w.perm_seed, 1, w.trials, n_surrogates, R)
    return w


def nonlinear_ensemble(R=500, T=300, n_points=100, window=10, k=4, n_surrogates=0,
                       name="nonlinear_ar"):
    """Nonlinear coupled AR pair, many analysis windows, all trials pooled.

    x_t = 0.5 x_{t-1} + e;  y_t = 0.5 y_{t-1} + 0.3 tanh(x_{t-3}) + e;
    d_y = d_x = 3, tau = 1, u = 3; w_c = 5 + floor(c (T - window - 5) / (C - 1)).
    """
    seed = BASE_SEED + 1000 * 2
    x, y = coupled_ar(seed, R, T, coupling=0.3, delay=3, nonlinear=True)
    h = 5
    span = T - window - h
    starts = np.array([h + (c * span) // max(n_points - 1, 1) for c in range(n_points)], np.int32)
    w = Workload(name=name, x=x[None], y=y[None], d_y=3, d_x=3, tau=1, u=3, k=k,
                 window_start=starts, window_len=np.full(n_points, window, np.int32),
                 trials=np.full(n_points, R, np.int32), n_surrogates=n_surrogates,
                 meta=dict(seed=seed))
    if n_surrogates:
        w.perm_seed = int(seed)
        w.perms = make_perms(w.perm_seed, 1, w.trials, n_surrogates, R)
    return w


def uneven_surrogates(R=5000, T=400, n_points=60, n_surrogates=200, n_lo=1000, n_hi=50000,
                      k=4, name="uneven_surrogates"):
    """Linear AR pair, d = 3, uneven pooled sizes, many source-shuffled surrogates.

    Per point: N*_c ~ U[n_lo, n_hi], W_c ~ U{10..20}, R_c = clamp(round(N*_c / W_c), 50, R),
    N_c = R_c W_c; w_c = 3 + floor(c (T - 20 - 3) / (C - 1)).
    """
    seed = BASE_SEED + 1000 * 3
    x, y = coupled_ar(seed, R, T, coupling=0.4, delay=1)
    u = uniform01(derive_key(seed, 5), 2 * n_points)
    n_star = n_lo + u[:n_points] * (n_hi - n_lo)
    wl = (10 + np.floor(u[n_points:] * 11)).astype(np.int32)
    rc = np.clip(np.rint(n_star / wl), min(50, R), R).astype(np.int32)
    h = 3
    span = T - 20 - h
    starts = np.array([h + (c * span) // max(n_points - 1, 1) for c in range(n_points)], np.int32)
    w = Workload(name=name, x=x[None], y=y[None], d_y=3, d_x=3, tau=1, u=1, k=k,
                 window_start=starts, window_len=wl, trials=rc, n_surrogates=n_surrogates,
                 meta=dict(seed=seed))
    w.perm_seed = int(seed)
    w.perms = make_perms(w.perm_seed, 1, rc, n_surrogates, R)
    return w


def meg_like(n_pairs=16, R=120, T=1200, n_points=40, window=20, n_surrogates=100, k=4,
             on=400, off=800, name="meg_like"):
    """Pink-noise channel pairs with a switched coupling 0.4 x_{t-5} for on <= t < off.

    d_y = d_x = 4, tau = 2, u = 5 (history 11); w_c = 11 + floor(c (T - window - 11) / (C - 1)).
    """
    pairs = []
    seeds = []
    for p in range(n_pairs):
        seed = BASE_SEED + 1000 * 4 + p
        seeds.append(seed)
        pairs.append(switched_pink_pair(seed, R, T, on=min(on, T), off=min(off, T)))
    x, y = _stack(pairs)
    h = 11
    span = T - window - h
    starts = np.array([h + (c * span) // max(n_points - 1, 1) for c in range(n_points)], np.int32)
    w = Workload(name=name, x=x, y=y, d_y=4, d_x=4, tau=2, u=5, k=k,
                 window_start=starts, window_len=np.full(n_points, window, np.int32),
                 trials=np.full(n_points, R, np.int32), n_surrogates=n_surrogates,
                 meta=dict(seeds=seeds, on=on, off=off))
    w.perm_seed = int(seeds[0])
    w.perms = make_perms(w.perm_seed, n_pairs, w.trials, n_surrogates, R)
    return w


def generic(seed_ids, *, n_pairs=1, R=40, T=60, d_y=2, d_x=2, tau=1, u=1, k=4, starts=(30,),
            windows=None, trials=None, n_surrogates=0, coupling=0.4, name="generic"):
    """Small linear-AR workload with arbitrary geometry, for edge-case tests."""
    pairs = []
    for p in range(n_pairs):
        seed = int(derive_key(*seed_ids, p) % np.uint64(1 << 31))
        pairs.append(coupled_ar(seed, R, T, coupling=coupling, delay=max(u, 1)))
    x, y = _stack(pairs)
    C = len(starts)
    wl = np.array(windows if windows is not None else [10] * C, np.int32)
    tr = np.array(trials if trials is not None else [R] * C, np.int32)
    w = Workload(name=name, x=x, y=y, d_y=d_y, d_x=d_x, tau=tau, u=u, k=k,
                 window_start=np.array(starts, np.int32), window_len=wl, trials=tr,
                 n_surrogates=n_surrogates)
    if n_surrogates:
        w.perm_seed = int(int(derive_key(*seed_ids) % np.uint64(1 << 31)))
        w.perms = make_perms(w.perm_seed, n_pairs, tr, n_surrogates, R)
    return w


def ar_scenarios(scenario=1, R=50, T=3000, window=300, n_surrogates=500, d_y=2, d_x=1, k=4, n_points=None,
                 name=None):
    """AR(1) coupling scenarios (Table 1, eq. 12-16): 50 trials x 3000 samples, windows of 300
    samples from sample 200 on (4 windows for scenario 1, 8 for scenarios 2 and 3), both
    directions as two pairs (pair 0: X -> Y, pair 1: Y -> X), assumed delays u = 1..20
    (1..30 for scenario 3) in meta["u_values"], trial-shuffled surrogates.
    """
    seed = BASE_SEED + 1000 * 6 + scenario
    x, y = ar_scenario(seed, R, T, scenario)
    C = 4 if scenario == 1 else 8
    if n_points is not None:
        C = n_points
    starts = np.array([200 + window * c for c in range(C)], np.int32)
    u_max = 30 if scenario == 3 else 20
    w = Workload(name=name or f"ar_scenario{scenario}", x=np.stack([x, y]), y=np.stack([y, x]), d_y=d_y,
                 d_x=d_x, tau=1, u=1, k=k, window_start=starts, window_len=np.full(C, window, np.int32),
                 trials=np.full(C, R, np.int32), n_surrogates=n_surrogates,
                 meta=dict(seed=seed, scenario=scenario, u_values=list(range(1, u_max + 1)),
                           directions=["X->Y", "Y->X"]))
    if n_surrogates:
        w.perm_seed = int(seed)
        w.perms = make_perms(w.perm_seed, 2, w.trials, n_surrogates, R)
    return w


def ar_robustness(R=100, T=3000, window=300, start=1100, trials=(2, 7, 17, 34, 100), n_surrogates=100, d_y=2,
                  d_x=1, k=4, name="ar_robustness"):
    """Robustness against the amount of data (the sweep over M pooled points in the
    robustness evaluation, here on AR scenario 1 instead of Lorenz systems): one
    coupled window [start, start + window) analysed with the first R_c trials for
    each R_c in `trials`, i.e. M = R_c * window points; assumed delays u = 1..20
    (true delay 10); X -> Y only.
    """
    seed = BASE_SEED + 1000 * 7
    x, y = ar_scenario(seed, R, T, 1)
    C = len(trials)
    w = Workload(name=name, x=x[None], y=y[None], d_y=d_y, d_x=d_x, tau=1, u=1, k=k,
                 window_start=np.full(C, start, np.int32), window_len=np.full(C, window, np.int32),
                 trials=np.array(trials, np.int32), n_surrogates=n_surrogates,
                 meta=dict(seed=seed, scenario=1, u_values=list(range(1, 21)), directions=["X->Y"],
                           points=[int(r) * window for r in trials]))
    if n_surrogates:
        w.perm_seed = int(seed)
        w.perms = make_perms(w.perm_seed, 1, w.trials, n_surrogates, R)
    return w


def history(d_y: int, d_x: int, tau: int, u: int) -> int:
    """Samples of history a window start needs: max(1 + (d_y-1) tau, u + (d_x-1) tau)."""
    return max(1 + (d_y - 1) * tau, u + (d_x - 1) * tau)


def served_jobs(n_jobs=2000, rate=200.0, n_lo=1000, n_hi=100000, s_max=500, seed_offset=0):
    """Poisson arrival trace of single (pair, point) jobs of mixed shapes.

    Returns a list of dicts: arrival time (s), d (d_y = d_x), window W in {10, 20},
    trials R = max(k + 1, round(N / W)) with N log-uniform in [n_lo, n_hi], S ~ U{0..s_max}.
    The series themselves are generated per job by ``job_workload``.
    """
    seed = BASE_SEED + 1000 * 5 + seed_offset
    u = uniform01(derive_key(seed, 1), 5 * n_jobs).reshape(n_jobs, 5)
    gaps = -np.log(1.0 - u[:, 0]) / rate
    t = np.cumsum(gaps)
    jobs = []
    for j in range(n_jobs):
        d = (2, 3, 4)[min(int(u[j, 1] * 3), 2)]
        W = (10, 20)[min(int(u[j, 2] * 2), 1)]
        n = math.exp(math.log(n_lo) + u[j, 3] * (math.log(n_hi) - math.log(n_lo)))
        R = max(8, int(round(n / W)))
        S = min(int(u[j, 4] * (s_max + 1)), s_max)
        jobs.append(dict(id=j, t=float(t[j]), d=d, W=W, R=R, S=S, seed=seed * 100003 + j))
    return jobs


def job_workload(job: dict, k: int = 4, with_perms: bool = True) -> Workload:
    """The series of one served job: linear AR pair, u = 1, tau = 1, one window at the end.
    with_perms=False leaves ``perms`` unset (the library draws the same ones from perm_seed)."""
    d, W, R, S = job["d"], job["W"], job["R"], job["S"]
    h = history(d, d, 1, 1)
    T = h + W
    seed = int(job["seed"] % (1 << 31))
    x, y = coupled_ar(seed, R, T, coupling=0.4, delay=1)
    w = Workload(name=f"job{job['id']}", x=x[None], y=y[None], d_y=d, d_x=d, tau=1, u=1, k=k,
                 window_start=np.array([h], np.int32), window_len=np.array([W], np.int32),
                 trials=np.array([R], np.int32), n_surrogates=S, meta=dict(job=job))
    w.perm_seed = int(seed)
    if with_perms:
        w.perms = make_perms(w.perm_seed, 1, w.trials, S, R)
    return w
