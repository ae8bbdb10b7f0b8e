"""Python front end of the brute-force KSG oracle (oracle/ksg_oracle.c).

TEST INFRASTRUCTURE ONLY: imported by the tests, the smoke check and the CPU
baseline leg of the benchmark, never by the library.  It shares no code with
the GPU path; both sides only read the same synthetic inputs.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "ksg_oracle.c")
LIB = os.path.join(HERE, "libksg_oracle.so")

_lib = None


def build(force: bool = True) -> str:
    """Compile the oracle with gcc (IEEE semantics: no fast-math, no contraction)."""
    if force or not os.path.exists(LIB):
        tmp = LIB + ".tmp%d" % os.getpid()
        cmd = ["gcc", "-O2", "-std=c11", "-fPIC", "-shared", "-pthread", "-ffp-contract=off",
               "-fno-fast-math", "-Wall", "-Wextra", "-o", tmp, SRC, "-lm"]
        subprocess.run(cmd, check=True)
        os.replace(tmp, LIB)
    return LIB


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB):
            build(force=True)
        L = ctypes.CDLL(LIB)
        f32p = ctypes.POINTER(ctypes.c_float)
        f64p = ctypes.POINTER(ctypes.c_double)
        i32p = ctypes.POINTER(ctypes.c_int32)
        i64p = ctypes.POINTER(ctypes.c_int64)
        ci = ctypes.c_int
        L.ksg_embed.argtypes = [f32p, f32p, ci, ci, ci, ci, ci, ci, ci, ci, ci, i32p, i32p, f32p]
        L.ksg_embed.restype = ci
        L.ksg_counts.argtypes = [f32p, ci, ci, ci, ci, ci, f64p, i32p, i32p, i32p]
        L.ksg_counts.restype = ci
        L.ksg_counts_points.argtypes = [f32p, ci, ci, ci, ci, ci, i64p, ci, f64p, i32p, i32p, i32p]
        L.ksg_counts_points.restype = ci
        L.ksg_counts_split.argtypes = [f32p, ci, ci, ci, ci, ci, ci, f64p, i32p, i32p, i32p]
        L.ksg_counts_split.restype = ci
        L.ksg_digamma_int.argtypes = [ci]
        L.ksg_digamma_int.restype = ctypes.c_double
        L.ksg_te_from_counts.argtypes = [i32p, i32p, i32p, ci, ci]
        L.ksg_te_from_counts.restype = ctypes.c_double
        L.ksg_local_from_counts.argtypes = [i32p, i32p, i32p, ci, ci, f64p]
        L.ksg_local_from_counts.restype = None
        L.ksg_p_value.argtypes = [ctypes.c_double, f64p, ci]
        L.ksg_p_value.restype = ctypes.c_double
        L.ksg_te_batch.argtypes = [f32p, f32p, ci, ci, ci, ci, ci, ci, ci, ci, ci,
                                   i32p, i32p, i32p, i32p, i32p, i32p, ci, f64p]
        L.ksg_te_batch.restype = ci
        L.ksg_counts_batch.argtypes = [f32p, i64p, ci, ci, ci, ci, ci, ci, f64p, i32p]
        L.ksg_counts_batch.restype = ci
        _lib = L
    return _lib


def _p(a, ct):
    return a.ctypes.data_as(ctypes.POINTER(ct))


def embed(x, y, d_y, d_x, tau, u, w, W, Rc=None, src_perm=None, tgt_perm=None, cond=False) -> np.ndarray:
    """Pooled points of one window as float32 [Rc*W, 1+d_y+d_x] (eq. 6-7, eq. 10).

    cond: the current source sample x_t joins the conditioning set (the note on
    instantaneous mixing with Fig. 2): it is inserted as the last target-past
    coordinate, giving [Rc*W, 2+d_y+d_x] points for d_y + 1 target-past columns."""
    x = np.ascontiguousarray(x, np.float32)
    y = np.ascontiguousarray(y, np.float32)
    R, T = x.shape
    Rc = R if Rc is None else int(Rc)
    D = 1 + d_y + d_x
    out = np.empty((Rc * W, D), np.float32)
    sp = None if src_perm is None else np.ascontiguousarray(src_perm[:Rc], np.int32)
    tp = None if tgt_perm is None else np.ascontiguousarray(tgt_perm[:Rc], np.int32)
    st = lib().ksg_embed(_p(x, ctypes.c_float), _p(y, ctypes.c_float), R, T, d_y, d_x, tau, u,
                         int(w), int(W), Rc,
                         None if sp is None else _p(sp, ctypes.c_int32),
                         None if tp is None else _p(tp, ctypes.c_int32),
                         _p(out, ctypes.c_float))
    if st != 0:
        raise ValueError("window geometry out of range")
    if cond:
        rs = np.arange(Rc) if sp is None else sp.astype(np.int64)
        xt = x[rs][:, int(w):int(w) + int(W)].reshape(-1)          # point order r * W + (t' - w)
        out = np.ascontiguousarray(np.insert(out, 1 + d_y, xt, axis=1))
    return out


def counts(pts, d_y, d_x, k, mode=0, n_threads=1):
    """(eps float64 [N], counts int32 [3, N] as (n_P, n_TP, n_PS)) of one chunk [N, D].

    n_threads != 1 splits the reference points of the chunk into contiguous ranges
    over that many threads (0: all online cores); the result is the same."""
    pts = np.ascontiguousarray(pts, np.float32)
    N = pts.shape[0]
    eps = np.empty(N, np.float64)
    cnt = np.empty((3, N), np.int32)
    args = (_p(eps, ctypes.c_double), _p(cnt[0], ctypes.c_int32), _p(cnt[1], ctypes.c_int32),
            _p(cnt[2], ctypes.c_int32))
    if n_threads == 1:
        st = lib().ksg_counts(_p(pts, ctypes.c_float), N, d_y, d_x, k, mode, *args)
    else:
        st = lib().ksg_counts_split(_p(pts, ctypes.c_float), N, d_y, d_x, k, mode, int(n_threads), *args)
    if st != 0:
        raise ValueError("need k >= 1 and N > k")
    return eps, cnt


def counts_points(pts, d_y, d_x, k, idx, mode=0):
    """Radius and counts of the listed reference points only (each by brute force over
    the whole chunk): (eps float64 [len(idx)], counts int32 [3, len(idx)])."""
    pts = np.ascontiguousarray(pts, np.float32)
    idx = np.ascontiguousarray(idx, np.int64)
    N = pts.shape[0]
    n = idx.shape[0]
    eps = np.empty(n, np.float64)
    cnt = np.empty((3, n), np.int32)
    st = lib().ksg_counts_points(_p(pts, ctypes.c_float), N, d_y, d_x, k, mode, _p(idx, ctypes.c_int64), n,
                                 _p(eps, ctypes.c_double), _p(cnt[0], ctypes.c_int32), _p(cnt[1], ctypes.c_int32),
                                 _p(cnt[2], ctypes.c_int32))
    if st != 0:
        raise ValueError("need k >= 1, N > k and indices in [0, N)")
    return eps, cnt


def counts_batch(chunks, d_y, d_x, k, mode=0, n_threads=0):
    """Neighbour statistics of several chunks in parallel: lists of (eps, counts)."""
    D = 1 + d_y + d_x
    sizes = [c.shape[0] for c in chunks]
    off = np.zeros(len(chunks) + 1, np.int64)
    off[1:] = np.cumsum(sizes)
    pts = np.ascontiguousarray(np.concatenate([np.asarray(c, np.float32).reshape(-1, D) for c in chunks]))
    total = int(off[-1])
    eps = np.empty(total, np.float64)
    cnt = np.empty((3, total), np.int32)
    bad = lib().ksg_counts_batch(_p(pts, ctypes.c_float), _p(off, ctypes.c_int64), len(chunks), d_y, d_x,
                                 k, mode, n_threads, _p(eps, ctypes.c_double), _p(cnt, ctypes.c_int32))
    if bad:
        raise ValueError("%d chunks rejected (need N > k)" % bad)
    return [(eps[off[c]:off[c + 1]], cnt[:, off[c]:off[c + 1]]) for c in range(len(chunks))]


def digamma_int(n: int) -> float:
    return lib().ksg_digamma_int(int(n))


def te_from_counts(cnt, k) -> float:
    cnt = np.ascontiguousarray(cnt, np.int32)
    N = cnt.shape[1]
    return lib().ksg_te_from_counts(_p(cnt[0], ctypes.c_int32), _p(cnt[1], ctypes.c_int32),
                                    _p(cnt[2], ctypes.c_int32), N, k)


def local_from_counts(cnt, k) -> np.ndarray:
    """Per-point local TE (eq. 17 on the pooled ensemble; mean = eq. 9, eq. 18)."""
    cnt = np.ascontiguousarray(cnt, np.int32)
    N = cnt.shape[1]
    out = np.empty(N, np.float64)
    lib().ksg_local_from_counts(_p(cnt[0], ctypes.c_int32), _p(cnt[1], ctypes.c_int32),
                                _p(cnt[2], ctypes.c_int32), N, k, _p(out, ctypes.c_double))
    return out


def local_te(pts, d_y, d_x, k, mode=0) -> np.ndarray:
    """Local TE of every point of one pooled chunk [N, D], in the chunk's point order."""
    return local_from_counts(counts(pts, d_y, d_x, k, mode)[1], k)


def p_value(te_orig: float, te_surr) -> float:
    s = np.ascontiguousarray(te_surr, np.float64)
    return lib().ksg_p_value(float(te_orig), _p(s, ctypes.c_double), len(s))


def te_jobs(x, y, d_y, d_x, tau, u, k, jobs, perms=None, n_threads=0, mode=0):
    """TE of independent (pair, w, W, Rc, perm_row) jobs on [P, R, T] series, threaded."""
    x = np.ascontiguousarray(x, np.float32)
    y = np.ascontiguousarray(y, np.float32)
    P, R, T = x.shape
    J = len(jobs)
    cols = np.array(jobs, np.int32).reshape(J, 5).T.copy() if J else np.zeros((5, 0), np.int32)
    pair, w, W, Rc, prow = (np.ascontiguousarray(c) for c in cols)
    if perms is None:
        perms = np.zeros((1, R), np.int32)
    perms = np.ascontiguousarray(perms.reshape(-1, R), np.int32)
    te = np.full(J, np.nan)
    bad = lib().ksg_te_batch(_p(x, ctypes.c_float), _p(y, ctypes.c_float), R, T, d_y, d_x, tau, u, k, mode,
                             J, _p(pair, ctypes.c_int32), _p(w, ctypes.c_int32), _p(W, ctypes.c_int32),
                             _p(Rc, ctypes.c_int32), _p(prow, ctypes.c_int32), _p(perms, ctypes.c_int32),
                             n_threads, _p(te, ctypes.c_double))
    if bad:
        raise ValueError("%d jobs rejected" % bad)
    return te


def workload_jobs(wl, pairs=None, points=None, surrogates=None):
    """Job list for a synth Workload: (pair, w, W, Rc, perm_row) per chunk, originals as s = 0.

    The permutation rows index ``wl.perms.reshape(-1, R)``; surrogate s >= 1 uses
    perms[pair, point, s-1].
    """
    P, C, S = wl.n_pairs, wl.n_points, wl.n_surrogates
    pairs = range(P) if pairs is None else pairs
    points = range(C) if points is None else points
    surrogates = range(S + 1) if surrogates is None else surrogates
    jobs, keys = [], []
    for p in pairs:
        for c in points:
            for s in surrogates:
                row = -1 if s == 0 else (p * C + c) * S + (s - 1)
                jobs.append((p, int(wl.window_start[c]), int(wl.window_len[c]), int(wl.trials[c]), row))
                keys.append((p, c, s))
    return jobs, keys


def te_cond_jobs(x, y, d_y, d_x, tau, u, k, jobs, perms=None, mode=0):
    """TE conditioned on the current source sample as well, for (pair, w, W, Rc, perm_row) jobs."""
    x = np.ascontiguousarray(x, np.float32)
    y = np.ascontiguousarray(y, np.float32)
    R = x.shape[1]
    prow = None if perms is None else np.ascontiguousarray(perms, np.int32).reshape(-1, R)
    out = np.empty(len(jobs))
    for i, (p, w, W, Rc, row) in enumerate(jobs):
        sp = None if row < 0 else prow[row]
        pts = embed(x[p], y[p], d_y, d_x, tau, u, w, W, Rc, src_perm=sp, cond=True)
        out[i] = te_from_counts(counts(pts, d_y + 1, d_x, k, mode)[1], k)
    return out


def te_workload(wl, pairs=None, points=None, surrogates=None, n_threads=0, mode=0):
    """Oracle TE for the selected chunks of a workload: dict (pair, point, s) -> TE."""
    jobs, keys = workload_jobs(wl, pairs, points, surrogates)
    if getattr(wl, "cond_source", 0):
        te = te_cond_jobs(wl.x, wl.y, wl.d_y, wl.d_x, wl.tau, wl.u, wl.k, jobs, wl.perms, mode)
        return dict(zip(keys, te.tolist()))
    te = te_jobs(wl.x, wl.y, wl.d_y, wl.d_x, wl.tau, wl.u, wl.k, jobs, wl.perms, n_threads, mode)
    return dict(zip(keys, te.tolist()))


def delay_scan(wl, u_values, pairs=None, points=None, n_threads=0, mode=0):
    """Delay reconstruction (eq. 5): the original TE at every assumed delay, the
    maximizing delay (first maximum in u_values order), and the surrogate TE and
    p-value (surrogate test of eq. 10) at that delay.

    Returns dicts keyed by (pair, point): te_scan -> [n_u] array, u_best -> int,
    te_surr -> [S] array, p_value -> float (NaN without surrogates).
    """
    u_values = [int(u) for u in u_values]
    jobs, keys = workload_jobs(wl, pairs, points, surrogates=[0])
    keys = [key[:2] for key in keys]
    scan = np.empty((len(keys), len(u_values)))
    for j, u in enumerate(u_values):
        scan[:, j] = te_jobs(wl.x, wl.y, wl.d_y, wl.d_x, wl.tau, u, wl.k, jobs, wl.perms, n_threads, mode)
    te_scan = {key: scan[i] for i, key in enumerate(keys)}
    u_best = {key: u_values[int(np.argmax(scan[i]))] for i, key in enumerate(keys)}
    S = wl.n_surrogates
    te_surr, pv = {}, {}
    for u in sorted(set(u_best.values())):
        sel = [key for key in keys if u_best[key] == u]
        sj, sk = [], []
        for (p, c) in sel:
            sub, subk = workload_jobs(wl, [p], [c], range(1, S + 1))
            sj += sub
            sk += subk
        te = te_jobs(wl.x, wl.y, wl.d_y, wl.d_x, wl.tau, u, wl.k, sj, wl.perms, n_threads, mode) if sj else []
        got = dict(zip(sk, list(te)))
        for (p, c) in sel:
            te_surr[(p, c)] = np.array([got[(p, c, s)] for s in range(1, S + 1)])
            pv[(p, c)] = p_value(te_scan[(p, c)][u_values.index(u)], te_surr[(p, c)]) if S else float("nan")
    return te_scan, u_best, te_surr, pv


def timed_te_jobs(*args, **kw):
    t0 = time.perf_counter()
    te = te_jobs(*args, **kw)
    return te, time.perf_counter() - t0
