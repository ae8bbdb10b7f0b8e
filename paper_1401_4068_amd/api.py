"""Python front end of libte: argument marshalling only.

PyTorch provides device memory (workspaces, inputs, outputs) and streams;
every step of the computation runs in the library's HIP kernels.
"""
from __future__ import annotations

import ctypes

import numpy as np

from ._lib import TE_SERVE_DRY_RUN, TE_SERVE_HOLD, Problem, ServeStats, check, lib


def _torch():
    import torch
    return torch


def _dev_ptr(t, dtype, name):
    torch = _torch()
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise TypeError("%s must be a CUDA (HIP) tensor" % name)
    if t.dtype != dtype:
        raise TypeError("%s must be %s, got %s" % (name, dtype, t.dtype))
    if not t.is_contiguous():
        raise ValueError("%s must be contiguous" % name)
    return ctypes.c_void_p(t.data_ptr())


def _stream_handle(stream):
    torch = _torch()
    cur = torch.cuda.current_stream()
    if stream is None:
        stream = cur
    elif stream != cur:
        stream.wait_stream(cur)      # inputs written on the current stream are visible
    return ctypes.c_void_p(stream.cuda_stream), stream


def _dp(a):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def _local_offsets(plan):
    off = np.empty(plan.n_pairs * plan.n_points + 1, np.int64)
    check(lib().te_plan_local_offsets(plan._h, off.ctypes.data_as(ctypes.POINTER(ctypes.c_int64))))
    return off


def _problem(n_pairs, n_trials, n_samples, d_y, d_x, tau, u, k, window_start, window_len=None, trials=None,
             n_surrogates=0, window=0, cond_source=0, seed=0):
    """A te_problem and the arrays it points to (keep both alive while it is used)."""
    keep = []
    ws = np.ascontiguousarray(window_start, np.int32)
    p = Problem()
    p.n_pairs, p.n_trials, p.n_samples = n_pairs, n_trials, n_samples
    p.d_y, p.d_x, p.tau, p.u, p.k = d_y, d_x, tau, u, k
    p.n_points = int(ws.shape[0])
    p.window = int(window)
    p.n_surrogates = int(n_surrogates)
    p.cond_source = int(cond_source)
    p.seed = int(seed) & 0xFFFFFFFFFFFFFFFF
    I32P = ctypes.POINTER(ctypes.c_int32)
    p.window_start = ws.ctypes.data_as(I32P)
    keep.append(ws)
    if window_len is not None:
        wl = np.ascontiguousarray(window_len, np.int32)
        p.window_len = wl.ctypes.data_as(I32P)
        keep.append(wl)
    if trials is not None:
        tr = np.ascontiguousarray(trials, np.int32)
        p.trials = tr.ctypes.data_as(I32P)
        keep.append(tr)
    return p, keep


class Plan:
    """An analysis plan (te_plan): geometry of one job, validated on creation.

    Parameters follow te_problem in include/te.h: series of n_pairs pairs,
    n_trials repetitions and n_samples samples; embedding d_y, d_x, tau; delay
    u; k neighbours; per analysis point the window start, length and number of
    pooled repetitions; n_surrogates shuffled surrogates; cond_source = 1 conditions
    on the current source sample x_t as well; seed keys the surrogate permutations
    the library draws when a call is given none.
    """

    def __init__(self, n_pairs, n_trials, n_samples, d_y, d_x, tau, u, k, window_start, window_len=None,
                 trials=None, n_surrogates=0, window=0, cond_source=0, seed=0):
        p, self._keep = _problem(n_pairs, n_trials, n_samples, d_y, d_x, tau, u, k, window_start, window_len,
                                 trials, n_surrogates, window, cond_source, seed)
        self.n_points = int(p.n_points)
        self.n_pairs = int(n_pairs)
        self.n_surrogates = int(n_surrogates)
        h = ctypes.c_void_p()
        check(lib().te_plan_create(ctypes.byref(p), ctypes.byref(h)))
        self._h = h
        self._ws = None
        self.shape = dict(n_trials=n_trials, n_samples=n_samples)

    @classmethod
    def from_workload(cls, wl, n_surrogates=None):
        """A plan for a synth Workload; its seed is the one the workload's own permutations were
        drawn from, so calls without permutations draw the same ones on the device."""
        return cls(wl.n_pairs, wl.n_trials, wl.n_samples, wl.d_y, wl.d_x, wl.tau, wl.u, wl.k, wl.window_start,
                   wl.window_len, wl.trials, wl.n_surrogates if n_surrogates is None else n_surrogates,
                   cond_source=int(getattr(wl, "cond_source", 0)), seed=int(getattr(wl, "perm_seed", 0)))

    def close(self):
        if getattr(self, "_h", None):
            lib().te_plan_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def autotune(self, x, y, perms=None, ws=None, stream=None):
        """Pick the search kernel's launch shape on this plan's own data (te_plan_autotune)."""
        torch = _torch()
        self._check_series(x, y)
        sl, wpg, wg = ctypes.c_int32(), ctypes.c_int32(), ctypes.c_int32()
        ms = ctypes.c_double()
        pp = _dev_ptr(perms, torch.int32, "perms") if perms is not None else None
        wsp, wsn = self._ws_args(ws)
        sh, _ = _stream_handle(stream)
        check(lib().te_plan_autotune(self._h, _dev_ptr(x, torch.float32, "x"), _dev_ptr(y, torch.float32, "y"), pp,
                                     wsp, wsn, sh, ctypes.byref(sl), ctypes.byref(wpg), ctypes.byref(wg),
                                     ctypes.byref(ms)))
        return dict(slots=sl.value, waves_per_wg=wpg.value, wg_per_cu=wg.value, ms=ms.value)

    def workspace_bytes(self):
        f, m, p = ctypes.c_size_t(), ctypes.c_size_t(), ctypes.c_size_t()
        check(lib().te_plan_workspace_bytes(self._h, ctypes.byref(f), ctypes.byref(m), ctypes.byref(p)))
        return f.value, m.value, p.value

    def workspace(self, nbytes=None):
        """A device workspace tensor (uint8) of nbytes (default: the full batched size)."""
        torch = _torch()
        if nbytes is None:
            nbytes = max(self.workspace_bytes()[0], self.workspace_bytes()[2])
        return torch.empty(int(nbytes), dtype=torch.uint8, device="cuda")

    def _ws_args(self, ws):
        torch = _torch()
        if ws is None:
            if self._ws is None:
                self._ws = self.workspace()
            ws = self._ws
        return _dev_ptr(ws, torch.uint8, "ws"), ws.numel()

    def _check_series(self, x, y):
        want = self.n_pairs * self.shape["n_trials"] * self.shape["n_samples"]
        for name, t in (("x", x), ("y", y)):
            if t.numel() != want:
                raise ValueError("%s must hold n_pairs*n_trials*n_samples = %d values, got %d"
                                 % (name, want, t.numel()))

    def _check_perms(self, perms):
        """perms: None (the library draws them from the plan's seed) or int32 [P, C, S, R]."""
        if perms is None or self.n_surrogates == 0:
            return
        want = self.n_pairs * self.n_points * self.n_surrogates * self.shape["n_trials"]
        if perms.numel() != want:
            raise ValueError("perms must be int32 [n_pairs, n_points, S, n_trials] (%d values)" % want)

    def permutations(self, stream=None):
        """The permutations the library draws from the plan's seed: CUDA int32 [P, C, S, R]
        (te_plan_permutations)."""
        torch = _torch()
        P, C, S, R = self.n_pairs, self.n_points, self.n_surrogates, self.shape["n_trials"]
        out = torch.empty((P, C, max(S, 0), R), dtype=torch.int32, device="cuda")
        nb = int(lib().te_plan_permutations_workspace_bytes(self._h))
        ws = torch.empty(max(nb, 256), dtype=torch.uint8, device="cuda")
        sh, _ = _stream_handle(stream)
        check(lib().te_plan_permutations(self._h, ctypes.c_void_p(ws.data_ptr()), ws.numel(), sh,
                                         ctypes.c_void_p(out.data_ptr())))
        return out

    def estimate(self, x, y, ws=None, stream=None):
        """Plain per-window path: float64 [n_pairs, n_points] original estimates."""
        torch = _torch()
        self._check_series(x, y)
        out = np.empty((self.n_pairs, self.n_points), np.float64)
        wsp, wsn = self._ws_args(ws)
        sh, _ = _stream_handle(stream)
        check(lib().te_estimate(self._h, _dev_ptr(x, torch.float32, "x"), _dev_ptr(y, torch.float32, "y"), wsp, wsn,
                                sh, _dp(out)))
        return out

    def estimate_each(self, x, y, perms=None, ws=None, stream=None):
        """Plain per-chunk path over originals and surrogates (te_estimate_each):
        (te_orig [P, C], te_surr [P, C, S], p_value [P, C]), equal to surrogates()."""
        torch = _torch()
        self._check_series(x, y)
        self._check_perms(perms)
        S = self.n_surrogates
        te_orig = np.empty((self.n_pairs, self.n_points), np.float64)
        te_surr = np.empty((self.n_pairs, self.n_points, S), np.float64)
        pv = np.empty((self.n_pairs, self.n_points), np.float64)
        if ws is None:
            ws = self.workspace(self.workspace_bytes()[2])
        sh, _ = _stream_handle(stream)
        pp = ctypes.c_void_p(0) if perms is None else _dev_ptr(perms, torch.int32, "perms")
        check(lib().te_estimate_each(self._h, _dev_ptr(x, torch.float32, "x"), _dev_ptr(y, torch.float32, "y"), pp,
                                     _dev_ptr(ws, torch.uint8, "ws"), ws.numel(), sh, _dp(te_orig),
                                     _dp(te_surr) if S > 0 else None, _dp(pv)))
        return te_orig, te_surr, pv

    def local(self, x, y, ws=None, stream=None):
        """Local TE of every pooled point (eq. 17-18): (list over (pair, point) of CUDA float64
        arrays in window order, te float64 [P, C])."""
        torch = _torch()
        self._check_series(x, y)
        off = _local_offsets(self)
        lte = torch.empty(max(int(off[-1]), 1), dtype=torch.float64, device="cuda")
        te_out = np.empty((self.n_pairs, self.n_points), np.float64)
        wsp, wsn = self._ws_args(ws)
        sh, _ = _stream_handle(stream)
        check(lib().te_local(self._h, _dev_ptr(x, torch.float32, "x"), _dev_ptr(y, torch.float32, "y"), wsp, wsn, sh,
                             ctypes.c_void_p(lte.data_ptr()), _dp(te_out)))
        parts = [lte[off[g]:off[g + 1]] for g in range(self.n_pairs * self.n_points)]
        return parts, te_out

    def delay_scan_workspace_bytes(self, u_values):
        u = np.ascontiguousarray(u_values, np.int32)
        f, m = ctypes.c_size_t(), ctypes.c_size_t()
        check(lib().te_delay_scan_workspace_bytes(self._h, ctypes.c_void_p(u.ctypes.data), len(u), ctypes.byref(f),
                                                  ctypes.byref(m)))
        return f.value, m.value

    def delay_scan(self, x, y, u_values, perms=None, ws=None, stream=None):
        """Delay reconstruction (eq. 5): (te_scan [P, C, n_u], u_best int32 [P, C],
        te_surr [P, C, S] at u_best, p_value [P, C])."""
        torch = _torch()
        self._check_series(x, y)
        u = np.ascontiguousarray(u_values, np.int32)
        P, C, S = self.n_pairs, self.n_points, self.n_surrogates
        if ws is None:
            ws = torch.empty(int(self.delay_scan_workspace_bytes(u)[0]), dtype=torch.uint8, device="cuda")
        te_scan = np.empty((P, C, len(u)), np.float64)
        u_best = np.empty((P, C), np.int32)
        te_surr = np.empty((P, C, S), np.float64) if S else None
        pv = np.empty((P, C), np.float64)
        pp = _dev_ptr(perms, torch.int32, "perms") if perms is not None else None
        sh, _ = _stream_handle(stream)
        check(lib().te_delay_scan(self._h, _dev_ptr(x, torch.float32, "x"), _dev_ptr(y, torch.float32, "y"), pp,
                                  ctypes.c_void_p(u.ctypes.data), len(u), _dev_ptr(ws, torch.uint8, "ws"),
                                  ws.numel(), sh, _dp(te_scan), ctypes.c_void_p(u_best.ctypes.data),
                                  _dp(te_surr) if S else None, _dp(pv)))
        return te_scan, u_best, te_surr, pv

    def surrogates(self, x, y, perms=None, ws=None, stream=None, use_graph=False):
        """Batched path: (te_orig [P, C], te_surr [P, C, S], p_value [P, C])."""
        torch = _torch()
        self._check_series(x, y)
        S = self.n_surrogates
        self._check_perms(perms)
        te_orig = np.empty((self.n_pairs, self.n_points), np.float64)
        te_surr = np.empty((self.n_pairs, self.n_points, S), np.float64)
        pv = np.empty((self.n_pairs, self.n_points), np.float64)
        wsp, wsn = self._ws_args(ws)
        sh, _ = _stream_handle(stream)
        pp = ctypes.c_void_p(0) if perms is None else _dev_ptr(perms, torch.int32, "perms")
        check(lib().te_surrogates(self._h, _dev_ptr(x, torch.float32, "x"), _dev_ptr(y, torch.float32, "y"), pp,
                                  wsp, wsn, sh, int(bool(use_graph)), _dp(te_orig),
                                  _dp(te_surr) if S > 0 else None, _dp(pv)))
        return te_orig, te_surr, pv

    def surrogates_async(self, x, y, perms=None, ws=None, stream=None, out=None):
        """te_surrogates_async: the batched path queued on `stream` without waiting.
        Returns `out`, a CUDA float64 tensor [G * (S + 1) + G] (G = n_pairs * n_points):
        estimates [G, S + 1] (original first), then p-values [G]; valid once the stream
        has run the work.  ws must hold the full batch (workspace_bytes()["full"])."""
        torch = _torch()
        self._check_series(x, y)
        S = self.n_surrogates
        G = self.n_pairs * self.n_points
        self._check_perms(perms)
        if out is None:
            out = torch.empty(G * (S + 1) + G, dtype=torch.float64, device="cuda")
        elif out.dtype != torch.float64 or out.numel() != G * (S + 1) + G or not out.is_contiguous():
            raise ValueError("out must be a contiguous float64 tensor of %d values" % (G * (S + 1) + G))
        wsp, wsn = self._ws_args(ws)
        sh, _ = _stream_handle(stream)
        pp = ctypes.c_void_p(0) if perms is None else _dev_ptr(perms, torch.int32, "perms")
        check(lib().te_surrogates_async(self._h, _dev_ptr(x, torch.float32, "x"), _dev_ptr(y, torch.float32, "y"),
                                        pp, wsp, wsn, sh, ctypes.c_void_p(out.data_ptr())))
        return out


class Server:
    """Continuous-batching server (te_serve_*): jobs are submitted with host arrays and
    run on a device arena allocated here (a torch uint8 tensor) unless dry_run."""

    def __init__(self, arena_bytes, max_slots=64, max_queue=1 << 20, step_pairs=0, dry_run=False, hold=False):
        self._arena = None
        ptr = ctypes.c_void_p(0)
        if not dry_run:
            torch = _torch()
            self._arena = torch.empty(int(arena_bytes), dtype=torch.uint8, device="cuda")
            ptr = ctypes.c_void_p(self._arena.data_ptr())
        flags = (TE_SERVE_DRY_RUN if dry_run else 0) | (TE_SERVE_HOLD if hold else 0)
        h = ctypes.c_void_p()
        check(lib().te_serve_open(ptr, int(arena_bytes), int(max_slots), int(max_queue), int(step_pairs), flags,
                                  ctypes.byref(h)))
        self._h = h
        self._shapes = {}

    def submit(self, wl, draw_perms=False):
        """Submit a synth Workload-like object (series, geometry, perms); returns a ticket.
        draw_perms (or a workload without perms): the server draws the permutations on the
        device from the workload's seed instead of copying them in."""
        p, keep = _problem(wl.n_pairs, wl.n_trials, wl.n_samples, wl.d_y, wl.d_x, wl.tau, wl.u, wl.k,
                           wl.window_start, wl.window_len, wl.trials, wl.n_surrogates,
                           cond_source=int(getattr(wl, "cond_source", 0)), seed=int(getattr(wl, "perm_seed", 0)))
        x = np.ascontiguousarray(wl.x, np.float32)
        y = np.ascontiguousarray(wl.y, np.float32)
        perms = None
        if wl.n_surrogates > 0 and not draw_perms and getattr(wl, "perms", None) is not None:
            perms = np.ascontiguousarray(wl.perms, np.int32)
            if perms.size != wl.n_pairs * wl.n_points * wl.n_surrogates * wl.n_trials:
                raise ValueError("perms must be [n_pairs, n_points, S, n_trials]")
        t = ctypes.c_uint64()
        check(lib().te_serve_submit(self._h, ctypes.byref(p), ctypes.c_void_p(x.ctypes.data),
                                    ctypes.c_void_p(y.ctypes.data),
                                    None if perms is None else ctypes.c_void_p(perms.ctypes.data), ctypes.byref(t)))
        self._shapes[t.value] = (wl.n_pairs, int(p.n_points), wl.n_surrogates)
        return t.value

    def wait(self, ticket, timeout_s=None):
        """(te_orig [P, C], te_surr [P, C, S], p_value [P, C]) of a finished ticket."""
        P, C, S = self._shapes[ticket]
        te_orig = np.empty((P, C), np.float64)
        te_surr = np.empty((P, C, max(S, 0)), np.float64)
        pv = np.empty((P, C), np.float64)
        us = -1 if timeout_s is None else int(timeout_s * 1e6)
        st = lib().te_serve_wait(self._h, ctypes.c_uint64(ticket), us, _dp(te_orig), _dp(te_surr) if S > 0 else None,
                                 _dp(pv))
        if st != 5:     # anything but a timeout releases the ticket
            self._shapes.pop(ticket, None)
        check(st)
        return te_orig, te_surr, pv

    def resume(self):
        check(lib().te_serve_resume(self._h))

    def cancel(self, ticket):
        check(lib().te_serve_cancel(self._h, ctypes.c_uint64(ticket)))

    def stats(self):
        s = ServeStats()
        check(lib().te_serve_stats(self._h, ctypes.byref(s)))
        return {name: getattr(s, name) for name, _ in ServeStats._fields_}

    def close(self):
        if getattr(self, "_h", None):
            check(lib().te_serve_close(self._h))
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def knn_counts(pts, offsets, d_y, d_x, k, stream=None, ws=None, want_te=True):
    """Neighbour statistics of pre-embedded chunks (te_knn_counts).

    pts: CUDA float32 [D, stride] coordinate-major; offsets: host int64 [C+1].
    Returns (eps float32 CUDA [total], counts int32 CUDA [3, total], te float64 [C] or None).
    """
    torch = _torch()
    off = np.ascontiguousarray(offsets, np.int64)
    C = off.shape[0] - 1
    total = int(off[-1])
    D = 1 + d_y + d_x
    if pts.dim() != 2 or pts.shape[0] != D:
        raise ValueError("pts must be [1 + d_y + d_x, stride]")
    eps = torch.empty(max(total, 1), dtype=torch.float32, device=pts.device)
    cnt = torch.empty((3, max(total, 1)), dtype=torch.int32, device=pts.device)
    need = lib().te_knn_counts_workspace_bytes(C, total)
    if ws is None:
        ws = torch.empty(need, dtype=torch.uint8, device=pts.device)
    te = np.empty(C, np.float64) if want_te else None
    sh, _ = _stream_handle(stream)
    check(lib().te_knn_counts(_dev_ptr(pts, torch.float32, "pts"), pts.shape[1],
                              off.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)), C, d_y, d_x, k,
                              _dev_ptr(ws, torch.uint8, "ws"), ws.numel(), sh, ctypes.c_void_p(eps.data_ptr()),
                              ctypes.c_void_p(cnt.data_ptr()), _dp(te) if want_te else None))
    return eps[:total], cnt[:, :total], te


def knn_counts_noalloc(pts, offsets, d_y, d_x, k, eps, counts, stream=None, want_te=True):
    """te_knn_counts with the library's static device scratch (te_knn_counts_noalloc): the
    call itself allocates no device memory.  eps (CUDA float32 [>= total]) and counts (CUDA
    int32 [3, stride >= total], rows counts[s, :total]) are the caller's outputs; the counts
    use the row stride total, so pass counts of shape [3, total].  Returns te float64 [C] or None."""
    torch = _torch()
    off = np.ascontiguousarray(offsets, np.int64)
    C = off.shape[0] - 1
    total = int(off[-1])
    D = 1 + d_y + d_x
    if pts.dim() != 2 or pts.shape[0] != D:
        raise ValueError("pts must be [1 + d_y + d_x, stride]")
    if eps.numel() < total or counts.dim() != 2 or counts.shape[0] != 3 or counts.shape[1] != total:
        raise ValueError("eps must hold >= total points and counts must be [3, total]")
    te = np.empty(C, np.float64) if want_te else None
    sh, _ = _stream_handle(stream)
    check(lib().te_knn_counts_noalloc(_dev_ptr(pts, torch.float32, "pts"), pts.shape[1],
                                      off.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)), C, d_y, d_x, k, sh,
                                      _dev_ptr(eps, torch.float32, "eps"), _dev_ptr(counts, torch.int32, "counts"),
                                      _dp(te) if want_te else None))
    return te


def ragwitz(y, window_start, window_len, candidates, k, stream=None, ws=None, want_pred=False):
    """Local-predictor scores of candidate target embeddings (te_ragwitz).

    y: CUDA float32 [n_trials, n_samples]; candidates: sequence of (d, tau).  Returns
    (scores float64 [n_cand] (the smallest marks the chosen embedding), predictions CUDA
    float64 [n_cand, n_trials * window_len] or None)."""
    torch = _torch()
    if y.dim() != 2:
        raise ValueError("y must be [n_trials, n_samples]")
    dims = np.ascontiguousarray([int(d) for d, _ in candidates], np.int32)
    taus = np.ascontiguousarray([int(t) for _, t in candidates], np.int32)
    R, T = int(y.shape[0]), int(y.shape[1])
    n = len(dims)
    i32p = ctypes.POINTER(ctypes.c_int32)
    if ws is None:
        need = ctypes.c_size_t()
        check(lib().te_ragwitz_workspace_bytes(R, window_len, dims.ctypes.data_as(i32p), n, ctypes.byref(need)))
        ws = torch.empty(need.value, dtype=torch.uint8, device=y.device)
    pred = torch.empty((n, R * window_len), dtype=torch.float64, device=y.device) if want_pred else None
    scores = np.empty(n, np.float64)
    sh, _ = _stream_handle(stream)
    check(lib().te_ragwitz(_dev_ptr(y, torch.float32, "y"), R, T, window_start, window_len,
                           dims.ctypes.data_as(i32p), taus.ctypes.data_as(i32p), n, k,
                           _dev_ptr(ws, torch.uint8, "ws"), ws.numel(), sh,
                           ctypes.c_void_p(pred.data_ptr()) if want_pred else None, _dp(scores)))
    return scores, pred


def autotune(d_y, d_x, k, n_points, n_chunks=None, stream=None):
    """Time every search launch shape on synthetic chunks (te_autotune); the winner is
    used by plans created afterwards.  Returns the chosen shape and its time."""
    torch = _torch()
    if n_chunks is None:
        n_chunks = max(1, int(4096 * 64 // max(n_points, 1)))       # about one GPU-full of work items
    D = 1 + d_y + d_x
    npad = 1 << max(0, (n_points - 1).bit_length())
    need = (8 * n_points * n_chunks * D + 4 * n_points * n_chunks + 8 * npad * n_chunks + 160 * n_chunks
            + 8 * (n_points // 64 + 2) * n_chunks + (1 << 20))
    ws = torch.empty(need, dtype=torch.uint8, device="cuda")
    sl, wpg, wg = ctypes.c_int32(), ctypes.c_int32(), ctypes.c_int32()
    ms = ctypes.c_double()
    sh, _ = _stream_handle(stream)
    check(lib().te_autotune(d_y, d_x, k, n_points, n_chunks, ctypes.c_void_p(ws.data_ptr()), need, sh,
                            ctypes.byref(sl), ctypes.byref(wpg), ctypes.byref(wg), ctypes.byref(ms)))
    return dict(slots=sl.value, waves_per_wg=wpg.value, wg_per_cu=wg.value, ms=ms.value, n_points=n_points,
                n_chunks=n_chunks)


def tune_save(path):
    check(lib().te_tune_save(str(path).encode()))


def tune_load(path):
    check(lib().te_tune_load(str(path).encode()))


def tune_clear():
    check(lib().te_tune_clear())


def profile_enable(on: bool = True, work: bool = False):
    """te_profile_enable: on brackets search-kernel launches with HIP events; work makes the
    launches count the pairs they evaluate (profile_work)."""
    check(lib().te_profile_enable((1 if on else 0) | (2 if work else 0)))


def profile_read(reset: bool = False):
    """(summed search-kernel milliseconds, launches) since the last reset."""
    ms = ctypes.c_double()
    n = ctypes.c_int64()
    check(lib().te_profile_read(ctypes.byref(ms), ctypes.byref(n), int(bool(reset))))
    return ms.value, n.value


def profile_work(reset: bool = False):
    """(pass-1 pairs, pass-2 pairs) evaluated by timed search launches since the last reset."""
    a, b = ctypes.c_int64(), ctypes.c_int64()
    check(lib().te_profile_work(ctypes.byref(a), ctypes.byref(b), int(bool(reset))))
    return a.value, b.value


def profile_work_all(reset: bool = False):
    """(pass-1 pairs, pass-2 pairs, pass-1 shared pairs, pass-2 shared pairs): the first two
    count a pair once per chunk, the last two once per set of chunks searched together."""
    w = (ctypes.c_int64 * 4)()
    check(lib().te_profile_work_all(w, int(bool(reset))))
    return tuple(int(v) for v in w)


def version() -> str:
    return lib().te_version().decode()
