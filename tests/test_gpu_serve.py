"""GPU serving: every job's result is the same alone and in the continuous-batching mix.

A job run alone goes through te_surrogates; in the mix it is admitted by the
server while other jobs of other shapes are resident, its reference blocks are
spread over several search launches shared with those jobs, and it is reduced
per job in block order.  Estimates, surrogate estimates and p-values must be
bitwise identical, and within 1e-6 (checked at 1e-9) of the oracle.
"""
import sys
import time

import numpy as np
import pytest

import synth
from oracle import oracle

pytestmark = pytest.mark.gpu


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


def _jobs():
    out = []
    shapes = [(2, 60, 10, 4), (3, 90, 20, 2), (4, 50, 10, 6), (2, 130, 10, 0), (3, 40, 20, 3), (4, 70, 20, 1),
              (2, 33, 10, 5), (3, 150, 10, 2)]
    for i, (d, R, W, S) in enumerate(shapes):
        h = synth.history(d, d, 1, 1)
        out.append(synth.generic((9100, i), R=R, T=h + W + 5, d_y=d, d_x=d, starts=(h + 3,), windows=(W,),
                                 n_surrogates=S))
    return out


def _alone(te, wl):
    import torch
    x = torch.from_numpy(wl.x).cuda()
    y = torch.from_numpy(wl.y).cuda()
    perms = torch.from_numpy(wl.perms).cuda() if wl.n_surrogates else None
    return te.Plan.from_workload(wl).surrogates(x, y, perms)


def test_alone_equals_mix(te):
    jobs = _jobs()
    alone = [_alone(te, wl) for wl in jobs]
    say("alone done", [float(a[0][0, 0]) for a in alone])
    srv = te.Server(arena_bytes=256 << 20, max_slots=5, step_pairs=2_000_000)
    tickets = []
    for i, wl in enumerate(jobs):
        tickets.append(srv.submit(wl))
        if i % 3 == 2:
            time.sleep(0.002)            # later jobs arrive while earlier ones run
    for wl, t, ref in zip(jobs, tickets, alone):
        got = srv.wait(t, timeout_s=60)
        for u, v in zip(ref, got):
            np.testing.assert_array_equal(u, v)
    st = srv.stats()
    say("stats", st)
    assert st["completed"] == len(jobs) and st["failed"] == 0
    assert st["steps"] >= len(set((wl.d_y for wl in jobs)))  # at least one step per kernel class
    assert st["peak_slots"] <= 5
    srv.close()
    # two jobs against the oracle
    for wl, ref in list(zip(jobs, alone))[:2]:
        o = oracle.te_workload(wl)
        assert abs(ref[0][0, 0] - o[(0, 0, 0)]) <= 1e-9
        for s in range(1, wl.n_surrogates + 1):
            assert abs(ref[1][0, 0, s - 1] - o[(0, 0, s)]) <= 1e-9


def test_small_arena_queues_and_still_matches(te):
    jobs = _jobs()[:5]
    alone = [_alone(te, wl) for wl in jobs]
    # probe: the jobs one at a time -> step tables of every kernel class + the largest job
    probe = te.Server(arena_bytes=256 << 20, max_slots=1)
    for t in [probe.submit(wl) for wl in jobs]:
        probe.wait(t, timeout_s=60)
    one = probe.stats()["peak_bytes"]
    probe.close()
    srv = te.Server(arena_bytes=one + (64 << 10), max_slots=8, step_pairs=1_000_000)
    tickets = [srv.submit(wl) for wl in jobs]
    for t, ref in zip(tickets, alone):
        got = srv.wait(t, timeout_s=60)
        for u, v in zip(ref, got):
            np.testing.assert_array_equal(u, v)
    st = srv.stats()
    assert st["peak_bytes"] <= one + (64 << 10)
    srv.close()


def test_invalid_job_fails_alone(te):
    good = _jobs()[0]
    bad = _jobs()[1]
    bad.y[0, 5, int(bad.window_start[0]) + 2] = np.nan
    srv = te.Server(arena_bytes=64 << 20, max_slots=4)
    tg, tb = srv.submit(good), srv.submit(bad)
    with pytest.raises(te.TEError) as ei:
        srv.wait(tb, timeout_s=60)
    assert ei.value.status == 1
    ref = _alone(te, good)
    got = srv.wait(tg, timeout_s=60)
    for u, v in zip(ref, got):
        np.testing.assert_array_equal(u, v)
    srv.close()


def test_chunks_split_across_steps_match_alone(te, monkeypatch):
    """With one wave per CU a step holds 4 to 16 items per CU (1 024 to 4 096 items on 256 CUs),
    so the two jobs' chunk sets of 80 000 points (an original and a surrogate each, 1 250 blocks,
    2 500 items) are spread over at least three steps in pieces; each piece is searched over its
    own blocks only and the results equal the jobs run alone."""
    monkeypatch.setenv("TE_WAVES_PER_WG", "1")
    monkeypatch.setenv("TE_WG_PER_CU", "1")
    jobs = []
    for i in range(2):
        h = synth.history(2, 2, 1, 1)
        jobs.append(synth.generic((9200, i), R=4000, T=h + 25, d_y=2, d_x=2, starts=(h + 3,), windows=(20,),
                                  n_surrogates=1))
    alone = [_alone(te, wl) for wl in jobs]
    srv = te.Server(arena_bytes=512 << 20, max_slots=2, step_pairs=1)
    tickets = [srv.submit(wl) for wl in jobs]
    for t, ref in zip(tickets, alone):
        got = srv.wait(t, timeout_s=120)
        for u, v in zip(ref, got):
            np.testing.assert_array_equal(u, v)
    st = srv.stats()
    say("split steps", st)
    assert st["steps"] >= 3
    srv.close()
