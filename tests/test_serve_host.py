"""Server admission and queueing logic on the CPU (dry-run mode: no device work).

Dry-run jobs go through the same admission (FIFO, job slots, arena footprint) and
step scheduling as real ones but launch nothing; their estimates are NaN.
"""
import math

import numpy as np
import pytest

import synth


@pytest.fixture(scope="module")
def te():
    import paper_1401_4068_amd as te
    from paper_1401_4068_amd import build
    import os
    if not os.path.exists(te.LIB_PATH):
        build.build()
    return te


def _job(i, R=20, W=10, S=2, d=2):
    return synth.generic((777, i), R=R, T=40, d_y=d, d_x=d, starts=(20,), windows=(W,), n_surrogates=S)


def test_dry_run_completes_every_job_within_slot_limit(te):
    srv = te.Server(arena_bytes=64 << 20, max_slots=3, dry_run=True)
    tickets = [srv.submit(_job(i)) for i in range(12)]
    for t in tickets:
        a, b, p = srv.wait(t, timeout_s=30)
        assert a.shape == (1, 1) and b.shape == (1, 1, 2) and math.isnan(a[0, 0])
    st = srv.stats()
    assert st["completed"] == 12 and st["failed"] == 0
    assert 1 <= st["peak_slots"] <= 3
    assert st["steps"] >= 1
    srv.close()


def test_footprint_bounds_residency(te):
    one = _job(0, R=40, S=20)
    probe = te.Server(arena_bytes=1 << 30, max_slots=64, dry_run=True, hold=True)
    t = probe.submit(one)
    probe.resume()
    probe.wait(t, timeout_s=30)
    need = probe.stats()["peak_bytes"]          # one job plus its class's step tables
    probe.close()
    srv = te.Server(arena_bytes=need + need // 2, max_slots=64, dry_run=True)
    ts = [srv.submit(_job(i, R=40, S=20)) for i in range(8)]
    for t in ts:
        srv.wait(t, timeout_s=30)
    st = srv.stats()
    assert st["completed"] == 8
    assert st["peak_bytes"] <= need + need // 2
    srv.close()


def test_submit_rejections(te):
    srv = te.Server(arena_bytes=1 << 20, max_slots=2, max_queue=2, dry_run=True, hold=True)
    bad = _job(1)
    bad.window_start = np.array([1], np.int32)         # not enough history
    with pytest.raises(te.TEError) as ei:
        srv.submit(bad)
    assert ei.value.status == 1
    big = _job(2, R=400, S=50)                           # never fits a 1 MiB arena
    with pytest.raises(te.TEError) as ei:
        srv.submit(big)
    assert ei.value.status == 2
    t1 = srv.submit(_job(3))
    t2 = srv.submit(_job(4))
    with pytest.raises(te.TEError) as ei:                # queue holds 2
        srv.submit(_job(5))
    assert ei.value.status == 4
    with pytest.raises(te.TEError) as ei:                # held: nothing is admitted yet
        srv.wait(t1, timeout_s=0.05)
    assert ei.value.status == 5
    srv.cancel(t2)
    with pytest.raises(te.TEError) as ei:
        srv.wait(t2)
    assert ei.value.status == 6
    srv.resume()
    a, _, _ = srv.wait(t1, timeout_s=30)
    assert a.shape == (1, 1)
    st = srv.stats()
    assert st["completed"] == 1 and st["cancelled"] == 1
    srv.close()


def test_close_cancels_queued_jobs(te):
    srv = te.Server(arena_bytes=1 << 20, max_slots=1, dry_run=True, hold=True)
    t = srv.submit(_job(6))
    srv.close()


def test_failed_staging_releases_the_job_and_the_queue_moves_on(te, monkeypatch):
    """An admission whose pinned staging fails (injected) fails only its own job, with
    TE_ERR_NOMEM; its arena region is returned and the jobs behind it complete."""
    monkeypatch.setenv("TE_SERVE_FAULT_STAGING", "2")
    srv = te.Server(arena_bytes=64 << 20, max_slots=2, dry_run=True)
    tickets = [srv.submit(_job(i)) for i in range(5)]
    outcomes = []
    for t in tickets:
        try:
            srv.wait(t, timeout_s=30)
            outcomes.append("ok")
        except te.TEError as e:
            outcomes.append(e.status)
    st = srv.stats()
    srv.close()
    assert outcomes.count(2) == 1 and outcomes.count("ok") == 4, outcomes
    assert st["completed"] == 4 and st["failed"] == 1 and st["resident"] == 0 and st["queued"] == 0


def test_mixed_classes_in_a_tight_arena_all_complete(te):
    """Jobs of five kernel classes (dimensions, with and without surrogates) through an arena
    just large enough for the classes' step tables and the largest job: class tables are
    taken from the top of the arena, so job regions never fragment around them and every
    job is admitted in turn."""
    jobs = [_job(50 + i, R=R, S=S, d=d) for i, (R, S, d) in
            enumerate([(30, 4, 2), (45, 2, 3), (25, 6, 4), (60, 0, 2), (20, 3, 3), (35, 1, 4), (50, 0, 3)])]
    probe = te.Server(arena_bytes=1 << 30, max_slots=1, dry_run=True)
    for t in [probe.submit(wl) for wl in jobs]:
        probe.wait(t, timeout_s=30)
    need = probe.stats()["peak_bytes"]
    probe.close()
    srv = te.Server(arena_bytes=need + (64 << 10), max_slots=8, dry_run=True)
    tickets = [srv.submit(wl) for wl in jobs]
    for t in tickets:
        srv.wait(t, timeout_s=30)
    st = srv.stats()
    assert st["completed"] == len(jobs) and st["peak_bytes"] <= need + (64 << 10)
    srv.close()
