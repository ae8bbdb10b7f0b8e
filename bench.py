#!/usr/bin/env python3
"""Benchmark: ensemble transfer-entropy estimates per second on one MI355X.

Workload (the plain GPU ensemble configuration): nonlinear coupled AR pair,
500 trials x 300 samples; 100 analysis windows of 10 samples, each pooling all
trials (N = 5000 points), d_y = d_x = 3, tau = 1, u = 3 (joint dimension 7),
k = 4, float32 data, no surrogates.  One step = the whole hot path (embed,
k-NN radius search, three range counts, digamma sums) for all 100 windows,
i.e. 100 TE estimates, with the series already resident in HBM.

The timed steps run through te_surrogates_async (batched: one persistent search
launch per step, queued back to back on one stream, results left in HBM);
--sync times synchronous te_surrogates calls instead (a host round trip per
step).  latency_s is the latency of synchronous calls in either mode.  The plain
per-window path (te_estimate) is timed beside it.  The JSON line adds the search
kernel's roofline (FP32 VALU, measured with HIP events around each launch) and
the CPU oracle timed on the host cores on a bounded sample.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "TE estimates/s and distance evals/s (% FP32 VALU peak); p50/p99 latency"

# MI355X: 256 CUs at 2.4 GHz; a wave64 VALU instruction issues at 64 lanes/clk/CU.
N_CU = 256
CLOCK_HZ = 2.4e9
VALU_LANE_INSTR_PER_S = N_CU * 64 * CLOCK_HZ                 # 39.3e12
PEAK_FP32_OPS = 2 * VALU_LANE_INSTR_PER_S / 1e12             # 78.6 T ops/s: 3-input op (max3 / FMA) per lane
PEAK_FP32_HEADLINE = 157.3                                   # AMD headline (packed FMA), T flop/s


# HBM bytes per search launch of this workload from rocprofv3 --pmc FETCH_SIZE and WRITE_SIZE runs, scaled by a
# plain 256 MiB copy (factors 2.000 and 1.000), keyed by the kernel source they were taken on; any other kernel
# source reports null.
RECORDED_TRAFFIC = {"152d275deeea": 8918.05 * 1024 * 2.0 + 1319.97 * 1024 * 1.0}
KERNEL_SRC = os.path.join(ROOT, "paper_1401_4068_amd", "csrc", "te_kernels.hip")


def kernel_traffic():
    import hashlib
    try:
        h = hashlib.sha1(open(KERNEL_SRC, "rb").read()).hexdigest()[:12]
    except OSError:
        return None
    v = RECORDED_TRAFFIC.get(h)
    return None if v is None else int(v)


def ops_per_pair(D: int) -> int:
    """Algorithmic FP32 ops per directed pair over both passes: (2D) + (2D + 2)."""
    return 4 * D + 2


def host_threads() -> int:
    try:
        n = len(os.sched_getaffinity(0))
    except AttributeError:
        n = os.cpu_count() or 1
    return max(1, min(16, n))


def cpu_baseline(wl, budget_s: float = 12.0):
    """The oracle on the host cores on a bounded, seeded sample of the workload's chunks.

    Chunks are taken in a seeded random order, a batch of one chunk per thread at a
    time, until about budget_s seconds have passed.  The rate is scaled by directed
    pairs (the oracle's work grows as N^2): estimates/s = sample pairs/s divided by
    the workload's mean pairs per estimate."""
    from oracle import oracle
    from synth.rng import derive_key, permutation
    threads = host_threads()
    jobs, _ = oracle.workload_jobs(wl)
    order = permutation(derive_key(4068, len(jobs)), len(jobs))
    jobs = [jobs[i] for i in order]
    done = 0
    pairs = 0
    t_total = 0.0
    while done < len(jobs) and t_total < budget_s:
        sel = jobs[done:done + threads]
        t0 = time.perf_counter()
        oracle.te_jobs(wl.x, wl.y, wl.d_y, wl.d_x, wl.tau, wl.u, wl.k, sel, wl.perms, n_threads=threads)
        t_total += time.perf_counter() - t0
        done += len(sel)
        pairs += sum(j[3] * j[2] * (j[3] * j[2] - 1) for j in sel)
    mean_pairs = wl.directed_pairs() / wl.n_estimates()
    return dict(value=(pairs / t_total) / mean_pairs, unit="estimates/s", cores=threads, kind="oracle",
                sample="%d of %d chunks (seeded random order; %.3g directed pairs), %.1f s wall on %d threads; "
                       "scaled by directed pairs" % (done, len(jobs), pairs, t_total, threads))


def make_workload(name):
    import synth
    if name == "nonlinear":
        return synth.nonlinear_ensemble(), "nonlinear_ar_ensemble"
    if name == "linear":
        return synth.linear_pair(), "linear_ar_single_estimate"
    if name == "uneven":
        return synth.uneven_surrogates(), "uneven_chunks_200_surrogates"
    if name == "meg":
        return synth.meg_like(), "meg_like_16_pairs_100_surrogates"
    raise SystemExit("unknown workload " + name)


def batched_record(args, wl, wname):
    import torch
    import paper_1401_4068_amd as te

    D = wl.dim
    n = wl.chunk_sizes()
    pairs_per_pass = int(wl.directed_pairs())                 # Σ over all chunks of N(N-1)
    x = torch.from_numpy(wl.x).cuda()
    y = torch.from_numpy(wl.y).cuda()
    perms = torch.from_numpy(wl.perms).cuda() if wl.n_surrogates else None
    plan = te.Plan.from_workload(wl)
    full, minimum, plain_bytes = plan.workspace_bytes()
    ws = plan.workspace()
    tuned = None
    if not args.no_tune:
        # launch shape tuned on the plan's own data before anything is timed
        t0 = time.perf_counter()
        tuned = plan.autotune(x, y, perms, ws=ws)
        tuned["tuning_s"] = round(time.perf_counter() - t0, 3)
    stream = torch.cuda.Stream() if args.graph else torch.cuda.current_stream()
    pipelined = not (args.graph or args.sync)

    def step():
        return plan.surrogates(x, y, perms, ws=ws, stream=stream, use_graph=args.graph)

    G, S = wl.n_pairs * wl.n_points, wl.n_surrogates
    dev_out = torch.empty(G * (S + 1) + G, dtype=torch.float64, device="cuda")

    def step_async():
        # the same hot path queued on the stream: results stay in HBM, no host round trip
        return plan.surrogates_async(x, y, perms, ws=ws, stream=stream, out=dev_out)

    for _ in range(args.warmup):
        step_async() if pipelined else step()
    te.profile_enable(True)
    te.profile_read(reset=True)
    te.profile_work(reset=True)
    lat = []
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        s0 = time.perf_counter()
        if pipelined:
            step_async()
        else:
            out = step()
        lat.append(time.perf_counter() - s0)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    k_ms, k_n = te.profile_read(reset=True)
    w1, w2 = te.profile_work(reset=True)
    te.profile_enable(False)
    if pipelined:
        # results of the last queued step against a synchronous call (bit for bit), and the
        # latency of synchronous calls (one call = one step with its host round trip)
        out = step()
        got = dev_out.cpu().numpy()
        assert np.array_equal(got[:G * (S + 1)].reshape(wl.n_pairs, wl.n_points, S + 1)[..., 0], out[0]), \
            "queued and synchronous calls disagree"
        lat = []
        for _ in range(min(args.steps, 20)):
            s0 = time.perf_counter()
            step()
            lat.append(time.perf_counter() - s0)
    est = wl.n_estimates()
    value = est * args.steps / dt
    evals_per_s = 2 * pairs_per_pass * args.steps / dt

    # dominant kernel: the persistent search launch (one per step when the workspace holds the batch)
    roof = None
    if k_n > 0:
        avg_s = k_ms / k_n / 1e3
        # algorithmic ops of the pairs each launch evaluates: 2D per pass-1 pair, 2D + 2 per pass-2 pair
        p1, p2 = w1 / k_n, w2 / k_n
        ops = p1 * 2 * D + p2 * (2 * D + 2)
        method_ops = pairs_per_pass * ops_per_pair(D) * args.steps / k_n
        achieved = ops / avg_s / 1e12
        roof = dict(bound="alu", achieved=round(achieved, 3), peak=PEAK_FP32_OPS, unit="TFLOP/s",
                    frac=round(achieved / PEAK_FP32_OPS, 4),
                    traffic=kernel_traffic() if wname == "nonlinear_ar_ensemble" else None,
                    kernel="search_kernel<%d,%d,k=%d,slots=%d,sorted>" % (wl.d_y, wl.d_x, wl.k,
                                                                          tuned["slots"] if tuned else 4),
                    avg_launch_ms=round(avg_s * 1e3, 4), launches=k_n, ops_per_launch=int(ops),
                    pairs_evaluated_per_launch=[int(p1), int(p2)],
                    method_pairs_per_launch=int(pairs_per_pass * args.steps / k_n),
                    method_equivalent_tops=round(method_ops / avg_s / 1e12, 3),
                    frac_of_headline_157_3=round(achieved / PEAK_FP32_HEADLINE, 4))

    # plain per-time-point path on the same workload
    plain_rec = None
    if args.plain_steps > 0:
        if wl.n_surrogates == 0:
            run_plain = lambda: plan.estimate(x, y, ws=ws)                          # noqa: E731
            label = "te_estimate, one window at a time"
        else:
            ws_min = torch.empty(minimum, dtype=torch.uint8, device="cuda")
            run_plain = lambda: plan.surrogates(x, y, perms, ws=ws_min)              # noqa: E731
            label = "te_surrogates with the minimum workspace: one window's S+1 chunks per launch"
        run_plain()
        torch.cuda.synchronize()
        p0 = time.perf_counter()
        for _ in range(args.plain_steps):
            plain = run_plain()
        torch.cuda.synchronize()
        pdt = time.perf_counter() - p0
        ref = out[0] if wl.n_surrogates == 0 else out
        if wl.n_surrogates == 0:
            assert np.array_equal(plain, ref), "plain and batched paths disagree"
        else:
            for u, v in zip(plain, ref):
                assert np.array_equal(u, v), "plain and batched paths disagree"
        plain_rec = dict(value=round(est * args.plain_steps / pdt, 2), unit="estimates/s",
                         ms_per_step=round(pdt / args.plain_steps * 1e3, 3), path=label)

    rec = dict(
        metric=METRIC, value=round(value, 2), unit="estimates/s", n_gpus=1, steps=args.steps,
        warmup=args.warmup, ms_per_step=round(dt / args.steps * 1e3, 4), higher_is_better=True,
        scaling="weak", vs_baseline=None, dtype="f32", data="synthetic",
        config=dict(workload=wname, pairs=wl.n_pairs, trials=wl.n_trials, samples=wl.n_samples,
                    windows=wl.n_points, points_per_window_min=int(n.min()), points_per_window_max=int(n.max()),
                    d_y=wl.d_y, d_x=wl.d_x, tau=wl.tau, u=wl.u, dim=D, k=wl.k, surrogates=wl.n_surrogates,
                    estimates_per_step=est, workspace_bytes=int(full),
                    path=("batched (te_surrogates_async: one persistent search launch per step, steps queued "
                          "back to back, results left in HBM)" if pipelined else
                          "batched (te_surrogates, one persistent search launch)" + (", hipGraph" if args.graph
                                                                                    else ""))),
        distance_evals_per_s=round(evals_per_s, 1),
        pct_fp32_valu_peak=None if roof is None else round(100 * roof["frac"], 2),
        latency_s=dict(p50=float(np.percentile(lat, 50)), p99=float(np.percentile(lat, 99))),
        plain=plain_rec,
        tuned_shape=tuned,
        roofline=roof,
    )
    if pipelined and not args.no_two_stream:
        rec["pipelined_two_streams"] = two_stream_record(plan, wl, x, y, perms, ws, dev_out, args.steps)
    if not args.no_cpu:
        rec["cpu_baseline"] = cpu_baseline(wl)
    return rec


def two_stream_record(plan, wl, x, y, perms, ws, out, steps):
    """The same queued steps alternating over two streams, each with its own workspace
    and output buffer: a step's search launch then fills the tail of the previous one.
    Reported beside `value` (which, with the roofline, is measured on one stream, where
    each launch runs alone)."""
    import torch
    wss = [ws, plan.workspace()]
    outs = [out, torch.empty_like(out)]
    streams = [torch.cuda.Stream(), torch.cuda.Stream()]

    def run(n):
        for i in range(n):
            plan.surrogates_async(x, y, perms, ws=wss[i % 2], stream=streams[i % 2], out=outs[i % 2])

    # the overlap takes a while to settle (first passes on new streams measured up to 25 %
    # slower): two passes of warm-up, then the median of three timed passes
    run(2 * max(steps, 4))
    times = []
    for _ in range(3):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        run(steps)
        torch.cuda.synchronize()
        times.append(time.perf_counter() - t0)
    ref = outs[(steps - 1) % 2].cpu().numpy()
    other = outs[steps % 2].cpu().numpy()
    assert np.array_equal(ref, other, equal_nan=True), "the two streams' results disagree"
    dt = float(np.median(times))
    return dict(value=round(wl.n_estimates() * steps / dt, 2), unit="estimates/s",
                ms_per_step=round(dt / steps * 1e3, 4), streams=2, steps=steps,
                ms_per_step_passes=[round(t / steps * 1e3, 4) for t in times])


def scan_record(args, scenario):
    """Delay reconstruction over an AR coupling scenario (eq. 5, eq. 12-16): one step is
    te_delay_scan over both directions, every window and every assumed delay, then the
    surrogate test at the chosen delays.  Estimates per step: P C n_u originals plus
    P C (S + 1) at the chosen delays.  scenario 0: the robustness sweep over the amount
    of data (one coupled window, M = R_c * W points for several R_c)."""
    import torch
    import synth
    import paper_1401_4068_amd as te

    wl = synth.ar_robustness() if scenario == 0 else synth.ar_scenarios(scenario)
    u_values = wl.meta["u_values"]
    n_u = len(u_values)
    D = wl.dim
    sizes = wl.chunk_sizes()
    N = int(sizes.max())
    G = wl.n_pairs * wl.n_points
    est = G * n_u + G * (wl.n_surrogates + 1)
    pairs_per_step = int(np.sum(sizes * (sizes - 1))) * wl.n_pairs * (n_u + wl.n_surrogates + 1)
    x = torch.from_numpy(wl.x).cuda()
    y = torch.from_numpy(wl.y).cuda()
    perms = torch.from_numpy(wl.perms).cuda()
    plan = te.Plan.from_workload(wl)
    tuned = None
    if not args.no_tune:
        t0 = time.perf_counter()
        tuned = plan.autotune(x, y, perms)
        tuned["tuning_s"] = round(time.perf_counter() - t0, 3)
    full, _ = plan.delay_scan_workspace_bytes(u_values)
    ws = torch.empty(full, dtype=torch.uint8, device="cuda")
    step = lambda: plan.delay_scan(x, y, u_values, perms, ws=ws)                 # noqa: E731
    for _ in range(args.warmup):
        step()
    te.profile_enable(True)
    te.profile_read(reset=True)
    te.profile_work(reset=True)
    lat = []
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        s0 = time.perf_counter()
        out = step()
        lat.append(time.perf_counter() - s0)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    k_ms, k_n = te.profile_read(reset=True)
    w1, w2 = te.profile_work(reset=True)
    te.profile_enable(False)
    roof = None
    if k_n > 0:
        # two search launches per step (all delays; the chosen delay's test): their mean
        avg_s = k_ms / k_n / 1e3
        ops = (w1 * 2 * D + w2 * (2 * D + 2)) / k_n
        achieved = ops / avg_s / 1e12
        roof = dict(bound="alu", achieved=round(achieved, 3), peak=PEAK_FP32_OPS, unit="TFLOP/s",
                    frac=round(achieved / PEAK_FP32_OPS, 4), traffic=None, avg_launch_ms=round(avg_s * 1e3, 4),
                    launches=k_n, pairs_evaluated_per_launch=[int(w1 / k_n), int(w2 / k_n)],
                    method_pairs_per_launch=int(pairs_per_step * args.steps / k_n))
    te_scan, u_best, _, pv = out
    findings = []
    for p in range(wl.n_pairs):
        for c in range(wl.n_points):
            w0 = int(wl.window_start[c])
            findings.append(dict(direction=wl.meta["directions"][p], window=[w0, w0 + int(wl.window_len[c])],
                                 points=int(sizes[c]), u_best=int(u_best[p, c]),
                                 te_max=round(float(te_scan[p, c].max()), 4), p_value=float(pv[p, c])))
    rec = dict(
        metric=METRIC, value=round(est * args.steps / dt, 2), unit="estimates/s", n_gpus=1, steps=args.steps,
        warmup=args.warmup, ms_per_step=round(dt / args.steps * 1e3, 4), higher_is_better=True, scaling="weak",
        vs_baseline=None, dtype="f32", data="synthetic",
        config=dict(workload=("ar_robustness_delay_scan" if scenario == 0 else "ar_scenario%d_delay_scan" % scenario),
                    pairs=wl.n_pairs, trials=wl.n_trials, samples=wl.n_samples, windows=wl.n_points,
                    points_per_window=[int(v) for v in sorted(set(sizes.tolist()))], d_y=wl.d_y, d_x=wl.d_x,
                    tau=wl.tau, u_values=[u_values[0], u_values[-1]], dim=D, k=wl.k, surrogates=wl.n_surrogates,
                    estimates_per_step=est, workspace_bytes=int(full), path="te_delay_scan"),
        distance_evals_per_s=round(2 * pairs_per_step * args.steps / dt, 1),
        latency_s=dict(p50=float(np.percentile(lat, 50)), p99=float(np.percentile(lat, 99))),
        tuned_shape=tuned, roofline=roof, findings=findings)
    if not args.no_cpu:
        rec["cpu_baseline"] = scan_cpu_baseline(wl, u_values, est, pairs_per_step)
    return rec


def scan_cpu_baseline(wl, u_values, est_per_step, pairs_per_step, budget_s: float = 12.0):
    """The oracle on a seeded sample of (direction, window, delay) originals, scaled by pairs:
    estimates/s = sample pairs/s divided by the step's mean pairs per estimate."""
    from oracle import oracle
    from synth.rng import derive_key, permutation
    threads = host_threads()
    jobs = [(p, c, u) for p in range(wl.n_pairs) for c in range(wl.n_points) for u in u_values]
    order = permutation(derive_key(4068, len(jobs)), len(jobs))
    sizes = wl.chunk_sizes()
    done, t_total, pairs = 0, 0.0, 0
    while done < len(jobs) and t_total < budget_s:
        sel = [jobs[i] for i in order[done:done + threads]]
        t0 = time.perf_counter()
        for u in sorted(set(j[2] for j in sel)):
            js = [(p, int(wl.window_start[c]), int(wl.window_len[c]), int(wl.trials[c]), -1)
                  for (p, c, uu) in sel if uu == u]
            oracle.te_jobs(wl.x, wl.y, wl.d_y, wl.d_x, wl.tau, u, wl.k, js, wl.perms, n_threads=threads)
        t_total += time.perf_counter() - t0
        done += len(sel)
        pairs += sum(int(sizes[c]) * (int(sizes[c]) - 1) for (_, c, _) in sel)
    mean_pairs = pairs_per_step / est_per_step
    return dict(value=(pairs / t_total) / mean_pairs, unit="estimates/s", cores=threads, kind="oracle",
                sample="%d of %d original (direction, window, delay) chunks (%.3g directed pairs), %.1f s wall on "
                       "%d threads; scaled by directed pairs" % (done, len(jobs), pairs, t_total, threads))


def served_record(args):
    """Poisson-arriving jobs through te_serve_* (continuous batching) and the same trace
    through te_surrogates one job at a time (FIFO)."""
    import threading

    import torch
    import paper_1401_4068_amd as te
    import synth

    def replay(jobs, rate_label):
        wls = [synth.job_workload(j) for j in jobs]
        warm_srv = te.Server(arena_bytes=256 << 20, max_slots=4)     # module load, first launches
        for d in (2, 3, 4):
            warm = synth.job_workload(dict(id=-d, t=0.0, d=d, W=10, R=30, S=2, seed=d))
            warm_srv.wait(warm_srv.submit(warm), timeout_s=120)
        warm_srv.close()
        srv = te.Server(arena_bytes=args.arena_gb << 30, max_slots=args.slots, step_pairs=args.step_pairs)
        tickets = [None] * len(jobs)
        t_sub = [0.0] * len(jobs)
        t0 = time.perf_counter() + 0.01

        def submitter():
            for i, (j, wl) in enumerate(zip(jobs, wls)):
                d = t0 + j["t"] - time.perf_counter()
                if d > 0:
                    time.sleep(d)
                t_sub[i] = time.perf_counter()
                tickets[i] = srv.submit(wl)

        th = threading.Thread(target=submitter)
        th.start()
        th.join()
        for i in range(len(jobs)):
            srv.wait(tickets[i], timeout_s=3600)
        st = srv.stats()
        t_end = time.perf_counter()
        served_est_per_s = sum(1 + j["S"] for j in jobs) / (t_end - t_sub[0])
        srv.close()
        est = sum((1 + j["S"]) for j in jobs)
        pairs = sum((1 + j["S"]) * (j["R"] * j["W"]) * (j["R"] * j["W"] - 1) for j in jobs)
        # FIFO through the batched path, one job at a time (arrival-ordered, queueing included)
        done = 0.0
        fifo_lat = []
        for j, wl in zip(jobs, wls):
            # service = what the job costs on its own: plan, upload of its host arrays, batched run
            torch.cuda.synchronize()
            s0 = time.perf_counter()
            plan = te.Plan.from_workload(wl)
            x = torch.from_numpy(wl.x).cuda()
            y = torch.from_numpy(wl.y).cuda()
            perms = torch.from_numpy(wl.perms).cuda() if wl.n_surrogates else None
            plan.surrogates(x, y, perms)
            svc = time.perf_counter() - s0
            start = max(j["t"], done)
            done = start + svc
            fifo_lat.append(done - j["t"])
            plan.close()
        fifo_span = done - jobs[0]["t"]
        return dict(rate_per_s=rate_label, jobs=len(jobs), estimates=est, directed_pairs=int(pairs),
                    served=dict(p50_s=st["p50_s"], p99_s=st["p99_s"], est_per_s=served_est_per_s,
                                span_s=t_end - t_sub[0], steps=st["steps"], peak_slots=st["peak_slots"],
                                peak_arena_bytes=st["peak_bytes"]),
                    fifo=dict(p50_s=float(np.percentile(fifo_lat, 50)), p99_s=float(np.percentile(fifo_lat, 99)),
                              est_per_s=est / fifo_span, span_s=fifo_span))

    trace = synth.served_jobs(n_jobs=args.jobs, rate=200.0)
    r1 = replay(trace, 200.0)
    # second trace: arrival rate rescaled to 0.8 x the measured served capacity (jobs/s)
    cap_jobs = r1["jobs"] / r1["served"]["span_s"]
    rate2 = 0.8 * cap_jobs
    trace2 = synth.served_jobs(n_jobs=args.jobs, rate=rate2, seed_offset=1)
    r2 = replay(trace2, round(rate2, 3))
    rec = dict(metric=METRIC, value=round(r1["served"]["est_per_s"], 2), unit="estimates/s", n_gpus=1,
               steps=1, warmup=1, ms_per_step=round(r1["served"]["span_s"] * 1e3, 1), higher_is_better=True,
               scaling="weak", vs_baseline=None, dtype="f32", data="synthetic",
               config=dict(workload="served_mix", arrivals="poisson", jobs=args.jobs, dims=[5, 7, 9],
                           points_per_job="log-uniform 1000..100000", surrogates="0..500", k=4,
                           arena_gb=args.arena_gb, max_slots=args.slots, step_pairs=args.step_pairs),
               latency_s=dict(p50=r1["served"]["p50_s"], p99=r1["served"]["p99_s"]),
               traces=[r1, r2])
    return rec


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=50)
    ap.add_argument("--warmup", type=int, default=10)
    ap.add_argument("--workload", default="nonlinear",
                    choices=["nonlinear", "linear", "uneven", "meg", "served", "ar0", "ar1", "ar2", "ar3"],
                    help="ar0: delay recovery against the amount of data; ar1-ar3: the AR coupling scenarios")
    ap.add_argument("--no-cpu", action="store_true", help="skip the oracle CPU baseline")
    ap.add_argument("--plain-steps", type=int, default=3)
    ap.add_argument("--graph", action="store_true", help="replay the batched step as a hipGraph")
    ap.add_argument("--no-two-stream", action="store_true",
                    help="skip the two-stream pipelined measurement (profiled runs: its launches overlap)")
    ap.add_argument("--sync", action="store_true",
                    help="time synchronous te_surrogates calls (a host round trip per step) instead of queued steps")
    ap.add_argument("--no-tune", action="store_true", help="skip the launch-shape autotuner")
    ap.add_argument("--jobs", type=int, default=60, help="served workload: jobs per trace")
    ap.add_argument("--arena-gb", type=int, default=32, help="served workload: device arena")
    ap.add_argument("--slots", type=int, default=64, help="served workload: resident job slots")
    ap.add_argument("--step-pairs", type=int, default=0, help="served workload: pairs per search launch")
    ap.add_argument("--copy-calibration", type=int, default=0, metavar="BYTES",
                    help="only run a plain device-to-device copy of BYTES, 5 times (HBM counter calibration)")
    args = ap.parse_args()
    if args.copy_calibration:
        import torch
        a = torch.ones(args.copy_calibration // 4, dtype=torch.float32, device="cuda")
        b = torch.empty_like(a)
        for _ in range(5):
            b.copy_(a)
        torch.cuda.synchronize()
        print(json.dumps(dict(copy_bytes=args.copy_calibration, launches=5)))
        return
    if args.gpus != 1:
        print("bench.py measures one GPU: this build has no multi-GPU path (chunks shard independently "
              "across GPUs by design; run one process per GPU).", file=sys.stderr)
        sys.exit(2)
    import torch
    torch.cuda.set_device(0)
    if args.workload == "served":
        rec = served_record(args)
    elif args.workload.startswith("ar"):
        rec = scan_record(args, int(args.workload[2:]))
    else:
        wl, wname = make_workload(args.workload)
        rec = batched_record(args, wl, wname)
    print(json.dumps(rec), flush=True)


if __name__ == "__main__":
    main()
