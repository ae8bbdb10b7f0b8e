#!/usr/bin/env python3
"""Benchmark: ensemble transfer-entropy estimates per second on one MI355X.

Default workload (batched surrogates): linear coupled AR pair, 5000 trials x 400
samples; 60 analysis time points whose windows pool 1 014 to 49 400 points
(R_c trials x W_c samples, uneven), d_y = d_x = 3, tau = 1, u = 1 (joint
dimension 7), k = 4, float32 data, 200 trial-shuffled source surrogates per time
point: 12 060 estimates per step.  One step = the whole hot path on device-
resident series: the surrogate permutations drawn from the plan's seed, sorting
and embedding every window, the k-NN radius search, the three range counts, the
digamma sums and the p-values of all 60 x 201 chunks, in one persistent search
launch (te_surrogates_async, steps queued back to back on one stream).

The JSON line adds the search kernel's roofline (FP32 VALU; kernel time from HIP
events around every timed launch, evaluated pairs from device counters in a
separate untimed step), the plain per-time-point path on the same work, and the
CPU oracle timed on the host cores on a bounded sample.  --workload selects the
other configurations (nonlinear ensemble without surrogates, MEG-shaped batch,
linear pair, AR delay scans, served mix).
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

# MI355X: 256 CUs in 8 XCDs, 4 SIMDs per CU, 2.4 GHz peak engine clock.  FP32 VALU instructions run
# 32 lanes per SIMD per clock (a wave64 instruction in 2 clocks): 256 x 4 x 32 x 2.4e9 = 78.6e12
# lane-instructions/s, which is AMD's 157.3 TFLOP/s FP32 vector figure when each is a 2-flop FMA.
# (The search kernel's own counters confirm the rate: on the uneven-surrogate batch it issues 1.51e12
# wave64 VALU instructions in 1.65 s, more than one per SIMD every 4 clocks.)
N_CU = 256
CLOCK_HZ = 2.4e9
FP32_LANE_INSTR_PER_S = N_CU * 4 * 32 * CLOCK_HZ              # 78.6e12
PEAK_FP32_HEADLINE = 157.3                                   # AMD headline (FMA = 2 flops), T flop/s


def ops_per_pair(D: int) -> int:
    """Algorithmic FP32 ops per directed pair over both passes: pass 1 D sub + (D-1) max + 1 cmp = 2D,
    pass 2 D sub + (D-1) max + 3 cmp = 2D + 2."""
    return 4 * D + 2


def executed_ops(DT: int, DX: int, w):
    """FP32 ops the search executed, by kind, from its four work counters w = (pass-1 and pass-2
    (reference, candidate, chunk) triples, pass-1 and pass-2 (reference, candidate) pairs whose
    target coordinates were compared once for a set of chunks).  Per shared pair: DT subtractions
    and DT - 1 maxes in either pass (pass 2: the target-past max and max(d_T, d_P)); per triple,
    pass 1: DX subtractions, DX maxes (source block, then the joint max), 1 compare; pass 2: DX
    subtractions, DX maxes (source block, then max(d_P, d_S)), 3 compares.  Without sets (shared
    pairs = triples) this is 2D per pass-1 pair and 2D + 2 per pass-2 pair."""
    p1, p2, s1, s2 = (float(v) for v in w)
    sub = (s1 + s2) * DT + (p1 + p2) * DX
    mx = (s1 + s2) * (DT - 1) + (p1 + p2) * DX
    cmp = p1 + 3 * p2
    return sub, mx, cmp


def valu_ceiling(sub: float, mx: float, cmp: float) -> float:
    """FP32 VALU roofline of an op mix (T ops/s): 78.6e12 lane-instructions/s times the ops per
    instruction of its fewest-instruction form without packed math -- a subtraction or a compare
    is one op per instruction, two maxes fold into one 3-input v_max3 (abs is a free source
    modifier).  Without sets at D = 7: 30 ops in 24 instructions, 98.3 T."""
    return FP32_LANE_INSTR_PER_S * (sub + mx + cmp) / (sub + mx / 2 + cmp) / 1e12


# HBM bytes per search launch from rocprofv3 --pmc FETCH_SIZE and WRITE_SIZE runs, scaled by a plain 256 MiB
# device copy measured the same way (factors 2.000 and 1.000), keyed by (kernel source, workload); any other
# kernel source reports null.
RECORDED_TRAFFIC = {
    ("e2709849861a", "uneven_chunks_200_surrogates"): 171724200872,
    ("e2709849861a", "nonlinear_ar_ensemble"): 19403050,
}
KERNEL_SRC = os.path.join(ROOT, "paper_1401_4068_amd", "csrc", "te_kernels.hip")


def kernel_sha() -> str:
    import hashlib
    try:
        return hashlib.sha1(open(KERNEL_SRC, "rb").read()).hexdigest()[:12]
    except OSError:
        return ""


def kernel_traffic(workload: str):
    v = RECORDED_TRAFFIC.get((kernel_sha(), workload))
    return None if v is None else int(v)


def host_info() -> dict:
    """Host cores: nproc, this process's CPU affinity, the threads the oracle uses (the
    process's share, at most 16 per GPU on the test hosts) and the CPU model."""
    nproc = os.cpu_count() or 1
    try:
        aff = len(os.sched_getaffinity(0))
    except AttributeError:
        aff = nproc
    env = os.environ.get("OMP_NUM_THREADS", "")
    threads = max(1, min(aff, int(env) if env.isdigit() and int(env) > 0 else aff, 16))
    model = ""
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                model = line.split(":", 1)[1].strip()
                break
    except OSError:
        pass
    return dict(nproc=nproc, affinity=aff, threads=threads, cpu_model=model)


def _oracle_chunk(wl, job, threads):
    """TE of one (pair, w, W, Rc, perm_row) chunk by the oracle, its reference points split over threads."""
    from oracle import oracle
    p, w, W, Rc, row = job
    perm = None if row < 0 else wl.perms.reshape(-1, wl.n_trials)[row]
    pts = oracle.embed(wl.x[p], wl.y[p], wl.d_y, wl.d_x, wl.tau, wl.u, w, W, Rc=Rc, src_perm=perm)
    _, cnt = oracle.counts(pts, wl.d_y, wl.d_x, wl.k, n_threads=threads)
    return oracle.te_from_counts(cnt, wl.k)


def cpu_baseline(wl, budget_s: float = 20.0, plan_c3: bool = False):
    """The oracle (untuned) on the host cores on a bounded, seeded sample of the workload's chunks.

    plan_c3 (the uneven-surrogate batch): every original of at most 10 000 points and the three
    largest chunks first, then surrogate chunks in a seeded order while the time budget lasts.
    Otherwise chunks in a seeded order, one per thread at a time, while the budget lasts.
    Chunks of more than 10 000 points split their reference points over all threads; smaller
    ones run one chunk per thread.  The rate is scaled by directed pairs (the oracle's work grows
    as N^2): estimates/s = sample pairs/s divided by the workload's mean pairs per estimate."""
    from oracle import oracle
    from synth.rng import derive_key, permutation
    info = host_info()
    threads = info["threads"]
    jobs, keys = oracle.workload_jobs(wl)
    size = lambda j: j[2] * j[3]                                         # noqa: E731
    if plan_c3:
        orig = [i for i, k in enumerate(keys) if k[2] == 0]
        first = [i for i in orig if size(jobs[i]) <= 10000]
        big = sorted(orig, key=lambda i: -size(jobs[i]))[:3]
        rest = [i for i, k in enumerate(keys) if k[2] > 0]
        order = [rest[i] for i in permutation(derive_key(4068, len(rest)), len(rest))]
        queue = first + [i for i in big if i not in first] + order
        label = "all originals of <= 10 000 points, the 3 largest chunks, then surrogate chunks in seeded order"
    else:
        queue = [int(i) for i in permutation(derive_key(4068, len(jobs)), len(jobs))]
        label = "chunks in seeded order"
    done, pairs, t_total, npick = 0, 0, 0.0, 0
    while done < len(queue) and t_total < budget_s:
        j = jobs[queue[done]]
        if size(j) > 10000:
            t0 = time.perf_counter()
            _oracle_chunk(wl, j, threads)
            t_total += time.perf_counter() - t0
            sel = [j]
            done += 1
        else:
            sel = []
            while done < len(queue) and len(sel) < threads and size(jobs[queue[done]]) <= 10000:
                sel.append(jobs[queue[done]])
                done += 1
            t0 = time.perf_counter()
            oracle.te_jobs(wl.x, wl.y, wl.d_y, wl.d_x, wl.tau, wl.u, wl.k, sel, wl.perms, n_threads=threads)
            t_total += time.perf_counter() - t0
        npick += len(sel)
        pairs += sum(size(j) * (size(j) - 1) for j in sel)
    mean_pairs = wl.directed_pairs() / wl.n_estimates()
    rate = pairs / t_total
    return dict(value=rate / mean_pairs, unit="estimates/s", cores=threads, kind="oracle",
                sample="%s: %d of %d chunks, %.3g of %.3g directed pairs per pass (%.2f %%), %.1f s wall on %d "
                       "threads; scaled by directed pairs" % (label, npick, len(jobs), pairs, wl.directed_pairs(),
                                                              100.0 * pairs / wl.directed_pairs(), t_total, threads),
                pairs_per_s=rate, pairs_per_s_per_core=rate / threads, nproc=info["nproc"],
                affinity=info["affinity"], cpu_model=info["cpu_model"])


WORKLOADS = {
    "uneven": "uneven_chunks_200_surrogates",
    "nonlinear": "nonlinear_ar_ensemble",
    "linear": "linear_ar_single_estimate",
    "meg": "meg_like_16_pairs_100_surrogates",
}


def make_workload(name):
    import synth
    if name == "nonlinear":
        return synth.nonlinear_ensemble(), WORKLOADS[name]
    if name == "linear":
        return synth.linear_pair(), WORKLOADS[name]
    if name == "uneven":
        return synth.uneven_surrogates(), WORKLOADS[name]
    if name == "meg":
        return synth.meg_like(), WORKLOADS[name]
    raise SystemExit("unknown workload " + name)


def set_kernel_name(d_y: int, d_x: int) -> str:
    """Name of the library's chunk-set search kernel for these dimensions: sets of as many chunks (2-4) as keep
    4 (1 + d_y + V d_x) coordinates within 64 scalar registers; the wide form for 1 + d_y + V d_x >= 16."""
    q = (15 - d_y) // d_x
    v = 4 if q >= 4 else (2 if q <= 2 else q)
    return "sets_wide_kernel" if 1 + d_y + v * d_x >= 16 else "sets_kernel"


def roofline_record(wl, wname, k_ms, k_n, w, work_launches, slots, pairs_per_pass_step):
    """The search kernel on the FP32 VALU roofline.  achieved = FP32 ops the launch executed (device
    work counters of an untimed step, see executed_ops) / the average launch duration of the timed
    steps (HIP events on the launch stream); peak = the VALU ceiling of that op mix."""
    D = wl.dim
    DT, DX = 1 + wl.d_y + wl.cond_source, wl.d_x
    avg_s = k_ms / k_n / 1e3
    w = [v / work_launches for v in w]
    sub, mx, cmp = executed_ops(DT, DX, w)
    ops = sub + mx + cmp
    method_ops = pairs_per_pass_step * ops_per_pair(D)
    achieved = ops / avg_s / 1e12
    method_tops = method_ops / avg_s / 1e12
    ceil = valu_ceiling(sub, mx, cmp)
    return dict(
        bound="alu", achieved=round(achieved, 3), peak=round(ceil, 3), unit="TFLOP/s",
        frac=round(achieved / ceil, 4), traffic=kernel_traffic(wname),
        peak_derivation="78.64e12 FP32 lane-instr/s (256 CU x 4 SIMD x 32 lanes x 2.4 GHz) x executed ops per "
                        "instruction of their fewest-instruction form (%.3g sub + %.3g max + %.3g cmp per launch; "
                        "sub and cmp one op per instruction, two maxes per v_max3; no packed FP32)" % (sub, mx, cmp),
        kernel="search_%s<%d,%d,k=%d,slots=%d,sorted>" % (set_kernel_name(DT - 1, DX) if w[2] < w[0] else "kernel",
                                                           DT - 1, DX, wl.k, slots),
        kernel_src=kernel_sha(), avg_launch_ms=round(avg_s * 1e3, 4), launches=k_n,
        pairs_evaluated_per_launch=[int(w[0]), int(w[1])], shared_pairs_per_launch=[int(w[2]), int(w[3])],
        ops_per_launch=int(ops), method_pairs_per_launch=int(pairs_per_pass_step),
        method_equivalent_tops=round(method_tops, 3),
        frac_method_equivalent=round(method_tops / ceil, 4),
        frac_of_headline_157_3=round(achieved / PEAK_FP32_HEADLINE, 4),
        method_frac_of_headline_157_3=round(method_tops / PEAK_FP32_HEADLINE, 4))


def batched_record(args, wl, wname):
    import torch
    import paper_1401_4068_amd as te

    D = wl.dim
    n = wl.chunk_sizes()
    pairs_per_pass = int(wl.directed_pairs())                 # Σ over all chunks of N(N-1)
    x = torch.from_numpy(wl.x).cuda()
    y = torch.from_numpy(wl.y).cuda()
    S = wl.n_surrogates
    G = wl.n_pairs * wl.n_points
    # surrogate permutations: drawn by the library from the plan's seed inside every step (the
    # default), or the input module's copy of the same permutations uploaded once (--given-perms)
    host_perms = torch.from_numpy(wl.perms).cuda() if S else None
    perms = host_perms if args.given_perms else None
    plan = te.Plan.from_workload(wl)
    full, minimum, plain_bytes = plan.workspace_bytes()
    ws = plan.workspace()
    if S:
        assert torch.equal(plan.permutations(), host_perms), "drawn permutations differ from the input module's"
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

    dev_out = torch.empty(G * (S + 1) + G, dtype=torch.float64, device="cuda")

    def step_async():
        # the same hot path queued on the stream: results stay in HBM, no host round trip
        return plan.surrogates_async(x, y, perms, ws=ws, stream=stream, out=dev_out)

    for _ in range(args.warmup):
        step_async() if pipelined else step()
    # timed steps: HIP events around every search launch, no work counters
    te.profile_enable(True)
    te.profile_read(reset=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        if pipelined:
            step_async()
        else:
            out = step()
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    k_ms, k_n = te.profile_read(reset=True)
    te.profile_enable(False)
    print("timed %d steps: %.4f s per step" % (args.steps, dt / args.steps), file=sys.stderr, flush=True)
    # one untimed step with the device counters of evaluated pairs
    te.profile_enable(False, work=True)
    te.profile_work_all(reset=True)
    step_async() if pipelined else step()
    work = te.profile_work_all(reset=True)
    te.profile_enable(False)
    # results of the last queued step against a synchronous call with the input module's
    # permutations (bit for bit), and the latency of synchronous calls (a step and its host round trip)
    ref = plan.surrogates(x, y, host_perms, ws=ws)
    if pipelined:
        got = dev_out.cpu().numpy()
        est_dev = got[:G * (S + 1)].reshape(wl.n_pairs, wl.n_points, S + 1)
        assert np.array_equal(est_dev[..., 0], ref[0]), "queued and synchronous calls disagree"
        if S:
            assert np.array_equal(est_dev[..., 1:], ref[1]), "queued and synchronous calls disagree"
            assert np.array_equal(got[G * (S + 1):].reshape(wl.n_pairs, wl.n_points), ref[2])
    else:
        for u, v in zip(out, ref):
            assert np.array_equal(u, v, equal_nan=True), "drawn and given permutations disagree"
    lat = []
    for _ in range(args.latency_calls):
        s0 = time.perf_counter()
        step()
        lat.append(time.perf_counter() - s0)
    est = wl.n_estimates()
    value = est * args.steps / dt
    evals_per_s = 2 * pairs_per_pass * args.steps / dt
    env_slots = os.environ.get("TE_SLOTS", "")
    slots = tuned["slots"] if tuned else (int(env_slots) if env_slots.isdigit() else 4)
    roof = None
    if k_n > 0:
        roof = roofline_record(wl, wname, k_ms, k_n, work, 1, slots, pairs_per_pass * args.steps / k_n)

    # plain per-time-point paths on the same work
    plain_rec = None
    if args.plain_steps > 0:
        plain_rec = {}
        ws_min = torch.empty(minimum, dtype=torch.uint8, device="cuda")
        if S:
            run_pt = lambda: plan.surrogates(x, y, perms, ws=ws_min)                 # noqa: E731
            run_pt()
            torch.cuda.synchronize()
            p0 = time.perf_counter()
            for _ in range(args.plain_steps):
                r = run_pt()
            torch.cuda.synchronize()
            pdt = time.perf_counter() - p0
            for u, v in zip(r, ref):
                assert np.array_equal(u, v, equal_nan=True), "per-time-point and batched paths disagree"
            plain_rec["per_time_point"] = dict(
                value=round(est * args.plain_steps / pdt, 2), unit="estimates/s",
                ms_per_step=round(pdt / args.plain_steps * 1e3, 3),
                path="te_surrogates with the minimum workspace: one time point (its S+1 chunks) per launch")
        # te_estimate: one chunk per launch sequence (sort, embed, search, reduce), originals; every
        # chunk of a time point costs the same, so its rate per estimate stands for the surrogates too
        plan.estimate(x, y, ws=ws)
        torch.cuda.synchronize()
        p0 = time.perf_counter()
        for _ in range(args.plain_steps):
            r0 = plan.estimate(x, y, ws=ws)
        torch.cuda.synchronize()
        pdt = time.perf_counter() - p0
        assert np.array_equal(r0, ref[0]), "plain and batched paths disagree"
        plain_rec["per_chunk"] = dict(
            value=round(G * args.plain_steps / pdt, 2), unit="estimates/s",
            ms_per_step=round(pdt / args.plain_steps * 1e3, 3),
            path="te_estimate, one chunk at a time (the %d originals; same chunk sizes as the surrogates)" % G)
        if S == 0:
            plain_rec["value"] = plain_rec["per_chunk"]["value"]
        else:
            plain_rec["value"] = plain_rec["per_time_point"]["value"]

    rec = dict(
        metric=METRIC, value=round(value, 2), unit="estimates/s", n_gpus=1, steps=args.steps,
        warmup=args.warmup, ms_per_step=round(dt / args.steps * 1e3, 4), higher_is_better=True,
        scaling="weak", vs_baseline=None, dtype="f32", data="synthetic",
        config=dict(workload=wname, pairs=wl.n_pairs, trials=wl.n_trials, samples=wl.n_samples,
                    windows=wl.n_points, points_per_window_min=int(n.min()), points_per_window_max=int(n.max()),
                    d_y=wl.d_y, d_x=wl.d_x, tau=wl.tau, u=wl.u, dim=D, k=wl.k, surrogates=S,
                    permutations=("given (uploaded once)" if args.given_perms else
                                  "drawn on the device from the plan's seed in every step") if S else None,
                    estimates_per_step=est, workspace_bytes=int(full),
                    path=("batched (te_surrogates_async: one persistent search launch per step, steps queued "
                          "back to back, results left in HBM)" if pipelined else
                          "batched (te_surrogates, one persistent search launch)" + (", hipGraph" if args.graph
                                                                                    else ""))),
        distance_evals_per_s=round(evals_per_s, 1),
        pct_fp32_valu_peak=None if roof is None else round(100 * roof["frac"], 2),
        latency_s=dict(p50=float(np.percentile(lat, 50)), p99=float(np.percentile(lat, 99)),
                       calls=len(lat)) if lat else None,
        plain=plain_rec,
        tuned_shape=tuned,
        roofline=roof,
    )
    if pipelined and not args.no_two_stream and wname != WORKLOADS["uneven"]:
        rec["pipelined_two_streams"] = two_stream_record(plan, wl, x, y, perms, ws, dev_out, args.steps)
    if not args.no_cpu:
        rec["cpu_baseline"] = cpu_baseline(wl, plan_c3=(wname == WORKLOADS["uneven"]))
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
    # one untimed step with the device counters of evaluated pairs (two launches)
    te.profile_enable(False, work=True)
    te.profile_work_all(reset=True)
    step()
    work = te.profile_work_all(reset=True)
    te.profile_enable(False)
    roof = None
    if k_n > 0:
        # two search launches per step (all delays; the chosen delay's test): their mean
        roof = roofline_record(wl, "ar_scan", k_ms, k_n, work, 2, tuned["slots"] if tuned else 4,
                               pairs_per_step / 2)
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
    threads = host_info()["threads"]
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
    """The served mix: Poisson-arriving single-time-point jobs of mixed shapes through the
    continuous-batching server (te_serve_*), and the same trace replayed in real time, one job
    at a time in arrival order, through the batched path (te_surrogates) and through the plain
    per-chunk path (te_estimate_each).  Every job's permutations are drawn on the device from its
    seed.  Latency = arrival (submission) -> result; estimates/s = the trace's estimates / the
    span from the first arrival to the last result."""
    import threading

    import torch
    import paper_1401_4068_amd as te
    import synth

    def progress(*a):
        print(*a, file=sys.stderr, flush=True)

    trace = synth.served_jobs(n_jobs=args.jobs, rate=args.served_rate, seed_offset=args.served_seed)
    progress("trace: %d jobs at %.3f/s" % (len(trace), args.served_rate))
    wls = [synth.job_workload(j, with_perms=False) for j in trace]
    est = sum(1 + j["S"] for j in trace)
    pairs = sum((1 + j["S"]) * (j["R"] * j["W"]) * (j["R"] * j["W"] - 1) for j in trace)
    offered_pairs_per_s = pairs / max(trace[-1]["t"], 1e-9)

    # warm-up: module load and the first launches of every kernel class
    warm_srv = te.Server(arena_bytes=256 << 20, max_slots=4)
    for d in (2, 3, 4):
        warm = synth.job_workload(dict(id=-d, t=0.0, d=d, W=10, R=30, S=2, seed=d), with_perms=False)
        warm_srv.wait(warm_srv.submit(warm, draw_perms=True), timeout_s=120)
        p = te.Plan.from_workload(warm)
        xw, yw = torch.from_numpy(warm.x).cuda(), torch.from_numpy(warm.y).cuda()
        p.surrogates(xw, yw)
        p.estimate_each(xw, yw)
        p.close()
    warm_srv.close()

    # served: a submitter thread replays the arrival times
    srv = te.Server(arena_bytes=args.arena_gb << 30, max_slots=args.slots, step_pairs=args.step_pairs)
    tickets = [None] * len(trace)
    t_sub = [0.0] * len(trace)
    t0 = time.perf_counter() + 0.05

    def submitter():
        for i, (j, wl) in enumerate(zip(trace, wls)):
            d = t0 + j["t"] - time.perf_counter()
            if d > 0:
                time.sleep(d)
            t_sub[i] = time.perf_counter()
            tickets[i] = srv.submit(wl, draw_perms=True)

    th = threading.Thread(target=submitter)
    th.start()
    th.join()
    served_te = []
    for i in range(len(trace)):
        served_te.append(srv.wait(tickets[i], timeout_s=3600)[0][0, 0])
        if i % 200 == 199:
            progress("served: %d jobs done" % (i + 1))
    t_end = time.perf_counter()
    st = srv.stats()
    srv.close()
    served = dict(p50_s=st["p50_s"], p99_s=st["p99_s"], est_per_s=est / (t_end - t0),
                  span_s=t_end - t0, steps=st["steps"], peak_slots=st["peak_slots"],
                  peak_arena_bytes=st["peak_bytes"])
    progress("served: %.1f s, %.1f estimates/s" % (served["span_s"], served["est_per_s"]))

    def replay(label, run):
        """Real-time replay, one job at a time in arrival order: a job starts at its arrival or
        when the previous one is done; its service is plan, upload and the call."""
        lat = []
        r0 = time.perf_counter()
        for i, (j, wl) in enumerate(zip(trace, wls)):
            d = r0 + j["t"] - time.perf_counter()
            if d > 0:
                time.sleep(d)
            plan = te.Plan.from_workload(wl)
            x = torch.from_numpy(wl.x).cuda()
            y = torch.from_numpy(wl.y).cuda()
            out = run(plan, x, y)
            lat.append(time.perf_counter() - (r0 + j["t"]))
            assert out[0][0, 0] == served_te[i], "%s and served estimates differ (job %d)" % (label, i)
            plan.close()
            if i % 200 == 199:
                progress("%s: %d jobs done" % (label, i + 1))
        span = time.perf_counter() - r0
        progress("%s: %.1f s" % (label, span))
        return dict(p50_s=float(np.percentile(lat, 50)), p99_s=float(np.percentile(lat, 99)),
                    est_per_s=est / span, span_s=span)

    fifo = replay("fifo", lambda plan, x, y: plan.surrogates(x, y))
    plain = replay("plain", lambda plan, x, y: plan.estimate_each(x, y)) if not args.no_plain_replay else None
    capacity_jobs_per_s = len(trace) / served["span_s"]
    rec = dict(metric=METRIC, value=round(served["est_per_s"], 2), unit="estimates/s", n_gpus=1,
               steps=1, warmup=1, ms_per_step=round(served["span_s"] * 1e3, 1), higher_is_better=True,
               scaling="weak", vs_baseline=None, dtype="f32", data="synthetic",
               config=dict(workload="served_mix", arrivals="poisson", rate_per_s=args.served_rate,
                           trace_seed_offset=args.served_seed, jobs=len(trace), dims=[5, 7, 9],
                           points_per_job="log-uniform 1000..100000", surrogates="0..500", k=4,
                           estimates=est, directed_pairs_per_pass=int(pairs),
                           offered_pairs_per_s=offered_pairs_per_s, arena_gb=args.arena_gb,
                           max_slots=args.slots, step_pairs=args.step_pairs,
                           permutations="drawn on the device from each job's seed"),
               latency_s=dict(p50=served["p50_s"], p99=served["p99_s"]),
               served=served, fifo_batched=fifo, plain_per_chunk=plain,
               served_capacity_jobs_per_s=capacity_jobs_per_s,
               rate_for_0_8_capacity=0.8 * capacity_jobs_per_s)
    return rec


def ragwitz_record(args):
    """Choice of the target embedding by the local-predictor score (te_ragwitz) on one
    window of AR scenario 1's target (50 trials x 300 samples: N = 15 000 pooled points),
    candidates d = 1..6 x tau = 1..2, k = 4.  One step scores every candidate."""
    import torch
    import synth
    import paper_1401_4068_amd as te

    wl = synth.ar_scenarios(1)
    y = torch.from_numpy(np.ascontiguousarray(wl.y[0])).cuda()
    w, W, k = int(wl.window_start[0]), int(wl.window_len[0]), 4
    cands = [(d, tau) for tau in (1, 2) for d in range(1, 7)]
    R = int(y.shape[0])
    N = R * W
    dims = np.array([d for d, _ in cands], np.int32)
    import ctypes
    need = ctypes.c_size_t()
    te._lib.check(te.lib().te_ragwitz_workspace_bytes(R, W, dims.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)),
                                                      len(cands), ctypes.byref(need)))
    ws = torch.empty(need.value, dtype=torch.uint8, device="cuda")
    for _ in range(args.warmup):
        te.ragwitz(y, w, W, cands, k, ws=ws)
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    ev0.record()
    for _ in range(args.steps):
        scores, _ = te.ragwitz(y, w, W, cands, k, ws=ws)
    ev1.record()
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    dev_ms = ev0.elapsed_time(ev1) / args.steps
    # executed FP32 operations: per (reference, candidate point) pair d subtractions, d - 1
    # maxes and one min or compare (abs is an operand modifier)
    ops = sum(2 * d for d, _ in cands) * float(N) * float(N)
    achieved = ops / (dev_ms * 1e-3) / 1e12
    peak = FP32_LANE_INSTR_PER_S / 1e12
    best = int(np.argmin(scores))
    rec = dict(
        metric="embedding candidates scored/s (local-predictor error, k nearest of all pooled points)",
        value=round(len(cands) * args.steps / dt, 2), unit="candidates/s", n_gpus=1, steps=args.steps,
        warmup=args.warmup, ms_per_step=round(dt / args.steps * 1e3, 4), higher_is_better=True, scaling="weak",
        vs_baseline=None, dtype="f32", data="synthetic",
        config=dict(workload="ragwitz_ar_scenario1_window", trials=R, window=[w, w + W], points=N,
                    candidates=[list(c) for c in cands], k=k, workspace_bytes=int(need.value),
                    path="te_ragwitz (synchronous)"),
        distance_evals_per_s=round(len(cands) * N * (N - 1) * args.steps / dt, 1),
        roofline=dict(bound="alu", achieved=round(achieved, 3), peak=round(peak, 3), unit="TFLOP/s",
                      frac=round(achieved / peak, 4), traffic=None,
                      peak_derivation="78.64e12 FP32 lane-instr/s (256 CU x 4 SIMD x 32 lanes x 2.4 GHz), one "
                                      "executed op per instruction",
                      kernel="rag_knn_kernel<d> (+ embed, score)", device_ms_per_step=round(dev_ms, 4),
                      ops_per_step=ops),
        findings=dict(scores=[round(float(v), 6) for v in scores], chosen=list(cands[best])))
    if not args.no_cpu:
        from oracle import ragwitz as rg
        from synth.rng import derive_key, permutation
        yh = np.ascontiguousarray(wl.y[0])
        done, t_cpu = 0, 0.0
        order = permutation(derive_key(4069, N), N)
        prep = {}
        while t_cpu < 10.0 and done < N:
            idx = order[done:done + 25]
            t1 = time.perf_counter()
            for d, tau in cands:
                if (d, tau) not in prep:
                    prep[(d, tau)] = rg.states(yh, d, tau, w, W)
                S, tgt = prep[(d, tau)]
                rg.predictions_points(S, tgt, k, idx)
            t_cpu += time.perf_counter() - t1
            done += len(idx)
        rec["cpu_baseline"] = dict(value=len(cands) * done / N / t_cpu, unit="candidates/s", cores=1, kind="oracle",
                                   sample="%d of %d points' predictions for each of the %d candidates (numpy, one "
                                          "thread), %.1f s; scaled by points" % (done, N, len(cands), t_cpu))
    return rec


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="uneven",
                    choices=["uneven", "nonlinear", "linear", "meg", "served", "ar0", "ar1", "ar2", "ar3",
                             "ragwitz"],
                    help="uneven: batched surrogates (60 time points x 201 chunks of 1 000-49 400 points); "
                         "ar0: delay recovery against the amount of data; ar1-ar3: the AR coupling scenarios")
    ap.add_argument("--no-cpu", action="store_true", help="skip the oracle CPU baseline")
    ap.add_argument("--plain-steps", type=int, default=1)
    ap.add_argument("--latency-calls", type=int, default=3, help="synchronous calls timed for latency_s")
    ap.add_argument("--given-perms", action="store_true",
                    help="pass the input module's permutations instead of drawing them in the library")
    ap.add_argument("--graph", action="store_true", help="replay the batched step as a hipGraph")
    ap.add_argument("--no-two-stream", action="store_true",
                    help="skip the two-stream pipelined measurement (profiled runs: its launches overlap)")
    ap.add_argument("--sync", action="store_true",
                    help="time synchronous te_surrogates calls (a host round trip per step) instead of queued steps")
    ap.add_argument("--no-tune", action="store_true", help="skip the launch-shape autotuner")
    ap.add_argument("--jobs", type=int, default=2000, help="served workload: jobs per trace")
    ap.add_argument("--served-rate", type=float, default=200.0, help="served workload: Poisson arrivals per second")
    ap.add_argument("--served-seed", type=int, default=0, help="served workload: trace seed offset")
    ap.add_argument("--no-plain-replay", action="store_true", help="served workload: skip the plain-path replay")
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
    elif args.workload == "ragwitz":
        rec = ragwitz_record(args)
    elif args.workload.startswith("ar"):
        rec = scan_record(args, int(args.workload[2:]))
    else:
        wl, wname = make_workload(args.workload)
        rec = batched_record(args, wl, wname)
    print(json.dumps(rec), flush=True)


if __name__ == "__main__":
    main()
