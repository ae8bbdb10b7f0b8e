#!/usr/bin/env python3
"""Benchmark: ensemble transfer-entropy estimates per second on one MI355X.

Workload (the plain GPU ensemble configuration): nonlinear coupled AR pair,
500 trials x 300 samples; 100 analysis windows of 10 samples, each pooling all
trials (N = 5000 points), d_y = d_x = 3, tau = 1, u = 3 (joint dimension 7),
k = 4, float32 data, no surrogates.  One step = the whole hot path (embed,
k-NN radius search, three range counts, digamma sums) for all 100 windows,
i.e. 100 TE estimates, with the series already resident in HBM.

The step runs through te_surrogates (batched: one persistent search launch);
the plain per-window path (te_estimate) is timed beside it.  The JSON line adds
the search kernel's roofline (FP32 VALU, measured with HIP events around each
launch) and the CPU oracle timed on the host cores on a bounded sample.
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
RECORDED_TRAFFIC = {"04d073ef47f2": 151226.875 * 1024 * 2.0 + 564.125 * 1024 * 1.0}
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
    """Oracle TE for as many windows as fit in about budget_s seconds on the host cores."""
    from oracle import oracle
    threads = host_threads()
    jobs, _ = oracle.workload_jobs(wl)
    done = 0
    t_total = 0.0
    batch = threads
    while done < len(jobs) and t_total < budget_s:
        sel = jobs[done:done + batch]
        t0 = time.perf_counter()
        oracle.te_jobs(wl.x, wl.y, wl.d_y, wl.d_x, wl.tau, wl.u, wl.k, sel, wl.perms, n_threads=threads)
        t_total += time.perf_counter() - t0
        done += len(sel)
    return dict(value=done / t_total, unit="estimates/s", cores=threads, kind="oracle",
                sample="%d of %d windows (N = %d each), %.1f s wall on %d threads"
                % (done, len(jobs), int(wl.chunk_sizes()[0]), t_total, threads))


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--no-cpu", action="store_true", help="skip the oracle CPU baseline")
    ap.add_argument("--plain-steps", type=int, default=3)
    ap.add_argument("--graph", action="store_true", help="replay the batched step as a hipGraph")
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
    import paper_1401_4068_amd as te
    import synth

    torch.cuda.set_device(0)
    wl = synth.nonlinear_ensemble()
    D = wl.dim
    n = wl.chunk_sizes()
    pairs_per_pass = int(np.sum(n * (n - 1)))                 # directed pairs, one pass
    x = torch.from_numpy(wl.x).cuda()
    y = torch.from_numpy(wl.y).cuda()
    plan = te.Plan.from_workload(wl)
    ws = plan.workspace()
    stream = torch.cuda.Stream() if args.graph else torch.cuda.current_stream()

    def step():
        return plan.surrogates(x, y, ws=ws, stream=stream, use_graph=args.graph)

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
    te.profile_enable(False)
    est = wl.n_estimates()
    value = est * args.steps / dt
    evals_per_s = 2 * pairs_per_pass * args.steps / dt

    # dominant kernel: the persistent search launch (one per step)
    roof = None
    if k_n > 0:
        avg_s = k_ms / k_n / 1e3
        ops = pairs_per_pass * ops_per_pair(D)
        achieved = ops / avg_s / 1e12
        roof = dict(bound="alu", achieved=round(achieved, 3), peak=PEAK_FP32_OPS, unit="TFLOP/s",
                    frac=round(achieved / PEAK_FP32_OPS, 4), traffic=kernel_traffic(),
                    kernel="search_kernel<3,3,k=4,slots=8>", avg_launch_ms=round(avg_s * 1e3, 4),
                    launches=k_n, ops_per_launch=ops,
                    frac_of_headline_157_3=round(achieved / PEAK_FP32_HEADLINE, 4))

    # plain per-window path on the same workload
    plain_rec = None
    if args.plain_steps > 0:
        plan.estimate(x, y, ws=ws)
        torch.cuda.synchronize()
        p0 = time.perf_counter()
        for _ in range(args.plain_steps):
            plain = plan.estimate(x, y, ws=ws)
        torch.cuda.synchronize()
        pdt = time.perf_counter() - p0
        assert np.array_equal(plain, out[0]), "plain and batched paths disagree"
        plain_rec = dict(value=round(est * args.plain_steps / pdt, 2), unit="estimates/s",
                         ms_per_step=round(pdt / args.plain_steps * 1e3, 3), path="te_estimate, one window at a time")

    rec = dict(
        metric=METRIC, value=round(value, 2), unit="estimates/s", n_gpus=1, steps=args.steps,
        warmup=args.warmup, ms_per_step=round(dt / args.steps * 1e3, 4), higher_is_better=True,
        scaling="weak", vs_baseline=None, dtype="f32", data="synthetic",
        config=dict(workload="nonlinear_ar_ensemble", trials=wl.n_trials, samples=wl.n_samples,
                    windows=wl.n_points, window_len=int(wl.window_len[0]), points_per_window=int(n[0]),
                    d_y=wl.d_y, d_x=wl.d_x, tau=wl.tau, u=wl.u, dim=D, k=wl.k, surrogates=0,
                    path="batched (te_surrogates, one persistent search launch)" + (", hipGraph" if args.graph else "")),
        distance_evals_per_s=round(evals_per_s, 1),
        pct_fp32_valu_peak=None if roof is None else round(100 * roof["frac"], 2),
        latency_s=dict(p50=float(np.percentile(lat, 50)), p99=float(np.percentile(lat, 99))),
        plain=plain_rec,
        roofline=roof,
    )
    if not args.no_cpu:
        rec["cpu_baseline"] = cpu_baseline(wl)
    print(json.dumps(rec), flush=True)


if __name__ == "__main__":
    main()
