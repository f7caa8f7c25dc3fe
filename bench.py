"""Throughput benchmark of the HIP LQT solver on one MI355X.

Headline workload (``value``): one long tracking instance, n = 4 states,
m = 2 controls, T = 1,000,000 steps, FP64 (sinusoid-reference generator:
F = I + 0.1 G rescaled to spectral radius 0.99, X = 10 I, U = 0.1 I,
X_T = 10 I).  One "step" of this benchmark is one full solve: element build,
reverse scan, gain extraction, forward trajectory scan; every output family
(S, v, K, d, x, u) is written to device memory.  Inputs are resident in HBM
before the timed region.  ``value`` = time steps solved per second
(T x solves / elapsed) over the timed region, in which only the dominant
kernel is bracketed by HIP events (its average duration gives ``roofline``).

Secondary results in the same JSON line (``--workload all``, the default):
the same instance with float results (MIXED), the uneven batch of 4096
instances (MIXED), and the serving run with Poisson arrivals (p50/p99
latency, served steps/s).  ``cpu_baseline`` times the FP64 CPU oracle on
the host.
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

HBM_PEAK_GBS = 8000.0        # MI355X HBM3E, GB/s
FP64_PEAK_TFLOPS = 78.6      # MI355X FP64 vector and FP64 matrix (dense)
FP32_PEAK_TFLOPS = 157.3     # MI355X FP32 vector and FP32 matrix (dense)

# Measured HBM traffic per launch of the dominant kernel (rocprofv3 --pmc
# FETCH_SIZE, then WRITE_SIZE, on `bench.py --workload single`), scaled by the
# plain-copy calibration (`bench.py --workload copy`: FETCH_SIZE x 2.0,
# WRITE_SIZE x 1.0).  Reported only while the kernel sources hash to the
# version the counters were taken on.
TRAFFIC_SOURCES = ("lqt_small.hip", "lqt_lane.hpp", "lqt_ops.hpp", "lqt_regmath.hpp")
TRAFFIC = {
    ("bwd_final", "fp64", 1_000_000): {
        "bytes_per_launch": 310_378_720,
        "fetch_kib": 26487.2, "write_kib": 250129.8, "fetch_scale": 2.0, "write_scale": 1.0,
        "src_sha256": "41c9c1b31124fb8f344f38941f461f844bf0ab5fad57ae237c6977be31bbdd0f",
    },
}


def sources_sha256():
    import hashlib

    h = hashlib.sha256()
    for f in TRAFFIC_SOURCES:
        with open(os.path.join(ROOT, "paper_2104_03186_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def measured_traffic(kernel, prec, T):
    rec = TRAFFIC.get((kernel, prec, T))
    if rec is None or rec["src_sha256"] != sources_sha256():
        return None
    return rec["bytes_per_launch"]


def algorithmic_bytes_per_step(n, m, p, osz=8):
    """Bytes a step must move by the path's contract: reference r_k read once
    (FP64); S_k, v_k, K_k, d_k, x_k, u_k written once (osz bytes each: 8 for
    FP64 results, 4 for MIXED)."""
    return 8 * p + osz * (n * n + n + m * n + m + n + m)


def stage_bytes_per_step(stage, n, m, p, osz=8):
    """Algorithmic bytes of one kernel's own contract, per step."""
    if stage == "bwd_final":   # reads r_k, writes S_k, v_k, K_k, d_k
        return 8 * p + osz * (n * n + n + m * n + m)
    if stage == "fwd_final":   # reads K_k, d_k, writes x_k, u_k
        return osz * (m * n + m + n + m)
    if stage in ("bwd_reduce", "prep_varying", "m2_reduce"):   # reads r_k
        return 8 * p
    if stage == "m2_final":    # reads r_k, S_k, v_k, K_k, d_k, writes x_k, u_k
        return 8 * p + osz * (n * n + n + m * n + m + n + m)
    if stage == "gen_transform":  # reads r_k, s_k, writes c~_k
        return 8 * (p + m + n)
    if stage == "gen_post":    # reads r_k, s_k, x_k; updates K_k, d_k, u_k in place
        return 8 * (p + m) + osz * (n + 2 * (m * n + m + m))
    return 0


def path_flops_per_step(n, m):
    """Algorithmic flops per step of the parallel path: two applications of
    the LQT combination rule per element (work-efficient scan), the gain
    extraction and two affine-map compositions."""
    comb = (56.0 / 3.0) * n ** 3 + 14 * n ** 2
    extract = 6 * n * n * m + 4 * n * m * m + m ** 3 / 3.0 + 4 * n * n
    aff = 2 * n ** 3 + 2 * n ** 2
    return 2 * comb + extract + 2 * aff


def rel(a, b):
    """Relative error over all steps stacked and, where it is larger, per step
    (the largest step error against max(step size, RMS step size)); the
    parity measure of the GPU tests."""
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    nb = float(np.linalg.norm(b))
    stacked = float(np.linalg.norm(a - b) / nb) if nb > 0 else float(np.linalg.norm(a))
    if a.ndim == 0 or a.shape[0] == 0:
        return stacked
    d = np.linalg.norm((a - b).reshape(a.shape[0], -1), axis=1)
    ns = np.linalg.norm(b.reshape(b.shape[0], -1), axis=1)
    rms = float(np.sqrt(np.mean(ns ** 2)))
    step = float(np.max(d)) if rms == 0.0 else float(np.max(d / np.maximum(ns, rms)))
    return max(stacked, step)


def host_cpu():
    """CPU model and logical CPU count of the host the oracle runs on."""
    model = "unknown"
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    return f"{model}; {os.cpu_count()} logical CPUs visible"


def note(msg):
    """A progress line on stderr (the JSON result stays alone on stdout)."""
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def timing_stats(ms_list):
    a = np.asarray(ms_list, dtype=np.float64)
    return {"mean": round(float(a.mean()), 4), "median": round(float(np.median(a)), 4),
            "p99": round(float(np.percentile(a, 99)), 4), "min": round(float(a.min()), 4), "runs": int(a.size)}


def timed_solves(torch, stream, fn, runs):
    """Per-solve device times (ms) of `runs` calls of fn, each bracketed by
    events on the solve stream."""
    evs = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(runs)]
    for a, b in evs:
        a.record(stream)
        fn()
        b.record(stream)
    torch.cuda.synchronize()
    return [a.elapsed_time(b) for a, b in evs]


def run_single(args, api, inputs, torch, prec, steps, warmup, with_cpu, trajectory="maps", cost="standard"):
    """One instance n=4, m=2, T=args.T.  Returns the result dict.  trajectory:
    the forward pass (closed-loop maps, or forward prefixes of the elements).
    cost: "standard" (the tracking workload), or "generalised" (a random
    instance with the cross term M and control reference s of Section IV-D,
    four tracked outputs)."""
    n, m, T = 4, 2, args.T
    if cost == "generalised":
        prob = inputs.generalised_problem(n, m, T, seed=1, p=4)
    else:
        prob = inputs.tracking_problem(n=n, m=m, T=T, workload=1)
    osz = 8 if prec == "fp64" else 4
    plan = api.Plan(n, m, prec=prec, device=0, max_steps=T, trajectory=trajectory)
    dp = api.DeviceProblem(prob)
    do = api.DeviceOutputs(n, m, T, dtype=torch.float64 if osz == 8 else torch.float32)
    stream = torch.cuda.current_stream(0)
    for _ in range(warmup):
        plan.solve([dp], [do], stream)
    torch.cuda.synchronize()
    status = int(do.status.item())
    rel_err = None
    if not args.no_parity:
        import oracle

        ref = oracle.solve(prob)
        got = do.host()
        rel_err = {f: rel(got[f], ref[f]) for f in api.FAMILIES}

    # Pass 1 (short): every kernel bracketed by events, to find the dominant one.
    plan.profile(True)
    plan.profile_read()
    for _ in range(max(3, steps // 10)):
        plan.solve([dp], [do], stream)
    stages_all = plan.profile_read()
    dom_name = max(stages_all.items(), key=lambda kv: kv[1][1] / max(kv[1][0], 1))[0]

    # Timed region: K solves; only the dominant kernel is bracketed by events.
    plan.profile_select(dom_name)
    plan.profile_read()
    torch.cuda.synchronize()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    t0 = time.perf_counter()
    e0.record(stream)
    for _ in range(steps):
        plan.solve([dp], [do], stream)
    e1.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    ms_total = e0.elapsed_time(e1)
    dom_launches, dom_ms = plan.profile_read()[dom_name]
    plan.profile(False)
    plan.profile_select(None)
    per_solve = timing_stats(timed_solves(torch, stream, lambda: plan.solve([dp], [do], stream), 10))
    alt = None
    if T <= 16384:  # the default route here is the batched lane kernel; the lane pipeline beside it
        plan.set_routing(path="small")
        for _ in range(3):
            plan.solve([dp], [do], stream)
        alt = timing_stats(timed_solves(torch, stream, lambda: plan.solve([dp], [do], stream), 10))
        plan.set_routing()
    plan.close()

    ms_per_step = ms_total / steps
    value = T * steps / (ms_total / 1e3)
    dom_avg_s = dom_ms / dom_launches / 1e3
    dom_bytes = stage_bytes_per_step(dom_name, n, m, prob.p, osz) * T
    achieved = dom_bytes / dom_avg_s / 1e9
    roofline = {"kernel": dom_name, "bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS,
                "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4),
                "traffic": measured_traffic(dom_name, prec, T),
                "avg_us": round(dom_avg_s * 1e6, 2), "launches": dom_launches,
                "algorithmic_bytes_per_launch": dom_bytes}
    bytes_step = algorithmic_bytes_per_step(n, m, prob.p, osz)
    flops_step = path_flops_per_step(n, m)
    t_bound = max(bytes_step * T / (HBM_PEAK_GBS * 1e9), flops_step * T / (FP64_PEAK_TFLOPS * 1e12))
    path = {"t_bound_us": round(t_bound * 1e6, 2), "t_measured_us": round(ms_per_step * 1e3, 2),
            "frac": round(t_bound / (ms_per_step / 1e3), 4), "bytes_per_step": bytes_step,
            "flops_per_step": round(flops_step, 1)}
    cpu = None
    if with_cpu:
        import oracle

        sps, secs, reps = oracle.time_solve([prob], min_seconds=args.cpu_seconds)
        cpu = {"value": round(sps, 1), "unit": "steps/s", "cores": 1, "kind": "oracle", "host": host_cpu(),
               "sample": f"{reps} full sequential FP64 solve(s) of the same T={T} instance ({secs:.1f} s)"}
    return {"value": value, "ms_per_step": ms_per_step, "ms_per_solve_stats": per_solve,
            "lane_pipeline_ms_per_solve_stats": alt, "status": status,
            "rel_err": rel_err,
            "stages_avg_ms": {k: round(v[1] / max(v[0], 1), 4) for k, v in stages_all.items()},
            "roofline": roofline, "path_roofline": path, "cpu_baseline": cpu, "wall_s": wall}


def run_batched(args, api, inputs, torch, prec, with_cpu=False):
    """Uneven batch: 4096 instances, T log-uniform on [256, 16384], n in
    {4, 8, 16}, m = n / 2, diagonal costs, random-walk references; one
    lqt_solve call per step (all instances, every output family).  The
    plan's chunk lengths are chosen by lqt_tune on the batch first (outside
    the timed region, as plan creation)."""
    count = args.count
    shapes = inputs.batched_shapes(count)
    probs = [inputs.diag_problem(n, n // 2, T, 2, i) for i, (n, T) in enumerate(shapes)]
    steps_total = sum(p.T for p in probs)
    plan = api.Plan(16, 8, prec=prec, device=0)
    dtype = torch.float64 if prec == "fp64" else torch.float32
    dps = [api.DeviceProblem(p) for p in probs]
    dos = [api.DeviceOutputs(p.n, p.m, p.T, dtype=dtype) for p in probs]
    stream = torch.cuda.current_stream(0)
    tuned = plan.tune(dps, dos, stream) if not args.no_tune else None
    for _ in range(args.batched_warmup):
        plan.solve(dps, dos, stream)
    torch.cuda.synchronize()
    status_bad = sum(int(o.status.item()) != 0 for o in dos)
    rel_err = None
    if not args.no_parity:
        import oracle

        # every size class sampled: 6 instances of each n, spread over the batch
        worst = {}
        for n in (4, 8, 16):
            idx = [i for i, p in enumerate(probs) if p.n == n]
            for i in idx[::max(1, len(idx) // 6)]:
                ref = oracle.solve(probs[i])
                got = dos[i].host()
                w = worst.setdefault(f"n{n}", {f: 0.0 for f in api.FAMILIES})
                for f in api.FAMILIES:
                    w[f] = max(w[f], rel(got[f], ref[f]))
        rel_err = worst
    plan.profile(True)
    plan.profile_read()
    plan.solve(dps, dos, stream)
    stages = plan.profile_read()
    plan.profile(False)
    times = timed_solves(torch, stream, lambda: plan.solve(dps, dos, stream), args.batched_steps)
    # the same batch replayed from a recorded graph (lqt_set_graphs)
    plan.set_graphs(True)
    plan.solve(dps, dos, stream)
    torch.cuda.synchronize()
    st_graph = timing_stats(timed_solves(torch, stream, lambda: plan.solve(dps, dos, stream), args.batched_steps))
    plan.close()
    st = timing_stats(times)
    ms = st["mean"]
    # the paper's work-efficient scan count (as for the single instance), at
    # the FP64 peak: the batch's algorithmic bound
    flops = sum(path_flops_per_step(p.n, p.m) * p.T for p in probs)
    t_bound_ms = flops / (FP64_PEAK_TFLOPS * 1e12) * 1e3
    cpu = None
    if with_cpu:
        import oracle

        sps, secs, used = oracle.time_solve_parallel(probs, oracle.host_threads())
        cpu = {"value": round(sps, 1), "unit": "steps/s", "cores": used, "kind": "oracle", "host": host_cpu(),
               "sample": f"the whole batch ({count} instances, {steps_total} steps) over the host threads "
                         f"({secs:.1f} s)"}
    return {"workload": f"batched {count} uneven instances, n in {{4,8,16}}, m = n/2, T log-uniform "
                        f"[256, 16384], {prec}",
            "steps_per_solve": steps_total, "ms_per_solve": ms, "ms_per_solve_stats": st,
            "algorithmic_tflops": round(flops / (ms / 1e3) / 1e12, 3),
            "algorithmic_fp64_bound_ms": round(t_bound_ms, 2),
            "algorithmic_fp64_peak_frac": round(t_bound_ms / ms, 4),
            "algorithmic_fp64_peak_frac_by_median": round(t_bound_ms / st["median"], 4),
            "value": round(steps_total / (ms / 1e3), 1), "unit": "steps/s", "status_failures": status_bad,
            "graph_replay_ms_per_solve_stats": st_graph,
            "tuned_chunk_divisors": tuned, "cpu_baseline": cpu,
            "rel_err_sampled": rel_err,
            "stage_ms_one_solve": {k: round(v[1], 4) for k, v in stages.items()}}


def dense_flops_per_step(n, m):
    """Algorithmic flops per step of the dense path (as path_flops_per_step)."""
    return path_flops_per_step(n, m)


def run_dense(args, api, inputs, torch, prec, with_cpu=False):
    """Dense batch: 64 instances, n = 64, m = 32, T = 8192, dense SPD costs
    (Q = W W^T + 0.1 I), spectral radius 0.98, random-walk references."""
    probs = [inputs.dense_problem(64, 32, args.dense_T, instance=i) for i in range(args.dense_count)]
    steps_total = sum(p.T for p in probs)
    plan = api.Plan(64, 32, prec=prec, device=0)
    dtype = torch.float64 if prec == "fp64" else torch.float32
    dps = [api.DeviceProblem(p) for p in probs]
    dos = [api.DeviceOutputs(p.n, p.m, p.T, dtype=dtype) for p in probs]
    stream = torch.cuda.current_stream(0)
    for _ in range(args.batched_warmup):
        plan.solve(dps, dos, stream)
    torch.cuda.synchronize()
    status_bad = sum(int(o.status.item()) != 0 for o in dos)
    rel_err = None
    if not args.no_parity:
        import oracle

        worst = {f: 0.0 for f in api.FAMILIES}
        for i in (0, len(probs) - 1):
            ref = oracle.solve(probs[i])
            got = dos[i].host()
            for f in api.FAMILIES:
                worst[f] = max(worst[f], rel(got[f], ref[f]))
        rel_err = worst
    plan.profile(True)
    plan.profile_read()
    plan.solve(dps, dos, stream)
    stages = plan.profile_read()
    plan.profile(False)
    st = timing_stats(timed_solves(torch, stream, lambda: plan.solve(dps, dos, stream), args.batched_steps))
    plan.close()
    ms = st["mean"]
    flops = dense_flops_per_step(64, 32) * steps_total
    tfs = flops / (ms / 1e3) / 1e12
    cpu = None
    if with_cpu:
        import oracle

        th = oracle.host_threads()
        sample = probs[:th]
        sps, secs, used = oracle.time_solve_parallel(sample, th)
        cpu = {"value": round(sps, 1), "unit": "steps/s", "cores": used, "kind": "oracle", "host": host_cpu(),
               "sample": f"{len(sample)} of the {len(probs)} instances (T={args.dense_T}), one per host thread "
                         f"({secs:.1f} s)"}
    return {"workload": f"dense batch {args.dense_count} x (n=64, m=32, T={args.dense_T}), {prec}",
            "steps_per_solve": steps_total, "ms_per_solve": ms, "ms_per_solve_stats": st,
            "value": round(steps_total / (ms / 1e3), 1), "unit": "steps/s", "status_failures": status_bad,
            "rel_err_sampled": rel_err, "algorithmic_tflops": round(tfs, 3),
            "algorithmic_fp64_peak_frac": round(tfs / FP64_PEAK_TFLOPS, 4),
            "algorithmic_fp32_peak_frac": round(tfs / FP32_PEAK_TFLOPS, 4),
            "stage_ms_one_solve": {k: round(v[1], 4) for k, v in stages.items()}, "cpu_baseline": cpu}


def run_nonlinear(args, api, inputs, torch, prec, with_cpu=True):
    """Iterated linearisation (the nonlinear extension of Section IV-D) on the unicycle of the nonlinear
    experiment (Section VI-E): T = args.nl_T steps, args.nl_rounds rounds per
    solve (the experiment: T = 1e5, 10 rounds), synthetic race track.  One
    timed solve = restore the nominal trajectory (device copy) + all rounds.
    The oracle's sequential iteration (the same rounds) is the parity
    reference and, timed, the CPU baseline."""
    T, rounds = args.nl_T, args.nl_rounds
    prob = inputs.unicycle_problem(T, seed=0)
    plan = api.Plan(4, 2, prec=prec, device=0, max_steps=T)
    dt = torch.float64 if prec == "fp64" else torch.float32
    dp = api.DeviceNLProblem(prob)
    x0 = torch.from_numpy(prob.xbar).to("cuda:0", dt).contiguous()
    u0 = torch.from_numpy(prob.ubar).to("cuda:0", dt).contiguous()
    x, u = x0.clone(), u0.clone()
    change = torch.zeros(rounds, dtype=torch.float64, device="cuda:0")
    status = torch.zeros(1, dtype=torch.int32, device="cuda:0")
    stream = torch.cuda.current_stream(0)

    def one():
        x.copy_(x0)
        u.copy_(u0)
        plan.nl_iterate(dp, rounds, x, u, change, status, stream)

    one()
    torch.cuda.synchronize()
    st = int(status.item())
    rel_err, cpu = None, None
    if not args.no_parity or with_cpu:
        from oracle import iterated

        t0 = time.perf_counter()
        rx, ru, rch = iterated.iterate(prob, rounds)
        secs = time.perf_counter() - t0
        if not args.no_parity:
            rel_err = {"x": rel(x.double().cpu().numpy(), rx), "u": rel(u.double().cpu().numpy(), ru),
                       "last_change_gpu": float(change[-1].item()), "last_change_oracle": rch[-1]}
        if with_cpu:
            cpu = {"value": round(T * rounds / secs, 1), "unit": "steps*rounds/s", "cores": 1, "kind": "oracle", "host": host_cpu(),
                   "sample": f"one full sequential FP64 iteration ({rounds} rounds, T={T}; {secs:.1f} s)"}
    plan.profile(True)
    plan.profile_read()
    one()
    stages = plan.profile_read()
    plan.profile(False)
    st_direct = timing_stats(timed_solves(torch, stream, one, args.nl_steps))
    # the same solves replayed from a recorded graph (lqt_set_graphs)
    plan.set_graphs(True)
    one()
    torch.cuda.synchronize()
    st_graph = timing_stats(timed_solves(torch, stream, one, args.nl_steps))
    recorded = plan.graphs_recorded()
    plan.close()
    ms = st_direct["mean"]
    return {"workload": f"iterated nonlinear LQT, unicycle, T={T}, {rounds} rounds, {prec}",
            "ms_per_solve": ms, "ms_per_round": round(ms / rounds, 4), "ms_per_solve_stats": st_direct,
            "graph_replay": {"ms_per_solve_stats": st_graph, "ms_per_round": round(st_graph["mean"] / rounds, 4),
                             "graphs_recorded": recorded},
            "value": round(T * rounds / (ms / 1e3), 1), "unit": "steps*rounds/s", "status": st,
            "rel_err": rel_err, "cpu_baseline": cpu,
            "stage_ms_one_solve": {k: round(v[1], 4) for k, v in stages.items()}}


def run_finite(args, api, inputs, torch, with_cpu=True):
    """Finite state and control spaces (Section III-D), the routing workload
    of the finite-state experiment (Section VI-D) at its state counts
    D_x = 5, 11, 21 and T = args.fs_T.  Integer-valued costs: parity with the
    oracle is exact.  Algorithmic bytes per step: the cost table row read
    twice (product fold and final walk, 8 D_x D_u each), the closed-loop map
    written once and read once (4 D_x each), V_k, u_k written (12 D_x), x_k
    and the applied control written (8)."""
    import oracle.finite as fin

    T = args.fs_T
    out = {}
    for D in (5, 11, 21):
        prob = inputs.routing_problem(T, nstates=D, seed=0)
        plan = api.Plan(4, 4, prec="fp64", device=0)
        dp = api.DeviceFSProblem(prob)
        do = api.DeviceFSOutputs(D, T)
        stream = torch.cuda.current_stream(0)
        plan.fs_solve(dp, do, stream)
        torch.cuda.synchronize()
        st = int(do.status.item())
        exact, cpu = None, None
        if not args.no_parity or with_cpu:
            t0 = time.perf_counter()
            ref = fin.solve(prob)
            secs = time.perf_counter() - t0
            if not args.no_parity:
                got = do.host()
                exact = all(np.array_equal(got[f], ref[f]) for f in got)
            if with_cpu:
                cpu = {"value": round(T / secs, 1), "unit": "steps/s", "cores": 1, "kind": "oracle", "host": host_cpu(),
                       "sample": f"one full sequential solve (T={T}; {secs:.2f} s)"}
        plan.profile(True)
        plan.profile_read()
        plan.fs_solve(dp, do, stream)
        stages = plan.profile_read()
        plan.profile(False)
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        for _ in range(args.fs_steps):
            plan.fs_solve(dp, do, stream)
        e1.record(stream)
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1) / args.fs_steps
        plan.close()
        Du = prob.ncontrols
        bytes_step = 2 * 8 * D * Du + 8 * D + 12 * D + 8
        out[f"D{D}"] = {"workload": f"finite-state routing, D_x={D}, D_u={Du}, T={T}", "ms_per_solve": round(ms, 4),
                        "value": round(T / (ms / 1e3), 1), "unit": "steps/s", "status": st, "exact_parity": exact,
                        "algorithmic_bytes_per_step": bytes_step,
                        "hbm_frac": round(bytes_step * T / (ms / 1e3) / 1e9 / HBM_PEAK_GBS, 4),
                        "cpu_baseline": cpu,
                        "stage_ms_one_solve": {k: round(v[1], 4) for k, v in stages.items()}}
    return out


def run_blocks(args, api, inputs, torch):
    """Block processing (Section V-C): every lane of the n <= 4 pipeline folds
    a block of B consecutive elements sequentially before the parallel scan
    over the blocks.  Time of the T = args.T tracking solve (FP64) for
    B = 1 .. 64 (the library's default for this T is 16)."""
    n, m, T = 4, 2, args.T
    prob = inputs.tracking_problem(n=n, m=m, T=T, workload=1)
    plan = api.Plan(n, m, prec="fp64", device=0, max_steps=T)
    dp = api.DeviceProblem(prob)
    do = api.DeviceOutputs(n, m, T)
    stream = torch.cuda.current_stream(0)
    res = {}
    try:
        for B in (1, 2, 4, 8, 12, 16, 24, 32, 64):
            plan.set_routing(lane_chunk=B)
            for _ in range(2):
                plan.solve([dp], [do], stream)
            torch.cuda.synchronize()
            e0 = torch.cuda.Event(enable_timing=True)
            e1 = torch.cuda.Event(enable_timing=True)
            e0.record(stream)
            for _ in range(args.block_steps):
                plan.solve([dp], [do], stream)
            e1.record(stream)
            torch.cuda.synchronize()
            res[str(B)] = round(e0.elapsed_time(e1) / args.block_steps, 4)
    finally:
        plan.close()
    best = min(res, key=res.get)
    return {"workload": f"block length sweep, tracking n=4 m=2 T={T} fp64", "ms_per_solve_by_block": res,
            "best_block": int(best)}


def condensed_problem(prob, B):
    """Partial condensing (Section V-C) of a time-invariant instance with block
    length B: the LQT over the block boundaries x_{jB}, j = 0..T/B, whose
    control is the block's B controls stacked (dimension B m) and whose stage
    cost is the block's B stage costs written in (x_{jB}, U_j).  With the
    outputs of the block stacked, Y = H_B x + G_B U + h, H_B = [H F^i]_i,
    G_B[i][l] = H F^(i-1-l) L (l < i), h_i = H sum_{l<i} F^(i-1-l) c, the
    cost is the generalised stage cost of Section IV-D with H' = H_B,
    r' = r_B - h, X' = blockdiag(X), M' = X' G_B, U' = G_B^T X' G_B +
    blockdiag(U), s' = 0; the dynamics are F' = F^B, L' = [F^(B-1-l) L]_l,
    c' = sum_l F^(B-1-l) c.  Host-side set-up of the condensing experiment
    (the library does not condense)."""
    import dataclasses

    from paper_2104_03186_amd import inputs as _inputs

    n, m, p, T = prob.n, prob.m, prob.p, prob.T
    if prob.per_step or prob.M is not None or prob.s is not None or T % B:
        raise ValueError("condensing needs a time-invariant standard-cost instance with B dividing T")
    F, L, H, X, U = prob.F, prob.L, prob.H, prob.X, prob.U
    c = np.zeros(n) if prob.c is None else np.asarray(prob.c, dtype=np.float64)
    Fp = [np.eye(n)]
    for _ in range(B):
        Fp.append(Fp[-1] @ F)
    HB = np.concatenate([H @ Fp[i] for i in range(B)], axis=0)
    GB = np.zeros((B * p, B * m))
    h = np.zeros(B * p)
    for i in range(B):
        for l in range(i):
            GB[i * p:(i + 1) * p, l * m:(l + 1) * m] = H @ Fp[i - 1 - l] @ L
        h[i * p:(i + 1) * p] = H @ sum((Fp[i - 1 - l] @ c for l in range(i)), np.zeros(n))
    XB = np.kron(np.eye(B), X)
    UB = np.kron(np.eye(B), U)
    Fc = Fp[B]
    Lc = np.concatenate([Fp[B - 1 - l] @ L for l in range(B)], axis=1)
    cc = sum((Fp[B - 1 - l] @ c for l in range(B)), np.zeros(n))
    rB = np.ascontiguousarray(prob.r.reshape(T // B, B * p) - h[None, :])
    Mc = XB @ GB
    Uc = GB.T @ XB @ GB + UB
    Uc = 0.5 * (Uc + Uc.T)
    return _inputs.LQTProblem(n=n, m=B * m, p=B * p, pT=prob.pT, T=T // B, per_step=0, F=Fc,
                              c=None if prob.c is None else cc, L=Lc, H=HB, X=XB, U=Uc, r=rB,
                              HT=prob.HT, XT=prob.XT, rT=prob.rT, x0=prob.x0, M=Mc,
                              s=np.zeros((T // B, B * m)))


def run_condensing(args, api, inputs, torch):
    """Partial condensing against the block fold (Section V-C): the headline
    tracking instance (n = 4, m = 2, T = args.T, FP64) condensed with block
    length B into T / B steps of B m controls and B n outputs, solved through
    the generalised-cost path (S, v, K, d, x, u of the condensed LQT), beside
    the direct solve, whose lanes fold blocks of B steps themselves.  The
    condensed instance's set-up (host) is outside the timed region."""
    n, m, T = 4, 2, args.T
    prob = inputs.tracking_problem(n=n, m=m, T=T, workload=1)
    stream = torch.cuda.current_stream(0)
    res = {}
    for B in (2, 4, 8, 16):
        cp = condensed_problem(prob, B)
        plan = api.Plan(cp.n, cp.m, prec="fp64", device=0, max_steps=cp.T)
        try:
            dp = api.DeviceProblem(cp)
            do = api.DeviceOutputs(cp.n, cp.m, cp.T)
            for _ in range(2):
                plan.solve([dp], [do], stream)
            torch.cuda.synchronize()
            st = int(do.status.item())
            plan.profile(True)
            plan.profile_read()
            plan.solve([dp], [do], stream)
            stages = plan.profile_read()
            plan.profile(False)
            times = timing_stats(timed_solves(torch, stream, lambda: plan.solve([dp], [do], stream),
                                              args.block_steps))
        finally:
            plan.close()
        res[str(B)] = {"condensed_steps": cp.T, "controls": cp.m, "outputs": cp.p, "status": st,
                       "ms_per_solve_stats": times,
                       "stage_ms_one_solve": {k: round(v[1], 4) for k, v in stages.items()}}
    return {"workload": f"partial condensing, tracking n=4 m=2 T={T} fp64, block length B", "by_block": res}


def run_state_scaling(args, api, inputs, torch, with_cpu=True):
    """State dimension (Section VI-C): the chain of N masses (n = 2N, m = 2)
    over a 10 s horizon in T steps, one instance per solve, FP64; device time
    per solve (median of args.block_steps solves) with the default routing
    and with the chunk scans as trees (routing tree=True, the latency setting
    for a lone instance), beside the oracle's sequential solve of the same
    instance on one host core."""
    res = {}
    for N in (2, 4, 8, 16, 32):
        for T in (100, 1000):
            prob = inputs.mass_spring_problem(N, T)
            row = {"n": 2 * N}
            for key, tree in (("gpu_ms_per_solve", None), ("gpu_ms_per_solve_trees", True)):
                plan = api.Plan(2 * N, 2, prec="fp64", device=0)
                try:
                    plan.set_routing(tree=tree)
                    dp = api.DeviceProblem(prob)
                    do = api.DeviceOutputs(prob.n, prob.m, T)
                    stream = torch.cuda.current_stream(0)
                    for _ in range(3):
                        plan.solve([dp], [do], stream)
                    torch.cuda.synchronize()
                    row["status" if tree is None else "status_trees"] = int(do.status.item())
                    row[key] = timing_stats(timed_solves(torch, stream, lambda: plan.solve([dp], [do], stream),
                                                         args.block_steps))
                finally:
                    plan.close()
            g = row["gpu_ms_per_solve"] if row["gpu_ms_per_solve"]["median"] <= row["gpu_ms_per_solve_trees"]["median"] \
                else row["gpu_ms_per_solve_trees"]
            if with_cpu:
                import oracle

                ts = []
                for _ in range(3):
                    t0 = time.perf_counter()
                    oracle.solve(prob)
                    ts.append((time.perf_counter() - t0) * 1e3)
                row["oracle_ms_per_solve"] = round(float(np.median(ts)), 3)
                row["oracle_over_gpu_best"] = round(row["oracle_ms_per_solve"] / g["median"], 1)
            res[f"N{N}_T{T}"] = row
    return {"workload": "mass-spring-damper chain, n = 2N, m = 2, 10 s horizon, FP64, one instance", "by_size": res,
            "oracle_host": host_cpu() if with_cpu else None}


def run_copy(args, torch):
    """Plain device copy of 256 MiB (float64), three times: the calibration of
    the HBM byte counters (a copy moves exactly its size in each direction)."""
    n = (256 << 20) // 8
    a = torch.ones(n, dtype=torch.float64, device="cuda")
    b = torch.empty_like(a)
    torch.cuda.synchronize()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(3):
        b.copy_(a)
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / 3
    return {"workload": "device copy of 256 MiB (counter calibration)", "bytes_each_way": n * 8,
            "ms_per_copy": round(ms, 4), "GBps_each_way": round(n * 8 / (ms / 1e3) / 1e9, 1)}


def run_serving(args, api, inputs, torch, prec, with_cpu=False):
    """Poisson arrivals (args.rate req/s for args.serve_seconds s), nx ~ U{4..32},
    nu = ceil(nx / 2), T log-uniform on [64, 65536], diagonal costs and
    random-walk references; each request asks for K, d, x, u.  One instance
    of T = 65536 per nx is kept on the device and every request solves its
    own horizon as a prefix of it, so every request has its own (nx, T);
    outputs are allocated per request.  Latency: submit to completed poll."""
    reqs = inputs.serving_requests(args.rate, args.serve_seconds)
    dtype = torch.float64 if prec == "fp64" else torch.float32
    want = ("K", "d", "x", "u")
    Tmax = 65536
    base = {}
    for n in range(4, 33):
        p = inputs.diag_problem(n, (n + 1) // 2, Tmax, 4, n)
        base[n] = (p, api.DeviceProblem(p))
    torch.cuda.synchronize()
    plan = api.Plan(32, 16, prec=prec, device=0, hbm_budget_bytes=args.serve_pool_gb << 30)

    def wait(t):
        while plan.poll(t) is None:
            pass

    # warm-up, then the latency of representative shapes served alone
    for n in (4, 16, 32):
        o = api.DeviceOutputs(n, (n + 1) // 2, 512, dtype=dtype, want=want, status=False)
        wait(plan.submit(base[n][1], o, T=512))
    alone = {}
    for n, T in ((4, 64), (4, 65536), (8, 1024), (16, 1024), (16, 65536), (32, 64), (32, 4096), (32, 65536)):
        ts = []
        for _ in range(5):
            o = api.DeviceOutputs(n, (n + 1) // 2, T, dtype=dtype, want=want, status=False)
            t0 = time.perf_counter()
            wait(plan.submit(base[n][1], o, T=T))
            ts.append((time.perf_counter() - t0) * 1e3)
        alone[f"n{n}_T{T}"] = round(float(np.median(ts)), 3)
    N = len(reqs)
    inflight = {}
    lat, lat_short, lat_long = [], [], []
    served_steps = 0
    keep = {}  # a few cheap requests kept for the parity check
    i = 0
    t0 = time.perf_counter()
    last_done = 0.0
    next_note = 5.0
    while i < N or inflight:
        now = time.perf_counter() - t0
        if now > next_note:
            print(f"[serving] t={now:.1f}s submitted={i}/{N} in_flight={len(inflight)}", file=sys.stderr, flush=True)
            next_note += 5.0
        while i < N and reqs[i][0] <= now:
            _, n, m, T = reqs[i]
            o = api.DeviceOutputs(n, m, T, dtype=dtype, want=want, status=False)
            tk = plan.submit(base[n][1], o, T=T)
            inflight[tk] = (reqs[i][0], n, T, o, i)
            i += 1
        for tk in list(inflight):
            st = plan.poll(tk)
            if st is not None:
                t_done = time.perf_counter() - t0
                arr, n, T, o, idx = inflight.pop(tk)
                if st != 0:
                    raise RuntimeError(f"served request failed with status {st}")
                ms = (t_done - arr) * 1e3
                lat.append(ms)
                (lat_long if T >= 4096 else lat_short).append(ms)
                served_steps += T
                last_done = t_done
                if len(keep) < 4 and n ** 3 * T < 4e6:
                    keep[idx] = (n, T, o)
    stats = plan.serve_stats()
    plan.close()
    lat_ms = np.array(lat)
    offered = sum(r[3] for r in reqs) / args.serve_seconds
    rel_err = None
    if not args.no_parity:
        import oracle

        worst = {f: 0.0 for f in want}
        for idx, (n, T, o) in keep.items():
            p = inputs.diag_problem(n, (n + 1) // 2, Tmax, 4, n)
            sub = inputs.prefix_problem(p, T)
            ref = oracle.solve(sub)
            got = o.host()
            for f in want:
                worst[f] = max(worst[f], rel(got[f], ref[f]))
        rel_err = worst

    def pct(a, q):
        return round(float(np.percentile(np.asarray(a), q)), 3) if len(a) else None

    cpu = None
    if with_cpu:
        import oracle

        # the first requests of the stream, solved over the host threads
        sample = [inputs.prefix_problem(inputs.diag_problem(n, m, Tmax, 4, n), T) for _, n, m, T in reqs[:256]]
        sps, secs, used = oracle.time_solve_parallel(sample, oracle.host_threads())
        cpu = {"value": round(sps, 1), "unit": "steps/s", "cores": used, "kind": "oracle", "host": host_cpu(),
               "sample": f"the first {len(sample)} requests of the stream over the host threads ({secs:.1f} s)"}

    return {"workload": f"serving: Poisson {args.rate:g} req/s for {args.serve_seconds:g} s, nx ~ U{{4..32}}, "
                        f"nu = ceil(nx/2), T log-uniform [64, 65536], {prec}, outputs K d x u",
            "requests": len(lat), "p50_ms": pct(lat_ms, 50), "p99_ms": pct(lat_ms, 99),
            "max_ms": round(float(lat_ms.max()), 3),
            "p50_p99_ms_T_below_4096": [pct(lat_short, 50), pct(lat_short, 99)],
            "p50_p99_ms_T_from_4096": [pct(lat_long, 50), pct(lat_long, 99)],
            "alone_ms_by_shape": alone,
            "served_steps_per_s": round(served_steps / last_done, 1),
            "offered_steps_per_s": round(offered, 1), "elapsed_s": round(last_done, 3),
            "serve_stats": stats, "rel_err_sampled": rel_err, "cpu_baseline": cpu}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=50)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--T", type=int, default=1_000_000)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-seconds", type=float, default=10.0)
    ap.add_argument("--no-parity", action="store_true")
    ap.add_argument("--workload", choices=("all", "single", "batched", "dense", "serving", "nonlinear", "finite",
                                           "blocks", "condensing", "scaling", "copy"), default="all")
    ap.add_argument("--prec", choices=("fp64", "mixed"), default=None,
                    help="precision of a --workload single/batched/serving run")
    ap.add_argument("--trajectory", choices=("maps", "prefix"), default="maps",
                    help="forward pass of a --workload single run: closed-loop maps or forward prefixes")
    ap.add_argument("--cost", choices=("standard", "generalised"), default="standard",
                    help="--workload single: stage cost of the instance (generalised: cross term M and control "
                         "reference s)")
    ap.add_argument("--nl-T", type=int, default=100_000)
    ap.add_argument("--nl-rounds", type=int, default=10)
    ap.add_argument("--nl-steps", type=int, default=10)
    ap.add_argument("--block-steps", type=int, default=20)
    ap.add_argument("--fs-T", type=int, default=100_000)
    ap.add_argument("--fs-steps", type=int, default=20)
    ap.add_argument("--count", type=int, default=4096)
    ap.add_argument("--batched-steps", type=int, default=10)
    ap.add_argument("--batched-warmup", type=int, default=3)
    ap.add_argument("--no-tune", action="store_true", help="batched leg: keep the default chunk lengths")
    ap.add_argument("--dense-count", type=int, default=64)
    ap.add_argument("--dense-T", type=int, default=8192)
    ap.add_argument("--rate", type=float, default=2000.0)
    ap.add_argument("--serve-seconds", type=float, default=60.0)
    ap.add_argument("--serve-pool-gb", type=int, default=16)
    args = ap.parse_args()

    if args.gpus != 1:
        print(f"bench.py measures one GPU only (got --gpus {args.gpus}); the library solves on one device.",
              file=sys.stderr)
        sys.exit(2)

    import torch

    from paper_2104_03186_amd import api, inputs

    with_cpu = not args.no_cpu_baseline
    if args.workload == "batched":
        print(json.dumps(run_batched(args, api, inputs, torch, args.prec or "mixed", with_cpu)), flush=True)
        return
    if args.workload == "copy":
        print(json.dumps(run_copy(args, torch)), flush=True)
        return
    if args.workload == "dense":
        print(json.dumps(run_dense(args, api, inputs, torch, args.prec or "mixed", with_cpu)), flush=True)
        return
    if args.workload == "nonlinear":
        print(json.dumps(run_nonlinear(args, api, inputs, torch, args.prec or "fp64",
                                       not args.no_cpu_baseline)), flush=True)
        return
    if args.workload == "blocks":
        print(json.dumps(run_blocks(args, api, inputs, torch)), flush=True)
        return
    if args.workload == "condensing":
        print(json.dumps(run_condensing(args, api, inputs, torch)), flush=True)
        return
    if args.workload == "scaling":
        print(json.dumps(run_state_scaling(args, api, inputs, torch, not args.no_cpu_baseline)), flush=True)
        return
    if args.workload == "finite":
        print(json.dumps(run_finite(args, api, inputs, torch, not args.no_cpu_baseline)), flush=True)
        return
    if args.workload == "serving":
        print(json.dumps(run_serving(args, api, inputs, torch, args.prec or "mixed", with_cpu)), flush=True)
        return
    prec = args.prec or "fp64"
    main_res = run_single(args, api, inputs, torch, prec, args.steps, args.warmup, not args.no_cpu_baseline,
                          trajectory=args.trajectory if args.workload == "single" else "maps",
                          cost=args.cost if args.workload == "single" else "standard")
    out = {
        "metric": "LQT time-steps solved/s (single long instance, parallel scan)",
        "value": round(main_res["value"], 1),
        "unit": "steps/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(main_res["ms_per_step"], 4),
        "ms_per_solve_stats": main_res["ms_per_solve_stats"],
        "lane_pipeline_ms_per_solve_stats": main_res["lane_pipeline_ms_per_solve_stats"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64" if prec == "fp64" else "f64 arithmetic, f32 results",
        "data": "synthetic (seeded generators: sinusoid-reference tracking; diagonal-cost random-walk batches)",
        "config": {"workload": f"single LQT instance nx=4 nu=2 T={args.T} {prec}"
                               + (", trajectory by forward prefixes" if args.trajectory == "prefix" else "")
                               + (", generalised cost (M, s)" if args.cost == "generalised" else ""),
                   "nx": 4, "nu": 2, "T": args.T, "precision": prec},
        "status": main_res["status"],
        "rel_err": main_res["rel_err"],
        "stages_avg_ms": main_res["stages_avg_ms"],
        "roofline": main_res["roofline"],
        "path_roofline": main_res["path_roofline"],
        "cpu_baseline": main_res["cpu_baseline"],
    }
    note(f"single fp64 T={args.T}: {main_res['ms_per_step']:.4f} ms per solve")
    if args.workload == "all":
        mixed = run_single(args, api, inputs, torch, "mixed", args.steps, args.warmup, False)
        out["single_mixed"] = {k: mixed[k] for k in ("value", "ms_per_step", "ms_per_solve_stats", "status", "rel_err",
                                                     "roofline")}
        note("single mixed done")
        m2 = run_single(args, api, inputs, torch, "fp64", max(10, args.steps // 2), 2, False, trajectory="prefix")
        out["single_fp64_forward_prefixes"] = {k: m2[k] for k in ("value", "ms_per_step", "status", "rel_err",
                                                                  "stages_avg_ms")}
        note("single forward prefixes done")
        gen = run_single(args, api, inputs, torch, "fp64", max(10, args.steps // 2), 2, False, cost="generalised")
        out["single_fp64_generalised_cost"] = {k: gen[k] for k in ("value", "ms_per_step", "status", "rel_err",
                                                                   "stages_avg_ms")}
        note("single generalised cost done")
        out["nonlinear_fp64"] = run_nonlinear(args, api, inputs, torch, "fp64", not args.no_cpu_baseline)
        note("nonlinear done")
        out["finite_state"] = run_finite(args, api, inputs, torch, not args.no_cpu_baseline)
        note("finite state done")
        out["block_sweep"] = run_blocks(args, api, inputs, torch)
        note("block sweep done")
        out["partial_condensing"] = run_condensing(args, api, inputs, torch)
        note("partial condensing done")
        out["state_scaling"] = run_state_scaling(args, api, inputs, torch, not args.no_cpu_baseline)
        note("state scaling done")
        out["batched_mixed"] = run_batched(args, api, inputs, torch, "mixed", with_cpu)
        note("batched done")
        out["dense_mixed"] = run_dense(args, api, inputs, torch, "mixed", with_cpu)
        note("dense mixed done")
        out["dense_fp64"] = run_dense(args, api, inputs, torch, "fp64")
        note("dense fp64 done")
        out["serving_mixed"] = run_serving(args, api, inputs, torch, "mixed", with_cpu)
        note("serving done")
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
