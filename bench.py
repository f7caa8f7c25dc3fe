"""Throughput benchmark of the HIP LQT solver on one MI355X.

Workload (default): one long tracking instance, n = 4 states, m = 2 controls,
T = 1,000,000 steps, FP64 (the sinusoid-reference generator with
F = I + 0.1 G rescaled to spectral radius 0.99, X = 10 I, U = 0.1 I,
X_T = 10 I).  One "step" of this benchmark is one full solve: element build,
reverse scan, gain extraction, forward trajectory scan; every output family
(S, v, K, d, x, u) is written to device memory.  Inputs are resident in HBM
before the timed region.

Prints one JSON line.  ``value`` = time steps solved per second (T x solves /
elapsed).  ``roofline`` describes the kernel with the largest device time,
measured with HIP events recorded around every kernel launch in the timed
region.  ``cpu_baseline`` times the FP64 CPU oracle on the host.
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
FP64_PEAK_TFLOPS = 78.6      # MI355X FP64 vector


def algorithmic_bytes_per_step(n, m, p):
    """Bytes a step must move by the path's contract: reference r_k read once;
    S_k, v_k, K_k, d_k, x_k, u_k written once (FP64)."""
    return 8 * (p + n * n + n + m * n + m + n + m)


def stage_bytes_per_step(stage, n, m, p):
    """Algorithmic bytes of one kernel's own contract, per step."""
    if stage == "bwd_final":   # reads r_k, writes S_k, v_k, K_k, d_k
        return 8 * (p + n * n + n + m * n + m)
    if stage == "fwd_final":   # writes x_k, u_k
        return 8 * (n + m)
    if stage in ("bwd_reduce", "prep_varying"):   # reads r_k
        return 8 * p
    return 0


def path_flops_per_step(n, m):
    """Algorithmic flops per step of the parallel path: two applications of
    the LQT combination rule per element (work-efficient scan), the gain
    extraction and two affine-map compositions."""
    comb = (56.0 / 3.0) * n ** 3 + 14 * n ** 2
    extract = 6 * n * n * m + 4 * n * m * m + m ** 3 / 3.0 + 4 * n * n
    aff = 2 * n ** 3 + 2 * n ** 2
    return 2 * comb + extract + 2 * aff


def run_batched(args, api, inputs, torch):
    """Uneven batch: 4096 instances, T log-uniform on [256, 16384], n in
    {4, 8, 16}, m = n / 2, diagonal costs, random-walk references; one
    lqt_solve call per step (all instances, every output family)."""
    count = args.count
    shapes = inputs.batched_shapes(count)
    probs = [inputs.diag_problem(n, n // 2, T, 2, i) for i, (n, T) in enumerate(shapes)]
    steps_total = sum(p.T for p in probs)
    plan = api.Plan(16, 8, prec="fp64", device=0)
    dps = [api.DeviceProblem(p) for p in probs]
    dos = [api.DeviceOutputs(p.n, p.m, p.T) for p in probs]
    stream = torch.cuda.current_stream(0)
    for _ in range(args.warmup):
        plan.solve(dps, dos, stream)
    torch.cuda.synchronize()
    status_bad = sum(int(o.status.item()) != 0 for o in dos)
    rel_err = None
    if not args.no_parity:
        import oracle

        worst = {f: 0.0 for f in api.FAMILIES}
        for i in range(0, count, max(1, count // 16)):
            ref = oracle.solve(probs[i])
            got = dos[i].host()
            for f in api.FAMILIES:
                worst[f] = max(worst[f], float(np.linalg.norm(got[f] - ref[f]) / np.linalg.norm(ref[f])))
        rel_err = worst
    plan.profile(True)
    plan.profile_read()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    for _ in range(args.steps):
        plan.solve(dps, dos, stream)
    e1.record(stream)
    torch.cuda.synchronize()
    stages = plan.profile_read()
    plan.profile(False)
    e0.record(stream)
    for _ in range(args.steps):
        plan.solve(dps, dos, stream)
    e1.record(stream)
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / args.steps
    out = {"workload": f"batched {count} uneven instances, n in {{4,8,16}}, FP64", "steps_per_solve": steps_total,
           "ms_per_solve": round(ms, 3), "value": round(steps_total / (ms / 1e3), 1), "unit": "steps/s",
           "status_failures": status_bad, "rel_err_sampled": rel_err,
           "stages_ms_per_solve": {k: round(v[1] / max(v[0], 1), 4) for k, v in stages.items()}}
    plan.close()
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=50)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--T", type=int, default=1_000_000)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-seconds", type=float, default=10.0)
    ap.add_argument("--no-parity", action="store_true")
    ap.add_argument("--workload", choices=("single", "batched"), default="single")
    ap.add_argument("--count", type=int, default=4096)
    args = ap.parse_args()

    if args.gpus != 1:
        print(f"bench.py measures one GPU only (got --gpus {args.gpus}); this build has no multi-GPU path.",
              file=sys.stderr)
        sys.exit(2)

    import torch

    from paper_2104_03186_amd import api, inputs

    if args.workload == "batched":
        print(json.dumps(run_batched(args, api, inputs, torch)), flush=True)
        return

    n, m, T = 4, 2, args.T
    prob = inputs.tracking_problem(n=n, m=m, T=T, workload=1)
    dev = "cuda:0"
    plan = api.Plan(n, m, prec="fp64", device=0, max_steps=T)
    dp = api.DeviceProblem(prob, dev)
    do = api.DeviceOutputs(n, m, T, dev)
    stream = torch.cuda.current_stream(0)

    for _ in range(args.warmup):
        plan.solve([dp], [do], stream)
    torch.cuda.synchronize()
    status = int(do.status.item())

    rel_err = None
    if not args.no_parity:
        import oracle

        ref = oracle.solve(prob)
        got = do.host()
        rel_err = {f: float(np.linalg.norm(got[f] - ref[f]) / np.linalg.norm(ref[f])) for f in api.FAMILIES}

    # Timed region: K solves, every kernel bracketed by HIP events on `stream`.
    plan.profile(True)
    plan.profile_read()
    torch.cuda.synchronize()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    t0 = time.perf_counter()
    e0.record(stream)
    for _ in range(args.steps):
        plan.solve([dp], [do], stream)
    e1.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    ms_total = e0.elapsed_time(e1)
    stages = plan.profile_read()
    plan.profile(False)

    # Same loop without per-kernel events, for reference.
    torch.cuda.synchronize()
    e0.record(stream)
    for _ in range(args.steps):
        plan.solve([dp], [do], stream)
    e1.record(stream)
    torch.cuda.synchronize()
    ms_total_plain = e0.elapsed_time(e1)

    ms_per_step = ms_total / args.steps
    value = T * args.steps / (ms_total / 1e3)

    dom = max(stages.items(), key=lambda kv: kv[1][1])
    dom_name, (dom_launches, dom_ms) = dom
    dom_avg_s = dom_ms / dom_launches / 1e3
    dom_bytes = stage_bytes_per_step(dom_name, n, m, prob.p) * T
    achieved = dom_bytes / dom_avg_s / 1e9
    roofline = {"kernel": dom_name, "bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS,
                "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": None,
                "avg_us": round(dom_avg_s * 1e6, 2), "algorithmic_bytes_per_launch": dom_bytes}

    bytes_step = algorithmic_bytes_per_step(n, m, prob.p)
    flops_step = path_flops_per_step(n, m)
    t_bound = max(bytes_step * T / (HBM_PEAK_GBS * 1e9), flops_step * T / (FP64_PEAK_TFLOPS * 1e12))
    path = {"t_bound_us": round(t_bound * 1e6, 2), "t_measured_us": round(ms_per_step * 1e3, 2),
            "frac": round(t_bound / (ms_per_step / 1e3), 4), "bytes_per_step": bytes_step,
            "flops_per_step": round(flops_step, 1)}

    cpu = None
    if not args.no_cpu_baseline:
        import oracle

        sps, secs, reps = oracle.time_solve([prob], min_seconds=args.cpu_seconds)
        cpu = {"value": round(sps, 1), "unit": "steps/s", "cores": 1, "kind": "oracle",
               "sample": f"{reps} full sequential FP64 solve(s) of the same T={T} instance ({secs:.1f} s)"}

    out = {
        "metric": "LQT time-steps solved/s (single long instance, FP64 parallel scan)",
        "value": round(value, 1),
        "unit": "steps/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_per_step, 4),
        "ms_per_step_no_events": round(ms_total_plain / args.steps, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic (seeded sinusoid-reference tracking generator)",
        "config": {"workload": f"single LQT instance nx=4 nu=2 T={T} FP64", "nx": n, "nu": m, "T": T,
                   "precision": "fp64"},
        "status": status,
        "rel_err": rel_err,
        "stages_ms_per_solve": {k: round(v[1] / max(v[0], 1), 4) for k, v in stages.items()},
        "roofline": roofline,
        "path_roofline": path,
        "cpu_baseline": cpu,
        "wall_s": round(wall, 3),
    }
    plan.close()
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
