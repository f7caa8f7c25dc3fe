"""GPU parity of the forward-prefix trajectory (Method 2 of Section IV-C) on
the lane pipeline: x and u against the FP64 oracle and against the
closed-loop-map trajectory (Method 1) of the same backward pass; FP64 and
MIXED; default and forced chunk lengths; time-varying data; outputs without
S and v (library workspace); and on the chunked engines (wavefront engine,
classes 8-32, and workgroup engines, classes 16-64): against the oracle and
against Method 1 at n from 6 to 64, time-varying data, partial outputs and
a batch that mixes the paths.

Tolerance: relative error per output family, over all steps stacked (Frobenius) and
per step (largest step error against the RMS step size; tests/helpers.err),
1e-10 (FP64) and 1e-5 (MIXED).
"""
import sys

import numpy as np
import pytest

import oracle
from paper_2104_03186_amd import inputs
from tests.helpers import FAMILIES, err

pytestmark = pytest.mark.gpu

TOL = {"fp64": 1e-10, "mixed": 1e-5}


def _say(*a):
    print("[case]", *a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def api():
    import torch

    assert torch.cuda.is_available(), "GPU tests need a GPU"
    from paper_2104_03186_amd import api as _api

    return _api


@pytest.fixture(scope="module")
def plans(api):
    ps = {(pr, tr): api.Plan(4, 4, prec=pr, device=0, trajectory=tr)
          for pr in ("fp64", "mixed") for tr in ("maps", "prefix")}
    yield ps
    for p in ps.values():
        p.close()


@pytest.fixture(autouse=True)
def _routing(plans):
    yield
    for p in plans.values():
        p.set_routing()


def run(api, plan, prob, prec, want=FAMILIES, chunk=None, path="small"):
    """Solve on the lane pipeline (path "small", any T) unless path says
    otherwise; chunk fixes the steps per lane."""
    import torch

    plan.set_routing(path=path, lane_chunk=chunk or 0)
    dt = torch.float64 if prec == "fp64" else torch.float32
    dp = api.DeviceProblem(prob)
    do = api.DeviceOutputs(prob.n, prob.m, prob.T, want=want, dtype=dt)
    plan.solve([dp], [do])
    torch.cuda.synchronize()
    assert int(do.status.item()) == 0
    return do.host()


@pytest.mark.parametrize("prec", ["fp64", "mixed"])
@pytest.mark.parametrize("T,chunk", [(1, None), (2, None), (5, 2), (64, 1), (65, 3), (1000, None), (4097, 16),
                                     (20000, 1), (70000, None)])
def test_prefix_trajectory(api, plans, prec, T, chunk):
    _say("method 2 tracking n=4 m=2 T=", T, "chunk=", chunk, prec)
    prob = inputs.tracking_problem(n=4, m=2, T=T, instance=3)
    got = run(api, plans[(prec, "prefix")], prob, prec, chunk=chunk)
    ref = oracle.solve(prob)
    errs = {f: err(got[f], ref[f]) for f in FAMILIES}
    assert max(errs.values()) <= TOL[prec], errs
    alt = run(api, plans[(prec, "maps")], prob, prec, chunk=chunk)
    for f in ("S", "v", "K", "d"):  # same backward pass
        assert np.array_equal(got[f], alt[f]), f
    for f in ("x", "u"):
        assert err(got[f], alt[f]) <= TOL[prec], (f, err(got[f], alt[f]))


@pytest.mark.parametrize("nm", [(1, 1), (2, 2), (3, 1), (4, 1), (4, 3), (4, 4)])
@pytest.mark.parametrize("per_step", [0, 1 | 2 | 4 | 8 | 16 | 32])
def test_prefix_shapes_and_time_varying(api, plans, nm, per_step):
    n, m = nm
    T = 300
    _say("method 2 random n=", n, "m=", m, "per_step=", per_step)
    prob = inputs.random_problem(n, m, T, seed=40 + 7 * n + m + per_step, p=n, pT=n, per_step=per_step,
                                 scale=0.95)
    got = run(api, plans[("fp64", "prefix")], prob, "fp64", chunk=7)
    ref = oracle.solve(prob)
    errs = {f: err(got[f], ref[f]) for f in FAMILIES}
    assert max(errs.values()) <= TOL["fp64"], errs


@pytest.mark.parametrize("want", [("x", "u"), ("K", "d", "x"), ("u",)])
def test_prefix_without_value_outputs(api, plans, want):
    # S and v are not taken: the forward pass reads them from library workspace
    prob = inputs.tracking_problem(n=4, m=2, T=9000, instance=4)
    _say("method 2 outputs", want)
    got = run(api, plans[("fp64", "prefix")], prob, "fp64", want=want)
    assert set(got) == set(want)
    ref = oracle.solve(prob)
    for f in want:
        assert err(got[f], ref[f]) <= TOL["fp64"], f


def test_prefix_full_size(api, plans):
    T = 1_000_000
    _say("method 2 tracking n=4 m=2 T=", T, "(default launch configuration)")
    prob = inputs.tracking_problem(n=4, m=2, T=T, workload=1)
    got = run(api, plans[("fp64", "prefix")], prob, "fp64")
    ref = oracle.solve(prob)
    errs = {f: err(got[f], ref[f]) for f in FAMILIES}
    assert max(errs.values()) <= TOL["fp64"], errs


# chunked engines: (n, m, engine, T, chunk); the workgroup engines take
# time-invariant instances of the classes 16, 32 and 64 (end-aligned chunks;
# operator-form fold without offsets), the wavefront engine classes 8-32
CHUNKED = [(6, 3, "wavefront", 300, None), (8, 4, "wavefront", 1001, 17), (12, 5, "wavefront", 257, None),
           (16, 8, "workgroup", 300, None), (16, 8, "wavefront", 700, 33), (24, 8, "workgroup", 513, 40),
           (32, 16, "workgroup", 400, None), (32, 16, "wavefront", 129, 16), (48, 20, "workgroup", 150, None),
           (64, 32, "workgroup", 200, 24)]


@pytest.mark.parametrize("prec", ["fp64", "mixed"])
@pytest.mark.parametrize("n,m,engine,T,chunk", CHUNKED)
def test_prefix_chunked_engines(api, prec, n, m, engine, T, chunk):
    """Method 2 on the chunked engines against the oracle and against Method 1
    of the same backward pass."""
    import torch

    dt = torch.float64 if prec == "fp64" else torch.float32
    _say("method 2 chunked n=", n, "m=", m, engine, "T=", T, "chunk=", chunk, prec)
    prob = inputs.random_problem(n, m, T, seed=300 + n + m + T, p=n, pT=n)
    out = {}
    for traj in ("prefix", "maps"):
        plan = api.Plan(64, 32, prec=prec, trajectory=traj)
        try:
            plan.set_routing(path="wave", wave_engine_only=(engine == "wavefront"), wave_chunk=chunk or 0)
            dp = api.DeviceProblem(prob)
            do = api.DeviceOutputs(n, m, T, dtype=dt)
            plan.solve([dp], [do])
            torch.cuda.synchronize()
            assert int(do.status.item()) == 0
            out[traj] = do.host()
        finally:
            plan.close()
    got, alt = out["prefix"], out["maps"]
    ref = oracle.solve(prob)
    errs = {f: err(got[f], ref[f]) for f in FAMILIES}
    assert max(errs.values()) <= TOL[prec], errs
    for f in ("S", "v", "K", "d"):  # same backward pass
        if prec == "fp64":
            assert np.array_equal(got[f], alt[f]), f
        else:
            assert err(got[f], alt[f]) <= TOL[prec], f
    for f in ("x", "u"):
        assert err(got[f], alt[f]) <= TOL[prec], (f, err(got[f], alt[f]))


@pytest.mark.parametrize("per_step", [1 | 2, 4 | 8 | 16 | 32, 63])
def test_prefix_chunked_time_varying(api, per_step):
    import torch

    n, m, T = 10, 4, 333
    _say("method 2 wavefront engine, per_step=", per_step)
    prob = inputs.random_problem(n, m, T, seed=70 + per_step, p=n, pT=n, per_step=per_step, scale=0.95)
    plan = api.Plan(16, 8, prec="fp64", trajectory="prefix")
    try:
        plan.set_routing(path="wave", wave_chunk=20)
        dp = api.DeviceProblem(prob)
        do = api.DeviceOutputs(n, m, T, dtype=torch.float64)
        plan.solve([dp], [do])
        torch.cuda.synchronize()
        assert int(do.status.item()) == 0
        got = do.host()
    finally:
        plan.close()
    ref = oracle.solve(prob)
    errs = {f: err(got[f], ref[f]) for f in FAMILIES}
    assert max(errs.values()) <= TOL["fp64"], errs


@pytest.mark.parametrize("prec", ["fp64", "mixed"])
@pytest.mark.parametrize("want", [("x", "u"), ("u",), ("S", "x")])
def test_prefix_chunked_partial_outputs(api, prec, want):
    """S and v not taken (or only some families): the walk reads S, v from
    library workspace; a mixed batch of lane-pipeline and chunked instances."""
    import torch

    dt = torch.float64 if prec == "fp64" else torch.float32
    probs = [inputs.random_problem(12, 6, 400, seed=91, p=12, pT=12), inputs.tracking_problem(n=4, m=2, T=9000),
             inputs.dense_problem(64, 32, 120, instance=5), inputs.random_problem(4, 2, 600, seed=92)]
    _say("method 2 partial outputs", want, prec)
    plan = api.Plan(64, 32, prec=prec, trajectory="prefix")
    try:
        dps = [api.DeviceProblem(p) for p in probs]
        dos = [api.DeviceOutputs(p.n, p.m, p.T, dtype=dt, want=want) for p in probs]
        plan.solve(dps, dos)
        torch.cuda.synchronize()
        for p, do in zip(probs, dos):
            assert int(do.status.item()) == 0
            got = do.host()
            assert set(got) == set(want)
            ref = oracle.solve(p)
            for f in want:
                assert err(got[f], ref[f]) <= TOL[prec], (p.n, f, err(got[f], ref[f]))
    finally:
        plan.close()
