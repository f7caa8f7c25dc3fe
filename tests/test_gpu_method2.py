"""GPU parity of the forward-prefix trajectory (Method 2 of Section IV-C) on
the lane pipeline: x and u against the FP64 oracle and against the
closed-loop-map trajectory (Method 1) of the same backward pass; FP64 and
MIXED; default and forced chunk lengths; time-varying data; outputs without
S and v (library workspace); the LQT_ENOTSUP boundary for other paths.

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


def test_prefix_limits(api):
    from paper_2104_03186_amd import _lib

    plan = api.Plan(8, 4, prec="fp64", trajectory="prefix")
    try:
        prob = inputs.random_problem(6, 3, 50, seed=9)  # wavefront path
        _say("method 2 on the wavefront path: LQT_ENOTSUP")
        with pytest.raises(_lib.LQTError) as e:
            run(api, plan, prob, "fp64")
        assert e.value.code == _lib.ENOTSUP
        # no trajectory asked for: the backward pass alone is allowed
        got = run(api, plan, prob, "fp64", want=("S", "v", "K", "d"))
        ref = oracle.solve(prob)
        for f in ("S", "v", "K", "d"):
            assert err(got[f], ref[f]) <= TOL["fp64"], f
    finally:
        plan.close()
