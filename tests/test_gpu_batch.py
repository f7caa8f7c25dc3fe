"""GPU parity of the batched lane kernel (n <= 4, time-invariant except c:
one workgroup per instance, the whole scan of Sections II-C, IV-A, IV-B and
the trajectory of Section IV-C, Method 1, inside it) against the FP64 oracle:
every (n, m) <= 4, horizons around the chunk and wavefront boundaries
(T = 1 to 16384, and larger through the routing override), square and
general output maps, per-step offsets (the step-data modes), FP64 and MIXED,
optional outputs, a batch equal to its instances solved alone (bitwise),
status codes and failure isolation.

Tolerance: relative error per output family over all steps stacked and per
step (tests/helpers.err), 1e-10 (FP64) and 1e-5 (MIXED).
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
    ps = {pr: api.Plan(8, 4, prec=pr) for pr in ("fp64", "mixed")}
    yield ps
    for p in ps.values():
        p.close()


@pytest.fixture(autouse=True)
def _routing(plans):
    for p in plans.values():
        p.set_routing(path="batch")
    yield
    for p in plans.values():
        p.set_routing()


def run(api, plan, probs, prec, want=FAMILIES):
    import torch

    dt = torch.float64 if prec == "fp64" else torch.float32
    dps = [api.DeviceProblem(p) for p in probs]
    dos = [api.DeviceOutputs(p.n, p.m, p.T, want=want, dtype=dt) for p in probs]
    plan.solve(dps, dos)
    torch.cuda.synchronize()
    return dos


def check(got, ref, tol):
    errs = {f: err(got[f], ref[f]) for f in got}
    bad = {f: e for f, e in errs.items() if not e <= tol}
    assert not bad, f"errors above {tol}: {bad} (all: {errs})"


@pytest.mark.parametrize("prec", ["fp64", "mixed"])
@pytest.mark.parametrize("T", [1, 2, 5, 63, 64, 65, 255, 256, 257, 511, 1000, 4097, 16384, 40000])
def test_tracking_horizons(api, plans, prec, T):
    _say("batched lane tracking n=4 m=2 T=", T, prec)
    prob = inputs.tracking_problem(n=4, m=2, T=T, instance=T % 7)
    (do,) = run(api, plans[prec], [prob], prec)
    assert int(do.status.item()) == 0
    check(do.host(), oracle.solve(prob), TOL[prec])


@pytest.mark.parametrize("nm", [(1, 1), (2, 1), (2, 2), (3, 1), (3, 2), (3, 3), (4, 1), (4, 2), (4, 3), (4, 4)])
@pytest.mark.parametrize("kind", ["square", "general", "offsets"])
def test_shapes_and_modes(api, plans, nm, kind):
    n, m = nm
    p = n if kind != "general" else n + 1
    per_step = 2 if kind == "offsets" else 0
    T = 777
    _say("batched lane random n=", n, "m=", m, kind)
    prob = inputs.random_problem(n, m, T, seed=500 + 10 * n + m, p=p, pT=n, per_step=per_step, scale=0.95,
                                 with_c=(kind != "square"))
    (do,) = run(api, plans["fp64"], [prob], "fp64")
    assert int(do.status.item()) == 0
    check(do.host(), oracle.solve(prob), TOL["fp64"])


@pytest.mark.parametrize("want", [("S", "v", "K", "d"), ("x", "u"), ("u",), ("K", "d", "x"), ("S",)])
def test_optional_outputs(api, plans, want):
    prob = inputs.random_problem(4, 2, 3000, seed=61)
    _say("batched lane outputs", want)
    (do,) = run(api, plans["fp64"], [prob], "fp64", want=want)
    got = do.host()
    assert set(got) == set(want)
    check(got, oracle.solve(prob), TOL["fp64"])


@pytest.mark.parametrize("prec", ["fp64", "mixed"])
def test_batch_equals_alone(api, plans, prec):
    """A batch of uneven instances of the batched workload's generator: each
    equal to itself solved alone (bitwise) and to the oracle."""
    rng = np.random.default_rng(5)
    probs = [inputs.diag_problem(n, n // 2 if n > 1 else 1, int(T), 2, i) for i, (n, T) in
             enumerate(zip(rng.choice([2, 4], 24), np.exp(rng.uniform(np.log(1), np.log(16384), 24)).round()))]
    probs.append(inputs.random_problem(3, 2, 900, seed=3, p=2, pT=3))
    _say("batched lane mix of", len(probs), prec)
    dos = run(api, plans[prec], probs, prec)
    for i, (p, do) in enumerate(zip(probs, dos)):
        assert int(do.status.item()) == 0, i
        got = do.host()
        check(got, oracle.solve(p), TOL[prec])
        (alone,) = run(api, plans[prec], [p], prec)
        for f in FAMILIES:
            assert np.array_equal(got[f], alone.host()[f]), (i, f)


def test_status_and_isolation(api, plans):
    good = inputs.random_problem(4, 2, 500, seed=71)
    bad = inputs.random_problem(4, 2, 500, seed=72)
    bad.U = -np.eye(2)
    nan = inputs.random_problem(3, 1, 400, seed=73)
    nan.r[123, 1] = np.nan
    _say("batched lane status codes")
    dos = run(api, plans["fp64"], [good, bad, nan], "fp64")
    assert int(dos[0].status.item()) == 0
    assert int(dos[1].status.item()) == 3
    assert int(dos[2].status.item()) == 4
    check(dos[0].host(), oracle.solve(good), TOL["fp64"])


def test_default_routing(api):
    """Without an override, n <= 4 time-invariant instances up to T = 16384
    take the batched lane kernel; the result matches the oracle either way."""
    import torch

    plan = api.Plan(4, 2, prec="fp64")
    try:
        for T in (300, 9000, 16384, 16385):
            prob = inputs.tracking_problem(n=4, m=2, T=T, instance=1)
            _say("default routing T=", T)
            dp = api.DeviceProblem(prob)
            do = api.DeviceOutputs(4, 2, T)
            plan.solve([dp], [do])
            torch.cuda.synchronize()
            assert int(do.status.item()) == 0
            check(do.host(), oracle.solve(prob), TOL["fp64"])
    finally:
        plan.close()
