"""GPU parity of the workgroup class (32 < max(n, m, p, pT) <= 64, m <= 32)
against the FP64 oracle: dense SPD costs, zero-padding edge cases, per-step
offsets, the full dense batch shape, and batch independence.

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
    ps = {pr: api.Plan(64, 32, prec=pr, device=0) for pr in ("fp64", "mixed")}
    yield ps
    for p in ps.values():
        p.close()


@pytest.fixture(autouse=True)
def _routing(plans):
    yield
    for p in plans.values():
        p.set_routing()


def run(api, plan, probs, prec, want=FAMILIES, chunk=None):
    import torch

    plan.set_routing(wave_chunk=chunk or 0)
    dt = torch.float64 if prec == "fp64" else torch.float32
    dps = [api.DeviceProblem(p) for p in probs]
    dos = [api.DeviceOutputs(p.n, p.m, p.T, want=want, dtype=dt) for p in probs]
    plan.solve(dps, dos)
    torch.cuda.synchronize()
    return dos


def check(got, ref, tol):
    errs = {f: err(got[f], ref[f]) for f in got}
    bad = {f: e for f, e in errs.items() if not e <= tol}
    assert not bad, f"rel errors above {tol}: {bad} (all: {errs})"
    return errs


@pytest.mark.parametrize("prec", ["fp64", "mixed"])
@pytest.mark.parametrize("T,chunk", [(1, None), (2, None), (5, 2), (37, 8), (300, None), (301, 16)])
def test_dense_generator(api, plans, prec, T, chunk):
    _say("dense n=64 m=32 T=", T, "chunk=", chunk, prec)
    prob = inputs.dense_problem(64, 32, T, instance=T)
    do = run(api, plans[prec], [prob], prec, chunk=chunk)[0]
    assert int(do.status.item()) == 0
    check(do.host(), oracle.solve(prob), TOL[prec])


@pytest.mark.parametrize("prec", ["fp64", "mixed"])
@pytest.mark.parametrize("nm", [(33, 1), (40, 20), (48, 32), (64, 1), (64, 7), (17, 3)])
def test_padding_shapes(api, plans, prec, nm):
    n, m = nm
    # (17, 3) reaches the class through p = 50 > 32
    p = 50 if n == 17 else max(1, n - 3)
    _say("random n=", n, "m=", m, "p=", p, prec)
    prob = inputs.random_problem(n, m, 120, seed=n * 100 + m, p=p, pT=min(64, n + 2), scale=0.95)
    do = run(api, plans[prec], [prob], prec, chunk=16)[0]
    assert int(do.status.item()) == 0
    check(do.host(), oracle.solve(prob), TOL[prec])


@pytest.mark.parametrize("prec", ["fp64", "mixed"])
@pytest.mark.parametrize("T,chunk", [(130, 16), (257, 128), (64, 1)])
def test_operator_form_padding(api, plans, prec, T, chunk):
    # no offsets (operator-form fold) with padding: n = 40, m = 20, p = 33
    prob = inputs.random_problem(40, 20, T, seed=T + chunk, p=33, pT=40, with_c=False, scale=0.95)
    _say("operator form n=40 m=20 p=33 T=", T, "chunk=", chunk, prec)
    do = run(api, plans[prec], [prob], prec, chunk=chunk)[0]
    assert int(do.status.item()) == 0
    check(do.host(), oracle.solve(prob), TOL[prec])


@pytest.mark.parametrize("prec", ["fp64", "mixed"])
def test_per_step_offsets(api, plans, prec):
    prob = inputs.random_problem(40, 12, 200, seed=77, p=40, pT=40, per_step=2, scale=0.95)
    _say("per-step c, n=40", prec)
    do = run(api, plans[prec], [prob], prec, chunk=32)[0]
    assert int(do.status.item()) == 0
    check(do.host(), oracle.solve(prob), TOL[prec])


@pytest.mark.parametrize("want", [("K", "d", "x", "u"), ("S", "v"), ("x", "u")])
def test_optional_outputs(api, plans, want):
    prob = inputs.dense_problem(64, 32, 90, instance=5)
    _say("dense outputs", want)
    do = run(api, plans["fp64"], [prob], "fp64", want=want)[0]
    assert int(do.status.item()) == 0
    got = do.host()
    assert set(got) == set(want)
    check(got, oracle.solve(prob), TOL["fp64"])


def test_full_dense_batch_shape(api, plans):
    # the dense batch as measured: 64 instances of n=64, m=32, T=8192; two
    # instances checked against the oracle, every status checked
    probs = [inputs.dense_problem(64, 32, 8192, instance=i) for i in range(64)]
    _say("dense batch 64 x T=8192 (fp64)")
    dos = run(api, plans["fp64"], probs, "fp64")
    assert all(int(d.status.item()) == 0 for d in dos)
    for i in (0, 63):
        errs = check(dos[i].host(), oracle.solve(probs[i]), TOL["fp64"])
        _say("instance", i, "max rel err", max(errs.values()))


def test_mixed_classes_equal_alone(api, plans):
    probs = [inputs.dense_problem(64, 32, 150, instance=1), inputs.random_problem(12, 6, 200, seed=3),
             inputs.random_problem(50, 25, 77, seed=4, p=50, pT=50), inputs.tracking_problem(n=4, m=2, T=9000),
             inputs.random_problem(3, 2, 40, seed=5)]
    _say("classes 64, 16, 64, lane path, 8 in one call")
    dos = run(api, plans["fp64"], probs, "fp64")
    for i, (p, do) in enumerate(zip(probs, dos)):
        assert int(do.status.item()) == 0
        got = do.host()
        check(got, oracle.solve(p), TOL["fp64"])
        alone = run(api, plans["fp64"], [p], "fp64")[0].host()
        for f in FAMILIES:
            assert np.array_equal(got[f], alone[f]), (i, f)


def test_status_and_limits(api, plans):
    from paper_2104_03186_amd import _lib

    bad = inputs.dense_problem(64, 32, 50, instance=2)
    bad.U = -np.eye(32)
    nan = inputs.dense_problem(64, 32, 50, instance=3)
    nan.r[20, 5] = np.nan
    good = inputs.dense_problem(64, 32, 50, instance=4)
    _say("dense status codes")
    dos = run(api, plans["fp64"], [bad, nan, good], "fp64")
    assert [int(d.status.item()) for d in dos] == [3, 4, 0]
    check(dos[2].host(), oracle.solve(good), TOL["fp64"])
    # above the class limits: nu > 32 with nx > 32, per-step F with nx > 32
    wide = inputs.random_problem(40, 33, 10, seed=6)
    varying = inputs.random_problem(40, 8, 10, seed=7, per_step=1)
    big = api.Plan(64, 64, prec="fp64")
    try:
        for p in (wide, varying):
            with pytest.raises(_lib.LQTError) as e:
                run(api, big, [p], "fp64")
            assert e.value.code == _lib.ENOTSUP
    finally:
        big.close()
