"""GPU parity of the chunked paths for n up to 32 (wavefront engine, and the
workgroup engine for time-invariant instances of the classes 16 and 32)
against the FP64 oracle, batched solves, and batch independence.

Tolerance: relative error per output family, over all steps stacked (Frobenius) and
per step (largest step error against the RMS step size; tests/helpers.err), <= 1e-10 (FP64).
"""
import sys

import numpy as np
import pytest

import oracle
from paper_2104_03186_amd import inputs
from tests.helpers import FAMILIES, err

pytestmark = pytest.mark.gpu

TOL = 1e-10


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
def plan(api):
    p = api.Plan(32, 32, prec="fp64", device=0)
    yield p
    p.close()


@pytest.fixture(autouse=True, params=["workgroup", "wavefront"])
def _engine(request, plan):
    """Every test runs twice: time-invariant instances of the classes 16 and
    32 on the workgroup engine (default routing) and on the wavefront
    engine (routing override)."""
    plan.engine = request.param
    plan.set_routing(path="wave", wave_engine_only=(request.param == "wavefront"))
    yield
    plan.set_routing()


def run(api, plan, probs, want=FAMILIES, chunk=None, path="wave"):
    import torch

    plan.set_routing(path=path, wave_engine_only=(plan.engine == "wavefront"), wave_chunk=chunk or 0)
    dps = [api.DeviceProblem(p) for p in probs]
    dos = [api.DeviceOutputs(p.n, p.m, p.T, want=want) for p in probs]
    plan.solve(dps, dos)
    torch.cuda.synchronize()
    return dos


def check(got: dict, ref: dict, tol=TOL):
    errs = {f: err(got[f], ref[f]) for f in got}
    bad = {f: e for f, e in errs.items() if not e <= tol}
    assert not bad, f"rel errors above {tol}: {bad} (all: {errs})"
    return errs


NM = [(1, 1), (2, 1), (3, 2), (4, 2), (5, 2), (5, 5), (6, 3), (8, 4), (8, 1), (12, 6), (16, 8), (16, 16),
      (24, 12), (32, 16), (7, 9), (20, 18), (32, 32)]


@pytest.mark.parametrize("nm", NM)
def test_random_dims(api, plan, nm):
    n, m = nm
    for T, chunk in ((1, None), (5, 2), (37, 4), (300, None)):
        _say("wave random n=", n, "m=", m, "T=", T, "chunk=", chunk)
        prob = inputs.random_problem(n, m, T, seed=7 * n + m + T, p=max(1, n - 1), pT=n, scale=0.95)
        do = run(api, plan, [prob], chunk=chunk)[0]
        assert int(do.status.item()) == 0
        check(do.host(), oracle.solve(prob))


@pytest.mark.parametrize("nm,T,chunk", [((12, 5), 300, None), ((16, 16), 257, 16), ((24, 12), 1000, None),
                                        ((32, 16), 333, 32), ((17, 3), 64, 1), ((20, 18), 129, 16),
                                        ((32, 32), 200, None), ((30, 9), 47, 64)])
def test_operator_form(api, plan, nm, T, chunk):
    """Instances without offsets: on the workgroup engines the chunk fold runs
    in operator form (matrix fold once per instance, vector part as a GEMM);
    classes 16, 32 (16- and 32-wide control blocks), ragged first chunks,
    one-step chunks, a chunk longer than the horizon."""
    n, m = nm
    _say("operator form n=", n, "m=", m, "T=", T, "chunk=", chunk)
    prob = inputs.random_problem(n, m, T, seed=31 * n + m + T, p=max(1, n - 2), pT=n, with_c=False, scale=0.95)
    do = run(api, plan, [prob], chunk=chunk)[0]
    assert int(do.status.item()) == 0
    check(do.host(), oracle.solve(prob))


@pytest.mark.parametrize("per_step", [1 | 2 | 4 | 8 | 16 | 32, 4 | 32, 8 | 16, 1])
def test_time_varying(api, plan, per_step):
    for n, m, p in ((3, 2, 2), (6, 3, 5), (9, 4, 9)):
        _say("wave time-varying n=", n, "m=", m, "p=", p, "per_step=", per_step)
        prob = inputs.random_problem(n, m, 120, seed=per_step + n, p=p, pT=n, per_step=per_step, scale=0.95)
        do = run(api, plan, [prob], chunk=7)[0]
        assert int(do.status.item()) == 0
        check(do.host(), oracle.solve(prob))


@pytest.mark.parametrize("n", [4, 8, 16])
def test_batched_workload_instances(api, plan, n):
    shapes = [(nn, T) for nn, T in inputs.batched_shapes(4096) if nn == n][:24]
    probs = [inputs.diag_problem(nn, nn // 2, T, 2, i) for i, (nn, T) in enumerate(shapes)]
    _say("batched-workload instances n=", n, "count=", len(probs), "steps=", sum(p.T for p in probs))
    dos = run(api, plan, probs)
    for p, do in zip(probs, dos):
        assert int(do.status.item()) == 0
        check(do.host(), oracle.solve(p))


def test_mixed_batch_equals_alone(api, plan):
    rng = np.random.default_rng(5)
    probs = []
    for i in range(40):
        n = int(rng.integers(1, 17))
        m = int(rng.integers(1, n + 1))
        T = int(rng.integers(1, 400))
        probs.append(inputs.random_problem(n, m, T, seed=1000 + i, p=n, pT=n, scale=0.9))
    _say("mixed batch of", len(probs))
    dos = run(api, plan, probs)
    for i, (p, do) in enumerate(zip(probs, dos)):
        assert int(do.status.item()) == 0
        got = do.host()
        check(got, oracle.solve(p))
        if i % 8 == 0:
            alone = run(api, plan, [p])[0].host()
            for f in FAMILIES:
                assert np.array_equal(got[f], alone[f]), (i, f)


def test_failures_are_isolated(api, plan):
    good = inputs.random_problem(6, 3, 200, seed=1)
    bad_pd = inputs.random_problem(6, 3, 150, seed=2)
    bad_pd.U = -np.eye(3)
    bad_nan = inputs.random_problem(5, 2, 100, seed=3)
    bad_nan.r[50, 0] = np.nan
    _say("failure isolation")
    dos = run(api, plan, [good, bad_pd, bad_nan])
    assert int(dos[0].status.item()) == 0
    assert int(dos[1].status.item()) == 3
    assert int(dos[2].status.item()) == 4
    check(dos[0].host(), oracle.solve(good))


@pytest.mark.parametrize("want", [("K", "d", "x", "u"), ("S", "v", "K", "d"), ("x", "u"), ("S", "v")])
def test_optional_outputs(api, plan, want):
    prob = inputs.random_problem(8, 4, 90, seed=4)
    _say("wave outputs", want)
    do = run(api, plan, [prob], want=want, chunk=8)[0]
    assert int(do.status.item()) == 0
    got = do.host()
    assert set(got) == set(want)
    check(got, oracle.solve(prob))


def test_auto_routing_long_small_instance(api, plan):
    # with no forced path an n = 4 instance of T >= 8192 takes the
    # lane-per-element path, a short one the wavefront path; both agree with
    # the oracle
    for T in (9000, 3000):
        prob = inputs.tracking_problem(n=4, m=2, T=T, instance=T)
        _say("auto routing T=", T)
        do = run(api, plan, [prob], path=None)[0]
        assert int(do.status.item()) == 0
        check(do.host(), oracle.solve(prob))
