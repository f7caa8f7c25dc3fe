"""GPU parity: the HIP path through the C ABI against the FP64 CPU oracle.

Tolerance: relative error per output family, over all steps stacked (Frobenius) and
per step (largest step error against the RMS step size; tests/helpers.err), <= 1e-10 for every
family (S, v, K, d, x, u) of the FP64 path.  Inputs are the seeded generators; every case prints
its parameters before touching the GPU.
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
    p = api.Plan(4, 4, prec="fp64", device=0)
    yield p
    p.close()


@pytest.fixture(autouse=True)
def _small_path(plan):
    """These tests exercise the lane-per-element path (n <= 4) at every T."""
    plan.set_routing(path="small")
    yield
    plan.set_routing()


def solve(api, plan, prob, want=FAMILIES, chunk=None):
    import torch

    plan.set_routing(path="small", lane_chunk=chunk or 0)
    dp = api.DeviceProblem(prob)
    do = api.DeviceOutputs(prob.n, prob.m, prob.T, want=want)
    plan.solve([dp], [do])
    torch.cuda.synchronize()
    return do


def assert_parity(got: dict, ref: dict, tol=TOL):
    errs = {f: err(got[f], ref[f]) for f in got}
    bad = {f: e for f, e in errs.items() if not e <= tol}
    assert not bad, f"rel errors above {tol}: {bad} (all: {errs})"
    return errs


T_SET = [1, 2, 3, 5, 63, 64, 65, 127, 128, 129, 1000, 4095, 4096, 4097, 20000]


@pytest.mark.parametrize("T", T_SET)
def test_tracking_default_chunk(api, plan, T):
    _say("tracking n=4 m=2 T=", T)
    prob = inputs.tracking_problem(n=4, m=2, T=T)
    do = solve(api, plan, prob)
    assert int(do.status.item()) == 0
    assert_parity(do.host(), oracle.solve(prob))


@pytest.mark.parametrize("chunk", [1, 3, 4, 8, 16, 33])
@pytest.mark.parametrize("T", [1, 7, 64, 65, 1000, 4097, 20000])
def test_tracking_chunk_sizes(api, plan, T, chunk):
    _say("tracking n=4 m=2 T=", T, "chunk=", chunk)
    prob = inputs.tracking_problem(n=4, m=2, T=T, instance=1)
    do = solve(api, plan, prob, chunk=chunk)
    assert int(do.status.item()) == 0
    assert_parity(do.host(), oracle.solve(prob))


DIMS = [(1, 1), (2, 1), (2, 2), (3, 1), (3, 2), (3, 3), (4, 1), (4, 2), (4, 3), (4, 4)]


@pytest.mark.parametrize("T,chunk", [(16384, 1), (16385, 1), (16448, 1), (32769, 1), (49152, 1), (2_000_000, 2),
                                     (4_195_304, 1)])
def test_top_level_blocks(api, plan, T, chunk):
    """Wavefront-unit counts (64 chunks each) around the 256-unit blocks of
    the backward top levels: exactly one block, one unit more, several blocks
    with a ragged last one, and more than 256 blocks (several block totals per
    thread of the top scan)."""
    _say("tracking n=4 m=2 T=", T, "chunk=", chunk, "units=", -(-(-(-T // chunk)) // 64))
    prob = inputs.tracking_problem(n=4, m=2, T=T, instance=2)
    do = solve(api, plan, prob, chunk=chunk)
    assert int(do.status.item()) == 0
    assert_parity(do.host(), oracle.solve(prob))


@pytest.mark.parametrize("per_step", [0, 1 | 2 | 4 | 8 | 16 | 32, 1 | 8, 2])
@pytest.mark.parametrize("nm", DIMS)
def test_random_problems(api, plan, nm, per_step):
    n, m = nm
    for T, p, pT in ((7, max(1, n - 1), n), (300, n, max(1, n - 1))):
        _say("random n=", n, "m=", m, "T=", T, "p=", p, "pT=", pT, "per_step=", per_step)
        prob = inputs.random_problem(n, m, T, seed=100 * n + 10 * m + per_step % 7, p=p, pT=pT,
                                     per_step=per_step, scale=0.95)
        do = solve(api, plan, prob, chunk=3)
        assert int(do.status.item()) == 0
        assert_parity(do.host(), oracle.solve(prob))


def test_full_size_single_instance(api, plan):
    T = 1_000_000
    _say("tracking n=4 m=2 T=", T, "(full size, default launch configuration)")
    prob = inputs.tracking_problem(n=4, m=2, T=T, workload=1)
    do = solve(api, plan, prob)
    assert int(do.status.item()) == 0
    errs = assert_parity(do.host(), oracle.solve(prob))
    _say("max rel err", max(errs.values()))


@pytest.mark.parametrize("want", [("K", "d", "x", "u"), ("S", "v", "K", "d"), ("S", "v", "x", "u"), ("x",),
                                  ("S",)])
def test_optional_outputs(api, plan, want):
    _say("outputs", want)
    prob = inputs.random_problem(3, 2, 500, seed=5, p=2)
    do = solve(api, plan, prob, want=want, chunk=4)
    assert int(do.status.item()) == 0
    got = do.host()
    assert set(got) == set(want)
    assert_parity(got, oracle.solve(prob))


def test_deterministic(api, plan):
    _say("determinism T=50000")
    prob = inputs.tracking_problem(n=4, m=2, T=50000)
    a = solve(api, plan, prob).host()
    b = solve(api, plan, prob).host()
    for f in FAMILIES:
        assert np.array_equal(a[f], b[f]), f


def test_batch_call_equals_single(api, plan):
    import torch

    _say("two instances in one lqt_solve call")
    probs = [inputs.tracking_problem(n=4, m=2, T=3000, instance=i) for i in range(2)]
    probs.append(inputs.random_problem(2, 1, 777, seed=9))
    dps = [api.DeviceProblem(p) for p in probs]
    dos = [api.DeviceOutputs(p.n, p.m, p.T) for p in probs]
    plan.solve(dps, dos)
    torch.cuda.synchronize()
    for p, do in zip(probs, dos):
        assert int(do.status.item()) == 0
        single = solve(api, plan, p).host()
        got = do.host()
        for f in FAMILIES:
            assert np.array_equal(got[f], single[f])
        assert_parity(got, oracle.solve(p))


def test_status_not_positive_definite(api, plan):
    _say("U not positive definite")
    prob = inputs.random_problem(3, 2, 100, seed=2)
    prob.U = -np.eye(2)
    do = solve(api, plan, prob)
    assert int(do.status.item()) == 3   # LQT_ENOTPD


def test_status_nonfinite(api, plan):
    _say("NaN in the reference")
    prob = inputs.tracking_problem(n=4, m=2, T=500)
    prob.r[123, 1] = np.nan
    do = solve(api, plan, prob)
    assert int(do.status.item()) == 4   # LQT_ENONFINITE


def test_failing_instance_is_isolated(api, plan):
    import torch

    _say("bad instance next to a good one")
    good = inputs.tracking_problem(n=4, m=2, T=2000)
    bad = inputs.tracking_problem(n=4, m=2, T=2000, instance=3)
    bad.r[5, 0] = np.inf
    dps = [api.DeviceProblem(good), api.DeviceProblem(bad)]
    dos = [api.DeviceOutputs(4, 2, 2000), api.DeviceOutputs(4, 2, 2000)]
    plan.solve(dps, dos)
    torch.cuda.synchronize()
    assert int(dos[0].status.item()) == 0 and int(dos[1].status.item()) == 4
    assert_parity(dos[0].host(), oracle.solve(good))


def test_argument_errors(api, plan):
    from paper_2104_03186_amd import _lib

    _say("argument validation")
    prob = inputs.tracking_problem(n=4, m=2, T=10)
    dp = api.DeviceProblem(prob)
    do = api.DeviceOutputs(4, 2, 10)
    dp.T = 0
    with pytest.raises(_lib.LQTError) as e:
        plan.solve([dp], [do])
    assert e.value.code == _lib.EINVAL
    dp.T = 10
    dp.t["F"] = None
    with pytest.raises(_lib.LQTError) as e:
        plan.solve([dp], [do])
    assert e.value.code == _lib.EINVAL
    small = api.Plan(2, 1)
    with pytest.raises(_lib.LQTError) as e:
        small.solve([api.DeviceProblem(prob)], [do])
    assert e.value.code == _lib.EINVAL
    small.close()


def test_submit_poll(api, plan):
    import time

    _say("submit/poll")
    probs = [inputs.tracking_problem(n=4, m=2, T=T, instance=i) for i, T in enumerate((100, 5000, 40000))]
    dps = [api.DeviceProblem(p) for p in probs]
    dos = [api.DeviceOutputs(p.n, p.m, p.T) for p in probs]
    tickets = [plan.submit(dp, do) for dp, do in zip(dps, dos)]
    done = {}
    t0 = time.time()
    while len(done) < len(tickets) and time.time() - t0 < 60:
        for t in tickets:
            if t not in done:
                st = plan.poll(t)
                if st is not None:
                    done[t] = st
    assert all(v == 0 for v in done.values()) and len(done) == 3
    for p, do in zip(probs, dos):
        assert_parity(do.host(), oracle.solve(p))
