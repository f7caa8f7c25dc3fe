"""GPU parity of the MIXED precision mode (float results) against the FP64
oracle, on both pipelines.

Tolerance: relative error per output family, over all steps stacked (Frobenius) and
per step (largest step error against the RMS step size; tests/helpers.err), <= 1e-5.  MIXED keeps
the scan arithmetic in double and rounds the stored results to float, so the
expected error is the float rounding of the results (about 6e-8) plus, for x
and u, the effect of the rounded gains on the roll-out.
"""
import sys

import numpy as np
import pytest

import oracle
from paper_2104_03186_amd import inputs
from tests.helpers import FAMILIES, err

pytestmark = pytest.mark.gpu

TOL = 1e-5


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
    p = api.Plan(32, 32, prec="mixed", device=0)
    yield p
    p.close()


@pytest.fixture(autouse=True)
def _routing(plan):
    yield
    plan.set_routing()


def run(api, plan, probs, want=FAMILIES, path=None):
    import torch

    plan.set_routing(path=path)
    dps = [api.DeviceProblem(p) for p in probs]
    dos = [api.DeviceOutputs(p.n, p.m, p.T, want=want, dtype=torch.float32) for p in probs]
    plan.solve(dps, dos)
    torch.cuda.synchronize()
    for do in dos:
        for t in do.t.values():
            if t is not None:
                assert t.dtype == torch.float32
    return dos


def check(got: dict, ref: dict, tol=TOL):
    errs = {f: err(got[f], ref[f]) for f in got}
    bad = {f: e for f, e in errs.items() if not e <= tol}
    assert not bad, f"rel errors above {tol}: {bad} (all: {errs})"
    return errs


@pytest.mark.parametrize("T", [1, 2, 65, 1000, 4097, 20000])
def test_small_path_tracking(api, plan, T):
    _say("mixed small path tracking n=4 m=2 T=", T)
    prob = inputs.tracking_problem(n=4, m=2, T=T)
    do = run(api, plan, [prob], path="small")[0]
    assert int(do.status.item()) == 0
    check(do.host(), oracle.solve(prob))


@pytest.mark.parametrize("nm", [(1, 1), (2, 1), (3, 2), (3, 3), (4, 1), (4, 3)])
@pytest.mark.parametrize("per_step", [0, 63])
def test_small_path_dims(api, plan, nm, per_step):
    n, m = nm
    _say("mixed small path n=", n, "m=", m, "per_step=", per_step)
    prob = inputs.random_problem(n, m, 300, seed=11 * n + m, p=n, pT=max(1, n - 1), per_step=per_step, scale=0.95)
    do = run(api, plan, [prob], path="small")[0]
    assert int(do.status.item()) == 0
    check(do.host(), oracle.solve(prob))


def test_small_path_full_size(api, plan):
    T = 1_000_000
    _say("mixed small path tracking n=4 m=2 T=", T, "(full size, default launch configuration)")
    prob = inputs.tracking_problem(n=4, m=2, T=T, workload=1)
    do = run(api, plan, [prob])[0]
    assert int(do.status.item()) == 0
    errs = check(do.host(), oracle.solve(prob))
    _say("max rel err", max(errs.values()))


@pytest.mark.parametrize("nm", [(2, 1), (5, 2), (8, 4), (12, 6), (16, 8), (24, 12), (32, 16)])
def test_wave_path_dims(api, plan, nm):
    n, m = nm
    for T in (1, 37, 300):
        _say("mixed wave path n=", n, "m=", m, "T=", T)
        prob = inputs.random_problem(n, m, T, seed=3 * n + m + T, p=max(1, n - 1), pT=n, scale=0.95)
        do = run(api, plan, [prob], path="wave")[0]
        assert int(do.status.item()) == 0
        check(do.host(), oracle.solve(prob))


def test_wave_path_time_varying(api, plan):
    prob = inputs.random_problem(6, 3, 150, seed=8, p=5, pT=6, per_step=63, scale=0.95)
    _say("mixed wave path time-varying n=6 m=3")
    do = run(api, plan, [prob], path="wave")[0]
    assert int(do.status.item()) == 0
    check(do.host(), oracle.solve(prob))


@pytest.mark.parametrize("n", [4, 8, 16])
def test_batched_workload_instances(api, plan, n):
    shapes = [(nn, T) for nn, T in inputs.batched_shapes(4096) if nn == n][:12]
    probs = [inputs.diag_problem(nn, nn // 2, T, 2, i) for i, (nn, T) in enumerate(shapes)]
    _say("mixed batched-workload instances n=", n, "count=", len(probs))
    dos = run(api, plan, probs)
    for p, do in zip(probs, dos):
        assert int(do.status.item()) == 0
        check(do.host(), oracle.solve(p))


def test_mixed_batch_equals_alone(api, plan):
    rng = np.random.default_rng(17)
    probs = []
    for i in range(24):
        n = int(rng.integers(1, 17))
        m = int(rng.integers(1, n + 1))
        T = int(rng.integers(1, 300))
        probs.append(inputs.random_problem(n, m, T, seed=2000 + i, p=n, pT=n, scale=0.9))
    probs.append(inputs.tracking_problem(n=4, m=2, T=9000, instance=4))
    _say("mixed-precision batch of", len(probs))
    dos = run(api, plan, probs)
    for i, (p, do) in enumerate(zip(probs, dos)):
        assert int(do.status.item()) == 0
        got = do.host()
        check(got, oracle.solve(p))
        if i % 6 == 0 or i == len(probs) - 1:
            alone = run(api, plan, [p])[0].host()
            for f in FAMILIES:
                assert np.array_equal(got[f], alone[f]), (i, f)


@pytest.mark.parametrize("want", [("K", "d", "x", "u"), ("S", "v"), ("x", "u")])
def test_optional_outputs(api, plan, want):
    for path, prob in (("small", inputs.random_problem(3, 2, 500, seed=5, p=2)),
                       ("wave", inputs.random_problem(8, 4, 90, seed=4))):
        _say("mixed outputs", want, "path", path)
        do = run(api, plan, [prob], want=want, path=path)[0]
        assert int(do.status.item()) == 0
        got = do.host()
        assert set(got) == set(want)
        check(got, oracle.solve(prob))


def test_status_codes(api, plan):
    bad_pd = inputs.random_problem(6, 3, 150, seed=2)
    bad_pd.U = -np.eye(3)
    bad_nan = inputs.tracking_problem(n=4, m=2, T=9000)
    bad_nan.r[50, 0] = np.nan
    good = inputs.random_problem(5, 2, 100, seed=3)
    _say("mixed status codes")
    dos = run(api, plan, [bad_pd, bad_nan, good])
    assert int(dos[0].status.item()) == 3
    assert int(dos[1].status.item()) == 4
    assert int(dos[2].status.item()) == 0
    check(dos[2].host(), oracle.solve(good))
