"""GPU parity of the roll-out (u_k = d_k - K_k x_k, x_{k+1} = F x_k + L u_k +
c_k, Section II-B) on every chunked engine at state and control dimensions
that leave the padded blocks partly empty: the products of a step are split
over groups of lanes per row, so rows and terms beyond n and m must contribute
nothing.  Each class of the wavefront engine (8, 16, 32; time-varying data)
and of the workgroup engines (16, 32 with 16- and 32-wide control blocks,
64), offsets c on and off, FP64 and MIXED, against the FP64 oracle.

Tolerance: tests/helpers.err (stacked and per step), 1e-10 (FP64), 1e-5
(MIXED).
"""
import sys

import pytest

import oracle
from paper_2104_03186_amd import inputs
from tests.helpers import err

pytestmark = pytest.mark.gpu

TOL = {"fp64": 1e-10, "mixed": 1e-5}
T = 16 * 37 + 5

SHAPES = {
    "wave8": lambda: inputs.random_problem(5, 2, T, seed=201, scale=0.95),
    "wave16_varying": lambda: inputs.random_problem(13, 5, T, seed=202, per_step=1, scale=0.95),
    "wave32_varying": lambda: inputs.random_problem(30, 9, T, seed=203, per_step=4, scale=0.95),
    "block16": lambda: inputs.random_problem(13, 5, T, seed=204, scale=0.95),
    "block16_no_offsets": lambda: inputs.random_problem(11, 7, T, seed=205, with_c=False, scale=0.95),
    "block32_m16": lambda: inputs.random_problem(27, 11, T, seed=206, scale=0.95),
    "block32": lambda: inputs.random_problem(29, 23, T, seed=207, scale=0.95),
    "block64": lambda: inputs.random_problem(61, 29, T, seed=208, scale=0.95),
}


@pytest.fixture(scope="module")
def api():
    import torch

    assert torch.cuda.is_available(), "GPU tests need a GPU"
    from paper_2104_03186_amd import api as _api

    return _api


@pytest.mark.parametrize("prec", ["fp64", "mixed"])
@pytest.mark.parametrize("name", list(SHAPES))
def test_rollout_partly_empty_blocks(api, name, prec):
    import torch

    prob = SHAPES[name]()
    print("[case] roll-out", name, prec, "n", prob.n, "m", prob.m, "T", prob.T, flush=True)
    sys.stdout.flush()
    plan = api.Plan(64, 32, prec=prec)
    try:
        plan.set_routing(wave_chunk=16)
        dt = torch.float64 if prec == "fp64" else torch.float32
        dp = api.DeviceProblem(prob)
        do = api.DeviceOutputs(prob.n, prob.m, prob.T, dtype=dt)
        plan.solve([dp], [do])
        torch.cuda.synchronize()
        assert int(do.status.item()) == 0
        got = do.host()
    finally:
        plan.close()
    ref = oracle.solve(prob)
    errs = {f: err(got[f], ref[f]) for f in ("x", "u", "K", "d")}
    assert max(errs.values()) <= TOL[prec], errs
