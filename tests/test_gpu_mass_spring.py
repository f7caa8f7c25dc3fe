"""GPU parity on the state-dimension workload of Section VI-C: the chain of
N masses (n = 2N states, m = 2 forces) driven to the origin, N = 2..32
(n = 4..64: the batched lane kernel, the wavefront engine for class 8 and
the workgroup engines for classes 16, 32 and 64), T = 100 and 1000 steps
over the same 10 s horizon, against the FP64 oracle.

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


def _say(*a):
    print("[case]", *a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def api():
    import torch

    assert torch.cuda.is_available(), "GPU tests need a GPU"
    from paper_2104_03186_amd import api as _api

    return _api


@pytest.mark.parametrize("prec", ["fp64", "mixed"])
@pytest.mark.parametrize("T", [100, 1000])
@pytest.mark.parametrize("N", [2, 4, 8, 16, 32])
def test_mass_spring_chain(api, N, T, prec):
    import torch

    prob = inputs.mass_spring_problem(N, T)
    _say("mass-spring N=", N, "T=", T, prec)
    plan = api.Plan(64, 32, prec=prec, device=0)
    try:
        dt = torch.float64 if prec == "fp64" else torch.float32
        dp = api.DeviceProblem(prob)
        do = api.DeviceOutputs(prob.n, prob.m, T, dtype=dt)
        plan.solve([dp], [do])
        torch.cuda.synchronize()
        assert int(do.status.item()) == 0
        got, ref = do.host(), oracle.solve(prob)
        errs = {f: err(got[f], ref[f]) for f in got}
        assert max(errs.values()) <= TOL[prec], errs
    finally:
        plan.close()
