"""GPU parity of the finite state and control solve (Section III-D):
lqt_fs_solve against the oracle's sequential dynamic programme (pinned in
tests/test_finite_pins.py).

Integer-valued costs make every min-plus sum exact, so the values, the
control law (smallest minimising index), the trajectory and the applied
controls are compared bit for bit: the routing workload of the finite-state
experiment (D_x = 5, 11, 21 as in Section VI-D) and random tables (per-step
and shared, blocked controls, D_x and D_u up to 32), at horizons around the
chunk and group boundaries and at T = 10^5.  With real-valued costs the
association order of the scan changes the rounding: values are compared to
1e-12 relative, and the control law is checked to attain the minimum.
"""
import sys

import numpy as np
import pytest

from oracle import finite
from paper_2104_03186_amd import inputs

pytestmark = pytest.mark.gpu


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


def run(api, plan, prob, want=("V", "u", "x", "ux")):
    import torch

    dp = api.DeviceFSProblem(prob)
    do = api.DeviceFSOutputs(prob.nstates, prob.T, want=want)
    plan.fs_solve(dp, do)
    torch.cuda.synchronize()
    return do.host(), int(do.status.item())


def exact(got, ref):
    for f, g in got.items():
        assert np.array_equal(g, ref[f]), (f, np.argwhere(g != ref[f])[:5])


@pytest.mark.parametrize("D", [5, 11, 21])
@pytest.mark.parametrize("T", [1, 2, 15, 16, 17, 255, 256, 257, 4095, 4097, 65536, 100_000])
def test_routing(api, plan, D, T):
    _say("routing D=", D, "T=", T)
    prob = inputs.routing_problem(T, nstates=D, seed=T % 13 + D)
    got, st = run(api, plan, prob)
    assert st == 0
    exact(got, finite.solve(prob))


@pytest.mark.parametrize("D,Du", [(1, 1), (2, 3), (7, 4), (16, 16), (32, 32), (32, 1), (3, 32)])
@pytest.mark.parametrize("per_step", [0, 1, 2, 3])
def test_random_tables(api, plan, D, Du, per_step):
    for T in (37, 5000):
        _say("random tables D=", D, "Du=", Du, "per_step=", per_step, "T=", T)
        prob = inputs.random_finite_problem(T, D, Du, seed=D * 100 + Du + per_step + T, per_step=per_step)
        got, st = run(api, plan, prob)
        ref = finite.solve(prob)
        assert st == (0 if np.isfinite(ref["V"][0, prob.x0]) else 4)
        exact(got, ref)


@pytest.mark.parametrize("want", [("V",), ("u",), ("x",), ("ux",), ("x", "ux"), ("V", "x")])
def test_partial_outputs(api, plan, want):
    prob = inputs.routing_problem(3000, nstates=11, seed=5)
    _say("routing outputs", want)
    got, st = run(api, plan, prob, want=want)
    assert st == 0 and set(got) == set(want)
    exact(got, finite.solve(prob))


def test_no_admissible_path(api, plan):
    prob = inputs.random_finite_problem(300, 6, 3, seed=4, per_step=0)
    prob.next[prob.x0, :] = -1  # no control leaves x0
    _say("finite state: blocked start")
    got, st = run(api, plan, prob)
    ref = finite.solve(prob)
    assert st == 4
    exact(got, ref)
    assert np.all(got["x"][1:] == -1) and np.all(got["ux"] == -1)


def test_real_costs(api, plan):
    prob = inputs.random_finite_problem(20000, 12, 5, seed=6, per_step=3, integer=False, p_blocked=0.1)
    _say("finite state: real-valued costs")
    got, st = run(api, plan, prob)
    ref = finite.solve(prob)
    assert st == 0
    V, U = got["V"], got["u"]
    fin = np.isfinite(ref["V"])
    assert np.array_equal(np.isfinite(V), fin)
    assert np.max(np.abs(V[fin] - ref["V"][fin]) / np.abs(ref["V"][fin])) <= 1e-12
    # the control law attains the minimum of its own values
    for k in (0, 1, 777, 19999):
        nxt, cst = finite._step_tables(prob, k)
        for i in range(prob.nstates):
            if U[k, i] >= 0:
                val = cst[i, U[k, i]] + V[k + 1, nxt[i, U[k, i]]]
                assert abs(val - V[k, i]) <= 1e-12 * abs(V[k, i])


def test_argument_errors(api, plan):
    from paper_2104_03186_amd import _lib

    prob = inputs.routing_problem(50, nstates=5)
    dp = api.DeviceFSProblem(prob)
    do = api.DeviceFSOutputs(5, 50)
    _say("finite state argument errors")
    lib = _lib.load()
    for field, val in (("nstates", 33), ("ncontrols", 0), ("x0", 5), ("per_step", 4), ("T", 0)):
        s = dp.struct()
        setattr(s, field, val)
        assert lib.lqt_fs_solve(plan.handle, s, do.struct(), None) == _lib.EINVAL, field
