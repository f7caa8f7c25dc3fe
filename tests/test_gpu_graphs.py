"""Graph replay (lqt_set_graphs): a recorded call replayed several times,
with eager work and synchronisations between the replays and the input data
changed in place between them, equals the same call made directly on the
same data, bit for bit, every time -- for a batch that spans every path
(batched lane kernel, lane pipeline, wavefront and workgroup engines, the
chunk elements of a long instance scanned as a tree), for
the iterated linearisation of the nonlinear extension (Section IV-D) on the
lane pipeline and on the wavefront engine, and with the forward-prefix
trajectory (its element scan on a second stream).
"""
import sys

import numpy as np
import pytest

import oracle
from paper_2104_03186_amd import inputs
from tests.helpers import FAMILIES, err

pytestmark = pytest.mark.gpu

REPLAYS = 4


def _say(*a):
    print("[case]", *a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def api():
    import torch

    assert torch.cuda.is_available(), "GPU tests need a GPU"
    from paper_2104_03186_amd import api as _api

    return _api


def batch_problems():
    return [inputs.tracking_problem(n=4, m=2, T=3000, instance=1),        # batched lane kernel
            inputs.tracking_problem(n=4, m=2, T=20000, instance=2),       # lane pipeline
            inputs.random_problem(6, 3, 700, seed=31),                    # wavefront engine, class 8
            inputs.diag_problem(16, 8, 1500, 2, 7),                       # workgroup engine, class 16
            inputs.random_problem(12, 5, 400, seed=32, per_step=1 | 2),   # wavefront engine, per-step
            inputs.random_problem(3, 2, 900, seed=33),                    # batched lane kernel, offsets
            inputs.diag_problem(12, 6, 17000, 2, 8)]                      # workgroup engine, chunk tree


@pytest.mark.parametrize("traj", ["maps", "prefix"])
def test_batch_replays_equal_direct(api, traj):
    import torch

    probs = batch_problems()
    graph_plan = api.Plan(16, 8, prec="fp64", trajectory=traj)
    direct_plan = api.Plan(16, 8, prec="fp64", trajectory=traj)
    graph_plan.set_graphs(True)
    try:
        dps = [api.DeviceProblem(p) for p in probs]
        g_out = [api.DeviceOutputs(p.n, p.m, p.T) for p in probs]
        d_out = [api.DeviceOutputs(p.n, p.m, p.T) for p in probs]
        other = inputs.random_problem(5, 2, 300, seed=34)
        dpo, doo = api.DeviceProblem(other), api.DeviceOutputs(5, 2, 300)
        for rep in range(REPLAYS + 1):  # the first call records, the others replay
            _say("batch", traj, "call", rep)
            graph_plan.solve(dps, g_out)
            torch.cuda.synchronize()
            assert graph_plan.graphs_recorded() == 1  # recorded once, then replayed
            direct_plan.solve(dps, d_out)
            direct_plan.solve([dpo], [doo])  # eager work between the replays
            torch.cuda.synchronize()
            for i, (a, b) in enumerate(zip(g_out, d_out)):
                assert int(a.status.item()) == 0, (rep, i)
                ga, gb = a.host(), b.host()
                for f in FAMILIES:
                    assert np.array_equal(ga[f], gb[f]), (rep, i, f)
            if rep == REPLAYS:  # the last replay against the oracle on the data it saw
                for i in (0, 2, 3, 6):
                    ref = oracle.solve(probs[i])
                    got = g_out[i].host()
                    assert max(err(got[f], ref[f]) for f in FAMILIES) <= 1e-10, i
            # new data in the same buffers: the references move
            for p, dp in zip(probs, dps):
                dp.t["r"].mul_(1.05).add_(0.01)
                p.r = p.r * 1.05 + 0.01
    finally:
        graph_plan.close()
        direct_plan.close()


@pytest.mark.parametrize("path,T,traj", [("small", 20001, "maps"), ("wave", 2049, "maps"),
                                         ("small", 9000, "prefix")])
def test_nonlinear_replays_equal_direct(api, path, T, traj):
    import torch

    prob = inputs.unicycle_problem(T, seed=5)
    rounds = 4
    plans = {k: api.Plan(4, 2, prec="fp64", trajectory=traj) for k in ("graph", "direct")}
    plans["graph"].set_graphs(True)
    try:
        for p in plans.values():
            p.set_routing(path=path)
        dp = api.DeviceNLProblem(prob)
        x0 = torch.from_numpy(prob.xbar).cuda()
        u0 = torch.from_numpy(prob.ubar).cuda()
        res = {}
        for k, p in plans.items():
            res[k] = (x0.clone(), u0.clone(), torch.zeros(rounds, dtype=torch.float64, device="cuda:0"),
                      torch.full((1,), -1, dtype=torch.int32, device="cuda:0"))
        for rep in range(REPLAYS + 1):
            _say("nonlinear", path, "T=", T, traj, "call", rep)
            for k, p in plans.items():
                x, u, ch, st = res[k]
                x.copy_(x0)  # restore the nominal (eager work between the replays)
                u.copy_(u0)
                p.nl_iterate(dp, rounds, x, u, ch, st)
                torch.cuda.synchronize()
            assert plans["graph"].graphs_recorded() == 1 and plans["direct"].graphs_recorded() == 0
            for a, b in zip(res["graph"], res["direct"]):
                assert torch.equal(a, b), rep
            assert int(res["graph"][3].item()) == 0
            u0.mul_(0.9)  # a new nominal in the same buffer
    finally:
        for p in plans.values():
            p.close()
