"""GPU test of the chunk-length autotuner (lqt_tune): the chosen lengths come
from the candidate set, results of the tuned plan stay within the FP64
tolerance of the oracle, and a result is the same alone and in a batch."""
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


def test_tuned_plan():
    import torch

    assert torch.cuda.is_available()
    from paper_2104_03186_amd import api

    probs = [inputs.diag_problem(n, n // 2, T, 2, i) for i, (n, T) in
             enumerate([(4, 700), (8, 3000), (16, 2500), (16, 900), (6, 4000)])]
    probs.append(inputs.random_problem(12, 5, 800, seed=3, per_step=4))  # wavefront engine, class 16
    probs.append(inputs.dense_problem(64, 32, 600, instance=9))
    plan = api.Plan(64, 32, prec="fp64")
    dps = [api.DeviceProblem(p) for p in probs]
    dos = [api.DeviceOutputs(p.n, p.m, p.T) for p in probs]
    _say("tune on", len(probs), "instances")
    chosen = plan.tune(dps, dos)
    _say("chosen divisors", chosen)
    assert all(c in (0, 1, 4, 16, 64, 256) for c in chosen)
    assert any(c != 0 for c in chosen)
    plan.solve(dps, dos)
    torch.cuda.synchronize()
    for i, (p, do) in enumerate(zip(probs, dos)):
        assert int(do.status.item()) == 0
        got = do.host()
        ref = oracle.solve(p)
        errs = {f: err(got[f], ref[f]) for f in FAMILIES}
        assert max(errs.values()) <= TOL, (i, errs)
        if i % 3 == 0:
            alone = api.DeviceOutputs(p.n, p.m, p.T)
            plan.solve([dps[i]], [alone])
            torch.cuda.synchronize()
            a = alone.host()
            for f in FAMILIES:
                assert np.array_equal(got[f], a[f]), (i, f)
    plan.close()
