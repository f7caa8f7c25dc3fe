"""The allocation-free entry point (lqt_solve_noalloc) against lqt_solve.

Two calls in a row on one plan through the C ABI, the second with a smaller
instance, each compared with lqt_solve of the same instance (the same
kernels and chunking: equal bit for bit) and with the oracle (the FP64 gate
of the parity tests); a generalised-cost instance, a wavefront-engine
instance, a long instance whose chunk elements are scanned as a tree, both
chunked engines with the chunk scans as trees by request, the operator form
of the fold on both chunked engines, and a MIXED plan; the size limit of the
static workspace.
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


def both(api, plan, prob, dtype, want=FAMILIES):
    """(lqt_solve_noalloc outputs, lqt_solve outputs) of one instance."""
    import torch

    dp = api.DeviceProblem(prob)
    a = api.DeviceOutputs(prob.n, prob.m, prob.T, dtype=dtype, want=want)
    b = api.DeviceOutputs(prob.n, prob.m, prob.T, dtype=dtype, want=want)
    plan.solve_noalloc(dp, a)
    torch.cuda.synchronize()
    plan.solve([dp], [b])
    torch.cuda.synchronize()
    assert int(a.status.item()) == 0 and int(b.status.item()) == 0
    return a.host(), b.host()


def check(got, alone, ref, tol):
    for f in got:
        assert np.array_equal(got[f], alone[f]), f
    errs = {f: err(got[f], ref[f]) for f in got}
    assert max(errs.values()) <= tol, errs


@pytest.mark.parametrize("prec", ["fp64", "mixed"])
def test_two_calls_second_smaller(api, prec):
    import torch

    dtype = torch.float64 if prec == "fp64" else torch.float32
    plan = api.Plan(8, 4, prec=prec)
    try:
        # lane pipeline at T = 1e6 (the caller takes K and d), then a smaller
        # instance on the wavefront engine
        first = inputs.tracking_problem(n=4, m=2, T=1_000_000, workload=1)
        _say("noalloc T=1e6 n=4", prec)
        got, alone = both(api, plan, first, dtype)
        check(got, alone, oracle.solve(first), TOL[prec])
        second = inputs.random_problem(6, 3, 3001, seed=12)
        _say("noalloc T=3001 n=6 (second, smaller)", prec)
        got, alone = both(api, plan, second, dtype)
        check(got, alone, oracle.solve(second), TOL[prec])
    finally:
        plan.close()


def test_generalised_and_workgroup_engine(api):
    import torch

    plan = api.Plan(16, 8, prec="fp64")
    try:
        for prob in (inputs.generalised_problem(4, 2, 9000, seed=21, p=3),
                     inputs.diag_problem(16, 8, 2000, 2, 5),
                     inputs.diag_problem(12, 6, 20000, 2, 6),  # 313 chunks: scanned as a tree
                     inputs.generalised_problem(12, 5, 700, seed=22, p=8, per_step=2)):
            _say("noalloc", prob.n, prob.m, prob.T)
            got, alone = both(api, plan, prob, torch.float64)
            check(got, alone, oracle.solve(prob), TOL["fp64"])
    finally:
        plan.close()


def test_forced_trees(api):
    """Routing tree=True: the chunk scans of both chunked engines as trees,
    the same with and without allocation."""
    import torch

    plan = api.Plan(16, 8, prec="fp64")
    try:
        plan.set_routing(tree=True)
        for prob in (inputs.diag_problem(16, 8, 2000, 2, 7), inputs.random_problem(6, 3, 3001, seed=13)):
            _say("noalloc with trees", prob.n, prob.m, prob.T)
            got, alone = both(api, plan, prob, torch.float64)
            check(got, alone, oracle.solve(prob), TOL["fp64"])
    finally:
        plan.close()


@pytest.mark.parametrize("tree", [None, True])
def test_operator_form_fold(api, tree):
    """Time-invariant instances without offsets: the operator form of the
    fold (one matrix fold per instance, then the vector recursion per chunk)
    on the wavefront engine (class 8) and the workgroup engine (class 16),
    chains and trees, the same with and without allocation."""
    import torch

    plan = api.Plan(16, 8, prec="fp64")
    try:
        plan.set_routing(tree=tree)
        for prob in (inputs.diag_problem(8, 4, 2000, 2, 5), inputs.random_problem(7, 3, 1500, seed=97, with_c=False,
                                                                                  scale=0.95),
                     inputs.diag_problem(16, 8, 2500, 2, 6)):
            _say("noalloc operator-form fold", prob.n, prob.m, prob.T, "tree", tree)
            got, alone = both(api, plan, prob, torch.float64)
            check(got, alone, oracle.solve(prob), TOL["fp64"])
    finally:
        plan.close()


def test_workspace_limit(api):
    import torch

    from paper_2104_03186_amd import _lib

    plan = api.Plan(4, 2, prec="fp64")
    try:
        # without K and d the gains go to workspace: T = 4e6 needs > 64 MiB
        prob = inputs.tracking_problem(n=4, m=2, T=4_000_000, workload=1)
        dp = api.DeviceProblem(prob)
        do = api.DeviceOutputs(4, 2, prob.T, want=("x", "u"))
        _say("noalloc over the limit")
        with pytest.raises(_lib.LQTError) as e:
            plan.solve_noalloc(dp, do)
        assert e.value.code == _lib.ENOMEM
        assert "static workspace" in str(e.value)
        torch.cuda.synchronize()
    finally:
        plan.close()
