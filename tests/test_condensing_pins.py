"""Partial condensing (Section V-C) as set up by the benchmark's condensing
experiment: the condensed LQT over the block boundaries, with the block's
controls stacked and the block's stage costs written as the generalised stage
cost of Section IV-D, has the original optimum -- S, v and x at the block
boundaries and every control -- as the oracle solves both (the original with
the standard recursion, the condensed one with the generalised-cost
recursion)."""
import numpy as np
import pytest

import oracle
from bench import condensed_problem
from paper_2104_03186_amd import inputs


@pytest.mark.parametrize("B", [1, 2, 4, 8, 16])
@pytest.mark.parametrize("kind", ["tracking", "offsets_general_output"])
def test_condensed_optimum_equals_original(B, kind):
    if kind == "tracking":
        prob = inputs.tracking_problem(n=4, m=2, T=64, workload=1)
    else:
        prob = inputs.random_problem(3, 2, 48, seed=9, p=4, pT=3, with_c=True)
    ref = oracle.solve(prob)
    cp = condensed_problem(prob, B)
    assert (cp.T, cp.m, cp.p) == (prob.T // B, prob.m * B, prob.p * B)
    got = oracle.solve(cp)
    scale = max(1.0, float(np.abs(ref["S"]).max()))
    assert np.abs(got["S"] - ref["S"][::B]).max() <= 1e-11 * scale
    assert np.abs(got["v"] - ref["v"][::B]).max() <= 1e-11 * max(1.0, float(np.abs(ref["v"]).max()))
    assert np.abs(got["x"] - ref["x"][::B]).max() <= 1e-11 * max(1.0, float(np.abs(ref["x"]).max()))
    assert np.abs(got["u"].reshape(prob.T, prob.m) - ref["u"]).max() <= 1e-11 * max(1.0, float(np.abs(ref["u"]).max()))


def test_condensing_rejects_what_it_cannot_condense():
    prob = inputs.tracking_problem(n=4, m=2, T=10, workload=1)
    with pytest.raises(ValueError):
        condensed_problem(prob, 4)  # B does not divide T
    tv = inputs.random_problem(3, 2, 16, seed=1, per_step=1)
    with pytest.raises(ValueError):
        condensed_problem(tv, 4)  # per-step dynamics
