"""GPU parity of the chunk scan as a tree on the chunked engines: instances
with at least 128 chunks form the value at every chunk start by recursive
doubling over their chunk elements (the parallel scan of Section II-C with
the general combination rule of Section IV-A, anchored on the terminal value
of Section IV-B) instead of walking the chunks in sequence.  Checked against
the FP64 oracle: every workgroup class (16, 32 in both control widths, 64)
and every wavefront class (8, 16, 32; time-varying data), the operator-form
fold and the per-chunk fold (offsets c), chunk counts around the tree's
level boundaries, MIXED, the generalised cost, forward prefixes (Method 2,
which reads the untouched chunk elements), the default chunking of long
instances, and a batch of tree and chain instances equal to each instance
alone, bit for bit.

Tolerance: tests/helpers.err (stacked and per step), 1e-10 (FP64), 1e-5
(MIXED).
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


def solve(api, probs, prec="fp64", chunk=16, trajectory="maps"):
    import torch

    plan = api.Plan(64, 32, prec=prec, device=0, trajectory=trajectory)
    try:
        plan.set_routing(wave_chunk=chunk)
        dt = torch.float64 if prec == "fp64" else torch.float32
        dps = [api.DeviceProblem(p) for p in probs]
        dos = [api.DeviceOutputs(p.n, p.m, p.T, dtype=dt) for p in probs]
        plan.solve(dps, dos)
        torch.cuda.synchronize()
        return [(int(o.status.item()), o.host()) for o in dos]
    finally:
        plan.close()


def check(got, ref, tol):
    errs = {f: err(got[f], ref[f]) for f in got}
    bad = {f: e for f, e in errs.items() if not e <= tol}
    assert not bad, f"errors above {tol}: {bad} (all: {errs})"


SHAPES = {
    "class16": lambda T: inputs.diag_problem(16, 8, T, 2, 3),
    "class16_offsets": lambda T: inputs.random_problem(12, 6, T, seed=91, scale=0.95),
    "class32": lambda T: inputs.random_problem(24, 20, T, seed=92, scale=0.95, with_c=False),
    "class32_m16": lambda T: inputs.random_problem(28, 12, T, seed=93, p=30, pT=20, scale=0.95),
    "class64": lambda T: inputs.dense_problem(64, 32, T, instance=1),
    "wave8": lambda T: inputs.random_problem(6, 3, T, seed=94, scale=0.95),
    "wave16_varying": lambda T: inputs.random_problem(12, 5, T, seed=95, per_step=1 | 2, scale=0.95),
    "wave32_varying": lambda T: inputs.random_problem(20, 9, T, seed=96, p=22, per_step=1 | 4, scale=0.95),
}


@pytest.mark.parametrize("name", list(SHAPES))
@pytest.mark.parametrize("T", [16 * 128, 16 * 129 + 5, 16 * 257 - 3])
def test_classes_and_level_boundaries(api, name, T):
    prob = SHAPES[name](T)
    _say("tree", name, "T=", T, "chunk 16")
    ((st, got),) = solve(api, [prob])
    assert st == 0
    check(got, oracle.solve(prob), TOL["fp64"])


@pytest.mark.parametrize("name", ["class16_offsets", "class64", "wave8", "wave16_varying"])
def test_mixed(api, name):
    prob = SHAPES[name](16 * 140)
    _say("tree mixed", name)
    ((st, got),) = solve(api, [prob], prec="mixed")
    assert st == 0
    check(got, oracle.solve(prob), TOL["mixed"])


def test_generalised_cost(api):
    prob = inputs.generalised_problem(20, 10, 16 * 150, seed=7, p=24)
    _say("tree generalised cost")
    ((st, got),) = solve(api, [prob])
    assert st == 0
    check(got, oracle.solve(prob), TOL["fp64"])


@pytest.mark.parametrize("name", ["class16", "class32_m16", "wave8", "wave16_varying"])
def test_forward_prefixes(api, name):
    prob = SHAPES[name](16 * 133)
    _say("tree with forward prefixes", name)
    ((st, got),) = solve(api, [prob], trajectory="prefix")
    assert st == 0
    check(got, oracle.solve(prob), TOL["fp64"])


@pytest.mark.parametrize("name", ["class16", "wave8"])
def test_default_chunking_long_instance(api, name):
    """T = 40000: 625 chunks of 64 steps by default, on either engine."""
    prob = SHAPES[name](40000)
    _say("tree default chunking T=40000", name)
    ((st, got),) = solve(api, [prob], chunk=0)
    assert st == 0
    check(got, oracle.solve(prob), TOL["fp64"])


def test_batch_of_tree_and_chain_instances_equals_alone(api):
    probs = [SHAPES["class16"](16 * 150), SHAPES["class16"](16 * 60), SHAPES["class32_m16"](16 * 200),
             SHAPES["class64"](16 * 130), SHAPES["class64"](16 * 40), SHAPES["wave8"](16 * 170),
             SHAPES["wave8"](16 * 50), SHAPES["wave16_varying"](16 * 140)]
    _say("tree and chain instances in one batch")
    mix = solve(api, probs)
    for i, p in enumerate(probs):
        (alone,) = solve(api, [p])
        assert mix[i][0] == 0 and alone[0] == 0, i
        for f in FAMILIES:
            assert np.array_equal(mix[i][1][f], alone[1][f]), (i, f)
    check(mix[0][1], oracle.solve(probs[0]), TOL["fp64"])


def test_status_codes_and_isolation(api):
    """A tree instance whose U is not positive definite (LQT_ENOTPD) and one
    with a non-finite reference (LQT_ENONFINITE) fail alone; the instance
    beside them is unaffected."""
    good = SHAPES["class16_offsets"](16 * 140)
    bad = SHAPES["class16_offsets"](16 * 140)
    bad.U = -np.eye(bad.m)
    nan = SHAPES["wave8"](16 * 150)
    nan.r[700, 0] = np.nan
    _say("tree status codes")
    res = solve(api, [good, bad, nan])
    assert [st for st, _ in res] == [0, 3, 4]
    check(res[0][1], oracle.solve(good), TOL["fp64"])
