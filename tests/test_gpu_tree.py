"""GPU parity of the chunk scans as trees on the chunked engines: instances
with at least 128 chunks (or every instance of two chunks or more, with the
routing override tree=True) form the value at every chunk start by recursive
doubling over their chunk elements (the parallel scan of Section II-C with
the general combination rule of Section IV-A, anchored on the terminal value
of Section IV-B) and the state at every chunk start by recursive doubling
over the chunk maps (Method 1 of Section IV-C), instead of walking the
chunks in sequence.  Checked against the FP64 oracle: every workgroup class
(16, 32 in both control widths, 64) and every wavefront class (8, 16, 32;
time-varying data), the operator-form fold and the per-chunk fold (offsets
c), chunk counts around the trees' level boundaries (2, 3, 5, 17, 33, 128,
129, 257 chunks), MIXED, the generalised cost, forward prefixes (Method 2,
which reads the untouched chunk elements), the default chunking of long
instances, the override tree=False on a long instance, and a batch of tree
and chain instances equal to each instance alone, bit for bit.

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


def solve(api, probs, prec="fp64", chunk=16, trajectory="maps", tree=None):
    import torch

    plan = api.Plan(64, 32, prec=prec, device=0, trajectory=trajectory)
    try:
        plan.set_routing(wave_chunk=chunk, tree=tree)
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


@pytest.mark.parametrize("name", list(SHAPES))
@pytest.mark.parametrize("T", [16 + 3, 16 * 2 + 1, 16 * 4 + 7, 16 * 17, 16 * 32 + 9])
def test_forced_trees_few_chunks(api, name, T):
    """tree=True: 2, 3, 5, 17 and 33 chunks (one or two levels past a power
    of two, both trees with a ragged last chunk)."""
    prob = SHAPES[name](T)
    _say("forced trees", name, "T=", T, "chunk 16")
    ((st, got),) = solve(api, [prob], tree=True)
    assert st == 0
    check(got, oracle.solve(prob), TOL["fp64"])


@pytest.mark.parametrize("name", ["class16_offsets", "class64", "wave8", "wave32_varying"])
def test_forced_trees_mixed(api, name):
    prob = SHAPES[name](16 * 37 + 5)
    _say("forced trees mixed", name)
    ((st, got),) = solve(api, [prob], prec="mixed", tree=True)
    assert st == 0
    check(got, oracle.solve(prob), TOL["mixed"])


@pytest.mark.parametrize("name", ["class16", "class32_m16", "wave16_varying"])
def test_forced_trees_default_chunking(api, name):
    """tree=True with the default chunk length (T = 1000 and 5000)."""
    for T in (1000, 5000):
        prob = SHAPES[name](T)
        _say("forced trees default chunking", name, "T=", T)
        ((st, got),) = solve(api, [prob], chunk=0, tree=True)
        assert st == 0
        check(got, oracle.solve(prob), TOL["fp64"])


@pytest.mark.parametrize("name", ["class16", "wave8"])
def test_trees_off_long_instance(api, name):
    """tree=False: 200 chunks walked in sequence."""
    prob = SHAPES[name](16 * 200)
    _say("trees off", name)
    ((st, got),) = solve(api, [prob], tree=False)
    assert st == 0
    check(got, oracle.solve(prob), TOL["fp64"])


def test_forced_trees_batch_with_one_chunk_instances(api):
    """tree=True in a batch whose instances have 1 to 40 chunks (an instance
    of one chunk has nothing to scan and keeps the walks): each equals the
    instance alone, bit for bit, and the oracle."""
    probs = [SHAPES["class16"](10), SHAPES["class16"](16 * 40), SHAPES["class16"](16 * 3 - 2),
             SHAPES["wave8"](16), SHAPES["wave8"](16 * 21 + 1), SHAPES["class64"](16 * 9 + 4),
             SHAPES["class64"](7)]
    _say("forced trees, batch with one-chunk instances")
    mix = solve(api, probs, tree=True)
    for i, p in enumerate(probs):
        (alone,) = solve(api, [p], tree=True)
        assert mix[i][0] == 0 and alone[0] == 0, i
        for f in FAMILIES:
            assert np.array_equal(mix[i][1][f], alone[1][f]), (i, f)
        check(mix[i][1], oracle.solve(p), TOL["fp64"])


def test_routing_tree_field_validation(api):
    """lqt_set_routing rejects tree values outside 0..2 with LQT_EINVAL and
    leaves the plan's routing as it was."""
    import ctypes

    from paper_2104_03186_amd import _lib

    plan = api.Plan(16, 8)
    try:
        plan.set_routing(tree=True)
        for bad in (-1, 3):
            r = _lib.Routing(tree=bad)
            rc = _lib.load().lqt_set_routing(plan.handle, ctypes.byref(r))
            assert rc == _lib.EINVAL, bad
            assert "tree" in _lib.last_error(plan.handle)
        prob = SHAPES["class16"](16 * 9 + 3)
        _say("routing after rejected tree values")
        dp = api.DeviceProblem(prob)
        do = api.DeviceOutputs(prob.n, prob.m, prob.T)
        plan.solve([dp], [do])
        import torch

        torch.cuda.synchronize()
        assert int(do.status.item()) == 0
        check(do.host(), oracle.solve(prob), TOL["fp64"])
    finally:
        plan.close()


@pytest.mark.parametrize("prec", ["fp64", "mixed"])
@pytest.mark.parametrize("T", [16 * 5, 16 * 9 + 7, 16 * 130 + 3])
def test_wave8_operator_form_fold(api, prec, T):
    """Class-8 time-invariant instances without offsets (the operator form of
    the wavefront engine's fold: one matrix fold per instance, the vector
    recursion per chunk), full and ragged last chunks, chains and trees, and
    one alone against the same instance in a batch."""
    probs = [inputs.diag_problem(8, 4, T, 2, 5), inputs.random_problem(7, 3, T, seed=97, with_c=False, scale=0.95),
             inputs.diag_problem(6, 3, T + 33, 2, 6)]
    _say("wave8 operator form", prec, "T=", T)
    mix = solve(api, probs, prec=prec)
    for i, p in enumerate(probs):
        assert mix[i][0] == 0, i
        check(mix[i][1], oracle.solve(p), TOL[prec])
    (alone,) = solve(api, [probs[1]], prec=prec)
    for f in FAMILIES:
        assert np.array_equal(mix[1][1][f], alone[1][f]), f
    for tree in (True, False):
        (res,) = solve(api, [probs[0]], prec=prec, chunk=0, tree=tree)
        assert res[0] == 0
        check(res[1], oracle.solve(probs[0]), TOL[prec])
