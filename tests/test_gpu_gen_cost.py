"""GPU parity of the generalised stage cost (the extension to more general
cost functions, Section IV-D): a cross term M between the output error and
the control error and a control reference s, solved by the library as the
standard-form transform and mapped back.  Against the FP64 oracle's direct
recursion for that cost (pinned by dense KKT solves), on every path: the
lane pipeline (both trajectory methods), the wavefront engine and the
workgroup engines of the classes 16, 32 (m <= 16 and m > 16) and 64; FP64
and MIXED; per-step F and c; M alone and s alone; outputs taken in part (u
without x uses library scratch); mixed batches with standard instances;
the serving interface; the LQT_ENOTSUP boundary.

Tolerance: relative error per output family, over all steps stacked (Frobenius) and
per step (largest step error against the RMS step size; tests/helpers.err),
1e-10 (FP64) and 1e-5 (MIXED).
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


@pytest.fixture(scope="module")
def plans(api):
    ps = {(pr, tr): api.Plan(64, 32, prec=pr, device=0, trajectory=tr)
          for pr in ("fp64", "mixed") for tr in ("maps", "prefix")}
    yield ps
    for p in ps.values():
        p.close()


@pytest.fixture(autouse=True)
def _routing(plans):
    yield
    route(plans)


def route(plans, **kw):
    for p in plans.values():
        p.set_routing(**kw)


def run(api, plan, probs, prec="fp64", want=FAMILIES):
    import torch

    dt = torch.float64 if prec == "fp64" else torch.float32
    dps = [api.DeviceProblem(p) for p in probs]
    dos = [api.DeviceOutputs(p.n, p.m, p.T, want=want, dtype=dt) for p in probs]
    plan.solve(dps, dos)
    torch.cuda.synchronize()
    for do in dos:
        assert int(do.status.item()) == 0
    return [do.host() for do in dos]


def check(got, ref, tol, fams=None):
    errs = {f: err(got[f], ref[f]) for f in (fams or got)}
    bad = {f: e for f, e in errs.items() if not e <= tol}
    assert not bad, f"rel errors above {tol}: {bad} (all: {errs})"


@pytest.mark.parametrize("prec", ["fp64", "mixed"])
@pytest.mark.parametrize("traj", ["maps", "prefix"])
@pytest.mark.parametrize("nmp,T,per_step", [((4, 2, 3), 9000, 0), ((4, 2, 4), 20001, 1 | 2), ((3, 1, 2), 8192, 2),
                                            ((2, 2, 1), 10000, 1), ((1, 1, 1), 8193, 0), ((4, 4, 4), 12000, 0)])
def test_lane_pipeline(api, plans, prec, traj, nmp, T, per_step):
    n, m, p = nmp
    _say("gen cost lane pipeline n,m,p=", nmp, "T=", T, "per_step=", per_step, prec, traj)
    prob = inputs.generalised_problem(n, m, T, seed=3 * n + m + p + per_step, p=p, per_step=per_step)
    (got,) = run(api, plans[(prec, traj)], [prob], prec)
    check(got, oracle.solve(prob), TOL[prec])


@pytest.mark.parametrize("prec", ["fp64", "mixed"])
@pytest.mark.parametrize("engine", ["workgroup", "wavefront"])
@pytest.mark.parametrize("nmp,T,per_step", [((6, 3, 4), 700, 0), ((6, 3, 6), 333, 1 | 2), ((12, 5, 8), 500, 0),
                                            ((12, 5, 12), 257, 2), ((24, 8, 16), 400, 0), ((20, 20, 20), 300, 2),
                                            ((3, 2, 3), 100, 0)])
def test_chunked_paths(api, plans, prec, engine, nmp, T, per_step):
    n, m, p = nmp
    route(plans, path="wave", wave_engine_only=(engine == "wavefront"))
    _say("gen cost chunked n,m,p=", nmp, "T=", T, "per_step=", per_step, prec, engine)
    prob = inputs.generalised_problem(n, m, T, seed=5 * n + m + p + per_step, p=p, per_step=per_step)
    (got,) = run(api, plans[(prec, "maps")], [prob], prec)
    check(got, oracle.solve(prob), TOL[prec])


@pytest.mark.parametrize("prec", ["fp64", "mixed"])
def test_class_64(api, plans, prec):
    _say("gen cost class 64 n=40 m=8 p=30", prec)
    prob = inputs.generalised_problem(40, 8, 300, seed=64, p=30, per_step=2)
    (got,) = run(api, plans[(prec, "maps")], [prob], prec)
    check(got, oracle.solve(prob), TOL[prec])


@pytest.mark.parametrize("path", ["small", "wave"])
@pytest.mark.parametrize("which", ["M", "s"])
def test_cross_term_or_reference_alone(api, plans, path, which):
    n, m, T = (4, 2, 9000) if path == "small" else (10, 4, 600)
    route(plans, path=path)
    _say("gen cost", which, "alone on", path)
    prob = inputs.generalised_problem(n, m, T, seed=71, p=n, with_s=(which == "s"))
    if which == "s":
        prob.M = None
    (got,) = run(api, plans[("fp64", "maps")], [prob])
    check(got, oracle.solve(prob), TOL["fp64"])


@pytest.mark.parametrize("path", ["small", "wave"])
@pytest.mark.parametrize("traj", ["maps", "prefix"])
@pytest.mark.parametrize("want", [("u",), ("K", "d"), ("x", "u"), ("S", "v", "u"), ("v", "u")])
def test_partial_outputs(api, plans, path, traj, want):
    n, m, T = (4, 3, 10000) if path == "small" else (8, 3, 500)
    route(plans, path=path)
    _say("gen cost outputs", want, path, traj)
    prob = inputs.generalised_problem(n, m, T, seed=81, p=n - 1, per_step=2)
    (got,) = run(api, plans[("fp64", traj)], [prob], want=want)
    assert set(got) == set(want)
    check(got, oracle.solve(prob), TOL["fp64"])


def test_mixed_batch(api, plans):
    """Generalised and standard instances in one solve: each equals its own
    solution alone."""
    probs = [inputs.generalised_problem(4, 2, 9000, seed=91, p=2),
             inputs.random_problem(4, 2, 9000, seed=92, p=4),
             inputs.generalised_problem(6, 2, 300, seed=93, p=5, per_step=1),
             inputs.random_problem(12, 4, 400, seed=94, p=12),
             inputs.generalised_problem(12, 4, 401, seed=95, p=7),
             inputs.generalised_problem(24, 10, 200, seed=96, p=24, per_step=2)]
    _say("gen cost mixed batch of", len(probs))
    got = run(api, plans[("fp64", "maps")], probs)
    for g, prob in zip(got, probs):
        check(g, oracle.solve(prob), TOL["fp64"])


def test_serving(api, plans):
    import time

    import torch

    plan = plans[("fp64", "maps")]
    probs = [inputs.generalised_problem(4, 2, 8192 + 37 * i, seed=100 + i, p=3) for i in range(3)]
    probs += [inputs.generalised_problem(10, 3, 250, seed=110 + i, p=6) for i in range(3)]
    _say("gen cost serving", len(probs))
    dps = [api.DeviceProblem(p) for p in probs]
    dos = [api.DeviceOutputs(p.n, p.m, p.T) for p in probs]
    tickets = [plan.submit(a, b) for a, b in zip(dps, dos)]
    t0 = time.time()
    done = {}
    while len(done) < len(tickets):
        for t in tickets:
            if t not in done:
                st = plan.poll(t)
                if st is not None:
                    done[t] = st
        assert time.time() - t0 < 60, "serving did not finish"
        time.sleep(0.002)
    torch.cuda.synchronize()
    assert all(v == 0 for v in done.values()), done
    for do, prob in zip(dos, probs):
        check(do.host(), oracle.solve(prob), TOL["fp64"])


def test_full_size(api, plans):
    T = 1_000_000
    _say("gen cost lane pipeline n=4 m=2 p=4 T=", T)
    prob = inputs.generalised_problem(4, 2, T, seed=1, p=4)
    (got,) = run(api, plans[("fp64", "maps")], [prob])
    check(got, oracle.solve(prob), TOL["fp64"])


def test_time_varying_weights_are_not_supported(api, plans):
    from paper_2104_03186_amd import _lib

    prob = inputs.generalised_problem(4, 2, 50, seed=5, p=4)
    prob.H = np.ascontiguousarray(np.broadcast_to(prob.H, (50, 4, 4)))
    prob.per_step |= inputs.PS_H
    _say("gen cost with per-step H: LQT_ENOTSUP")
    with pytest.raises(_lib.LQTError) as e:
        run(api, plans[("fp64", "maps")], [prob])
    assert e.value.code == _lib.ENOTSUP
