"""Pins of the oracle's generalised stage cost (the extension to more general
cost functions, Section IV-D): a cross term M between the output error and
the control error, and a control reference s.  CPU only.

* brute force: dense KKT solves of the equality-constrained QP with that
  cost (tests/helpers.py), all six output families, tiny T;
* M = 0, s = 0 reduces to the standard recursion;
* the paper's transformation to the standard form (U^{-1} M^T folded into F,
  c and X, the control recovered afterwards), written here from its
  formulas and solved by the standard oracle, gives the same solution.
"""
import numpy as np
import pytest

import oracle
from paper_2104_03186_amd import inputs
from tests.helpers import FAMILIES, kkt_solution, rel


@pytest.mark.parametrize("n,m,p,T,per_step", [(2, 1, 2, 3, 0), (3, 2, 2, 4, 0), (4, 2, 3, 5, 1 | 2), (3, 3, 4, 4, 2),
                                              (1, 1, 1, 6, 0), (4, 1, 4, 3, 1)])
def test_generalised_oracle_matches_kkt(n, m, p, T, per_step):
    prob = inputs.generalised_problem(n, m, T, seed=10 * n + m + T, p=p, per_step=per_step)
    ref = kkt_solution(prob)
    got = oracle.solve(prob)
    for f in FAMILIES:
        assert rel(got[f], ref[f]) < 1e-9, (f, rel(got[f], ref[f]))


def test_generalised_reduces_to_standard():
    prob = inputs.random_problem(4, 2, 40, seed=5, p=3)
    std = oracle.solve(prob)
    prob.M = np.zeros((prob.p, prob.m))
    prob.s = np.zeros((prob.T, prob.m))
    gen = oracle.solve(prob)
    for f in FAMILIES:
        assert rel(gen[f], std[f]) < 1e-13, f


def transformed(prob):
    """The standard-form problem of the transformation: u~ = U^{-1} M^T (H x -
    r) + u - s, F~ = F - L U^{-1} M^T H, c~_k = c_k + L U^{-1} M^T r_k + L s_k,
    X~ = X - M U^{-1} M^T, U~ = U (time-invariant L, H, X, U, M)."""
    Z = np.linalg.solve(prob.U, prob.M.T)  # U^{-1} M^T, m x p
    T, n = prob.T, prob.n
    F = prob.F - prob.L @ Z @ prob.H  # broadcast over the time axis when F is per step
    c0 = np.zeros((T, n)) if prob.c is None else (prob.c if prob.per_step & inputs.PS_c else
                                                  np.broadcast_to(prob.c, (T, n)))
    s = np.zeros((T, prob.m)) if prob.s is None else prob.s
    c = c0 + prob.r @ (prob.L @ Z).T + s @ prob.L.T
    t = inputs.LQTProblem(n=n, m=prob.m, p=prob.p, pT=prob.pT, T=T, per_step=prob.per_step | inputs.PS_c,
                          F=np.ascontiguousarray(F), c=np.ascontiguousarray(c), L=prob.L, H=prob.H,
                          X=prob.X - prob.M @ Z, U=prob.U, r=prob.r, HT=prob.HT, XT=prob.XT, rT=prob.rT,
                          x0=prob.x0)
    return t, Z


@pytest.mark.parametrize("per_step", [0, 1, 2])
def test_paper_transformation_gives_the_same_solution(per_step):
    prob = inputs.generalised_problem(4, 2, 60, seed=7 + per_step, p=3, per_step=per_step)
    gen = oracle.solve(prob)
    t, Z = transformed(prob)
    std = oracle.solve(t)
    # value functions and states are those of the same problem
    for f in ("S", "v", "x"):
        assert rel(std[f], gen[f]) < 1e-11, f
    # controls and gains map back: u = u~ - Z (H x - r) + s, K = K~ + Z H, d = d~ + Z r + s
    s = prob.s
    u = std["u"] - (std["x"][:-1] @ prob.H.T - prob.r) @ Z.T + s
    K = std["K"] + (Z @ prob.H)[None]
    d = std["d"] + prob.r @ Z.T + s
    assert rel(u, gen["u"]) < 1e-11
    assert rel(K, gen["K"]) < 1e-11
    assert rel(d, gen["d"]) < 1e-11
