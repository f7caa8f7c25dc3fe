"""Pins of the oracle's finite state and control dynamic programme (Section
III-D).  CPU only.

* brute force: every control sequence of tiny problems enumerated; the
  least total cost from each start state is V_0, and the oracle's
  trajectory attains it;
* shortest paths: the layered graph of a medium problem (edges (k, x) ->
  (k+1, f_k(x, u)) weighted l_k(x, u), terminal edges weighted l_T) solved
  by scipy's Dijkstra gives every V_k(x);
* the scan formulation: the one-step conditional value functions combined
  by the min-plus product (Section III-B), in sequence and in a tree
  bracketing, reproduce V exactly (integer costs), and the product is
  associative with the two-sided identity (0 on the diagonal, +inf off);
* the control law attains the minimum with the smallest index;
* all-zero grid costs on the routing workload: zero values, straight flight.
"""
import itertools

import numpy as np
import pytest

from oracle import finite
from paper_2104_03186_amd import inputs


def _brute_force(prob, x_start):
    best = np.inf
    for seq in itertools.product(range(prob.ncontrols), repeat=prob.T):
        x, total = x_start, 0.0
        for k, u in enumerate(seq):
            nxt, cst = finite._step_tables(prob, k)
            j = int(nxt[x, u])
            if j < 0:
                total = np.inf
                break
            total += cst[x, u]
            x = j
        if np.isfinite(total):
            best = min(best, total + prob.cost_T[x])
    return best


@pytest.mark.parametrize("T,D,Du,per_step,seed", [(1, 3, 2, 3, 0), (3, 3, 3, 3, 1), (4, 4, 2, 1, 2), (5, 2, 3, 2, 3),
                                                  (4, 3, 3, 0, 4)])
def test_brute_force(T, D, Du, per_step, seed):
    prob = inputs.random_finite_problem(T, D, Du, seed=seed, per_step=per_step, integer=False)
    sol = finite.solve(prob)
    for x in range(D):
        assert sol["V"][0, x] == pytest.approx(_brute_force(prob, x), rel=1e-12, abs=0)
    if np.isfinite(sol["V"][0, prob.x0]):
        assert finite.path_cost(prob, sol["x"], sol["ux"]) == pytest.approx(sol["V"][0, prob.x0], rel=1e-12)


def test_layered_shortest_paths():
    from scipy.sparse import csr_matrix
    from scipy.sparse.csgraph import dijkstra

    prob = inputs.random_finite_problem(60, 11, 3, seed=7, per_step=3)
    T, D = prob.T, prob.nstates
    sink = (T + 1) * D
    edges = {}  # (from, to) -> least weight (controls reaching the same state share one edge)
    for k in range(T):
        nxt, cst = finite._step_tables(prob, k)
        for i in range(D):
            for u in range(prob.ncontrols):
                if nxt[i, u] >= 0:
                    e = (k * D + i, (k + 1) * D + int(nxt[i, u]))
                    edges[e] = min(edges.get(e, np.inf), cst[i, u])
    for i in range(D):
        edges[(T * D + i, sink)] = prob.cost_T[i]
    rows, cols = zip(*edges)
    w = [v + 1e-300 for v in edges.values()]  # keep zero-cost edges in the sparse graph
    G = csr_matrix((w, (rows, cols)), shape=(sink + 1, sink + 1))
    dist = dijkstra(G.T, indices=sink)  # distance of every node to the sink
    V = finite.solve(prob)["V"]
    for k in range(T + 1):
        assert np.allclose(V[k], dist[k * D:(k + 1) * D], rtol=0, atol=1e-9)


def test_scan_formulation_is_exact():
    prob = inputs.random_finite_problem(40, 6, 3, seed=8, per_step=3)
    V = finite.solve(prob)["V"]
    E = [finite.element(prob, k) for k in range(prob.T)]
    # suffix products applied to the terminal cost, in sequence
    acc = prob.cost_T.copy()
    for k in range(prob.T - 1, -1, -1):
        acc = np.min(E[k] + acc[None, :], axis=1)
        assert np.array_equal(acc, V[k])
    # tree bracketing of the products
    def tree(lo, hi):
        if hi - lo == 1:
            return E[lo]
        mid = (lo + hi) // 2
        return finite.combine(tree(lo, mid), tree(mid, hi))
    P = tree(0, prob.T)
    assert np.array_equal(np.min(P + prob.cost_T[None, :], axis=1), V[0])
    a, b, c = E[0], E[1], E[2]
    assert np.array_equal(finite.combine(finite.combine(a, b), c), finite.combine(a, finite.combine(b, c)))
    ident = np.where(np.eye(6) > 0, 0.0, np.inf)
    assert np.array_equal(finite.combine(ident, a), a) and np.array_equal(finite.combine(a, ident), a)


def test_control_law_is_smallest_minimiser():
    prob = inputs.routing_problem(50, nstates=7, seed=3)
    sol = finite.solve(prob)
    V, U = sol["V"], sol["u"]
    for k in range(prob.T):
        nxt, cst = finite._step_tables(prob, k)
        for i in range(prob.nstates):
            cand = [cst[i, u] + V[k + 1, nxt[i, u]] if nxt[i, u] >= 0 else np.inf for u in range(3)]
            assert V[k, i] == min(cand)
            assert U[k, i] == int(np.argmin(cand))


def test_flat_grid_flies_straight():
    prob = inputs.routing_problem(30, nstates=5, seed=0)
    prob.cost[:] = np.array([1.0, 0.0, 1.0])  # grid costs zero: only the moves cost
    prob.cost_T[:] = 0.0
    sol = finite.solve(prob)
    assert np.all(sol["V"] == 0.0)
    assert np.all(sol["ux"] == 1) and np.all(sol["x"] == prob.x0)
