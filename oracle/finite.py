"""Finite state and control spaces (Section III-D).

TEST INFRASTRUCTURE ONLY: imported by the tests, the smoke check and the
benchmark's CPU leg, never by the product package; it shares no code with
the HIP implementation.

The sequential dynamic programme of Section II-A written out over the finite
tables: V_T(x) = l_T(x); V_k(x) = min_u { l_k(x, u) + V_{k+1}(f_k(x, u)) }
with the minimising control u_k(x) (the smallest index among equal minima;
-1 and +inf when no control is admissible); then the optimal trajectory
x_{k+1} = f_k(x_k, u_k(x_k)) from x_0.  ``combine`` is the min-plus product
of two conditional value functions (the associative operator of
Section III-B), used by the pins.

Tables: next [Dx][Du] or [T][Dx][Du] (int, -1 = not admissible), cost of the
same shape (float), cost_T [Dx].
"""
from __future__ import annotations

import numpy as np


def _step_tables(prob, k):
    nxt = prob.next[k] if prob.next.ndim == 3 else prob.next
    cst = prob.cost[k] if prob.cost.ndim == 3 else prob.cost
    return nxt, cst


def solve(prob) -> dict:
    """V [T+1][Dx], u [T][Dx], x [T+1], ux [T]."""
    T, D = prob.T, prob.nstates
    V = np.empty((T + 1, D))
    U = np.empty((T, D), dtype=np.int32)
    V[T] = prob.cost_T
    rows = np.arange(D)[:, None]
    for k in range(T - 1, -1, -1):
        nxt, cst = _step_tables(prob, k)
        ok = (nxt >= 0) & (nxt < D)
        # l_k(x, u) + V_{k+1}(f_k(x, u)) over every (x, u); +inf where not admissible
        vals = np.where(ok, cst + V[k + 1][np.where(ok, nxt, 0)], np.inf)
        arg = np.argmin(vals, axis=1)  # first (smallest) index among equal minima
        best = vals[rows[:, 0], arg]
        V[k] = best
        U[k] = np.where(np.isfinite(best), arg, -1)
    x = np.empty(T + 1, dtype=np.int32)
    ux = np.empty(T, dtype=np.int32)
    x[0] = prob.x0
    for k in range(T):
        nxt, _ = _step_tables(prob, k)
        if x[k] < 0:
            x[k + 1], ux[k] = -1, -1
            continue
        ux[k] = U[k, x[k]]
        x[k + 1] = nxt[x[k], ux[k]] if ux[k] >= 0 else -1
    return {"V": V, "u": U, "x": x, "ux": ux}


def element(prob, k: int) -> np.ndarray:
    """V_{k->k+1}(x, y) = min { l_k(x, u) : f_k(x, u) = y } (+inf if none)."""
    D = prob.nstates
    nxt, cst = _step_tables(prob, k)
    E = np.full((D, D), np.inf)
    for i in range(D):
        for u in range(prob.ncontrols):
            j = int(nxt[i, u])
            if 0 <= j < D:
                E[i, j] = min(E[i, j], cst[i, u])
    return E


def combine(a: np.ndarray, b: np.ndarray) -> np.ndarray:
    """(a (x) b)(x, y) = min_z a(x, z) + b(z, y)."""
    return np.min(a[:, :, None] + b[None, :, :], axis=1)


def path_cost(prob, x: np.ndarray, ux: np.ndarray) -> float:
    """Total cost of a control sequence applied from x_0 (its states x)."""
    total = 0.0
    for k in range(prob.T):
        _, cst = _step_tables(prob, k)
        total += cst[x[k], ux[k]]
    return float(total + prob.cost_T[x[prob.T]])
