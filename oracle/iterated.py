"""Iterated linearisation for nonlinear control (the nonlinear extension of Section IV-D) with the
unicycle model of the nonlinear experiment (Section VI-E).

TEST INFRASTRUCTURE ONLY: imported by the tests, the smoke check and the
benchmark's CPU leg, never by the product package; it shares no code with
the HIP implementation.

Each iteration takes the nominal trajectory (xbar, ubar), linearises the
dynamics by a first-order Taylor expansion about it (the expansion of the
nonlinear section: f(x, u) ~ f(xbar, ubar) + J^x (x - xbar) + J^u (u - ubar),
i.e. x_{k+1} = F_k x_k + c_k + L_k u_k with F_k = J^x_k, L_k = J^u_k,
c_k = f(xbar_k, ubar_k) - F_k xbar_k - L_k ubar_k), solves that LQT with the
sequential FP64 oracle and takes its optimal (x, u) as the next nominal
trajectory.  Output and control maps are linear here (h(x) = H x, g(u) = u).
"""
from __future__ import annotations

import types

import numpy as np

from . import solve

PS_F, PS_c, PS_L, PS_X = 1, 2, 4, 16


def unicycle_f(x: np.ndarray, u: np.ndarray, dt: float) -> np.ndarray:
    """Discretised unicycle (Section VI-E): position advanced along the heading
    by speed * dt, heading by the turn rate, speed by the acceleration."""
    px, py, th, s = x
    a, w = u
    return np.array([px + s * np.cos(th) * dt, py + s * np.sin(th) * dt, th + w * dt, s + a * dt])


def unicycle_jacobians(x: np.ndarray, u: np.ndarray, dt: float):
    """J^x (4 x 4) and J^u (4 x 2) of unicycle_f at (x, u), differentiated by
    hand."""
    _, _, th, s = x
    Jx = np.eye(4)
    Jx[0, 2] = -s * np.sin(th) * dt
    Jx[0, 3] = np.cos(th) * dt
    Jx[1, 2] = s * np.cos(th) * dt
    Jx[1, 3] = np.sin(th) * dt
    Ju = np.zeros((4, 2))
    Ju[2, 1] = dt
    Ju[3, 0] = dt
    return Jx, Ju


def linearise(prob, xbar: np.ndarray, ubar: np.ndarray):
    """The LQT instance of one iteration (per-step F, L, c and X)."""
    T = prob.T
    F = np.empty((T, 4, 4))
    L = np.empty((T, 4, 2))
    c = np.empty((T, 4))
    for k in range(T):
        Jx, Ju = unicycle_jacobians(xbar[k], ubar[k], prob.dt[k])
        F[k], L[k] = Jx, Ju
        c[k] = unicycle_f(xbar[k], ubar[k], prob.dt[k]) - Jx @ xbar[k] - Ju @ ubar[k]
    return types.SimpleNamespace(n=4, m=2, p=3, pT=3, T=T, per_step=PS_F | PS_c | PS_L | PS_X, F=F, c=c, L=L,
                                 H=prob.H, X=prob.X, U=prob.U, r=prob.r, HT=prob.HT, XT=prob.XT, rT=prob.rT,
                                 x0=prob.x0)


def iterate(prob, iterations: int, xbar=None, ubar=None):
    """``iterations`` rounds of linearise-and-solve from (xbar, ubar)
    (default: the problem's nominal trajectory).  Returns x, u of the last
    round and, per round, max |u_new - u_nominal|."""
    x = np.array(prob.xbar if xbar is None else xbar, dtype=np.float64)
    u = np.array(prob.ubar if ubar is None else ubar, dtype=np.float64)
    changes = []
    for _ in range(iterations):
        sol = solve(linearise(prob, x, u))
        changes.append(float(np.max(np.abs(sol["u"] - u))) if u.size else 0.0)
        x, u = sol["x"], sol["u"]
    return x, u, changes


def rollout(prob, u: np.ndarray) -> np.ndarray:
    """States of the nonlinear model under the controls u, from x_0."""
    x = np.empty((prob.T + 1, 4))
    x[0] = prob.x0
    for k in range(prob.T):
        x[k + 1] = unicycle_f(x[k], u[k], prob.dt[k])
    return x


def nonlinear_cost(prob, u: np.ndarray) -> float:
    """Total cost of the nonlinear problem under u (states by rollout)."""
    x = rollout(prob, u)
    e = x[:-1] @ prob.H.T - prob.r
    run = 0.5 * np.einsum("ki,kij,kj->", e, prob.X, e) + 0.5 * np.einsum("ki,ij,kj->", u, prob.U, u)
    eT = prob.HT @ x[-1] - prob.rT
    return float(run + 0.5 * eT @ prob.XT @ eT)
