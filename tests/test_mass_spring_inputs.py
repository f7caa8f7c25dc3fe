"""The state-dimension workload (Section VI-C): the chain of N masses with
springs and dampers, discretised by zero-order hold.  The discrete model is
checked against a fine fourth-order Runge-Kutta integration of the
continuous equations of motion (written here from the equations, with the
middle masses' damper term read as d (y'_{i-1} - 2 y'_i + y'_{i+1})), the
initial state against the experiment's description, and the optimum of the
instance against a dense KKT solve on a short horizon."""
import numpy as np
import pytest

import oracle
from paper_2104_03186_amd import inputs
from tests.helpers import kkt_solution


def accel(y, v, u, N, k=1.0, d=0.2, mass=1.0):
    a = np.zeros(N)
    for i in range(N):
        left_y = y[i - 1] if i > 0 else 0.0
        left_v = v[i - 1] if i > 0 else 0.0
        right_y = y[i + 1] if i < N - 1 else 0.0
        right_v = v[i + 1] if i < N - 1 else 0.0
        a[i] = k / mass * (left_y - 2 * y[i] + right_y) + d / mass * (left_v - 2 * v[i] + right_v)
    a[0] += u[0] / mass
    a[N - 1] -= u[1] / mass
    return a


def rk4_step(x, u, N, h):
    def f(z):
        y, v = z[0::2], z[1::2]
        out = np.empty_like(z)
        out[0::2] = v
        out[1::2] = accel(y, v, u, N)
        return out

    k1 = f(x)
    k2 = f(x + 0.5 * h * k1)
    k3 = f(x + 0.5 * h * k2)
    k4 = f(x + h * k3)
    return x + h / 6.0 * (k1 + 2 * k2 + 2 * k3 + k4)


@pytest.mark.parametrize("N", [2, 3, 5])
def test_zero_order_hold_matches_integration(N):
    T = 50
    prob = inputs.mass_spring_problem(N, T)
    dt = 10.0 / T
    rng = np.random.default_rng(N)
    for _ in range(3):
        x = rng.normal(size=2 * N)
        u = rng.normal(size=2)
        z = x.copy()
        sub = 400
        for _ in range(sub):
            z = rk4_step(z, u, N, dt / sub)
        assert np.allclose(prob.F @ x + prob.L @ u, z, rtol=0, atol=1e-10)


def test_initial_state_and_shape():
    prob = inputs.mass_spring_problem(7, 100)
    assert (prob.n, prob.m, prob.T) == (14, 2, 100)
    expect = np.zeros(14)
    expect[0] = 1.0          # first mass
    expect[2 * (7 // 2)] = 1.0  # mass floor(N/2)+1 (1-based)
    assert np.array_equal(prob.x0, expect)


def test_optimum_matches_kkt():
    prob = inputs.mass_spring_problem(3, 5)
    ref = kkt_solution(prob)
    got = oracle.solve(prob)
    for f in ("x", "u"):
        assert np.allclose(got[f], ref[f], rtol=0, atol=1e-9)
