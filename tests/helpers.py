"""Shared test helpers: relative errors (stacked and per step) and a brute-force
KKT solver.

The KKT solver is independent of the oracle: it assembles the equality-
constrained quadratic program of the LQT problem statement (Section II-B of the
paper; Section IV-A notes that the conditional value function is such a QP)
and solves the dense KKT system with numpy.
"""
import numpy as np

FAMILIES = ("S", "v", "K", "d", "x", "u")


def rel(a, b):
    """Frobenius relative error ||a - b|| / ||b|| over all steps stacked."""
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    nb = np.linalg.norm(b)
    if nb == 0.0:
        return float(np.linalg.norm(a))
    return float(np.linalg.norm(a - b) / nb)


def step_rel(a, b):
    """Largest per-step relative error, time on the first axis:
    max_k ||a_k - b_k|| / max(||b_k||, rms), rms = sqrt(mean_k ||b_k||^2).

    Each step is held to its own size, or to the RMS step size where the step
    is smaller than that (a step near zero is not divided by its own tiny
    norm).  The stacked norm of rel() spreads one wrong step over all T of
    them (one bad step at T = 1e6 moves it by 1/1000 of that step's error);
    this one does not.  Where no step exceeds the RMS size it is never below
    rel()."""
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    if a.ndim == 0 or a.shape[0] == 0:
        return rel(a, b)
    d = np.linalg.norm((a - b).reshape(a.shape[0], -1), axis=1)
    nb = np.linalg.norm(b.reshape(b.shape[0], -1), axis=1)
    rms = float(np.sqrt(np.mean(nb ** 2)))
    if rms == 0.0:
        return float(np.max(d))
    return float(np.max(d / np.maximum(nb, rms)))


def err(a, b):
    """Parity gate of the GPU tests: the larger of the stacked relative error
    and the per-step error (step_rel), so every step is held to the bound."""
    return max(rel(a, b), step_rel(a, b))


def _mat(prob, name, bit, k):
    a = getattr(prob, name)
    return a[k] if (prob.per_step & bit) else a


def kkt_subproblem(prob, k0, xi):
    """Solve the LQT QP from step k0 with x_{k0} = xi by a dense KKT solve.

    Returns (x [T-k0+1, n], u [T-k0, m], mu0) where mu0 is the multiplier of
    the constraint x_{k0} = xi, so that grad V_{k0}(xi) = -mu0."""
    n, m, T = prob.n, prob.m, prob.T
    N = T - k0
    nxv, nuv = n * (N + 1), m * N
    nz = nxv + nuv
    P = np.zeros((nz, nz))
    q = np.zeros(nz)

    def xs(k):
        return slice(n * (k - k0), n * (k - k0 + 1))

    def us(k):
        return slice(nxv + m * (k - k0), nxv + m * (k - k0 + 1))

    M = getattr(prob, "M", None)
    s = getattr(prob, "s", None)
    for k in range(k0, T):
        H, X, U = _mat(prob, "H", 8, k), _mat(prob, "X", 16, k), _mat(prob, "U", 32, k)
        P[xs(k), xs(k)] += H.T @ X @ H
        q[xs(k)] += -H.T @ X @ prob.r[k]
        P[us(k), us(k)] += U
        # generalised stage cost: (H x - r)^T M (u - s) + 1/2 (u - s)^T U (u - s)
        sk = np.zeros(m) if s is None else s[k]
        if M is not None:
            Mk = _mat(prob, "M", 64, k)
            P[xs(k), us(k)] += H.T @ Mk
            P[us(k), xs(k)] += Mk.T @ H
            q[xs(k)] += -H.T @ Mk @ sk
            q[us(k)] += -Mk.T @ prob.r[k]
        q[us(k)] += -U @ sk
    P[xs(T), xs(T)] += prob.HT.T @ prob.XT @ prob.HT
    q[xs(T)] += -prob.HT.T @ prob.XT @ prob.rT

    ncons = n * (N + 1)
    G = np.zeros((ncons, nz))
    h = np.zeros(ncons)
    G[0:n, xs(k0)] = np.eye(n)
    h[0:n] = xi
    for k in range(k0, T):
        F, L = _mat(prob, "F", 1, k), _mat(prob, "L", 4, k)
        c = np.zeros(n) if prob.c is None else _mat(prob, "c", 2, k)
        rows = slice(n * (k - k0 + 1), n * (k - k0 + 2))
        G[rows, xs(k + 1)] = np.eye(n)
        G[rows, xs(k)] = -F
        G[rows, us(k)] = -L
        h[rows] = c
    KKT = np.block([[P, G.T], [G, np.zeros((ncons, ncons))]])
    sol = np.linalg.solve(KKT, np.concatenate([-q, h]))
    z, mu = sol[:nz], sol[nz:]
    return z[:nxv].reshape(N + 1, n), z[nxv:].reshape(N, m), mu[:n]


def kkt_solution(prob):
    """All of S, v, K, d, x, u from dense KKT solves (tiny T only).

    V_k is quadratic, so grad V_k(xi) = S_k xi - v_k = -mu0(xi) evaluated at
    xi in {0, e_1..e_n} recovers S_k and v_k exactly; the first optimal
    control u_k(xi) = -K_k xi + d_k recovers K_k and d_k."""
    n, m, T = prob.n, prob.m, prob.T
    S = np.zeros((T + 1, n, n))
    v = np.zeros((T + 1, n))
    K = np.zeros((T, m, n))
    d = np.zeros((T, m))
    for k0 in range(T + 1):
        _, u0, mu0 = kkt_subproblem(prob, k0, np.zeros(n))
        v[k0] = mu0
        if k0 < T:
            d[k0] = u0[0]
        for i in range(n):
            e = np.zeros(n)
            e[i] = 1.0
            _, ui, mui = kkt_subproblem(prob, k0, e)
            S[k0][:, i] = -mui + v[k0]
            if k0 < T:
                K[k0][:, i] = d[k0] - ui[0]
    x, u, _ = kkt_subproblem(prob, 0, prob.x0)
    return {"S": S, "v": v, "K": K, "d": d, "x": x, "u": u}


def rollout(prob, u):
    """x_{k+1} = F_k x_k + c_k + L_k u_k from x_0 (the problem's dynamics)."""
    n, T = prob.n, prob.T
    x = np.zeros((T + 1, n))
    x[0] = prob.x0
    for k in range(T):
        F, L = _mat(prob, "F", 1, k), _mat(prob, "L", 4, k)
        c = np.zeros(n) if prob.c is None else _mat(prob, "c", 2, k)
        x[k + 1] = F @ x[k] + c + L @ u[k]
    return x
