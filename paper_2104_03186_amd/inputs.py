"""Seeded synthetic LQT problem generators (inputs only, no solver arithmetic).

This module is shared by the tests, the benchmark and the CPU oracle's
callers.  It holds no step of the method: it only draws problem data of the
shapes and distributions of the workloads below and packs them into
``LQTProblem``.  It imports nothing from the rest of the package.

Problem (Section II-B of the paper): x_{k+1} = F_k x_k + c_k + L_k u_k with
running cost 1/2 (H_k x_k - r_k)^T X_k (H_k x_k - r_k) + 1/2 u_k^T U_k u_k for
k = 0..T-1 and terminal cost 1/2 (H_T x_T - r_T)^T X_T (H_T x_T - r_T).

Workloads (every generator draws from numpy PCG64 seeded with
SeedSequence([2104, workload_id, instance_id]); draw order is fixed below):

* ``tracking_problem`` (workloads 0 and 1): n x n dynamics F = I + 0.1 G,
  G ~ N(0, 1/n), rescaled to spectral radius rho (0.99); L ~ N(0, 1) (n x m);
  c = 0; H = H_T = I; X = 10 I, U = 0.1 I, X_T = 10 I; reference
  r_{k,i} = sin(2 pi k / 200 + phi_i) with phi ~ U[0, 2 pi); x_0 ~ N(0, I).
* ``batched_problems`` (workload 2): 4096 instances, T log-uniform on
  [256, 16384], n uniform on {4, 8, 16}, m = n / 2, F and L as above,
  X = diag(U[1, 10]), U = diag(U[0.01, 1]), X_T = X, random-walk reference
  r_0 ~ N(0, I), r_{k+1} = r_k + N(0, 0.1^2 I), x_0 ~ N(0, I).
* ``dense_problems`` (workload 3): 64 instances, n = 64, m = 32, T = 8192,
  F with spectral radius 0.98, L ~ N(0, 1), X = W W^T + 0.1 I with
  W ~ N(0, 1/n), U = W' W'^T + 0.1 I with W' ~ N(0, 1/m), X_T = X,
  random-walk reference.
* ``serving_requests`` (workload 4): Poisson arrivals at a given rate;
  n uniform on {4..32}, m = ceil(n / 2), T log-uniform on [64, 65536], data as
  workload 2.
"""
from __future__ import annotations

import dataclasses
import math
from typing import Optional

import numpy as np

BASE_SEED = 2104

PS_F, PS_c, PS_L, PS_H, PS_X, PS_U = 1, 2, 4, 8, 16, 32
PS_M = 64  # cross term of the generalised stage cost


@dataclasses.dataclass
class LQTProblem:
    """One LQT instance.  Arrays are float64, row-major.

    A matrix whose ``PS_*`` bit is set in ``per_step`` carries a leading time
    axis of length T; otherwise one matrix serves every step.  ``r`` is always
    per step ([T][p]); ``rT`` is the terminal reference ([pT])."""
    n: int
    m: int
    p: int
    pT: int
    T: int
    per_step: int
    F: np.ndarray
    c: Optional[np.ndarray]
    L: np.ndarray
    H: np.ndarray
    X: np.ndarray
    U: np.ndarray
    r: np.ndarray
    HT: np.ndarray
    XT: np.ndarray
    rT: np.ndarray
    x0: np.ndarray
    # generalised stage cost (cross term and control reference); None: absent
    M: Optional[np.ndarray] = None   # [p][m] (or [T][p][m] with PS_M)
    s: Optional[np.ndarray] = None   # [T][m]

    @property
    def steps(self) -> int:
        return self.T


def prefix_problem(prob: LQTProblem, T: int) -> LQTProblem:
    """The instance over its first T steps: per-step arrays cut to T, the
    terminal data unchanged (what a device instance read as a prefix solves)."""
    if not 1 <= T <= prob.T:
        raise ValueError(f"T={T} outside 1..{prob.T}")
    bits = {"F": PS_F, "c": PS_c, "L": PS_L, "H": PS_H, "X": PS_X, "U": PS_U, "M": PS_M}
    kw = dataclasses.asdict(prob)
    for f, bit in bits.items():
        if kw[f] is not None and (prob.per_step & bit):
            kw[f] = np.ascontiguousarray(kw[f][:T])
    kw["r"] = np.ascontiguousarray(prob.r[:T])
    if kw["s"] is not None:
        kw["s"] = np.ascontiguousarray(prob.s[:T])
    kw["T"] = T
    return LQTProblem(**kw)


def _rng(workload: int, instance: int) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(np.random.SeedSequence([BASE_SEED, workload, instance])))


def _dynamics(rng: np.random.Generator, n: int, m: int, rho: float):
    """F = I + 0.1 G rescaled to spectral radius rho; L ~ N(0, 1)."""
    G = rng.normal(0.0, 1.0 / math.sqrt(n), size=(n, n))
    F0 = np.eye(n) + 0.1 * G
    F = F0 * (rho / np.max(np.abs(np.linalg.eigvals(F0))))
    L = rng.normal(0.0, 1.0, size=(n, m))
    return np.ascontiguousarray(F), np.ascontiguousarray(L)


def tracking_problem(n: int = 4, m: int = 2, T: int = 1000, workload: int = 0,
                     instance: int = 0, rho: float = 0.99) -> LQTProblem:
    """Sinusoidal-reference tracking problem (workloads 0 and 1)."""
    rng = _rng(workload, instance)
    F, L = _dynamics(rng, n, m, rho)
    phi = rng.uniform(0.0, 2.0 * math.pi, size=n)
    k = np.arange(T + 1, dtype=np.float64)[:, None]
    rr = np.sin(2.0 * math.pi * k / 200.0 + phi[None, :])
    x0 = rng.normal(0.0, 1.0, size=n)
    eye = np.eye(n)
    return LQTProblem(n=n, m=m, p=n, pT=n, T=T, per_step=0, F=F, c=None, L=L,
                      H=eye.copy(), X=10.0 * eye, U=0.1 * np.eye(m),
                      r=np.ascontiguousarray(rr[:T]), HT=eye.copy(), XT=10.0 * eye,
                      rT=np.ascontiguousarray(rr[T]), x0=x0)


def _random_walk(rng, T, p, sigma=0.1):
    r0 = rng.normal(0.0, 1.0, size=(1, p))
    steps = rng.normal(0.0, sigma, size=(T, p))
    return np.concatenate([r0, r0 + np.cumsum(steps, axis=0)], axis=0)


def diag_problem(n: int, m: int, T: int, workload: int, instance: int) -> LQTProblem:
    """Workload-2 style instance: diagonal costs, random-walk reference."""
    rng = _rng(workload, instance)
    F, L = _dynamics(rng, n, m, 0.99)
    q = rng.uniform(1.0, 10.0, size=n)
    ru = rng.uniform(0.01, 1.0, size=m)
    rr = _random_walk(rng, T, n)
    x0 = rng.normal(0.0, 1.0, size=n)
    Q = np.diag(q)
    return LQTProblem(n=n, m=m, p=n, pT=n, T=T, per_step=0, F=F, c=None, L=L,
                      H=np.eye(n), X=Q, U=np.diag(ru), r=np.ascontiguousarray(rr[:T]),
                      HT=np.eye(n), XT=Q.copy(), rT=np.ascontiguousarray(rr[T]), x0=x0)


def batched_shapes(count: int = 4096, workload: int = 2):
    """(n, T) for each instance of the uneven batch, drawn before the data."""
    rng = _rng(workload, 1 << 30)
    Ts = np.rint(np.exp(rng.uniform(math.log(256), math.log(16384), size=count))).astype(np.int64)
    ns = rng.choice(np.array([4, 8, 16]), size=count)
    return [(int(n), int(t)) for n, t in zip(ns, Ts)]


def batched_problems(count: int = 4096, workload: int = 2):
    return [diag_problem(n, n // 2, T, workload, i) for i, (n, T) in enumerate(batched_shapes(count, workload))]


def dense_problem(n: int = 64, m: int = 32, T: int = 8192, workload: int = 3, instance: int = 0) -> LQTProblem:
    """Workload-3 instance: dense SPD costs, spectral radius 0.98."""
    rng = _rng(workload, instance)
    F, L = _dynamics(rng, n, m, 0.98)
    W = rng.normal(0.0, 1.0 / math.sqrt(n), size=(n, n))
    Wu = rng.normal(0.0, 1.0 / math.sqrt(m), size=(m, m))
    Q = W @ W.T + 0.1 * np.eye(n)
    R = Wu @ Wu.T + 0.1 * np.eye(m)
    Q = 0.5 * (Q + Q.T)
    R = 0.5 * (R + R.T)
    rr = _random_walk(rng, T, n)
    x0 = rng.normal(0.0, 1.0, size=n)
    return LQTProblem(n=n, m=m, p=n, pT=n, T=T, per_step=0, F=F, c=None, L=L,
                      H=np.eye(n), X=Q, U=R, r=np.ascontiguousarray(rr[:T]),
                      HT=np.eye(n), XT=Q.copy(), rT=np.ascontiguousarray(rr[T]), x0=x0)


def serving_requests(rate_hz: float = 2000.0, seconds: float = 60.0, workload: int = 4):
    """Arrival times (s) and (n, m, T) of the request stream (data drawn lazily
    with ``diag_problem(n, m, T, workload, i)``)."""
    rng = _rng(workload, 1 << 30)
    t, out = 0.0, []
    while True:
        t += rng.exponential(1.0 / rate_hz)
        if t >= seconds:
            break
        n = int(rng.integers(4, 33))
        T = int(round(math.exp(rng.uniform(math.log(64), math.log(65536)))))
        out.append((t, n, (n + 1) // 2, T))
    return out


def random_problem(n: int, m: int, T: int, seed: int, p: Optional[int] = None, pT: Optional[int] = None,
                   per_step: int = 0, with_c: bool = True, scale: float = 1.0) -> LQTProblem:
    """Fully random instance for edge-case and parity tests: general H (p x n),
    SPD X and U, non-zero offsets c, optional per-step matrices."""
    rng = np.random.Generator(np.random.PCG64(np.random.SeedSequence([BASE_SEED, 99, seed])))
    p = n if p is None else p
    pT = n if pT is None else pT

    def mat(shape_one, bit, fn):
        if per_step & bit:
            return np.ascontiguousarray(np.stack([fn() for _ in range(T)]))
        return np.ascontiguousarray(fn())

    def spd(k, lo):
        W = rng.normal(0.0, 1.0 / math.sqrt(k), size=(k, k))
        A = W @ W.T + lo * np.eye(k)
        return 0.5 * (A + A.T)

    def dyn():
        G = rng.normal(0.0, 1.0 / math.sqrt(n), size=(n, n))
        F0 = np.eye(n) + 0.3 * G
        return F0 * (scale / max(1e-12, np.max(np.abs(np.linalg.eigvals(F0)))))

    F = mat((n, n), PS_F, dyn)
    c = mat((n,), PS_c, lambda: rng.normal(0.0, 0.3, size=n)) if with_c else None
    L = mat((n, m), PS_L, lambda: rng.normal(0.0, 1.0, size=(n, m)))
    H = mat((p, n), PS_H, lambda: rng.normal(0.0, 1.0, size=(p, n)))
    X = mat((p, p), PS_X, lambda: spd(p, 0.5))
    U = mat((m, m), PS_U, lambda: spd(m, 0.2))
    r = rng.normal(0.0, 1.0, size=(T, p))
    HT = rng.normal(0.0, 1.0, size=(pT, n))
    XT = spd(pT, 0.5)
    rT = rng.normal(0.0, 1.0, size=pT)
    x0 = rng.normal(0.0, 1.0, size=n)
    if not with_c:
        per_step &= ~PS_c
    return LQTProblem(n=n, m=m, p=p, pT=pT, T=T, per_step=per_step, F=F, c=c, L=L, H=H, X=X, U=U,
                      r=r, HT=HT, XT=XT, rT=rT, x0=x0)


def generalised_problem(n: int, m: int, T: int, seed: int, p: Optional[int] = None, per_step: int = 0,
                        with_c: bool = True, with_s: bool = True, scale: float = 0.95) -> LQTProblem:
    """random_problem with the generalised stage cost of the extension to more
    general cost functions: a cross term M ([p][m]) between the output error
    and the control error, and a control reference s ([T][m]).  X, M and U
    are the blocks of one random positive definite (p + m) x (p + m) matrix,
    so the stage cost stays convex; per_step bits F, c and r-like data only
    (the library's transformation keeps L, H, X, U, M time-invariant)."""
    base = random_problem(n, m, T, seed=seed, p=p, pT=n, per_step=per_step & (PS_F | PS_c), with_c=with_c,
                          scale=scale)
    rng = np.random.Generator(np.random.PCG64(np.random.SeedSequence([BASE_SEED, 98, seed])))
    q = base.p + m
    Wb = rng.normal(0.0, 1.0 / math.sqrt(q), size=(q, q))
    Bm = Wb @ Wb.T + 0.3 * np.eye(q)
    Bm = 0.5 * (Bm + Bm.T)
    base.X = np.ascontiguousarray(Bm[:base.p, :base.p])
    base.M = np.ascontiguousarray(Bm[:base.p, base.p:])
    base.U = np.ascontiguousarray(Bm[base.p:, base.p:])
    base.s = np.ascontiguousarray(rng.normal(0.0, 0.3, size=(T, m))) if with_s else None
    return base


@dataclasses.dataclass
class UnicycleProblem:
    """Nonlinear tracking with the unicycle model of the nonlinear experiment
    (Section VI-E): state (p_x, p_y, theta, speed), control (acceleration, turn
    rate), x_{k+1} = f(x_k, u_k; dt_k); running cost
    1/2 (H x - r_k)^T X_k (H x - r_k) + 1/2 u^T U u, terminal
    1/2 (H_T x - r_T)^T X_T (H_T x - r_T).  X carries a time axis (weights
    switch on at the steps with a reference point).  ``xbar``, ``ubar``: the
    nominal trajectory the iteration starts from."""
    T: int
    dt: np.ndarray     # [T]
    H: np.ndarray      # [3][4]
    X: np.ndarray      # [T][3][3]
    U: np.ndarray      # [2][2]
    r: np.ndarray      # [T][3]
    HT: np.ndarray     # [3][4]
    XT: np.ndarray     # [3][3]
    rT: np.ndarray     # [3]
    x0: np.ndarray     # [4]
    xbar: np.ndarray   # [T + 1][4]
    ubar: np.ndarray   # [T][2]
    n: int = 4
    m: int = 2
    p: int = 3


def mass_spring_problem(N: int, T: int, horizon: float = 10.0, mass: float = 1.0, spring: float = 1.0,
                        damper: float = 0.2, x_weight: float = 1.0, u_weight: float = 1.0) -> LQTProblem:
    """Chain of N masses joined by springs and dampers, forces on the first
    and the last mass (the state-dimension experiment, Section VI-C): state
    (y_1, y_1', ..., y_N, y_N'), n = 2N, m = 2, driven to the origin from
    y_1 = y_{floor(N/2)+1} = 1 over `horizon` seconds in T steps.  Zero-order
    hold discretisation in closed form: the exponential of the augmented
    matrix [[A_c, B_c], [0, 0]] dt gives F and L.  The cost weights are not
    given for this experiment; X = x_weight I (all states, reference 0),
    U = u_weight I, X_T = X."""
    import scipy.linalg

    n, m = 2 * N, 2
    Ac = np.zeros((n, n))
    Bc = np.zeros((n, m))
    k, d = spring / mass, damper / mass
    for i in range(N):
        yi, vi = 2 * i, 2 * i + 1
        Ac[yi, vi] = 1.0
        Ac[vi, yi] = -2.0 * k
        Ac[vi, vi] = -2.0 * d
        for j in (i - 1, i + 1):  # neighbours (the chain's ends have one)
            if 0 <= j < N:
                Ac[vi, 2 * j] = k
                Ac[vi, 2 * j + 1] = d
    Bc[1, 0] = 1.0 / mass
    Bc[2 * (N - 1) + 1, 1] = -1.0 / mass
    dt = horizon / T
    aug = np.zeros((n + m, n + m))
    aug[:n, :n] = Ac
    aug[:n, n:] = Bc
    E = scipy.linalg.expm(aug * dt)
    F = np.ascontiguousarray(E[:n, :n])
    L = np.ascontiguousarray(E[:n, n:])
    x0 = np.zeros(n)
    x0[0] = 1.0
    x0[2 * (N // 2)] = 1.0
    eye = np.eye(n)
    return LQTProblem(n=n, m=m, p=n, pT=n, T=T, per_step=0, F=F, c=None, L=L, H=eye.copy(),
                      X=x_weight * eye, U=u_weight * np.eye(m), r=np.zeros((T, n)), HT=eye.copy(),
                      XT=x_weight * eye, rT=np.zeros(n), x0=x0)


def race_track(T: int, dt: float = 0.1, omega: float = 0.12):
    """A closed synthetic track (the paper's track is shown only in a figure):
    P(phi) = (50 cos phi, 30 sin phi + 8 sin 2 phi), phi = omega t, driven
    round several times.  Returns positions [T+1][2], unwrapped heading
    [T+1] and speed [T+1] along it."""
    t = dt * np.arange(T + 1, dtype=np.float64)
    ph = omega * t
    pos = np.stack([50.0 * np.cos(ph), 30.0 * np.sin(ph) + 8.0 * np.sin(2.0 * ph)], axis=1)
    vel = omega * np.stack([-50.0 * np.sin(ph), 30.0 * np.cos(ph) + 16.0 * np.cos(2.0 * ph)], axis=1)
    heading = np.unwrap(np.arctan2(vel[:, 1], vel[:, 0]))
    speed = np.hypot(vel[:, 0], vel[:, 1])
    return pos, heading, speed


def unicycle_problem(T: int, seed: int = 0, ref_every: int = 5, dt: float = 0.1, noise: float = 0.5,
                     start: str = "track") -> UnicycleProblem:
    """Nonlinear unicycle tracking workload (Section VI, nonlinear experiment)
    on the synthetic race track: reference points (position and heading,
    jittered by N(0, noise^2) in position) every ``ref_every`` steps with the
    experiment's weights (100 on position, 1000 on heading; 1e-6 elsewhere and
    at the terminal step), U = diag(1, 100), dt = 0.1.  start = "track": the
    nominal trajectory is the noiseless track with zero controls; "x0": every
    nominal state is x_0 (one of the paper's suggested initialisations)."""
    rng = np.random.Generator(np.random.PCG64(np.random.SeedSequence([BASE_SEED, 7, seed])))
    pos, heading, speed = race_track(T, dt)
    r = np.concatenate([pos[:T] + rng.normal(0.0, noise, size=(T, 2)), heading[:T, None]], axis=1)
    has = (np.arange(T) % ref_every) == 0
    lo = 1e-6
    X = np.empty((T, 3, 3))
    X[:] = lo * np.eye(3)
    X[has] = np.diag([100.0, 100.0, 1000.0])
    H = np.zeros((3, 4))
    H[0, 0] = H[1, 1] = H[2, 2] = 1.0
    x0 = np.array([pos[0, 0], pos[0, 1], heading[0], speed[0]])
    if start == "track":
        xbar = np.concatenate([pos, heading[:, None], speed[:, None]], axis=1)
    else:
        xbar = np.broadcast_to(x0, (T + 1, 4)).copy()
    xbar[0] = x0
    return UnicycleProblem(T=T, dt=np.full(T, dt), H=H, X=np.ascontiguousarray(X), U=np.diag([1.0, 100.0]),
                           r=np.ascontiguousarray(r), HT=H.copy(), XT=lo * np.eye(3),
                           rT=np.array([pos[T, 0], pos[T, 1], heading[T]]), x0=x0,
                           xbar=np.ascontiguousarray(xbar), ubar=np.zeros((T, 2)))


@dataclasses.dataclass
class FiniteProblem:
    """Finite state and control spaces (Section III-D): next [Dx][Du] or
    [T][Dx][Du] (int32, -1 = not admissible), cost of the same shape
    (float64), cost_T [Dx], initial state x0."""
    nstates: int
    ncontrols: int
    T: int
    next: np.ndarray
    cost: np.ndarray
    cost_T: np.ndarray
    x0: int


def routing_problem(T: int, nstates: int = 11, seed: int = 0) -> FiniteProblem:
    """The aircraft-routing workload of the finite-state experiment (Section
    VI-D; its cost grid is shown only in a figure): states are altitude
    levels 0..Dx-1, controls up / straight / down (the two moves cost one
    unit, straight nothing, no move leaves the grid), every grid point costs
    0, 1 or 2 (seeded uniform), the terminal cost is the last column's grid
    cost, the start is the middle level.  Integer-valued costs."""
    rng = np.random.Generator(np.random.PCG64(np.random.SeedSequence([BASE_SEED, 8, seed])))
    D = nstates
    grid = rng.integers(0, 3, size=(T + 1, D)).astype(np.float64)
    nxt = np.empty((D, 3), dtype=np.int32)
    for i in range(D):
        nxt[i] = [i + 1 if i + 1 < D else -1, i, i - 1 if i >= 1 else -1]
    move = np.array([1.0, 0.0, 1.0])
    cost = grid[:T, :, None] + move[None, None, :]
    return FiniteProblem(nstates=D, ncontrols=3, T=T, next=nxt, cost=np.ascontiguousarray(cost),
                         cost_T=np.ascontiguousarray(grid[T]), x0=D // 2)


def random_finite_problem(T: int, nstates: int, ncontrols: int, seed: int, per_step: int = 3,
                          integer: bool = True, p_blocked: float = 0.2) -> FiniteProblem:
    """Random tables: next states uniform (a fraction p_blocked not
    admissible), costs uniform on 0..9 (integer-valued) or U[0, 10)."""
    rng = np.random.Generator(np.random.PCG64(np.random.SeedSequence([BASE_SEED, 9, seed])))
    D, Du = nstates, ncontrols
    shape_n = (T, D, Du) if per_step & 1 else (D, Du)
    shape_c = (T, D, Du) if per_step & 2 else (D, Du)
    nxt = rng.integers(0, D, size=shape_n).astype(np.int32)
    nxt[rng.random(size=shape_n) < p_blocked] = -1
    if integer:
        cost = rng.integers(0, 10, size=shape_c).astype(np.float64)
        cost_T = rng.integers(0, 10, size=D).astype(np.float64)
    else:
        cost = rng.uniform(0.0, 10.0, size=shape_c)
        cost_T = rng.uniform(0.0, 10.0, size=D)
    return FiniteProblem(nstates=D, ncontrols=Du, T=T, next=np.ascontiguousarray(nxt),
                         cost=np.ascontiguousarray(cost), cost_T=cost_T, x0=int(rng.integers(0, D)))
