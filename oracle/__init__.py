"""FP64 CPU oracle for the linear-quadratic tracker (LQT).

TEST INFRASTRUCTURE ONLY: the test suite, the smoke check and the CPU-baseline
leg of the benchmark may import this package; the product package never does.
It shares no code with the HIP implementation.

The arithmetic lives in ``lqt_oracle.c`` (plain C, IEEE double), a direct
transcription of:

* Section II-B: sequential backward recursion for S_k, v_k, the gain K_k, the
  control law u_k = -K_k x_k + K^v_k v_{k+1} - K^c_k c_k and the forward pass
  of the dynamics (``solve``);
* Section IV-B: the one-step elements (A, b, C, eta, J) of the backward scan
  and the terminal element (``element``);
* Section IV-A: the LQT associative combination rule (``combine``);
* Section II-B: the total tracking cost (``cost``).

This wrapper only marshals arrays; it builds the shared object with gcc on
first use when it is missing.

Problem objects are duck-typed: any object with the attributes
``n, m, p, pT, T, per_step, F, c, L, H, X, U, r, HT, XT, rT, x0`` (numpy
float64 arrays, ``c`` may be ``None``) is accepted.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
import time

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "lqt_oracle.c")
_BUILD = os.path.join(_HERE, "_build")
_SO = os.path.join(_BUILD, "liblqt_oracle.so")

OK, EINVAL, ENOTPD, ENONFINITE = 0, 1, 3, 4

_lib = None


def build(force: bool = True) -> str:
    """Compile the oracle with gcc (no fast-math: IEEE semantics)."""
    if not force and os.path.exists(_SO):
        return _SO
    os.makedirs(_BUILD, exist_ok=True)
    tmp = _SO + f".tmp{os.getpid()}"
    subprocess.check_call(
        ["gcc", "-O2", "-fno-fast-math", "-ffp-contract=off", "-shared", "-fPIC",
         "-o", tmp, _SRC, "-lm"])
    os.replace(tmp, _SO)
    return _SO


def _load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_SO) or os.path.getmtime(_SO) < os.path.getmtime(_SRC):
        build()
    lib = ctypes.CDLL(_SO)
    dp = ctypes.POINTER(ctypes.c_double)
    i32, i64, u32 = ctypes.c_int, ctypes.c_int64, ctypes.c_uint32
    lib.oracle_solve.argtypes = [i32, i32, i32, i32, i64, u32] + [dp] * 17
    lib.oracle_solve.restype = i32
    lib.oracle_solve_gen.argtypes = [i32, i32, i32, i32, i64, u32] + [dp] * 19
    lib.oracle_solve_gen.restype = i32
    lib.oracle_element.argtypes = [i32, i32, i32, i32, i64, u32, i64] + [dp] * 11
    lib.oracle_element.restype = i32
    lib.oracle_combine.argtypes = [i32, dp, dp, dp]
    lib.oracle_combine.restype = i32
    lib.oracle_cost.argtypes = [i32, i32, i32, i32, i64, u32] + [dp] * 9
    lib.oracle_cost.restype = ctypes.c_double
    _lib = lib
    return lib


def _p(a):
    if a is None:
        return ctypes.POINTER(ctypes.c_double)()
    assert a.dtype == np.float64 and a.flags["C_CONTIGUOUS"]
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def _arr(a):
    return None if a is None else np.ascontiguousarray(a, dtype=np.float64)


class OracleError(RuntimeError):
    def __init__(self, code):
        super().__init__(f"oracle returned status {code}")
        self.code = code


def _inputs(prob):
    return [_arr(getattr(prob, k)) for k in ("F", "c", "L", "H", "X", "U", "r", "HT", "XT", "rT")]


def solve(prob) -> dict:
    """Sequential FP64 solution (Section II-B; with a cross term M or control
    reference s, the generalised stage cost of Section IV-D).  Returns S, v,
    K, d, x, u."""
    lib = _load()
    n, m, T = int(prob.n), int(prob.m), int(prob.T)
    out = {
        "S": np.empty((T + 1, n, n)), "v": np.empty((T + 1, n)),
        "K": np.empty((T, m, n)), "d": np.empty((T, m)),
        "x": np.empty((T + 1, n)), "u": np.empty((T, m)),
    }
    ins = _inputs(prob)
    x0 = _arr(prob.x0)
    M = getattr(prob, "M", None)
    s = getattr(prob, "s", None)
    if M is None and s is None:
        rc = lib.oracle_solve(n, m, int(prob.p), int(prob.pT), T, int(prob.per_step),
                              *[_p(a) for a in ins], _p(x0),
                              *[_p(out[k]) for k in ("S", "v", "K", "d", "x", "u")])
    else:  # generalised stage cost (Section IV-D)
        Mz = _arr(M) if M is not None else np.zeros((int(prob.p), m))
        rc = lib.oracle_solve_gen(n, m, int(prob.p), int(prob.pT), T, int(prob.per_step),
                                  *[_p(a) for a in ins], _p(x0), _p(Mz), _p(_arr(s)),
                                  *[_p(out[k]) for k in ("S", "v", "K", "d", "x", "u")])
    if rc != OK:
        raise OracleError(rc)
    return out


def element(prob, k: int) -> np.ndarray:
    """Element a_k (k < T) or the terminal element (k == T), Section IV-B.

    Packed as A[n*n] | b[n] | C[n*n] | eta[n] | J[n*n]."""
    lib = _load()
    n = int(prob.n)
    e = np.empty(3 * n * n + 2 * n)
    rc = lib.oracle_element(n, int(prob.m), int(prob.p), int(prob.pT), int(prob.T),
                            int(prob.per_step), int(k), *[_p(a) for a in _inputs(prob)], _p(e))
    if rc != OK:
        raise OracleError(rc)
    return e


def combine(n: int, e1: np.ndarray, e2: np.ndarray) -> np.ndarray:
    """e1 (x) e2 with the LQT combination rule (Section IV-A); e1 is earlier."""
    lib = _load()
    e1, e2 = _arr(e1), _arr(e2)
    out = np.empty(3 * n * n + 2 * n)
    rc = lib.oracle_combine(int(n), _p(e1), _p(e2), _p(out))
    if rc != OK:
        raise OracleError(rc)
    return out


def unpack(n: int, e: np.ndarray):
    """Split a packed element into (A, b, C, eta, J)."""
    nn = n * n
    return (e[:nn].reshape(n, n), e[nn:nn + n], e[nn + n:2 * nn + n].reshape(n, n),
            e[2 * nn + n:2 * nn + 2 * n], e[2 * nn + 2 * n:].reshape(n, n))


def pack(A, b, C, eta, J) -> np.ndarray:
    return np.concatenate([np.ravel(A), np.ravel(b), np.ravel(C), np.ravel(eta), np.ravel(J)]).astype(np.float64)


def cost(prob, x: np.ndarray, u: np.ndarray) -> float:
    """Total cost sum_k l_k(x_k, u_k) + l_T(x_T) of Section II-B."""
    lib = _load()
    x, u = _arr(x), _arr(u)
    return float(lib.oracle_cost(int(prob.n), int(prob.m), int(prob.p), int(prob.pT), int(prob.T),
                                 int(prob.per_step), _p(_arr(prob.H)), _p(_arr(prob.X)), _p(_arr(prob.U)),
                                 _p(_arr(prob.r)), _p(_arr(prob.HT)), _p(_arr(prob.XT)), _p(_arr(prob.rT)),
                                 _p(x), _p(u)))


def time_solve_parallel(probs, threads: int):
    """Time the unmodified oracle over a list of problems on `threads` host
    threads, the instances partitioned statically (longest first, each to the
    least-loaded thread); one pass.  The C solve runs without the Python
    interpreter lock, so the threads solve concurrently.  Returns
    (steps_per_second, seconds, threads)."""
    import threading

    threads = max(1, min(threads, len(probs)))
    cost = [int(p.n) ** 3 * int(p.T) + 1 for p in probs]
    order = sorted(range(len(probs)), key=lambda i: -cost[i])
    parts = [[] for _ in range(threads)]
    load = [0] * threads
    for i in order:
        j = load.index(min(load))
        parts[j].append(probs[i])
        load[j] += cost[i]

    def work(ps):
        for p in ps:
            solve(p)

    ts = [threading.Thread(target=work, args=(ps,)) for ps in parts]
    t0 = time.perf_counter()
    for t in ts:
        t.start()
    for t in ts:
        t.join()
    el = time.perf_counter() - t0
    return sum(int(p.T) for p in probs) / el, el, threads


def host_threads(limit: int = 16) -> int:
    """Host threads for a parallel baseline: the CPUs this process may use,
    at most `limit`."""
    try:
        n = len(os.sched_getaffinity(0))
    except AttributeError:
        n = os.cpu_count() or 1
    return max(1, min(limit, n))


def time_solve(probs, min_seconds: float = 10.0, max_reps: int = 1000):
    """Time the unmodified oracle on one host core over a list of problems.

    Repeats the whole list until ``min_seconds`` of wall time have passed (at
    least once).  Returns (steps_per_second, seconds, repetitions)."""
    steps = sum(int(p.T) for p in probs)
    reps, t0 = 0, time.perf_counter()
    while True:
        for p in probs:
            solve(p)
        reps += 1
        el = time.perf_counter() - t0
        if el >= min_seconds or reps >= max_reps:
            break
    return steps * reps / el, el, reps
