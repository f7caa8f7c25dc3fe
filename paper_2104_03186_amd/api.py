"""Python front end of the HIP LQT solver (argument marshalling only).

PyTorch provides device memory and streams; every arithmetic step runs in the
HIP kernels of liblqt.so through the C ABI of include/lqt.h.
"""
from __future__ import annotations

import ctypes
from typing import Dict, Iterable, List, Optional, Sequence

import numpy as np
import torch

from . import _lib

FAMILIES = ("S", "v", "K", "d", "x", "u")
_PREC = {"fp64": _lib.PREC_FP64, "mixed": _lib.PREC_MIXED}
_TRAJ = {"maps": _lib.TRAJ_MAPS, "prefix": _lib.TRAJ_PREFIX}
_PATH = {None: 0, "auto": 0, "small": 1, "wave": 2, "batch": 3}


def _ptr(t: Optional[torch.Tensor]) -> Optional[int]:
    return None if t is None else t.data_ptr()


class DeviceProblem:
    """An LQT instance resident in device memory (float64 tensors)."""

    FIELDS = ("F", "c", "L", "H", "X", "U", "r", "HT", "XT", "rT", "x0", "M", "s")

    def __init__(self, prob, device="cuda:0"):
        self.n, self.m, self.p, self.pT = int(prob.n), int(prob.m), int(prob.p), int(prob.pT)
        self.T, self.per_step = int(prob.T), int(prob.per_step)
        self.t = {}
        for f in self.FIELDS:
            a = getattr(prob, f, None)  # M, s: generalised stage cost (Section IV-D)
            self.t[f] = None if a is None else torch.from_numpy(np.ascontiguousarray(a, dtype=np.float64)).to(device)

    def struct(self, T: Optional[int] = None) -> _lib.Problem:
        """The C struct; T (<= self.T) takes the instance over its first T
        steps (per-step arrays read as prefixes; the terminal data unchanged)."""
        s = _lib.Problem()
        if T is None:
            T = self.T  # passed as given: the library validates it
        elif not 1 <= int(T) <= self.T:
            raise ValueError(f"prefix T={T} outside 1..{self.T}")
        s.nx, s.nu, s.ny, s.nyT, s.T, s.per_step = self.n, self.m, self.p, self.pT, T, self.per_step
        for f in self.FIELDS:
            setattr(s, f, _ptr(self.t[f]))
        return s


class DeviceNLProblem:
    """A nonlinear tracking instance for the iterated linearisation (Section
    IV-D, nonlinear extension) resident in device memory; ``prob`` has the attributes of
    inputs.UnicycleProblem (model: the unicycle of Section VI-E)."""

    FIELDS = ("dt", "H", "X", "U", "r", "HT", "XT", "rT", "x0")

    def __init__(self, prob, device="cuda:0"):
        self.T, self.p, self.pT = int(prob.T), int(prob.p), int(np.asarray(prob.rT).shape[0])
        X = np.asarray(prob.X)
        self.per_step = _lib.PS_X if X.ndim == 3 else 0
        self.t = {f: torch.from_numpy(np.ascontiguousarray(getattr(prob, f), dtype=np.float64)).to(device)
                  for f in self.FIELDS}

    def struct(self) -> _lib.NLProblem:
        s = _lib.NLProblem()
        s.model, s.ny, s.nyT, s.T, s.per_step = _lib.NL_UNICYCLE, self.p, self.pT, self.T, self.per_step
        for f in self.FIELDS:
            setattr(s, f, _ptr(self.t[f]))
        return s


class DeviceFSProblem:
    """A finite state and control problem (Section III-D) resident in device
    memory; ``prob`` has the attributes of inputs.FiniteProblem."""

    def __init__(self, prob, device="cuda:0"):
        self.D, self.Du, self.T, self.x0 = int(prob.nstates), int(prob.ncontrols), int(prob.T), int(prob.x0)
        nxt, cost = np.asarray(prob.next), np.asarray(prob.cost)
        self.per_step = (_lib.FS_NEXT if nxt.ndim == 3 else 0) | (_lib.FS_COST if cost.ndim == 3 else 0)
        self.t = {"next": torch.from_numpy(np.ascontiguousarray(nxt, dtype=np.int32)).to(device),
                  "cost": torch.from_numpy(np.ascontiguousarray(cost, dtype=np.float64)).to(device),
                  "cost_T": torch.from_numpy(np.ascontiguousarray(prob.cost_T, dtype=np.float64)).to(device)}

    def struct(self) -> _lib.FSProblem:
        s = _lib.FSProblem()
        s.nstates, s.ncontrols, s.T, s.per_step, s.x0 = self.D, self.Du, self.T, self.per_step, self.x0
        for f, t in self.t.items():
            setattr(s, f, _ptr(t))
        return s


class DeviceFSOutputs:
    """Outputs of a finite-state solve: V [T+1][D] (float64), u [T][D], x
    [T+1], ux [T] (int32); ``want`` selects them (others NULL)."""

    def __init__(self, D: int, T: int, device="cuda:0", want: Iterable[str] = ("V", "u", "x", "ux")):
        want = set(want)
        spec = {"V": ((T + 1, D), torch.float64), "u": ((T, D), torch.int32), "x": ((T + 1,), torch.int32),
                "ux": ((T,), torch.int32)}
        self.t = {k: (torch.empty(sh, dtype=dt, device=device) if k in want else None) for k, (sh, dt) in spec.items()}
        self.status = torch.full((1,), -1, dtype=torch.int32, device=device)

    def struct(self) -> _lib.FSOutputs:
        s = _lib.FSOutputs()
        for k, t in self.t.items():
            setattr(s, k, _ptr(t))
        s.status = _ptr(self.status)
        return s

    def host(self) -> Dict[str, np.ndarray]:
        return {k: v.cpu().numpy() for k, v in self.t.items() if v is not None}


class DeviceOutputs:
    """Output buffers of one instance.  ``want`` lists the families to produce
    (the others are passed as NULL)."""

    def __init__(self, n: int, m: int, T: int, device="cuda:0", dtype=torch.float64,
                 want: Iterable[str] = FAMILIES, status: bool = True):
        want = set(want)
        shapes = {"S": (T + 1, n, n), "v": (T + 1, n), "K": (T, m, n), "d": (T, m), "x": (T + 1, n), "u": (T, m)}
        self.t: Dict[str, Optional[torch.Tensor]] = {
            k: (torch.empty(shapes[k], dtype=dtype, device=device) if k in want else None) for k in FAMILIES}
        self.status = torch.full((1,), -1, dtype=torch.int32, device=device) if status else None

    def struct(self) -> _lib.Outputs:
        s = _lib.Outputs()
        for k in FAMILIES:
            setattr(s, k, _ptr(self.t[k]))
        s.status = _ptr(self.status)
        return s

    def host(self) -> Dict[str, np.ndarray]:
        return {k: v.double().cpu().numpy() for k, v in self.t.items() if v is not None}


class Plan:
    """Owns an lqt_plan_t (workspace on one device)."""

    def __init__(self, max_nx: int, max_nu: int, prec: str = "fp64", device: int = 0, max_steps: int = 0,
                 hbm_budget_bytes: int = 0, max_inflight: int = 0, trajectory: str = "maps"):
        """trajectory: "maps" (Method 1, scan of the closed-loop affine maps) or
        "prefix" (Method 2, forward scan of the LQT elements from x_0)."""
        lib = _lib.load()
        if trajectory not in _TRAJ:
            raise ValueError(f"trajectory must be one of {sorted(_TRAJ)}")
        d = _lib.PlanDesc(device=device, max_nx=max_nx, max_nu=max_nu, prec=_PREC[prec],
                          hbm_budget_bytes=hbm_budget_bytes, max_steps=max_steps, max_inflight=max_inflight,
                          trajectory=_TRAJ[trajectory])
        h = ctypes.c_void_p()
        _lib.check(lib.lqt_plan(ctypes.byref(d), ctypes.byref(h)), None)
        self._h = h
        self.device = device
        self.prec = prec

    @property
    def handle(self):
        return self._h

    def solve(self, probs: Sequence[DeviceProblem], outs: Sequence[DeviceOutputs], stream=None) -> None:
        """Enqueue the solve of every instance on ``stream`` (default: torch's
        current stream).  Asynchronous."""
        if len(probs) != len(outs):
            raise ValueError("probs and outs differ in length")
        for o in outs:
            self._check_dtype(o)
        n = len(probs)
        P = (_lib.Problem * max(n, 1))(*[p.struct() for p in probs])
        O = (_lib.Outputs * max(n, 1))(*[o.struct() for o in outs])
        if stream is None:
            stream = torch.cuda.current_stream(self.device)
        sp = ctypes.c_void_p(stream.cuda_stream)
        _lib.check(_lib.load().lqt_solve(self._h, P, O, n, sp), self._h)

    def solve_noalloc(self, prob: DeviceProblem, out: DeviceOutputs, stream=None) -> None:
        """One instance through lqt_solve_noalloc: the library's fixed device
        workspace, no allocation.  Asynchronous."""
        self._check_dtype(out)
        if stream is None:
            stream = torch.cuda.current_stream(self.device)
        ps, os_ = prob.struct(), out.struct()
        _lib.check(_lib.load().lqt_solve_noalloc(self._h, ctypes.byref(ps), ctypes.byref(os_),
                                                 ctypes.c_void_p(stream.cuda_stream)), self._h)

    def tune(self, probs: Sequence[DeviceProblem], outs: Sequence[DeviceOutputs], stream=None) -> List[int]:
        """Pick the chunk length of every launch group present from timed
        solves of these instances (lqt_tune); returns the 8 chosen divisors."""
        if len(probs) != len(outs):
            raise ValueError("probs and outs differ in length")
        for o in outs:
            self._check_dtype(o)
        n = len(probs)
        P = (_lib.Problem * max(n, 1))(*[p.struct() for p in probs])
        O = (_lib.Outputs * max(n, 1))(*[o.struct() for o in outs])
        if stream is None:
            stream = torch.cuda.current_stream(self.device)
        ch = (ctypes.c_int32 * 8)()
        _lib.check(_lib.load().lqt_tune(self._h, P, O, n, ctypes.c_void_p(stream.cuda_stream), ch), self._h)
        return list(ch)

    def set_graphs(self, enable: bool = True) -> None:
        """Record repeated solve / nl_iterate calls as HIP graphs and replay
        them (lqt_set_graphs)."""
        _lib.check(_lib.load().lqt_set_graphs(self._h, 1 if enable else 0), self._h)

    def graphs_recorded(self) -> int:
        """Signatures currently recorded as graphs (lqt_graphs_recorded)."""
        n = _lib.load().lqt_graphs_recorded(self._h)
        if n < 0:
            raise _lib.LQTError(-n, _lib.last_error(self._h))
        return n

    def set_routing(self, path: Optional[str] = None, wave_engine_only: bool = False, lane_chunk: int = 0,
                    wave_chunk: int = 0, tree: Optional[bool] = None) -> None:
        """Routing and chunking overrides of this plan (lqt_set_routing):
        path "small" (lane pipeline wherever it applies), "wave" (chunked
        engines) or "batch" (batched lane kernel wherever it applies),
        wave_engine_only keeps the classes 16/32 off the workgroup
        engines, lane_chunk / wave_chunk fix the chunk lengths (0: automatic),
        tree True / False scans the chunks of every chunked instance as trees /
        as walks (None: trees from 128 chunks on).  Called with no arguments it
        restores the automatic choices."""
        r = _lib.Routing(path=_PATH[path], block=1 if wave_engine_only else 0, lane_chunk=int(lane_chunk or 0),
                         wave_chunk=int(wave_chunk or 0), tree=0 if tree is None else (1 if tree else 2))
        _lib.check(_lib.load().lqt_set_routing(self._h, ctypes.byref(r)), self._h)

    def _check_dtype(self, out: DeviceOutputs) -> None:
        want = torch.float64 if self.prec == "fp64" else torch.float32
        for k, t in out.t.items():
            if t is not None and t.dtype != want:
                raise TypeError(f"output {k} is {t.dtype}; a {self.prec} plan writes {want}")

    def nl_iterate(self, prob: "DeviceNLProblem", iterations: int, x: torch.Tensor, u: torch.Tensor,
                   change: Optional[torch.Tensor] = None, status: Optional[torch.Tensor] = None,
                   stream=None) -> None:
        """Iterated linearisation (lqt_nl_iterate): x ([T+1][4]) and u ([T][2])
        hold the nominal trajectory and receive the last round's solution;
        change ([iterations] float64) the per-round max |u_new - u_nominal|;
        status (int32) the first failing round's status.  Asynchronous."""
        want = torch.float64 if self.prec == "fp64" else torch.float32
        for name, t in (("x", x), ("u", u)):
            if t.dtype != want or not t.is_contiguous():
                raise TypeError(f"{name} must be a contiguous {want} tensor for a {self.prec} plan")
        if change is not None and change.dtype != torch.float64:
            raise TypeError("change must be float64")
        if status is not None and status.dtype != torch.int32:
            raise TypeError("status must be int32")
        if stream is None:
            stream = torch.cuda.current_stream(self.device)
        ps = prob.struct()
        _lib.check(_lib.load().lqt_nl_iterate(self._h, ctypes.byref(ps), int(iterations), _ptr(x), _ptr(u),
                                              _ptr(change), _ptr(status), ctypes.c_void_p(stream.cuda_stream)),
                   self._h)

    def fs_solve(self, prob: "DeviceFSProblem", out: "DeviceFSOutputs", stream=None) -> None:
        """Finite state and control problem (lqt_fs_solve).  Asynchronous."""
        if stream is None:
            stream = torch.cuda.current_stream(self.device)
        ps, os_ = prob.struct(), out.struct()
        _lib.check(_lib.load().lqt_fs_solve(self._h, ctypes.byref(ps), ctypes.byref(os_),
                                            ctypes.c_void_p(stream.cuda_stream)), self._h)

    def submit(self, prob: DeviceProblem, out: DeviceOutputs, T: Optional[int] = None) -> int:
        """Queue one instance (lqt_submit); T: solve the instance's first T
        steps (out sized for T).  Returns the ticket."""
        self._check_dtype(out)
        t = ctypes.c_uint64()
        ps, os_ = prob.struct(T), out.struct()
        _lib.check(_lib.load().lqt_submit(self._h, ctypes.byref(ps), ctypes.byref(os_), ctypes.byref(t)), self._h)
        return int(t.value)

    def poll(self, ticket: int) -> Optional[int]:
        """None while in flight, else the instance status (0 = LQT_OK)."""
        rc = _lib.load().lqt_poll(self._h, ticket)
        if rc == _lib.EAGAIN:
            return None
        if rc == _lib.EINVAL or rc == _lib.EHIP:
            raise _lib.LQTError(rc, _lib.last_error(self._h))
        return rc

    def serve_stats(self) -> Dict[str, int]:
        """Counters of the serving interface (lqt_serve_stats_read)."""
        st = _lib.ServeStats()
        _lib.check(_lib.load().lqt_serve_stats_read(self._h, ctypes.byref(st)), self._h)
        return {f: int(getattr(st, f)) for f, _ in _lib.ServeStats._fields_}

    def profile(self, enable: bool = True) -> None:
        """Bracket every kernel launch with HIP events (see profile_read)."""
        _lib.check(_lib.load().lqt_profile_enable(self._h, 1 if enable else 0), self._h)

    def profile_select(self, stage: Optional[str] = None) -> None:
        """Time only the launches of ``stage`` (None: every stage)."""
        _lib.check(_lib.load().lqt_profile_select(self._h, None if stage is None else stage.encode()), self._h)

    def profile_read(self) -> Dict[str, tuple]:
        """{stage: (launches, total_ms)} since the last read (synchronises)."""
        buf = (_lib.StageTime * 64)()
        n = _lib.load().lqt_profile_read(self._h, buf, 64)
        if n < 0:
            raise _lib.LQTError(-n, _lib.last_error(self._h))
        return {buf[i].name.decode(): (int(buf[i].launches), float(buf[i].total_ms)) for i in range(n)}

    def close(self):
        if self._h:
            _lib.load().lqt_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def solve_host(prob, prec: str = "fp64", device: int = 0) -> Dict[str, np.ndarray]:
    """Convenience: copy one host problem to the device, solve, copy back."""
    dev = f"cuda:{device}"
    plan = Plan(prob.n, prob.m, prec=prec, device=device)
    dp = DeviceProblem(prob, dev)
    do = DeviceOutputs(prob.n, prob.m, prob.T, dev,
                       dtype=torch.float64 if prec == "fp64" else torch.float32)
    plan.solve([dp], [do])
    torch.cuda.synchronize(device)
    st = int(do.status.item())
    plan.close()
    if st != _lib.OK:
        raise _lib.LQTError(st, "instance status")
    return do.host()
