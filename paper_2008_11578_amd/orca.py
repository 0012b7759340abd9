"""Python binding of liborca.so (ctypes).  Argument marshalling only: every
step of the computation runs in the library's HIP kernels.

Tensors are torch tensors on the current HIP device, contiguous, FP32 (class:
uint8); work is enqueued on ``torch.cuda.current_stream()``.  Loading fails
loudly when the library has not been built: there is no CPU fallback.
"""
from __future__ import annotations

import ctypes
import dataclasses
import os
from typing import Dict, Optional

import torch

from . import scenarios

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "liborca.so")

ORCA_OK = 0
ORCA_K_MAX = 32
STATE_FIELDS = ("px", "py", "vx", "vy", "pref_x", "pref_y", "radius", "max_speed", "cls")


class OrcaError(RuntimeError):
    def __init__(self, fn: str, code: int):
        super().__init__(f"{fn} failed: {status_string(code)} ({code})")
        self.code = code


class OrcaParams(ctypes.Structure):
    _fields_ = [("dt", ctypes.c_float), ("time_horizon", ctypes.c_float),
                ("neighbor_dist", ctypes.c_float), ("cell_size", ctypes.c_float),
                ("max_neighbors", ctypes.c_int32), ("pref_is_goal", ctypes.c_int32),
                ("f", (ctypes.c_float * 2) * 2), ("par_eps", ctypes.c_float),
                ("accel", ctypes.c_float * 2), ("turn", ctypes.c_float * 2)]


class AgentsIn(ctypes.Structure):
    _fields_ = [(k, ctypes.c_void_p) for k in STATE_FIELDS]


class AgentsOut(ctypes.Structure):
    _fields_ = [(k, ctypes.c_void_p) for k in ("px", "py", "vx", "vy", "status")]


class OrcaBatch(ctypes.Structure):
    _fields_ = [("scene_off", ctypes.c_void_p), ("n_scenes", ctypes.c_int32),
                ("params", ctypes.c_void_p), ("max_neighbors", ctypes.c_int32),
                ("mode", ctypes.c_int32), ("error_flag", ctypes.c_void_p),
                ("has_accel", ctypes.c_int32), ("block", ctypes.c_int32),
                ("k_tile", ctypes.c_int32)]


class Cotangents(ctypes.Structure):
    _fields_ = [(k, ctypes.c_void_p) for k in ("px", "py", "vx", "vy")]


class CotangentsOut(ctypes.Structure):
    _fields_ = [(k, ctypes.c_void_p) for k in ("px", "py", "vx", "vy", "pref_x", "pref_y", "tau")]


class AgentsBuf(ctypes.Structure):
    _fields_ = [(k, ctypes.c_void_p) for k in ("px", "py", "vx", "vy", "pref_x", "pref_y",
                                                "radius", "max_speed", "cls")]


class StepEvents(ctypes.Structure):
    _fields_ = [("grid_begin", ctypes.c_void_p), ("step_begin", ctypes.c_void_p),
                ("step_end", ctypes.c_void_p)]


_lib = None


def lib() -> ctypes.CDLL:
    """The loaded library; raises if it has not been built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(
                f"{LIB_PATH} is missing: build it with `python -m paper_2008_11578_amd.build` "
                "(the ORCA step has no CPU fallback)")
        L = ctypes.CDLL(LIB_PATH)
        vp, sz, i32 = ctypes.c_void_p, ctypes.c_size_t, ctypes.c_int32
        L.orca_workspace_bytes.restype = sz
        L.orca_workspace_bytes.argtypes = [i32, i32, i32]
        L.orca_workspace_init.restype = ctypes.c_int
        L.orca_workspace_init.argtypes = [vp, sz, vp]
        L.orca_build_grid.restype = ctypes.c_int
        L.orca_build_grid.argtypes = [ctypes.POINTER(AgentsIn), i32, ctypes.POINTER(OrcaParams),
                                      vp, sz, vp, vp, vp]
        L.orca_step.restype = ctypes.c_int
        L.orca_step.argtypes = [ctypes.POINTER(AgentsIn), ctypes.POINTER(AgentsOut), i32,
                                ctypes.POINTER(OrcaParams), vp, sz, vp]
        L.orca_step_ex.restype = ctypes.c_int
        L.orca_step_ex.argtypes = [ctypes.POINTER(AgentsIn), ctypes.POINTER(AgentsOut), i32,
                                   ctypes.POINTER(OrcaParams), vp, sz,
                                   ctypes.POINTER(StepEvents), vp]
        L.orca_step_nbr.restype = ctypes.c_int
        L.orca_step_nbr.argtypes = [ctypes.POINTER(AgentsIn), ctypes.POINTER(AgentsOut), i32,
                                    ctypes.POINTER(OrcaParams), vp, sz, vp, vp, vp]
        L.orca_step_batched.restype = ctypes.c_int
        L.orca_step_noalloc.restype = ctypes.c_int
        L.orca_step_noalloc.argtypes = [ctypes.POINTER(AgentsIn), ctypes.POINTER(AgentsOut), i32,
                                        ctypes.POINTER(OrcaParams), vp]
        L.orca_step_batched.argtypes = [ctypes.POINTER(AgentsIn), ctypes.POINTER(AgentsOut), i32,
                                        ctypes.POINTER(OrcaBatch), vp, sz, vp]
        L.orca_step_batched_ex.restype = ctypes.c_int
        L.orca_step_batched_ex.argtypes = [ctypes.POINTER(AgentsIn), ctypes.POINTER(AgentsOut),
                                           i32, ctypes.POINTER(OrcaBatch), vp, sz,
                                           ctypes.POINTER(StepEvents), vp]
        L.orca_step_backward_ex.restype = ctypes.c_int
        L.orca_step_backward_ex.argtypes = [ctypes.POINTER(AgentsIn), i32,
                                            ctypes.POINTER(OrcaParams), ctypes.POINTER(Cotangents),
                                            ctypes.POINTER(CotangentsOut), vp, sz,
                                            ctypes.POINTER(StepEvents), vp]
        L.orca_backward_workspace_bytes.restype = sz
        L.orca_backward_workspace_bytes.argtypes = [i32, i32]
        L.orca_step_backward.restype = ctypes.c_int
        L.orca_step_backward.argtypes = [ctypes.POINTER(AgentsIn), i32, ctypes.POINTER(OrcaParams),
                                         ctypes.POINTER(Cotangents), ctypes.POINTER(CotangentsOut),
                                         vp, sz, vp]
        L.orca_lifecycle_workspace_bytes.restype = sz
        L.orca_lifecycle_workspace_bytes.argtypes = [i32, i32]
        L.orca_remove_arrived.restype = ctypes.c_int
        L.orca_remove_arrived.argtypes = [ctypes.POINTER(AgentsIn), ctypes.POINTER(AgentsBuf), i32,
                                          vp, vp, vp, sz, vp]
        L.orca_spawn.restype = ctypes.c_int
        L.orca_spawn.argtypes = [ctypes.POINTER(AgentsBuf), i32, i32, ctypes.POINTER(AgentsIn), i32,
                                 ctypes.c_float, vp, vp, vp, sz, vp]
        L.orca_overlap_workspace_bytes.restype = sz
        L.orca_overlap_workspace_bytes.argtypes = [i32]
        L.orca_overlap_stats.restype = ctypes.c_int
        L.orca_overlap_stats.argtypes = [ctypes.POINTER(AgentsIn), i32, ctypes.c_float, vp, vp, sz,
                                         vp]
        L.orca_status_string.restype = ctypes.c_char_p
        L.orca_status_string.argtypes = [ctypes.c_int]
        L.orca_version.restype = ctypes.c_char_p
        L.orca_version.argtypes = []
        _lib = L
    return _lib


def status_string(code: int) -> str:
    return lib().orca_status_string(int(code)).decode()


def version() -> str:
    return lib().orca_version().decode()


def make_params(p) -> OrcaParams:
    """From a ``scenarios.Params`` or a dict with the same field names."""
    g = p.get if isinstance(p, dict) else (lambda k: getattr(p, k))
    out = OrcaParams()
    out.dt = g("dt")
    out.time_horizon = g("time_horizon")
    out.neighbor_dist = g("neighbor_dist")
    out.cell_size = g("cell_size") if (not isinstance(p, dict) or "cell_size" in p) else 0.0
    out.max_neighbors = int(g("max_neighbors"))
    out.pref_is_goal = int(g("pref_is_goal"))
    f = g("f")
    for a in range(2):
        for b in range(2):
            out.f[a][b] = float(f[a][b])
    out.par_eps = g("par_eps")
    try:
        acc = g("accel")
    except (AttributeError, KeyError):
        acc = None
    acc = (0.0, 0.0) if acc is None else acc
    for c in range(2):
        out.accel[c] = float(acc[c])
    try:
        turn = g("turn")
    except (AttributeError, KeyError):
        turn = None
    turn = (0.0, 0.0) if turn is None else turn
    for c in range(2):
        out.turn[c] = float(turn[c])
    return out


def _stream_handle(stream=None) -> int:
    s = stream if stream is not None else torch.cuda.current_stream()
    return int(s.cuda_stream)


def _ptr(t: Optional[torch.Tensor]) -> Optional[int]:
    return None if t is None else int(t.data_ptr())


def _check(t: torch.Tensor, name: str, dtype, n: int):
    if not isinstance(t, torch.Tensor) or t.device.type != "cuda":
        raise TypeError(f"{name} must be a device tensor")
    if t.dtype != dtype or not t.is_contiguous() or t.numel() != n:
        raise TypeError(f"{name} must be contiguous {dtype} with {n} elements")


@dataclasses.dataclass
class State:
    """Agent state on the device, caller order (SoA)."""

    px: torch.Tensor
    py: torch.Tensor
    vx: torch.Tensor
    vy: torch.Tensor
    pref_x: torch.Tensor
    pref_y: torch.Tensor
    radius: torch.Tensor
    max_speed: torch.Tensor
    cls: torch.Tensor

    @property
    def n(self) -> int:
        return int(self.px.numel())

    @classmethod
    def from_arrays(cls, arrays, device="cuda") -> "State":
        g = arrays.get if isinstance(arrays, dict) else (lambda k: getattr(arrays, k))
        kw = {}
        for k in STATE_FIELDS:
            dt = torch.uint8 if k == "cls" else torch.float32
            kw[k] = torch.as_tensor(g(k)).to(device=device, dtype=dt).contiguous()
        return cls(**kw)

    def clone(self) -> "State":
        return State(**{k: getattr(self, k).clone() for k in STATE_FIELDS})

    def to_numpy(self) -> Dict[str, "object"]:
        return {k: getattr(self, k).cpu().numpy() for k in STATE_FIELDS}

    def agents_in(self) -> AgentsIn:
        n = self.n
        for k in STATE_FIELDS:
            _check(getattr(self, k), k, torch.uint8 if k == "cls" else torch.float32, n)
        return AgentsIn(*[_ptr(getattr(self, k)) for k in STATE_FIELDS])


def workspace_bytes(n: int, n_scenes: int = 0, max_cells: int = 0) -> int:
    return int(lib().orca_workspace_bytes(int(n), int(n_scenes), int(max_cells)))


class Workspace:
    """A caller-owned device workspace, zero-filled once on creation.  With
    backward=True it is sized for orca_step_backward."""

    def __init__(self, n: int, n_scenes: int = 0, max_cells: int = 0, device="cuda",
                 backward: bool = False):
        if backward:
            self.nbytes = int(lib().orca_backward_workspace_bytes(int(n), int(max_cells)))
        else:
            self.nbytes = workspace_bytes(n, n_scenes, max_cells)
        self.buf = torch.empty(max(self.nbytes, 256), dtype=torch.uint8, device=device)
        rc = lib().orca_workspace_init(_ptr(self.buf), self.nbytes, _stream_handle())
        if rc != ORCA_OK:
            raise OrcaError("orca_workspace_init", rc)

    def ptr(self) -> int:
        return _ptr(self.buf)


def build_grid(state: State, params, ws: Workspace, want_neighbors: bool = True,
               stream=None):
    """Grid + exact neighbour lists.  Returns (nbr[n, k] int32, count[n] int32)."""
    p = make_params(params)
    n = state.n
    nbr = cnt = None
    if want_neighbors:
        nbr = torch.empty((n, p.max_neighbors), dtype=torch.int32, device=state.px.device)
        cnt = torch.empty(n, dtype=torch.int32, device=state.px.device)
    ain = state.agents_in()
    rc = lib().orca_build_grid(ctypes.byref(ain), n, ctypes.byref(p), ws.ptr(), ws.nbytes,
                               _ptr(nbr), _ptr(cnt), _stream_handle(stream))
    if rc != ORCA_OK:
        raise OrcaError("orca_build_grid", rc)
    return nbr, cnt


def step(state: State, params, ws: Workspace, out: Optional[State] = None,
         status: Optional[torch.Tensor] = None, stream=None, events=None) -> State:
    """One ORCA step.  ``out`` (default: a copy of ``state``) receives the new
    positions and velocities; it may be ``state`` itself (in-place step).
    ``events``: optional (grid_begin, step_begin, step_end) raw hipEvent_t
    handles recorded around the phases (timing only)."""
    p = make_params(params)
    n = state.n
    if out is None:
        out = state.clone()
    if status is not None:
        _check(status, "status", torch.uint8, n)
    for k in ("px", "py", "vx", "vy"):
        _check(getattr(out, k), "out." + k, torch.float32, n)
    ain = state.agents_in()
    aout = AgentsOut(_ptr(out.px), _ptr(out.py), _ptr(out.vx), _ptr(out.vy), _ptr(status))
    if events is None:
        rc = lib().orca_step(ctypes.byref(ain), ctypes.byref(aout), n, ctypes.byref(p),
                             ws.ptr(), ws.nbytes, _stream_handle(stream))
    else:
        ev = StepEvents(*events)
        rc = lib().orca_step_ex(ctypes.byref(ain), ctypes.byref(aout), n, ctypes.byref(p),
                                ws.ptr(), ws.nbytes, ctypes.byref(ev), _stream_handle(stream))
    if rc != ORCA_OK:
        raise OrcaError("orca_step", rc)
    return out


def step_nbr(state: State, params, ws: Workspace, out: Optional[State] = None,
             status: Optional[torch.Tensor] = None, stream=None):
    """``orca_step_nbr``: the same step as :func:`step`, also returning the
    neighbour lists it used, (out, nbr[n, k] int32, count[n] int32)."""
    p = make_params(params)
    n = state.n
    if out is None:
        out = state.clone()
    if status is not None:
        _check(status, "status", torch.uint8, n)
    for k in ("px", "py", "vx", "vy"):
        _check(getattr(out, k), "out." + k, torch.float32, n)
    nbr = torch.empty((n, p.max_neighbors), dtype=torch.int32, device=state.px.device)
    cnt = torch.empty(n, dtype=torch.int32, device=state.px.device)
    ain = state.agents_in()
    aout = AgentsOut(_ptr(out.px), _ptr(out.py), _ptr(out.vx), _ptr(out.vy), _ptr(status))
    rc = lib().orca_step_nbr(ctypes.byref(ain), ctypes.byref(aout), n, ctypes.byref(p),
                             ws.ptr(), ws.nbytes, _ptr(nbr), _ptr(cnt), _stream_handle(stream))
    if rc != ORCA_OK:
        raise OrcaError("orca_step_nbr", rc)
    return out, nbr, cnt


NOALLOC_N_MAX = 262144


def step_noalloc(state: State, params, out: Optional[State] = None,
                 status: Optional[torch.Tensor] = None, stream=None) -> State:
    """``orca_step_noalloc``: :func:`step` on the library's own per-GPU
    scratch array instead of a workspace (at most ``NOALLOC_N_MAX`` agents;
    calls on one GPU must not overlap)."""
    p = make_params(params)
    n = state.n
    if out is None:
        out = state.clone()
    if status is not None:
        _check(status, "status", torch.uint8, n)
    for k in ("px", "py", "vx", "vy"):
        _check(getattr(out, k), "out." + k, torch.float32, n)
    ain = state.agents_in()
    aout = AgentsOut(_ptr(out.px), _ptr(out.py), _ptr(out.vx), _ptr(out.vy), _ptr(status))
    rc = lib().orca_step_noalloc(ctypes.byref(ain), ctypes.byref(aout), n, ctypes.byref(p),
                                 _stream_handle(stream))
    if rc != ORCA_OK:
        raise OrcaError("orca_step_noalloc", rc)
    return out


def params_of(sc: "scenarios.Scenario"):
    return sc.params


class Batch:
    """Scene offsets, per-scene parameters and the error flag of a batch, on
    the device (``orca_batch``)."""

    def __init__(self, scene_off, scene_params, device="cuda", mode: int = 0, block: int = 0,
                 k_tile: int = 0):
        import numpy as np
        off = np.ascontiguousarray(np.asarray(scene_off), dtype=np.int32)
        self.n_scenes = int(off.shape[0] - 1)
        if self.n_scenes < 1 or len(scene_params) != self.n_scenes:
            raise ValueError("scene_off needs n_scenes + 1 entries and one Params per scene")
        self.off = torch.as_tensor(off).to(device)
        arr = (OrcaParams * self.n_scenes)(*[make_params(p) for p in scene_params])
        raw = np.frombuffer(bytes(arr), dtype=np.uint8).copy()
        self.params = torch.as_tensor(raw).to(device)
        self.max_neighbors = max(int(make_params(p).max_neighbors) for p in scene_params)
        self.has_accel = int(any(make_params(p).accel[c] > 0 or make_params(p).turn[c] > 0
                                 for p in scene_params for c in range(2)))
        self.mode = int(mode)
        self.block = int(block)    # lanes per workgroup (64, 128, 256; 0 = 128)
        self.k_tile = int(k_tile)  # compiled neighbour capacity (0 = smallest >= k)
        self.error = torch.zeros(1, dtype=torch.int32, device=device)

    def c_struct(self) -> OrcaBatch:
        return OrcaBatch(_ptr(self.off), self.n_scenes, _ptr(self.params), self.max_neighbors,
                         self.mode, _ptr(self.error), self.has_accel, self.block, self.k_tile)


def step_batched(state: State, batch: Batch, ws: Workspace, out: Optional[State] = None,
                 status: Optional[torch.Tensor] = None, stream=None, events=None) -> State:
    """One ORCA step of every scene of the batch (``orca_step_batched``).
    ``events``: optional (grid_begin, step_begin, step_end) raw hipEvent_t
    handles (``orca_step_batched_ex``; timing only)."""
    n = state.n
    if out is None:
        out = state.clone()
    if status is not None:
        _check(status, "status", torch.uint8, n)
    for k in ("px", "py", "vx", "vy"):
        _check(getattr(out, k), "out." + k, torch.float32, n)
    ain = state.agents_in()
    aout = AgentsOut(_ptr(out.px), _ptr(out.py), _ptr(out.vx), _ptr(out.vy), _ptr(status))
    b = batch.c_struct()
    if events is None:
        rc = lib().orca_step_batched(ctypes.byref(ain), ctypes.byref(aout), n, ctypes.byref(b),
                                     ws.ptr(), ws.nbytes, _stream_handle(stream))
    else:
        ev = StepEvents(*events)
        rc = lib().orca_step_batched_ex(ctypes.byref(ain), ctypes.byref(aout), n,
                                        ctypes.byref(b), ws.ptr(), ws.nbytes, ctypes.byref(ev),
                                        _stream_handle(stream))
    if rc != ORCA_OK:
        raise OrcaError("orca_step_batched", rc)
    return out


def step_backward(state: State, params, ws: Workspace, g_px, g_py, g_vx, g_vy,
                  g_pref_x: torch.Tensor, g_pref_y: torch.Tensor,
                  g_tau: Optional[torch.Tensor] = None, out=None, stream=None, events=None):
    """Adjoint of one step at `state` (``orca_step_backward``).  g_* are the
    cotangents of the step's outputs; returns (g_px0, g_py0, g_vx0, g_vy0),
    written into `out` (a 4-tuple of tensors, which may be the inputs) or new
    tensors.  g_pref_x/g_pref_y and g_tau (one float) are accumulated.
    ``events``: optional (grid_begin, step_begin, step_end) raw hipEvent_t
    handles around the grid build and the per-agent adjoint kernel
    (``orca_step_backward_ex``; timing only)."""
    n = state.n
    gin = (g_px, g_py, g_vx, g_vy)
    for k, t in zip(("g_px", "g_py", "g_vx", "g_vy"), gin):
        _check(t, k, torch.float32, n)
    if out is None:
        out = tuple(torch.empty_like(t) for t in gin)
    for t in out:
        _check(t, "out", torch.float32, n)
    _check(g_pref_x, "g_pref_x", torch.float32, n)
    _check(g_pref_y, "g_pref_y", torch.float32, n)
    if g_tau is not None:
        _check(g_tau, "g_tau", torch.float32, 1)
    p = make_params(params)
    ain = state.agents_in()
    c1 = Cotangents(*[_ptr(t) for t in gin])
    c0 = CotangentsOut(*[_ptr(t) for t in out], _ptr(g_pref_x), _ptr(g_pref_y), _ptr(g_tau))
    if events is None:
        rc = lib().orca_step_backward(ctypes.byref(ain), n, ctypes.byref(p), ctypes.byref(c1),
                                      ctypes.byref(c0), ws.ptr(), ws.nbytes,
                                      _stream_handle(stream))
    else:
        ev = StepEvents(*events)
        rc = lib().orca_step_backward_ex(ctypes.byref(ain), n, ctypes.byref(p), ctypes.byref(c1),
                                         ctypes.byref(c0), ws.ptr(), ws.nbytes, ctypes.byref(ev),
                                         _stream_handle(stream))
    if rc != ORCA_OK:
        raise OrcaError("orca_step_backward", rc)
    return out


# ---- agent lifecycle -------------------------------------------------------

SPAWN_MAX = 16384


def _buf_of(state: State, n_min: int) -> AgentsBuf:
    for k in STATE_FIELDS:
        t = getattr(state, k)
        if not isinstance(t, torch.Tensor) or t.device.type != "cuda" or not t.is_contiguous():
            raise TypeError(f"{k} must be a contiguous device tensor")
        if t.dtype != (torch.uint8 if k == "cls" else torch.float32) or t.numel() < n_min:
            raise TypeError(f"{k} must hold at least {n_min} elements of the state's dtype")
    return AgentsBuf(*[_ptr(getattr(state, k)) for k in STATE_FIELDS])


class LifecycleWorkspace(Workspace):
    """Workspace of remove_arrived / spawn for up to n agents and n_cand
    spawn candidates."""

    def __init__(self, n: int, n_cand: int = 0, device="cuda"):
        self.nbytes = int(lib().orca_lifecycle_workspace_bytes(int(n), int(n_cand)))
        self.n_max, self.cand_max = int(n), int(n_cand)
        self.buf = torch.empty(max(self.nbytes, 256), dtype=torch.uint8, device=device)
        rc = lib().orca_workspace_init(_ptr(self.buf), self.nbytes, _stream_handle())
        if rc != ORCA_OK:
            raise OrcaError("orca_workspace_init", rc)


def remove_arrived(state: State, out: State, ws: LifecycleWorkspace,
                   old_to_new: Optional[torch.Tensor] = None, stream=None) -> torch.Tensor:
    """Writes the agents of `state` that have not reached their goal (pref is
    read as the goal) to out[0:count], in order; returns count as a device
    int32 tensor of one element.  `out` must not overlap `state`."""
    n = state.n
    ain = state.agents_in()
    abuf = _buf_of(out, n)
    if old_to_new is not None:
        _check(old_to_new, "old_to_new", torch.int32, n)
    count = torch.empty(1, dtype=torch.int32, device=state.px.device)
    rc = lib().orca_remove_arrived(ctypes.byref(ain), ctypes.byref(abuf), n, _ptr(count),
                                   _ptr(old_to_new), ws.ptr(), ws.nbytes, _stream_handle(stream))
    if rc != ORCA_OK:
        raise OrcaError("orca_remove_arrived", rc)
    return count


def spawn(state: State, n: int, cand: State, t_clear: float, ws: LifecycleWorkspace,
          accepted: Optional[torch.Tensor] = None, stream=None) -> torch.Tensor:
    """Appends, in order, the candidates that keep clear of the first n agents
    of `state` (capacity-sized buffers) and of the candidates accepted before
    them for t_clear seconds; returns the new agent count as a device int32
    tensor of one element."""
    cap = state.n
    nc = cand.n
    abuf = _buf_of(state, n + nc)
    cin = cand.agents_in()
    if accepted is not None:
        _check(accepted, "accepted", torch.uint8, nc)
    total = torch.empty(1, dtype=torch.int32, device=state.px.device)
    rc = lib().orca_spawn(ctypes.byref(abuf), int(n), int(cap), ctypes.byref(cin), nc,
                          float(t_clear), _ptr(total), _ptr(accepted), ws.ptr(), ws.nbytes,
                          _stream_handle(stream))
    if rc != ORCA_OK:
        raise OrcaError("orca_spawn", rc)
    return total


class OverlapWorkspace(Workspace):
    """Workspace of overlap_stats for up to n agents."""

    def __init__(self, n: int, device="cuda"):
        self.nbytes = int(lib().orca_overlap_workspace_bytes(int(n)))
        self.buf = torch.empty(max(self.nbytes, 256), dtype=torch.uint8, device=device)
        rc = lib().orca_workspace_init(_ptr(self.buf), self.nbytes, _stream_handle())
        if rc != ORCA_OK:
            raise OrcaError("orca_workspace_init", rc)


def overlap_stats(state: State, reach: float, ws: OverlapWorkspace, out=None,
                  stream=None) -> torch.Tensor:
    """(overlapping pairs, agents in an overlap, smallest clearance) over the
    pairs closer than `reach`, as a device float64 tensor of 3."""
    if out is None:
        out = torch.empty(3, dtype=torch.float64, device=state.px.device)
    ain = state.agents_in()
    rc = lib().orca_overlap_stats(ctypes.byref(ain), state.n, float(reach), _ptr(out), ws.ptr(),
                                  ws.nbytes, _stream_handle(stream))
    if rc != ORCA_OK:
        raise OrcaError("orca_overlap_stats", rc)
    return out
