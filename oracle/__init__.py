"""FP64 CPU oracle for the ORCA step and its gradient (ctypes wrapper over
``orca_oracle.cpp``).

TEST INFRASTRUCTURE ONLY: the test suite, the smoke check and the CPU
baseline of the benchmark may use this package; the library path must not.
It shares no code with the GPU library.  Every scalar parameter is first
rounded to FP32 (the precision the GPU library receives it in) and then
widened to double, so both sides start from identical inputs.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from typing import Optional

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "orca_oracle.cpp")
_SRC_LIFE = os.path.join(_HERE, "lifecycle_oracle.cpp")
_LIB = os.path.join(_HERE, "liborca_oracle.so")
K_MAX = 64
NWORK = 12
WORK_FIELDS = ("candidates", "in_range", "neighbors", "lp2_checks", "lp2_solves", "lp2_inner",
               "lp3_used", "lp3_outer", "lp3_proj", "lp3_checks", "lp3_solves", "lp3_inner")


def build(force: bool = True) -> str:
    """Compile the oracle with g++ (FP64, no contraction, OpenMP)."""
    srcs = (_SRC, _SRC_LIFE)
    if force or not os.path.exists(_LIB) or \
            any(os.path.getmtime(_LIB) < os.path.getmtime(s) for s in srcs):
        tmp = _LIB + ".tmp"
        subprocess.check_call(["g++", "-O3", "-std=c++17", "-fopenmp", "-ffp-contract=off", "-fPIC",
                               "-shared", "-Wall", "-o", tmp, *srcs, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


class _OParams(ctypes.Structure):
    _fields_ = [("dt", ctypes.c_double), ("tau", ctypes.c_double), ("rn", ctypes.c_double),
                ("k", ctypes.c_int32), ("pref_is_goal", ctypes.c_int32),
                ("f", (ctypes.c_double * 2) * 2), ("eps", ctypes.c_double),
                ("accel", ctypes.c_double * 2), ("turn", ctypes.c_double * 2)]


_lib = None


def lib():
    global _lib
    if _lib is None:
        build(force=False)
        L = ctypes.CDLL(_LIB)
        dp = ctypes.POINTER(ctypes.c_double)
        L.oracle_halfplane.restype = ctypes.c_int
        L.oracle_halfplane.argtypes = [ctypes.c_double] * 13 + [ctypes.c_int, dp]
        L.oracle_lp2.restype = ctypes.c_int
        L.oracle_lp2.argtypes = [ctypes.c_int, dp, ctypes.c_double, ctypes.c_double,
                                 ctypes.c_double, ctypes.c_double, dp]
        L.oracle_lp_full.restype = ctypes.c_int
        L.oracle_lp_full.argtypes = L.oracle_lp2.argtypes
        L.oracle_knn.restype = ctypes.c_int
        L.oracle_knn.argtypes = [ctypes.c_int, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_float,
                                 ctypes.c_int, ctypes.c_void_p, ctypes.c_void_p]
        L.oracle_step.restype = ctypes.c_int
        L.oracle_step.argtypes = [ctypes.c_int] + [ctypes.c_void_p] * 9 + \
            [ctypes.POINTER(_OParams)] + [ctypes.c_void_p] * 11
        L.oracle_step_d.restype = ctypes.c_int
        L.oracle_step_d.argtypes = [ctypes.c_int] + [ctypes.c_void_p] * 9 + \
            [ctypes.POINTER(_OParams)] + [ctypes.c_void_p] * 6
        for name in ("oracle_step_vjp", "oracle_step_vjp_d"):
            fn = getattr(L, name)
            fn.restype = ctypes.c_int
            fn.argtypes = [ctypes.c_int] + [ctypes.c_void_p] * 9 + \
                [ctypes.POINTER(_OParams)] + [ctypes.c_void_p] * 11
        L.oracle_arrived.restype = ctypes.c_int
        L.oracle_arrived.argtypes = [ctypes.c_int] + [ctypes.c_void_p] * 6
        L.oracle_spawn.restype = ctypes.c_int
        L.oracle_spawn.argtypes = [ctypes.c_int] + [ctypes.c_void_p] * 4 + [ctypes.c_int] + \
            [ctypes.c_void_p] * 4 + [ctypes.c_float, ctypes.c_void_p]
        L.oracle_overlap_stats.restype = ctypes.c_int
        L.oracle_overlap_stats.argtypes = [ctypes.c_int] + [ctypes.c_void_p] * 3 + \
            [ctypes.c_float, ctypes.c_void_p]
        L.oracle_lp_full_hard.restype = ctypes.c_int
        L.oracle_lp_full_hard.argtypes = [ctypes.c_int, ctypes.c_int, dp] + \
            [ctypes.c_double] * 6 + [dp]
        L.oracle_accel_lines.restype = ctypes.c_int
        L.oracle_accel_lines.argtypes = [ctypes.c_double] * 5 + [dp]
        L.oracle_turn_lines.restype = ctypes.c_int
        L.oracle_turn_lines.argtypes = [ctypes.c_double] * 4 + [dp]
        L.oracle_set_threads.restype = ctypes.c_int
        L.oracle_set_threads.argtypes = [ctypes.c_int]
        L.oracle_step_batched.restype = ctypes.c_int
        L.oracle_step_batched.argtypes = [ctypes.c_int] + [ctypes.c_void_p] * 10 + \
            [ctypes.c_void_p] + [ctypes.c_void_p] * 6
        _lib = L
    return _lib


def arrived(state) -> np.ndarray:
    """1 where an agent's goal (its pref input) lies within its disc."""
    g = state.get if isinstance(state, dict) else (lambda k: getattr(state, k))
    a = [np.ascontiguousarray(g(k), dtype=np.float32) for k in ("px", "py", "pref_x", "pref_y",
                                                                "radius")]
    n = a[0].shape[0]
    out = np.zeros(n, np.uint8)
    if lib().oracle_arrived(n, *[x.ctypes.data for x in a], out.ctypes.data) != 0:
        raise ValueError("oracle_arrived failed")
    return out


def remove_arrived(state) -> dict:
    """The state without the agents that reached their goal, survivors in
    their order; also 'old_to_new' (new index or -1)."""
    g = state.get if isinstance(state, dict) else (lambda k: getattr(state, k))
    keep = arrived(state) == 0
    out = {k: np.asarray(g(k))[keep] for k in _STATE + ("cls",)}
    o2n = np.full(keep.shape[0], -1, np.int32)
    o2n[keep] = np.arange(int(keep.sum()), dtype=np.int32)
    out["old_to_new"] = o2n
    return out


def spawn(state, cand, t_clear: float) -> np.ndarray:
    """Acceptance (0/1 per candidate, in order) of spawn candidates
    cand = dict(px, py, radius, max_speed) against the agents of `state`
    and the candidates accepted before each one."""
    g = state.get if isinstance(state, dict) else (lambda k: getattr(state, k))
    a = [np.ascontiguousarray(g(k), dtype=np.float32) for k in ("px", "py", "radius", "max_speed")]
    c = [np.ascontiguousarray(cand[k], dtype=np.float32) for k in ("px", "py", "radius",
                                                                   "max_speed")]
    n, nc = a[0].shape[0], c[0].shape[0]
    acc = np.zeros(nc, np.uint8)
    rc = lib().oracle_spawn(n, *[x.ctypes.data for x in a], nc, *[x.ctypes.data for x in c],
                            float(np.float32(t_clear)), acc.ctypes.data)
    if rc < 0:
        raise ValueError("oracle_spawn failed")
    return acc


def overlap_stats(state, reach: float) -> dict:
    """Overlapping pairs, agents in an overlap, and the smallest clearance
    |p_i - p_j| - (r_i + r_j) over the pairs closer than `reach` (brute
    force)."""
    g = state.get if isinstance(state, dict) else (lambda k: getattr(state, k))
    a = [np.ascontiguousarray(g(k), dtype=np.float32) for k in ("px", "py", "radius")]
    out = np.zeros(3)
    if lib().oracle_overlap_stats(a[0].shape[0], *[x.ctypes.data for x in a],
                                  float(np.float32(reach)), out.ctypes.data):
        raise ValueError("oracle_overlap_stats failed")
    return {"pairs": int(out[0]), "agents": int(out[1]), "min_clearance": float(out[2])}


def overlap_stats_tree(state, reach: float) -> dict:
    """The same statistics as `overlap_stats`, for crowds too large for the
    all-pairs loop: a k-d tree (scipy) lists every pair closer than a reach
    widened by a relative 1e-9, then each listed pair is tested exactly as
    in the loop (FP64 of the FP32 inputs, |d|^2 < reach^2, overlap when
    |d|^2 < (r_i + r_j)^2, clearance sqrt(|d|^2) - (r_i + r_j))."""
    from scipy.spatial import cKDTree
    g = state.get if isinstance(state, dict) else (lambda k: getattr(state, k))
    px = np.asarray(g("px"), dtype=np.float32).astype(np.float64)
    py = np.asarray(g("py"), dtype=np.float32).astype(np.float64)
    rad = np.asarray(g("radius"), dtype=np.float32).astype(np.float64)
    n = px.shape[0]
    q = float(np.float32(reach))
    if n < 2:
        return {"pairs": 0, "agents": 0, "min_clearance": float("inf")}
    ij = cKDTree(np.stack([px, py], axis=1)).query_pairs(q * (1.0 + 1e-9) + 1e-300,
                                                         output_type="ndarray")
    i, j = ij[:, 0], ij[:, 1]
    dx = px[j] - px[i]
    dy = py[j] - py[i]
    d2 = dx * dx + dy * dy
    near = d2 < q * q
    i, j, d2 = i[near], j[near], d2[near]
    rr = rad[i] + rad[j]
    over = d2 < rr * rr
    hit = np.zeros(n, bool)
    hit[i[over]] = True
    hit[j[over]] = True
    gap = float(np.min(np.sqrt(d2) - rr)) if d2.size else float("inf")
    return {"pairs": int(over.sum()), "agents": int(hit.sum()), "min_clearance": gap}


def set_threads(t: int = 0) -> int:
    """Sets the oracle's OpenMP thread count when t > 0; returns the count in
    effect."""
    return int(lib().oracle_set_threads(int(t)))


def _f32d(x) -> float:
    """Round a scalar to FP32, then widen to double."""
    return float(np.float32(x))


def make_params(params) -> _OParams:
    """Accepts any object with the ``orca_params`` field names; scalars are
    rounded to FP32, as the GPU library receives them.  An ``_OParams``
    passes through unchanged (finite-difference pins perturb its FP64
    fields directly)."""
    if isinstance(params, _OParams):
        return params
    g = params.get if isinstance(params, dict) else (lambda k: getattr(params, k))
    p = _OParams()
    p.dt = _f32d(g("dt"))
    p.tau = _f32d(g("time_horizon"))
    p.rn = _f32d(g("neighbor_dist"))
    p.k = int(g("max_neighbors"))
    p.pref_is_goal = int(g("pref_is_goal"))
    f = g("f")
    for a in range(2):
        for b in range(2):
            p.f[a][b] = _f32d(f[a][b])
    p.eps = _f32d(g("par_eps"))
    try:
        acc = g("accel")
    except (AttributeError, KeyError):
        acc = None
    acc = (0.0, 0.0) if acc is None else acc
    for c in range(2):
        p.accel[c] = _f32d(acc[c])
    try:
        turn = g("turn")
    except (AttributeError, KeyError):
        turn = None
    turn = (0.0, 0.0) if turn is None else turn
    for c in range(2):
        p.turn[c] = _f32d(turn[c])
    return p


def _c(a, dtype):
    a = np.ascontiguousarray(a, dtype=dtype)
    return a, a.ctypes.data


def halfplane(pa, va, ra, pb, vb, rb, f, tau, dt, a_before_b=True):
    """ORCA_{A|B}: returns dict(q, d, u, n, branch) in FP64."""
    out = (ctypes.c_double * 8)()
    br = lib().oracle_halfplane(float(pa[0]), float(pa[1]), float(va[0]), float(va[1]), float(ra),
                                float(pb[0]), float(pb[1]), float(vb[0]), float(vb[1]), float(rb),
                                float(f), float(tau), float(dt), int(bool(a_before_b)), out)
    o = np.array(out[:])
    return {"q": o[0:2], "d": o[2:4], "u": o[4:6], "n": o[6:8], "branch": br}


def lp2(lines, vmax, opt, eps=1e-5):
    """Incremental closest-point LP.  lines: (m, 4) rows (qx, qy, dx, dy).
    Returns (v, fail) with fail == m when feasible."""
    lines = np.ascontiguousarray(lines, dtype=np.float64).reshape(-1, 4)
    v = (ctypes.c_double * 2)()
    fail = lib().oracle_lp2(lines.shape[0], lines.ctypes.data_as(ctypes.POINTER(ctypes.c_double)),
                            float(vmax), float(opt[0]), float(opt[1]), float(eps), v)
    if fail < 0:
        raise ValueError("oracle_lp2: bad arguments")
    return np.array(v[:]), fail


def lp_full(lines, vmax, opt, eps=1e-5):
    """LP2, then LP3 when LP2 is infeasible.  Returns (v, fail)."""
    lines = np.ascontiguousarray(lines, dtype=np.float64).reshape(-1, 4)
    v = (ctypes.c_double * 2)()
    fail = lib().oracle_lp_full(lines.shape[0],
                                lines.ctypes.data_as(ctypes.POINTER(ctypes.c_double)),
                                float(vmax), float(opt[0]), float(opt[1]), float(eps), v)
    if fail < 0:
        raise ValueError("oracle_lp_full: bad arguments")
    return np.array(v[:]), fail


def lp_full_hard(lines, n_hard, vmax, opt, centre, eps=1e-5):
    """LP2/LP3 with the first `n_hard` lines never relaxed (acceleration and
    heading lines); a failure among them takes v = centre.  Returns (v, fail)."""
    lines = np.ascontiguousarray(lines, dtype=np.float64).reshape(-1, 4)
    v = (ctypes.c_double * 2)()
    fail = lib().oracle_lp_full_hard(lines.shape[0], int(n_hard),
                                     lines.ctypes.data_as(ctypes.POINTER(ctypes.c_double)),
                                     float(vmax), float(opt[0]), float(opt[1]), float(eps),
                                     float(centre[0]), float(centre[1]), v)
    if fail < 0:
        raise ValueError("oracle_lp_full_hard: bad arguments")
    return np.array(v[:]), fail


def accel_lines(v, vmax, accel, dt):
    """The acceleration lines (8 x 4, or 0 x 4 when accel <= 0) of an agent
    with current velocity v."""
    out = (ctypes.c_double * 32)()
    m = lib().oracle_accel_lines(float(v[0]), float(v[1]), float(vmax), float(accel), float(dt),
                                 out)
    return np.array(out[:]).reshape(8, 4)[:m]


def turn_lines(v, turn, dt):
    """The heading lines (2 x 4, or 0 x 4 when turn <= 0 or v = 0) of an
    agent with current velocity v: the sides of the wedge of half-angle
    min(turn dt, pi/2) about its heading, through the origin."""
    out = (ctypes.c_double * 8)()
    m = lib().oracle_turn_lines(float(v[0]), float(v[1]), float(turn), float(dt), out)
    return np.array(out[:]).reshape(2, 4)[:m]


def knn(px, py, neighbor_dist, k):
    """Exact k nearest within the neighbour distance, ties by index."""
    px, ppx = _c(px, np.float32)
    py, ppy = _c(py, np.float32)
    n = px.shape[0]
    nbr = np.full((n, k), -1, np.int32)
    cnt = np.zeros(n, np.int32)
    rc = lib().oracle_knn(n, ppx, ppy, float(np.float32(neighbor_dist)), int(k),
                          nbr.ctypes.data, cnt.ctypes.data)
    if rc != 0:
        raise ValueError(f"oracle_knn failed ({rc})")
    return nbr, cnt


_STATE = ("px", "py", "vx", "vy", "pref_x", "pref_y", "radius", "max_speed")


def _state_ptrs(state):
    g = state.get if isinstance(state, dict) else (lambda k: getattr(state, k))
    keep = [np.ascontiguousarray(g(k), dtype=np.float32) for k in _STATE]
    keep.append(np.ascontiguousarray(g("cls"), dtype=np.uint8))
    return keep, [a.ctypes.data for a in keep]


def step(state, params, want_neighbors: bool = False, want_work: bool = False,
         want_lines: bool = False, want_trace: bool = False):
    """One synchronous step from an FP32 state.  Returns FP64 arrays
    px, py, vx, vy, the status byte (1 = least-penetration fallback used),
    and optionally the neighbour lists, per-agent work counters, and each
    agent's half-planes (n, k, 4) with its desired velocity (n, 2)."""
    keep, ptrs = _state_ptrs(state)
    n = keep[0].shape[0]
    p = make_params(params)
    out = {k: np.zeros(n, np.float64) for k in ("px", "py", "vx", "vy")}
    status = np.zeros(n, np.uint8)
    nbr = np.full((n, p.k), -1, np.int32) if want_neighbors else None
    cnt = np.zeros(n, np.int32) if want_neighbors else None
    work = np.zeros((n, NWORK), np.int64) if want_work else None
    lines = np.zeros((n, p.k, 4), np.float64) if want_lines else None
    pref = np.zeros((n, 2), np.float64) if want_lines else None
    if want_lines and not want_neighbors:
        cnt = np.zeros(n, np.int32)
    trace = np.zeros(n, np.uint64) if want_trace else None
    rc = lib().oracle_step(n, *ptrs, ctypes.byref(p), out["px"].ctypes.data,
                           out["py"].ctypes.data, out["vx"].ctypes.data, out["vy"].ctypes.data,
                           status.ctypes.data, nbr.ctypes.data if nbr is not None else None,
                           cnt.ctypes.data if cnt is not None else None,
                           work.ctypes.data if work is not None else None,
                           lines.ctypes.data if lines is not None else None,
                           pref.ctypes.data if pref is not None else None,
                           trace.ctypes.data if trace is not None else None)
    if rc != 0:
        raise ValueError(f"oracle_step failed ({rc})")
    out["status"] = status
    if want_neighbors:
        out["nbr"] = nbr
        out["cnt"] = cnt
    if want_work:
        out["work"] = work
    if want_lines:
        out["lines"] = lines
        out["pref"] = pref
        out["cnt"] = cnt
    if want_trace:
        out["trace"] = trace
    return out


def _d(a):
    a = np.ascontiguousarray(a, dtype=np.float64)
    return a, a.ctypes.data


def step_vjp(state, params, g_px1, g_py1, g_vx1, g_vy1, double_state: bool = False):
    """Vector-Jacobian product of one step at `state` (FP32 arrays, or double
    arrays with double_state=True).  Returns dict g_px, g_py, g_vx, g_vy (the
    cotangents of the step-t state), g_pref_x, g_pref_y (of the pref input:
    desired velocity, or goal in goal mode) and g_tau."""
    g = state.get if isinstance(state, dict) else (lambda k: getattr(state, k))
    if double_state:
        keep = [np.ascontiguousarray(g(k), dtype=np.float64) for k in _STATE]
    else:
        keep = [np.ascontiguousarray(g(k), dtype=np.float32) for k in _STATE]
    cls = np.ascontiguousarray(g("cls"), dtype=np.uint8)
    n = keep[0].shape[0]
    p = make_params(params)
    gin = [_d(x) for x in (g_px1, g_py1, g_vx1, g_vy1)]
    out = {k: np.zeros(n) for k in ("g_px", "g_py", "g_vx", "g_vy", "g_pref_x", "g_pref_y")}
    tau = np.zeros(1)
    fn = lib().oracle_step_vjp_d if double_state else lib().oracle_step_vjp
    rc = fn(n, *[a.ctypes.data for a in keep], cls.ctypes.data, ctypes.byref(p),
            *[x[1] for x in gin], out["g_px"].ctypes.data, out["g_py"].ctypes.data,
            out["g_vx"].ctypes.data, out["g_vy"].ctypes.data, out["g_pref_x"].ctypes.data,
            out["g_pref_y"].ctypes.data, tau.ctypes.data)
    if rc != 0:
        raise ValueError(f"oracle_step_vjp failed ({rc})")
    out["g_tau"] = float(tau[0])
    return out


def step_d(state, params):
    """One step from an FP64 state (no rounding of the state to FP32).
    Returns FP64 px, py, vx, vy and the per-agent trace hash of neighbour
    lists and branch outcomes."""
    g = state.get if isinstance(state, dict) else (lambda k: getattr(state, k))
    cur = [np.ascontiguousarray(g(k), dtype=np.float64) for k in _STATE]
    cls = np.ascontiguousarray(g("cls"), dtype=np.uint8)
    n = cur[0].shape[0]
    p = make_params(params)
    out = {k: np.zeros(n) for k in ("px", "py", "vx", "vy")}
    trace = np.zeros(n, np.uint64)
    rc = lib().oracle_step_d(n, *[a.ctypes.data for a in cur], cls.ctypes.data, ctypes.byref(p),
                             out["px"].ctypes.data, out["py"].ctypes.data, out["vx"].ctypes.data,
                             out["vy"].ctypes.data, None, trace.ctypes.data)
    if rc != 0:
        raise ValueError(f"oracle_step_d failed ({rc})")
    out["trace"] = trace
    return out


def rollout(state, params, steps: int, keep_states: bool = False):
    """FP64 rollout: `steps` oracle steps carrying the state in double.
    Returns dict px, py, vx, vy (final), trace (hash of every agent's
    neighbour lists and branch outcomes over all steps) and, with
    keep_states, the list of per-step double states (step 0 first)."""
    g = state.get if isinstance(state, dict) else (lambda k: getattr(state, k))
    cur = {k: np.ascontiguousarray(g(k), dtype=np.float64) for k in _STATE}
    cur["cls"] = np.ascontiguousarray(g("cls"), dtype=np.uint8)
    n = cur["px"].shape[0]
    p = make_params(params)
    hist = []
    h = np.uint64(1469598103934665603)
    for _ in range(steps):
        if keep_states:
            hist.append({k: cur[k].copy() for k in ("px", "py", "vx", "vy")})
        nxt = step_d(cur, p)
        with np.errstate(over="ignore"):
            h = np.uint64((int(h) * 1099511628211 + int(np.bitwise_xor.reduce(
                nxt["trace"] * np.arange(1, n + 1, dtype=np.uint64)))) % (1 << 64))
        cur.update({k: nxt[k] for k in ("px", "py", "vx", "vy")})
    out = {k: cur[k] for k in ("px", "py", "vx", "vy")}
    out["trace"] = int(h)
    if keep_states:
        out["states"] = hist
    return out


def rollout_grad(state, params, steps: int, target_x, target_y):
    """Loss L = mean_i |p_i(T) - target_i|^2 of an FP64 rollout and its
    gradient with respect to every agent's pref input and tau, by chaining
    the oracle's one-step VJPs backwards along the stored trajectory."""
    g = state.get if isinstance(state, dict) else (lambda k: getattr(state, k))
    base = {k: np.ascontiguousarray(g(k), dtype=np.float64) for k in _STATE}
    cls = np.ascontiguousarray(g("cls"), dtype=np.uint8)
    n = base["px"].shape[0]
    fw = rollout(dict(base, cls=cls), params, steps, keep_states=True)
    tx = np.asarray(target_x, np.float64)
    ty = np.asarray(target_y, np.float64)
    loss = float(np.mean((fw["px"] - tx) ** 2 + (fw["py"] - ty) ** 2))
    gpx = 2.0 * (fw["px"] - tx) / n
    gpy = 2.0 * (fw["py"] - ty) / n
    gvx = np.zeros(n)
    gvy = np.zeros(n)
    gprx = np.zeros(n)
    gpry = np.zeros(n)
    gtau = 0.0
    for t in range(steps - 1, -1, -1):
        st = dict(base, cls=cls)
        st.update(fw["states"][t])
        r = step_vjp(st, params, gpx, gpy, gvx, gvy, double_state=True)
        gpx, gpy, gvx, gvy = r["g_px"], r["g_py"], r["g_vx"], r["g_vy"]
        gprx += r["g_pref_x"]
        gpry += r["g_pref_y"]
        gtau += r["g_tau"]
    return {"loss": loss, "g_pref_x": gprx, "g_pref_y": gpry, "g_tau": gtau,
            "trace": fw["trace"], "final": fw}


def step_batched(state, scene_off, scene_params, want_work: bool = False):
    """One step of every scene; scene s owns [off[s], off[s+1])."""
    keep, ptrs = _state_ptrs(state)
    n = keep[0].shape[0]
    off = np.ascontiguousarray(scene_off, dtype=np.int32)
    S = off.shape[0] - 1
    parr = (_OParams * max(S, 1))()
    for s in range(S):
        parr[s] = make_params(scene_params[s])
    out = {k: np.zeros(n, np.float64) for k in ("px", "py", "vx", "vy")}
    status = np.zeros(n, np.uint8)
    work = np.zeros((n, NWORK), np.int64) if want_work else None
    rc = lib().oracle_step_batched(S, off.ctypes.data, *ptrs, ctypes.addressof(parr),
                                   out["px"].ctypes.data, out["py"].ctypes.data,
                                   out["vx"].ctypes.data, out["vy"].ctypes.data,
                                   status.ctypes.data,
                                   work.ctypes.data if work is not None else None)
    if rc != 0:
        raise ValueError(f"oracle_step_batched failed ({rc})")
    out["status"] = status
    if want_work:
        out["work"] = work
    return out
