"""Helpers shared by the GPU parity tests: run the HIP path and the FP64
oracle from the same FP32 state and compare them.

Velocity tolerance: 1e-4 m/s per agent for agents whose oracle solution is
well conditioned.  Conditioning is measured with the oracle alone: it is
re-run on copies of the state whose velocities are perturbed by 1e-6 m/s
and radii by one ulp; an agent whose oracle velocity moves by more than
``COND_TOL`` under such perturbations sits on a regime boundary (LP2/LP3
flip, nearly parallel active lines, arc/leg switch, non-unique LP3
minimiser) where FP32 rounding legitimately selects a different answer.
A second probe covers the rounding of the FP32 path itself: an agent whose
oracle LP answer moves by more than ``COND_TOL`` when each component of its
own half-planes is perturbed by a relative 1e-6 (a few FP32 ulps, the error
of half-planes formed in FP32) is ill-conditioned as well -- its LP path
(which line first fails, which interval end binds, which LP3 boundary wins)
is decided below FP32 resolution.  Such an agent must still hold a valid
answer to the oracle's FP64 problem (`valid_answer`), or match the oracle
across a contact within rounding (`contact_flipped`), or lie within twice
the distance the oracle's own answer moves under the two perturbations
above (`oracle_sensitivity`, `line_movement`: at a vertex of nearly
parallel lines or a tie of LP3 the answer moves with rounding itself);
these agents are counted and their share is bounded.
"""
from __future__ import annotations

import numpy as np

import oracle

V_TOL = 1e-4
COND_TOL = 1e-5


def gpu_step(state_np, params, status=True):
    import torch
    from paper_2008_11578_amd import orca
    st = orca.State.from_arrays(state_np)
    ws = orca.Workspace(st.n)
    stat = torch.zeros(st.n, dtype=torch.uint8, device="cuda") if status else None
    out = orca.step(st, params, ws, status=stat)
    torch.cuda.synchronize()
    res = {k: getattr(out, k).cpu().numpy() for k in ("px", "py", "vx", "vy")}
    if status:
        res["status"] = stat.cpu().numpy()
    return res


def gpu_neighbors(state_np, params):
    import torch
    from paper_2008_11578_amd import orca
    st = orca.State.from_arrays(state_np)
    ws = orca.Workspace(st.n)
    nbr, cnt = orca.build_grid(st, params, ws)
    torch.cuda.synchronize()
    return nbr.cpu().numpy(), cnt.cpu().numpy()


def perturbed(state_np, seed, dv=1e-6):
    """Copy of the state with velocities moved by up to `dv` m/s per
    component and radii by one FP32 ulp: the size of the rounding the FP32
    path makes in the half-plane geometry (relative positions are formed
    exactly in FP32, so positions are left alone)."""
    rng = np.random.default_rng(seed)
    out = dict(as_dict(state_np))
    for k in ("vx", "vy"):
        a = np.asarray(out[k], np.float64)
        out[k] = (a + rng.uniform(-dv, dv, size=a.shape)).astype(np.float32)
    r = np.asarray(out["radius"], np.float32)
    up = rng.random(r.shape) < 0.5
    out["radius"] = np.where(up, np.nextafter(r, np.float32(np.inf)),
                             np.nextafter(r, np.float32(0))).astype(np.float32)
    return out


def oracle_sensitivity(state_np, params, base, reps=2):
    """Per-agent max |v_perturbed - v_base| of the oracle."""
    sens = np.zeros_like(base["vx"])
    for r in range(reps):
        o = oracle.step(perturbed(state_np, 1000 + r), params)
        sens = np.maximum(sens, np.hypot(o["vx"] - base["vx"], o["vy"] - base["vy"]))
    return sens


def _accel(params):
    acc = params.get("accel") if isinstance(params, dict) else getattr(params, "accel", None)
    return (0.0, 0.0) if acc is None else tuple(float(np.float32(a)) for a in acc)


def _turn(params):
    t = params.get("turn") if isinstance(params, dict) else getattr(params, "turn", None)
    return (0.0, 0.0) if t is None else tuple(float(np.float32(a)) for a in t)


def _capped(params):
    return any(a > 0 for a in _accel(params) + _turn(params))


def _dt(params):
    return float(np.float32(params["dt"] if isinstance(params, dict) else params.dt))


def hard_lines(st, params, a):
    """Agent a's hard lines -- its acceleration lines (0 or 8), then its
    heading lines (0 or 2) -- and their centre, from the oracle."""
    cls = int(st["cls"][a]) & 1
    v = (float(st["vx"][a]), float(st["vy"][a]))
    vmax = float(np.float32(st["max_speed"][a]))
    h = np.concatenate([oracle.accel_lines(v, vmax, _accel(params)[cls], _dt(params)),
                        oracle.turn_lines(v, _turn(params)[cls], _dt(params))])
    sp = float(np.hypot(*v))
    c = np.array(v) * (vmax / sp if sp > vmax else 1.0)
    return h, c


def line_sensitive(o, st, idx, params=None, reps=4, rel=1e-6, seed=77):
    """For agents `idx`: whether the oracle LP answer on the agent's own
    lines (hard lines, when capped, then half-planes) moves by more
    than COND_TOL when every line component is scaled by (1 + U(-rel, rel))."""
    return line_movement(o, st, idx, params, reps, rel, seed) > COND_TOL


def line_movement(o, st, idx, params=None, reps=4, rel=1e-6, seed=77):
    """For agents `idx`: the farthest the oracle LP answer on the agent's own
    lines moves when every line component is scaled by (1 + U(-rel, rel)),
    a few FP32 ulps: how far FP32 rounding of the half-planes alone can
    carry the answer."""
    rng = np.random.default_rng(seed)
    out = np.zeros(len(idx))
    vmax = np.asarray(st["max_speed"], np.float64)
    for k, a in enumerate(idx):
        m = int(o["cnt"][a])
        hard, c = hard_lines(st, params, a) if params is not None else (np.zeros((0, 4)), None)
        lines = np.concatenate([hard, o["lines"][a, :m].astype(np.float64)])
        nh = hard.shape[0]
        pref = o["pref"][a]
        vm = float(np.float32(vmax[a]))

        def solve(ls):
            if nh:
                return oracle.lp_full_hard(ls, nh, vm, pref, c)[0]
            return oracle.lp_full(ls, vm, pref)[0]

        v0 = solve(lines)
        worst = 0.0
        for _ in range(reps):
            v1 = solve(lines * (1.0 + rng.uniform(-rel, rel, size=lines.shape)))
            worst = max(worst, float(np.hypot(*(v1 - v0))))
        out[k] = worst
    return out


def penetration(lines, cnt, vx, vy):
    """max_j det(d_j, q_j - v) over each agent's valid lines (-inf if none)."""
    q = lines[:, :, 0:2]
    d = lines[:, :, 2:4]
    rx = q[:, :, 0] - vx[:, None]
    ry = q[:, :, 1] - vy[:, None]
    pen = d[:, :, 0] * ry - d[:, :, 1] * rx
    valid = np.arange(lines.shape[1])[None, :] < cnt[:, None]
    pen = np.where(valid, pen, -np.inf)
    return pen.max(axis=1)


def valid_answer(o, g, vmax, tol=V_TOL, st=None, params=None):
    """Whether the GPU velocity solves the oracle's own FP64 problem to within
    `tol`: inside the speed disc and the hard lines (when capped),
    no more penetration of the half-planes than the oracle's answer (least
    penetration), and, when both sides found a permitted velocity, no
    farther from the desired velocity than the oracle's."""
    vg_x, vg_y = g["vx"].astype(np.float64), g["vy"].astype(np.float64)
    pen_g = penetration(o["lines"], o["cnt"], vg_x, vg_y)
    pen_o = penetration(o["lines"], o["cnt"], o["vx"], o["vy"])
    speed_ok = np.hypot(vg_x, vg_y) <= vmax * (1 + 1e-5) + 1e-6
    if params is not None and _capped(params):
        for a in range(len(vg_x)):
            hard, _ = hard_lines(st, params, a)
            if hard.shape[0]:
                ph = penetration(hard[None], np.array([hard.shape[0]]), vg_x[a:a + 1],
                                 vg_y[a:a + 1])[0]
                speed_ok[a] &= ph <= tol
    pen_ok = pen_g <= np.maximum(pen_o, 0.0) + tol
    obj_g = np.hypot(vg_x - o["pref"][:, 0], vg_y - o["pref"][:, 1])
    obj_o = np.hypot(o["vx"] - o["pref"][:, 0], o["vy"] - o["pref"][:, 1])
    both_lp2 = (o["status"] == 0) & (g["status"] == 0)
    obj_ok = ~both_lp2 | (obj_g <= obj_o + tol)
    return speed_ok & pen_ok & obj_ok


def as_dict(sc):
    if isinstance(sc, dict):
        return sc
    return {k: getattr(sc, k) for k in oracle._STATE + ("cls",)}


CONTACT_REL = 1e-6


def contact_flipped(st, params, a, g, tol=V_TOL):
    """Whether agent `a` touches a neighbour to within a relative CONTACT_REL
    of the sum of their radii, where the FP32 and the FP64 contact test
    |P| > R may pick different forms of the velocity obstacle (the overlap
    form below R, the look-ahead form above), and its GPU velocity is within
    `tol` of the oracle's answer after its radius moves by 1, 2, 4 or 8 FP32
    ulps, up or down, which moves the FP64 test across that contact."""
    px = np.asarray(st["px"], np.float32).astype(np.float64)
    py = np.asarray(st["py"], np.float32).astype(np.float64)
    rad = np.asarray(st["radius"], np.float32).astype(np.float64)
    d = np.hypot(px - px[a], py - py[a])
    R = rad + rad[a]
    near = np.abs(d - R) <= CONTACT_REL * R
    near[a] = False
    if not near.any():
        return False
    r0 = np.asarray(st["radius"], np.float32)
    for ulps in (1, 2, 4, 8):
        for up in (True, False):
            r = r0.copy()
            for _ in range(ulps):
                r[a] = np.nextafter(r[a], np.float32(np.inf if up else -np.inf))
            s2 = dict(st)
            s2["radius"] = r
            o2 = oracle.step(s2, params)
            if np.hypot(g["vx"][a] - o2["vx"][a], g["vy"][a] - o2["vy"][a]) <= tol:
                return True
    return False


def compare_step(state_np, params, *, require_all=False, max_ill_frac=0.01, reps=2, gpu=None):
    """Runs both sides one step from the same FP32 state and asserts the
    parity contract.  Returns (report, gpu, oracle).  `gpu` takes a GPU
    result already computed from this state (px, py, vx, vy, status): a step
    launched with a workspace kept across steps, or a scene of a batch."""
    st = as_dict(state_np)
    g = gpu_step(st, params) if gpu is None else gpu
    o = oracle.step(st, params, want_lines=True)
    dv = np.hypot(g["vx"] - o["vx"], g["vy"] - o["vy"])
    bad = dv > V_TOL
    rep = {"n": int(dv.size), "max_dv": float(dv.max()) if dv.size else 0.0,
           "n_bad": int(bad.sum()), "lp3_gpu": int(g["status"].sum()),
           "lp3_oracle": int(o["status"].sum()),
           "status_mismatch": int((g["status"] != o["status"]).sum())}
    ill = np.zeros_like(bad)
    if bad.any() and not require_all:
        sens = oracle_sensitivity(st, params, o, reps=reps)
        ill = sens > COND_TOL
        # how far each agent outside the tolerance would move with its own
        # half-planes rounded at FP32 size (eight draws)
        mv = np.zeros(dv.shape)
        idx = np.nonzero(bad)[0][:64]
        if idx.size:
            mv[idx] = line_movement(o, st, idx, params, reps=8)
            rep["n_line_sensitive"] = int(np.sum(~ill[idx] & (mv[idx] > COND_TOL)))
            ill[idx] |= mv[idx] > COND_TOL
        rep["n_ill"] = int(ill.sum())
        rep["n_bad_ill"] = int((bad & ill).sum())
        vmax = np.asarray(st["max_speed"], np.float64)
        ok = valid_answer(o, g, vmax, st=st, params=params)
        rep["n_bad_ill_invalid"] = int((bad & ill & ~ok).sum())
        # an agent in contact within rounding may solve the problem of the
        # other side of that contact: it must then match the oracle there
        for a in np.nonzero(bad & ill & ~ok)[0][:32]:
            ok[a] = contact_flipped(st, params, a, g)
        rep["n_contact_flipped"] = rep["n_bad_ill_invalid"] - int((bad & ill & ~ok).sum())
        # an ill-conditioned answer moves with rounding itself: an answer
        # within twice the distance the oracle's own answer moves when its
        # state (sens) or its own half-planes (mv) are perturbed at FP32 size
        # is as close as FP32 can come
        far = bad & ill & ~ok & (dv <= 2.0 * np.maximum(sens, mv))
        ok |= far
        rep["n_within_sensitivity"] = int(far.sum())
        # ill-conditioned agents must still hold a valid answer
        assert not (bad & ill & ~ok).any(), (rep, np.nonzero(bad & ill & ~ok)[0][:10])
    # every well-conditioned agent within tolerance
    assert not (bad & ~ill).any(), (rep, np.nonzero(bad & ~ill)[0][:10], dv[bad & ~ill][:10])
    assert ill.mean() <= max_ill_frac, rep
    # positions follow from the velocities: p' = p + v' dt (FP32 rounding of p)
    dt = float(np.float32(params.dt if hasattr(params, "dt") else params["dt"]))
    for k, kv in (("px", "vx"), ("py", "vy")):
        p0 = np.abs(np.asarray(st[k], np.float32))
        p1 = np.abs(o[k]).astype(np.float32)
        tol = (np.abs(g[kv] - o[kv]) * dt + np.spacing(p0).astype(np.float64)
               + np.spacing(p1).astype(np.float64) + 1e-12)
        assert (np.abs(g[k] - o[k]) <= tol).all(), k
    return rep, g, o
