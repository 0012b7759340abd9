"""Acceleration-limited agents on the GPU (Sec. 5: acceleration limits as
extra linear constraints in the same LP): the HIP path against the FP64
oracle through the C ABI, the batched form against single-scene steps, and
the relations to the uncapped step."""
import dataclasses

import numpy as np
import pytest

import oracle
from paper_2008_11578_amd import scenarios

from parity import as_dict, compare_step, gpu_step, perturbed

pytestmark = pytest.mark.gpu


def _print(*a):
    print(*a, flush=True)


def _crowd(n, side, seed, veh_share, accel, k=10, dt=0.1):
    p = scenarios.Params(dt=dt, neighbor_dist=5.0, max_neighbors=k, accel=accel)
    return scenarios.random_state(n, side, seed=seed, n_vehicles=int(veh_share * n), params=p)


@pytest.mark.parametrize("accel,k", [((0.0, 3.0), 10), ((2.0, 3.0), 16), ((0.5, 0.5), 10),
                                     ((8.0, 1.0), 20)])
def test_capped_step_matches_oracle(accel, k):
    sc = _crowd(6000, 70.0, seed=31 + k, veh_share=0.1, accel=accel, k=k)
    _print("accel", accel, "k", k, "n", sc.n)
    rep, g, o = compare_step(as_dict(sc), sc.params)
    _print(rep)
    # the caps bind: capped agents that changed relative to no cap exist
    o0 = oracle.step(as_dict(sc), dataclasses.replace(sc.params, accel=(0.0, 0.0)))
    moved = np.hypot(o["vx"] - o0["vx"], o["vy"] - o0["vy"]) > 1e-3
    assert moved.sum() > 50


def test_capped_step_full_size_measured_configuration():
    """The 1,048,576-agent dense crossing with caps of 2 m/s^2 for both
    classes, 0.6 m cells, one workspace kept across steps, as the
    throughput measurement steps it: every agent of the sixth step against
    the oracle."""
    import torch
    from paper_2008_11578_amd import orca
    sc = scenarios.c3_crossing()
    params = dataclasses.replace(sc.params, cell_size=0.6, accel=(2.0, 2.0))
    state = orca.State.from_arrays(sc)
    nxt = state.clone()
    ws = orca.Workspace(state.n)
    status = torch.zeros(state.n, dtype=torch.uint8, device="cuda")
    for _ in range(5):
        orca.step(state, params, ws, out=nxt, status=status)
        state, nxt = nxt, state
    torch.cuda.synchronize()
    snap = state.to_numpy()
    orca.step(state, params, ws, out=nxt, status=status)
    torch.cuda.synchronize()
    g = {k: getattr(nxt, k).cpu().numpy() for k in ("px", "py", "vx", "vy")}
    g["status"] = status.cpu().numpy()
    rep, _, _ = compare_step(snap, params, gpu=g)
    _print("capped c3 1M", rep)


def test_capped_step_every_velocity_within_its_octagon():
    """GPU velocities respect the acceleration lines the oracle forms for
    each agent (to FP32 rounding)."""
    from parity import hard_lines
    sc = _crowd(4000, 60.0, seed=5, veh_share=0.2, accel=(1.0, 2.0))
    st = as_dict(sc)
    g = gpu_step(st, sc.params)
    worst = 0.0
    for a in range(sc.n):
        h, _ = hard_lines(st, sc.params, a)
        q, d = h[:, 0:2], h[:, 2:4]
        r = q - np.array([g["vx"][a], g["vy"][a]], np.float64)
        worst = max(worst, float((d[:, 0] * r[:, 1] - d[:, 1] * r[:, 0]).max()))
    _print("worst hard-line penetration", worst)
    assert worst <= 1e-5


def test_cap_too_large_to_bind_equals_uncapped():
    """Same LP decisions and velocities as without caps.  (The two kernels
    run the same arithmetic but are separate instantiations whose
    multiply-adds the compiler may fuse differently, so agreement is to a
    few FP32 ulps rather than bit for bit; the oracle pins the exact
    equality.)"""
    sc = _crowd(5000, 60.0, seed=7, veh_share=0.1, accel=(0.0, 0.0))
    st = as_dict(sc)
    g0 = gpu_step(st, sc.params)
    g1 = gpu_step(st, dataclasses.replace(sc.params, accel=(1e6, 1e6)))
    np.testing.assert_array_equal(g0["status"], g1["status"])
    dv = np.hypot(g0["vx"] - g1["vx"], g0["vy"] - g1["vy"])
    _print("max |dv| huge cap vs none", float(dv.max()), "differing", int((dv > 0).sum()))
    assert dv.max() <= 1e-5


def test_uncapped_class_unchanged_by_other_class_cap():
    sc = _crowd(5000, 60.0, seed=8, veh_share=0.1, accel=(0.0, 0.0))
    st = as_dict(sc)
    g0 = gpu_step(st, sc.params)
    g1 = gpu_step(st, dataclasses.replace(sc.params, accel=(0.0, 2.0)))
    ped = st["cls"] == 0
    # pedestrians take no acceleration lines: same decisions, velocities to a
    # few ulps (separate kernel instantiations, see above)
    np.testing.assert_array_equal(g0["status"][ped], g1["status"][ped])
    dv = np.hypot(g0["vx"] - g1["vx"], g0["vy"] - g1["vy"])
    assert dv[ped].max() <= 1e-5
    assert dv[~ped].max() > 1e-3


@pytest.mark.parametrize("mode", [0, 1])
def test_batched_caps_equal_single_scene_steps(mode):
    import torch
    from paper_2008_11578_amd import orca
    caps = [(0.0, 0.0), (0.0, 3.0), (1.5, 1.5), (4.0, 0.0)]
    parts = [_crowd(n, np.sqrt(n / 0.4), seed=40 + s, veh_share=0.1, accel=caps[s % 4])
             for s, n in enumerate([500, 64, 3000, 1, 1200, 800])]
    off = np.zeros(len(parts) + 1, np.int32)
    off[1:] = np.cumsum([p.n for p in parts])
    cat = {k: np.concatenate([getattr(p, k) for p in parts]) for k in parts[0].arrays()}
    st = orca.State.from_arrays(cat)
    b = orca.Batch(off, [p.params for p in parts], mode=mode)
    assert b.has_accel == 1
    out = orca.step_batched(st, b, orca.Workspace(st.n, n_scenes=len(parts)))
    torch.cuda.synchronize()
    assert int(b.error.item()) == 0
    for s, p in enumerate(parts):
        o1 = orca.step(orca.State.from_arrays(p), p.params, orca.Workspace(p.n))
        torch.cuda.synchronize()
        for k in ("vx", "vy", "px", "py"):
            assert torch.equal(getattr(out, k)[off[s]:off[s + 1]], getattr(o1, k)), (s, k)


def test_batched_flags_caps_without_the_capped_kernel():
    import torch
    from paper_2008_11578_amd import orca
    sc = _crowd(300, 20.0, seed=3, veh_share=0.1, accel=(0.0, 2.0))
    st = orca.State.from_arrays(sc)
    b = orca.Batch(np.array([0, sc.n], np.int32), [sc.params])
    b.has_accel = 0   # a caller that claims no scene is capped
    orca.step_batched(st, b, orca.Workspace(st.n, n_scenes=1))
    torch.cuda.synchronize()
    assert int(b.error.item()) == 1


def test_head_on_vehicle_with_low_cap_brakes_late():
    """A vehicle with a low cap cannot turn away in time from a pedestrian it
    is assigned all avoidance of: its velocity changes by at most a dt each
    step (oracle and GPU agree every step), and the pair ends up closer than
    without the cap."""
    from paper_2008_11578_amd import orca
    import torch
    sc = scenarios.head_on_pairs(pairs=4)
    res = {}
    for acc in (0.0, 1.0):
        p = dataclasses.replace(sc.params, f=((0.5, 0.0), (1.0, 0.5)), accel=(0.0, acc))
        st = orca.State.from_arrays(sc)
        ws = orca.Workspace(sc.n)
        ost = {k: v.copy() for k, v in sc.arrays().items()}
        gap = np.inf
        for t in range(sc.steps):
            prev = (st.vx.cpu().numpy().copy(), st.vy.cpu().numpy().copy())
            st = orca.step(st, p, ws)
            torch.cuda.synchronize()
            o = oracle.step(ost, p)
            gv = np.stack([st.vx.cpu().numpy(), st.vy.cpu().numpy()], 1)
            assert np.abs(gv[:, 0] - o["vx"]).max() < 1e-3 and np.abs(gv[:, 1] - o["vy"]).max() < 1e-3, t
            if acc > 0:
                dv = np.hypot(gv[1::2, 0] - prev[0][1::2], gv[1::2, 1] - prev[1][1::2])
                assert (dv <= acc * float(np.float32(p.dt)) * (1 + 1e-5) + 1e-6).all(), t
            ost = {k: (st_k.cpu().numpy() if k in ("px", "py", "vx", "vy") else ost[k])
                   for k, st_k in ((k, getattr(st, k)) for k in ost)}
            d = np.hypot(ost["px"][0::2] - ost["px"][1::2], ost["py"][0::2] - ost["py"][1::2])
            gap = min(gap, float((d - 1.8).min()))
        res[acc] = gap
    _print("min clearance without / with cap", res)
    assert res[0.0] > -1e-4
    assert res[1.0] < res[0.0]


def _rel(a, b):
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-30))


@pytest.mark.parametrize("accel", [(1.0, 2.0), (2.5, 0.0)])
def test_capped_step_backward_matches_oracle(accel):
    """The adjoint through the acceleration lines (q = c + h n_k, c = v or v
    scaled onto the speed circle) against the oracle's forward-mode
    gradient, from a state where the caps bind for many agents (crowd
    accelerating from rest towards its goals)."""
    import torch
    from paper_2008_11578_amd import orca
    sc = scenarios.c5_rollout(seed=6, n=4096, side=120.0)
    params = dataclasses.replace(sc.params, accel=accel)
    st = orca.State.from_arrays(sc)
    nxt = st.clone()
    ws = orca.Workspace(st.n)
    for _ in range(6):
        orca.step(st, params, ws, out=nxt)
        st, nxt = nxt, st
    torch.cuda.synchronize()
    S = st.to_numpy()
    o_cap = oracle.step(S, params)
    o_free = oracle.step(S, dataclasses.replace(params, accel=(0.0, 0.0)))
    bind = np.hypot(o_cap["vx"] - o_free["vx"], o_cap["vy"] - o_free["vy"]) > 1e-4
    _print("accel", accel, "cap binds for", int(bind.sum()), "of", st.n)
    assert bind.mean() > 0.1
    rng = np.random.default_rng(4)
    cot = [rng.normal(size=st.n).astype(np.float32) for _ in range(4)]
    g = [torch.as_tensor(c).cuda() for c in cot]
    gpr = torch.zeros(st.n, device="cuda")
    gpy = torch.zeros(st.n, device="cuda")
    gt = torch.zeros(1, device="cuda")
    out = orca.step_backward(st, params, orca.Workspace(st.n, backward=True), *g, gpr, gpy, gt)
    torch.cuda.synchronize()
    gpx, gpy0, gvx, gvy = [t.cpu().numpy() for t in out]
    o = oracle.step_vjp(S, params, *[c.astype(np.float64) for c in cot])
    # Agents touching a neighbour (||P| - R| below 1e-4) sit where the velocity
    # obstacle switches to the overlap form: d leg / d P grows like
    # 1/sqrt(|P|^2 - R^2), so FP32 and FP64 position cotangents there differ
    # by whole percents (the oracle's own derivative already departs from its
    # finite differences).  They are left out of the position check and kept
    # rare; velocity and pref cotangents are checked for everyone.
    on = oracle.step(S, params, want_neighbors=True)
    gap = np.full(st.n, np.inf)
    for q in range(on["nbr"].shape[1]):
        j = on["nbr"][:, q]
        ok = (j >= 0) & (q < on["cnt"])
        jj = np.where(ok, j, 0)
        d = np.hypot(S["px"][jj].astype(np.float64) - S["px"], S["py"][jj].astype(np.float64) - S["py"])
        r = S["radius"].astype(np.float64) + S["radius"][jj]
        gap = np.where(ok, np.minimum(gap, d - r), gap)
    touch = np.abs(gap) < 1e-4
    _print("touching agents", int(touch.sum()))
    assert touch.mean() < 0.01
    keep = ~touch
    for a, k, tol, mask in ((gvx, "g_vx", 1e-4, None), (gvy, "g_vy", 1e-4, None),
                            (gpr.cpu().numpy(), "g_pref_x", 1e-4, None),
                            (gpy.cpu().numpy(), "g_pref_y", 1e-4, None),
                            (gpx, "g_px", 5e-3, keep), (gpy0, "g_py", 5e-3, keep)):
        if mask is not None:
            a, ref = a[mask], o[k][mask]
        else:
            ref = o[k]
        _print(k, _rel(a, ref))
        assert _rel(a, ref) <= tol, (k, _rel(a, ref))
        assert np.max(np.abs(a - ref)) <= 1e-3 * np.max(np.abs(ref)), k
    # tau's cotangent sums every agent's share, the touching agents' included,
    # whose derivatives FP32 resolves poorly: the bound is 1e-4 relative, or
    # twice what the oracle's own value moves on states perturbed by FP32-sized
    # amounts (velocities by 1e-6 m/s, radii by one ulp), whichever is larger
    moved = max(abs(oracle.step_vjp(perturbed(S, 600 + r), params,
                                    *[c.astype(np.float64) for c in cot])["g_tau"] - o["g_tau"])
                for r in range(2))
    _print("g_tau", float(gt.item()), o["g_tau"], "oracle moves by", moved)
    assert abs(float(gt.item()) - o["g_tau"]) <= max(1e-4 * abs(o["g_tau"]), 2.0 * moved)
