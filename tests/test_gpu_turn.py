"""Turn-rate-limited vehicles on the GPU (Sec. 5: non-holonomic motion as
extra linear constraints in the same LP): the HIP path against the FP64
oracle through the C ABI, over single steps and kept-workspace
trajectories, the batched form against single-scene steps, and the wedge
every capped velocity must stay in."""
import dataclasses

import numpy as np
import pytest

import oracle
from paper_2008_11578_amd import scenarios

from parity import as_dict, compare_step, gpu_step, hard_lines

pytestmark = pytest.mark.gpu


def _print(*a):
    print(*a, flush=True)


def _crowd(n, side, seed, veh_share, turn, accel=(0.0, 0.0), k=10, dt=0.1):
    p = scenarios.Params(dt=dt, neighbor_dist=5.0, max_neighbors=k, accel=accel, turn=turn)
    return scenarios.random_state(n, side, seed=seed, n_vehicles=int(veh_share * n), params=p)


@pytest.mark.parametrize("turn,accel,k", [((0.0, 1.0), (0.0, 0.0), 10),
                                          ((0.5, 2.0), (0.0, 0.0), 16),
                                          ((0.0, 1.5), (0.0, 3.0), 10),
                                          ((3.0, 0.3), (2.0, 1.0), 20)])
def test_turn_capped_step_matches_oracle(turn, accel, k):
    sc = _crowd(6000, 70.0, seed=61 + k, veh_share=0.15, turn=turn, accel=accel, k=k)
    _print("turn", turn, "accel", accel, "k", k, "n", sc.n)
    rep, g, o = compare_step(as_dict(sc), sc.params)
    _print(rep)
    # the wedges bind: agents that changed relative to no turn cap exist
    o0 = oracle.step(as_dict(sc), dataclasses.replace(sc.params, turn=(0.0, 0.0)))
    moved = np.hypot(o["vx"] - o0["vx"], o["vy"] - o0["vy"]) > 1e-3
    _print("moved by the wedge", int(moved.sum()))
    assert moved.sum() > 50


def test_turn_capped_trajectory_kept_workspace():
    """A mixed crowd with turn-limited vehicles stepped 30 times with one
    workspace, as a simulation runs it; every agent of steps 1, 10, 20 and
    30 against the oracle from the GPU's own state before that step."""
    import torch
    from paper_2008_11578_amd import orca
    sc = _crowd(8000, 80.0, seed=71, veh_share=0.2, turn=(0.0, 1.0), accel=(0.0, 2.0))
    params = sc.params
    state = orca.State.from_arrays(sc)
    nxt = state.clone()
    ws = orca.Workspace(state.n)
    status = torch.zeros(state.n, dtype=torch.uint8, device="cuda")
    for s in range(1, 31):
        if s in (1, 10, 20, 30):
            torch.cuda.synchronize()
            snap = state.to_numpy()
        orca.step(state, params, ws, out=nxt, status=status)
        if s in (1, 10, 20, 30):
            torch.cuda.synchronize()
            g = {k: getattr(nxt, k).cpu().numpy() for k in ("px", "py", "vx", "vy")}
            g["status"] = status.cpu().numpy()
            rep, _, _ = compare_step(snap, params, gpu=g)
            _print("step", s, rep)
        state, nxt = nxt, state


def test_turn_capped_step_full_size_measured_configuration():
    """The 1,048,576-agent dense crossing with a turn cap of 1 rad/s for
    everyone, 0.6 m cells, one workspace kept across steps: every agent of
    the sixth step against the oracle."""
    import torch
    from paper_2008_11578_amd import orca
    sc = scenarios.c3_crossing()
    params = dataclasses.replace(sc.params, cell_size=0.6, turn=(1.0, 1.0))
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
    _print("turn-capped c3 1M", rep)


def test_turn_capped_every_velocity_within_its_wedge():
    """GPU velocities respect the hard lines (acceleration octagon and
    heading wedge) the oracle forms for each agent, to FP32 rounding."""
    sc = _crowd(4000, 60.0, seed=75, veh_share=0.3, turn=(0.5, 1.5), accel=(0.0, 2.0))
    st = as_dict(sc)
    g = gpu_step(st, sc.params)
    worst = 0.0
    n_wedge = 0
    for a in range(sc.n):
        h, _ = hard_lines(st, sc.params, a)
        if h.shape[0] == 0:
            continue
        n_wedge += 1
        q, d = h[:, 0:2], h[:, 2:4]
        r = q - np.array([g["vx"][a], g["vy"][a]], np.float64)
        worst = max(worst, float((d[:, 0] * r[:, 1] - d[:, 1] * r[:, 0]).max()))
    _print("agents with hard lines", n_wedge, "worst hard-line penetration", worst)
    assert n_wedge > 1000
    assert worst <= 1e-5


def test_uncapped_class_unchanged_by_other_class_turn_cap():
    sc = _crowd(5000, 60.0, seed=78, veh_share=0.1, turn=(0.0, 0.0))
    st = as_dict(sc)
    g0 = gpu_step(st, sc.params)
    g1 = gpu_step(st, dataclasses.replace(sc.params, turn=(0.0, 1.0)))
    ped = st["cls"] == 0
    # pedestrians take no hard lines: same decisions, velocities to a few
    # ulps (the kernel with hard lines is a separate instantiation)
    np.testing.assert_array_equal(g0["status"][ped], g1["status"][ped])
    dv = np.hypot(g0["vx"] - g1["vx"], g0["vy"] - g1["vy"])
    assert dv[ped].max() <= 1e-5
    assert dv[~ped].max() > 1e-3


@pytest.mark.parametrize("mode", [0, 1])
def test_batched_turn_caps_equal_single_scene_steps(mode):
    import torch
    from paper_2008_11578_amd import orca
    caps = [((0.0, 0.0), (0.0, 0.0)), ((0.0, 1.0), (0.0, 0.0)), ((0.5, 0.5), (1.5, 1.5)),
            ((2.0, 0.0), (0.0, 3.0))]
    parts = [_crowd(n, np.sqrt(n / 0.4), seed=80 + s, veh_share=0.1, turn=caps[s % 4][0],
                    accel=caps[s % 4][1])
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


def test_batched_flags_turn_caps_without_the_capped_kernel():
    import torch
    from paper_2008_11578_amd import orca
    sc = _crowd(300, 20.0, seed=83, veh_share=0.1, turn=(0.0, 1.0))
    st = orca.State.from_arrays(sc)
    b = orca.Batch(np.array([0, sc.n], np.int32), [sc.params])
    assert b.has_accel == 1
    b.has_accel = 0      # claim no caps although the scene has one
    orca.step_batched(st, b, orca.Workspace(sc.n, n_scenes=1))
    torch.cuda.synchronize()
    assert int(b.error.item()) == 1


@pytest.mark.parametrize("turn", [(1.0, 1.0), (2.0, 0.0)])
def test_turn_capped_step_backward_matches_oracle(turn):
    """The adjoint through the heading wedge (sides along R(-+phi) v/|v|)
    against the oracle's forward-mode gradient, from a state where the
    wedges bind for many agents; touching agents are left out of the
    position check as in the acceleration case.  (Wedges much narrower than
    these -- 0.03 rad per step -- put LP vertices so close together that
    the active set, and with it the derivative, flips for some agents under
    FP32-sized perturbations of the state: the oracle's own gradient then
    moves by whole units there.)"""
    import torch
    from paper_2008_11578_amd import orca
    from test_gpu_accel import _rel
    sc = scenarios.c5_rollout(seed=7, n=4096, side=120.0)
    params = dataclasses.replace(sc.params, turn=turn)
    st = orca.State.from_arrays(sc)
    nxt = st.clone()
    ws = orca.Workspace(st.n)
    for _ in range(6):
        orca.step(st, params, ws, out=nxt)
        st, nxt = nxt, st
    torch.cuda.synchronize()
    S = st.to_numpy()
    o_cap = oracle.step(S, params)
    o_free = oracle.step(S, dataclasses.replace(params, turn=(0.0, 0.0)))
    bind = np.hypot(o_cap["vx"] - o_free["vx"], o_cap["vy"] - o_free["vy"]) > 1e-4
    _print("turn", turn, "wedge binds for", int(bind.sum()), "of", st.n)
    assert bind.mean() > 0.05
    rng = np.random.default_rng(14)
    cot = [rng.normal(size=st.n).astype(np.float32) for _ in range(4)]
    g = [torch.as_tensor(c).cuda() for c in cot]
    gpr = torch.zeros(st.n, device="cuda")
    gpy = torch.zeros(st.n, device="cuda")
    gt = torch.zeros(1, device="cuda")
    out = orca.step_backward(st, params, orca.Workspace(st.n, backward=True), *g, gpr, gpy, gt)
    torch.cuda.synchronize()
    gpx, gpy0, gvx, gvy = [t.cpu().numpy() for t in out]
    o = oracle.step_vjp(S, params, *[c.astype(np.float64) for c in cot])
    on = oracle.step(S, params, want_neighbors=True)
    gap = np.full(st.n, np.inf)
    for q in range(on["nbr"].shape[1]):
        j = on["nbr"][:, q]
        ok = (j >= 0) & (q < on["cnt"])
        jj = np.where(ok, j, 0)
        d = np.hypot(S["px"][jj].astype(np.float64) - S["px"],
                     S["py"][jj].astype(np.float64) - S["py"])
        r = S["radius"].astype(np.float64) + S["radius"][jj]
        gap = np.where(ok, np.minimum(gap, d - r), gap)
    keep = ~(np.abs(gap) < 1e-4)
    assert keep.mean() > 0.99
    for a, k, tol, mask in ((gvx, "g_vx", 1e-4, None), (gvy, "g_vy", 1e-4, None),
                            (gpr.cpu().numpy(), "g_pref_x", 1e-4, None),
                            (gpy.cpu().numpy(), "g_pref_y", 1e-4, None),
                            (gpx, "g_px", 5e-3, keep), (gpy0, "g_py", 5e-3, keep)):
        ref = o[k] if mask is None else o[k][mask]
        a = a if mask is None else a[mask]
        _print(k, _rel(a, ref))
        assert _rel(a, ref) <= tol, (k, _rel(a, ref))
        assert np.max(np.abs(a - ref)) <= 1e-3 * np.max(np.abs(ref)), k
