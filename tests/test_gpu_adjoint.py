"""GPU adjoint (orca_step_backward and the checkpointed rollout) against the
oracle's forward-mode gradient, from identical FP32 states.

The oracle VJP is itself pinned to closed forms and FP64 finite differences
(tests/test_oracle_adjoint.py); here the hand-written FP32 adjoint must agree
with it one step at a time, and a whole checkpointed rollout gradient must
agree with the oracle's VJPs chained backwards along the GPU's own
trajectory (which separates the adjoint's maths from FP32 trajectory drift).
"""
import numpy as np
import pytest

import oracle
from paper_2008_11578_amd import scenarios

from parity import perturbed

pytestmark = pytest.mark.gpu


def rel(a, b):
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-30))


def _advanced_state(n=4096, steps=8, seed=5):
    import torch
    from paper_2008_11578_amd import orca
    sc = scenarios.c5_rollout(seed=seed, n=n, side=240.0 * np.sqrt(n / 16384))
    st = orca.State.from_arrays(sc)
    nxt = st.clone()
    ws = orca.Workspace(st.n)
    for _ in range(steps):
        orca.step(st, sc.params, ws, out=nxt)
        st, nxt = nxt, st
    torch.cuda.synchronize()
    return sc, st


def _gpu_vjp(st, params, cot):
    import torch
    from paper_2008_11578_amd import orca
    n = st.n
    g = [torch.as_tensor(c).cuda() for c in cot]
    gpr = torch.zeros(n, device="cuda")
    gpy = torch.zeros(n, device="cuda")
    gt = torch.zeros(1, device="cuda")
    out = orca.step_backward(st, params, orca.Workspace(n, backward=True), *g, gpr, gpy, gt)
    torch.cuda.synchronize()
    return [t.cpu().numpy() for t in out], gpr.cpu().numpy(), gpy.cpu().numpy(), float(gt.item())


@pytest.mark.parametrize("goal", [0, 1])
def test_step_backward_matches_oracle(goal):
    import dataclasses
    sc, st = _advanced_state()
    params = dataclasses.replace(sc.params, pref_is_goal=goal)
    S = st.to_numpy()
    if goal:
        # goals far enough away that the desired speed is capped or arriving
        rng = np.random.default_rng(9)
        S["pref_x"] = (S["px"] + rng.uniform(-30, 30, st.n)).astype(np.float32)
        S["pref_y"] = (S["py"] + rng.uniform(-30, 30, st.n)).astype(np.float32)
        from paper_2008_11578_amd import orca
        st = orca.State.from_arrays(S)
    rng = np.random.default_rng(3)
    cot = [rng.normal(size=st.n).astype(np.float32) for _ in range(4)]
    (gpx, gpy, gvx, gvy), gprx, gpry, gtau = _gpu_vjp(st, params, cot)
    o = oracle.step_vjp(S, params, *[c.astype(np.float64) for c in cot])
    for a, k, tol in ((gvx, "g_vx", 1e-4), (gvy, "g_vy", 1e-4), (gprx, "g_pref_x", 1e-4),
                      (gpry, "g_pref_y", 1e-4), (gpx, "g_px", 5e-3), (gpy, "g_py", 5e-3)):
        assert rel(a, o[k]) <= tol, (k, rel(a, o[k]))
        # no single agent off by more than 1e-3 of the largest cotangent; in
        # goal mode v_pref depends on p with gain up to 1/dt and a derivative
        # kink at the arrival radius |g - p| = v_max dt, where FP32 and FP64
        # may take different sides, so the bound there is 1e-2
        per = 1e-2 if goal and k in ("g_px", "g_py") else 1e-3
        assert np.max(np.abs(a - o[k])) <= per * np.max(np.abs(o[k])), k
    assert abs(gtau - o["g_tau"]) <= 1e-4 * abs(o["g_tau"])


def test_step_backward_deterministic_and_inplace():
    import torch
    from paper_2008_11578_amd import orca
    sc, st = _advanced_state(n=2048)
    rng = np.random.default_rng(4)
    cot = [rng.normal(size=st.n).astype(np.float32) for _ in range(4)]
    a = _gpu_vjp(st, sc.params, cot)
    b = _gpu_vjp(st, sc.params, cot)
    for x, y in zip(a[0], b[0]):
        assert np.array_equal(x, y)
    assert a[3] == b[3]
    # in place: outputs overwrite the incoming cotangents
    g = [torch.as_tensor(c).cuda() for c in cot]
    gpr = torch.zeros(st.n, device="cuda")
    gpy = torch.zeros(st.n, device="cuda")
    orca.step_backward(st, sc.params, orca.Workspace(st.n, backward=True), *g, gpr, gpy,
                       None, out=tuple(g))
    torch.cuda.synchronize()
    for x, y in zip(a[0], g):
        assert np.array_equal(x, y.cpu().numpy())
    assert np.array_equal(a[1], gpr.cpu().numpy())


def component_err(g, ref):
    """Per-parameter error measure of the rollout gradient:
    |g - g_ref| / max(|g_ref|, 1e-3 max|g_ref|)."""
    g, ref = np.asarray(g, np.float64), np.asarray(ref, np.float64)
    return np.abs(g - ref) / np.maximum(np.abs(ref), 1e-3 * np.max(np.abs(ref)))


def touching(states, params, tol=1e-4):
    """Agents that at some state of the trajectory are within `tol` m of
    touching one of their neighbours (||P| - R| < tol): there the velocity
    obstacle changes form (reading 5) and its derivative grows like
    1 / sqrt(|P|^2 - R^2), so FP32 and FP64 Jacobians part."""
    flag = None
    for s in states:
        px = s["px"].astype(np.float64)
        py = s["py"].astype(np.float64)
        r = s["radius"].astype(np.float64)
        nb, cn = oracle.knn(s["px"], s["py"], params.neighbor_dist, params.max_neighbors)
        j = np.where(nb >= 0, nb, 0)
        d = np.hypot(px[j] - px[:, None], py[j] - py[:, None]) - (r[j] + r[:, None])
        near = (np.abs(d) < tol) & (nb >= 0)
        f = near.any(axis=1)
        flag = f if flag is None else (flag | f)
    return flag


def _rollout_vs_chain(sc, steps, ckpt, label):
    """GPU rollout gradient (autograd through the checkpointed rollout)
    against the oracle's VJPs chained backwards along the GPU's own FP32
    trajectory, per parameter (C-12's measure) for every desired-velocity
    component and tau."""
    import torch
    from paper_2008_11578_amd import orca, rollout
    p = sc.params
    n = sc.n
    st0 = orca.State.from_arrays(sc)
    vpx = st0.pref_x.clone().requires_grad_(True)
    vpy = st0.pref_y.clone().requires_grad_(True)
    tau = torch.tensor(float(np.float32(p.time_horizon)), device="cuda", requires_grad=True)
    tx = torch.as_tensor(sc.target_x).cuda()
    ty = torch.as_tensor(sc.target_y).cuda()
    px, py = rollout.rollout(vpx, vpy, tau, st0, p, steps=steps, ckpt=ckpt)
    rollout.trajectory_loss(px, py, tx, ty).backward()
    torch.cuda.synchronize()
    ws = orca.Workspace(n)
    s, s2 = st0.clone(), st0.clone()
    states = []
    for _ in range(steps):
        states.append(s.to_numpy())
        orca.step(s, p, ws, out=s2)
        s, s2 = s2, s
    fin = s.to_numpy()
    np.testing.assert_array_equal(fin["px"], px.detach().cpu().numpy())
    g = np.concatenate([vpx.grad.cpu().numpy(), vpy.grad.cpu().numpy()])
    ref, gtau = _oracle_chain(states, fin, sc, p)
    e = component_err(g, ref)
    e_tau = abs(tau.grad.item() - gtau) / abs(gtau)
    touch = touching(states, p)
    # conditioning of the FP64 chained gradient itself: the same chain on
    # states moved by FP32-sized amounts (velocities by 1e-6 m/s, radii by
    # one ulp, as the step parity contract does); a component that then
    # moves by more than a tenth of the tolerance depends on an interaction
    # decided below FP32 resolution (a contact, nearly parallel active
    # lines), directly or through a neighbour earlier in the rollout
    sens = np.zeros_like(e)
    for r in range(2):
        pert = [perturbed(s_, 4000 + 97 * t + r) for t, s_ in enumerate(states)]
        ref_p, _ = _oracle_chain(pert, fin, sc, p)
        sens = np.maximum(sens, component_err(ref_p, ref))
    ill = sens > 1e-4
    # agents whose forward step on the GPU took another answer than the
    # oracle's from the same state (allowed by the step parity contract for
    # ill-conditioned agents only): their Jacobian there belongs to another
    # active set, which reaches their own desired velocity and those of the
    # neighbours their half-planes were built from
    flip = np.zeros(n, bool)
    for t in range(steps):
        nxt_ = states[t + 1] if t + 1 < steps else fin
        o = oracle.step(states[t], p, want_neighbors=True)
        bad = np.hypot(o["vx"] - nxt_["vx"], o["vy"] - nxt_["vy"]) > 1e-5
        if bad.any():
            flip[bad] = True
            nb = o["nbr"][bad]
            flip[nb[nb >= 0]] = True
    flip2 = np.concatenate([flip, flip])
    # diagnostics of the components outside the tolerance that none of the
    # probes explains: the largest one-step velocity difference of the agent
    # and of its neighbours over the rollout
    unexpl = np.nonzero((e > 1e-3) & ~ill & ~flip2)[0] % n
    if unexpl.size:
        own = np.zeros(n)
        nbm = np.zeros(n)
        for t in range(steps):
            nxt_ = states[t + 1] if t + 1 < steps else fin
            o = oracle.step(states[t], p, want_neighbors=True)
            d = np.hypot(o["vx"] - nxt_["vx"], o["vy"] - nxt_["vy"])
            own = np.maximum(own, d)
            nb = o["nbr"]
            nbm = np.maximum(nbm, np.where(nb >= 0, d[np.where(nb >= 0, nb, 0)], 0).max(axis=1))
        print("  unexplained:", [(int(a), float(own[a]), float(nbm[a])) for a in unexpl[:12]],
              flush=True)
    touch2 = np.concatenate([touch, touch])
    exempt = ill | flip2
    worst = np.argsort(e)[-5:][::-1]
    print(f"{label}: {e.size} components, err max {e.max():.2e} median {np.median(e):.2e}, "
          f"over 1e-3: {int(np.sum(e > 1e-3))} ({int(np.sum((e > 1e-3) & exempt))} "
          f"ill-conditioned, {int(np.sum((e > 1e-3) & touch2 & ~exempt))} others touching, "
          f"{int(np.sum((e > 1e-3) & flip2 & ~exempt))} others near a differing step, "
          f"{int(np.sum((e > 1e-3) & ~flip2 & ~touch2 & ~exempt))} none of these); "
          f"{int(flip.sum())} agents near a differing step; "
          f"{int(touch.sum())} agents touch, {int(ill.sum())} components ill-conditioned; "
          f"tau {tau.grad.item():.6g} vs {gtau:.6g} (err {e_tau:.1e}); worst "
          f"{[(int(i % n), float(e[i]), float(sens[i]), bool(exempt[i])) for i in worst]}",
          flush=True)
    assert rel(g, ref) <= 1e-3
    assert e_tau <= 1e-3
    assert exempt.mean() <= 0.2, exempt.mean()
    return e, exempt


def _oracle_chain(states, fin, sc, p):
    """The oracle's one-step VJPs chained backwards along `states` from the
    loss gradient at the final positions `fin`: (d loss / d v_pref as
    [x components, y components], d loss / d tau)."""
    n = sc.n
    gpx = 2 * (fin["px"].astype(np.float64) - sc.target_x) / n
    gpy = 2 * (fin["py"].astype(np.float64) - sc.target_y) / n
    gvx = np.zeros(n)
    gvy = np.zeros(n)
    gprx = np.zeros(n)
    gpry = np.zeros(n)
    gtau = 0.0
    for t in range(len(states) - 1, -1, -1):
        r = oracle.step_vjp(states[t], p, gpx, gpy, gvx, gvy)
        gpx, gpy, gvx, gvy = r["g_px"], r["g_py"], r["g_vx"], r["g_vy"]
        gprx += r["g_pref_x"]
        gpry += r["g_pref_y"]
        gtau += r["g_tau"]
    return np.concatenate([gprx, gpry]), gtau


def test_rollout_gradient_matches_oracle_chain():
    sc = scenarios.c5_rollout(n=4096, side=120.0)
    e, exempt = _rollout_vs_chain(sc, 20, 6, "rollout 4096 x 20")
    assert (e[~exempt] <= 1e-3).all()


def test_rollout_gradient_full_shape_matches_oracle_chain():
    """16,384 agents, 50 steps, checkpoints every 10: the GPU gradient with
    respect to each of the 32,768 desired-velocity components and tau."""
    sc = scenarios.c5_rollout()
    e, exempt = _rollout_vs_chain(sc, sc.steps, 10, "rollout 16384 x 50")
    assert (e[~exempt] <= 1e-3).all()


def test_rollout_host_tau_equals_device_tau():
    """tau given as a host scalar (read without a device synchronisation)
    gives the same rollout and the same gradients, bit for bit, as tau on
    the device; its gradient comes back on the host."""
    import torch
    from paper_2008_11578_amd import orca, rollout
    sc = scenarios.c5_rollout(n=2048, side=240.0 * np.sqrt(2048 / 16384))
    p = sc.params
    st0 = orca.State.from_arrays(sc)
    tx = torch.as_tensor(sc.target_x).cuda()
    ty = torch.as_tensor(sc.target_y).cuda()
    res = []
    for dev in ("cuda", "cpu"):
        vpx = st0.pref_x.clone().requires_grad_(True)
        vpy = st0.pref_y.clone().requires_grad_(True)
        tau = torch.tensor(float(np.float32(p.time_horizon)), device=dev, requires_grad=True)
        px, py = rollout.rollout(vpx, vpy, tau, st0, p, steps=12, ckpt=5)
        loss = rollout.trajectory_loss(px, py, tx, ty)
        loss.backward()
        torch.cuda.synchronize()
        assert tau.grad.device.type == dev
        res.append((px.detach().cpu(), vpx.grad.cpu(), vpy.grad.cpu(), float(tau.grad)))
    assert torch.equal(res[0][0], res[1][0])
    assert torch.equal(res[0][1], res[1][1]) and torch.equal(res[0][2], res[1][2])
    assert res[0][3] == res[1][3]


def test_rollout_graph_replays_equal_eager_rollout():
    """The captured rollout (forward and backward graphs) gives the eager
    rollout's final positions and gradients bit for bit, on two replays with
    different desired velocities (with eager work in between)."""
    import torch
    from paper_2008_11578_amd import orca, rollout
    sc = scenarios.c5_rollout(n=2048, side=240.0 * np.sqrt(2048 / 16384))
    p = sc.params
    st0 = orca.State.from_arrays(sc)
    tx = torch.as_tensor(sc.target_x).cuda()
    ty = torch.as_tensor(sc.target_y).cuda()
    tau = float(np.float32(p.time_horizon))
    rg = rollout.RolloutGraph(st0, p, tau, steps=12, ckpt=5)
    for r in range(2):
        scale = 1.0 - 0.1 * r
        vpx = (st0.pref_x * scale).clone().requires_grad_(True)
        vpy = (st0.pref_y * scale).clone().requires_grad_(True)
        tt = torch.tensor(tau, requires_grad=True)
        px, py = rollout.rollout(vpx, vpy, tt, st0, p, steps=12, ckpt=5)
        # the cotangents autograd hands the rollout, for the graph's backward
        seen = {}
        px.register_hook(lambda g: seen.__setitem__("x", g.clone()))
        py.register_hook(lambda g: seen.__setitem__("y", g.clone()))
        rollout.trajectory_loss(px, py, tx, ty).backward()
        torch.cuda.synchronize()
        gx, gy = rg.forward(vpx.detach(), vpy.detach())
        assert torch.equal(gx, px.detach()) and torch.equal(gy, py.detach()), r
        g_prx, g_pry, g_tau = rg.backward(seen["x"], seen["y"])
        torch.cuda.synchronize()
        assert torch.equal(g_prx, vpx.grad) and torch.equal(g_pry, vpy.grad), r
        assert float(g_tau) == float(tt.grad), r
