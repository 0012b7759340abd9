"""Pins of the oracle's acceleration limit (Sec. 5: acceleration-limited
vehicles add linear constraints of their own motion to the same LP).

Reading under test: with cap a the new velocity lies in the regular octagon
inscribed in the disc of radius a dt about c (the current velocity, scaled
onto the speed circle when outside it); the octagon's edges are hard lines
ahead of the ORCA lines, never relaxed by the least-penetration fallback.

Sources of truth, none of them the oracle itself:
  * the geometry of the inscribed regular octagon (its vertices on the disc
    boundary, two edges through each vertex, the centre strictly inside);
  * closed forms for a lone agent (the desired velocity along an edge normal
    lands on the edge midpoint, along a vertex direction on the vertex);
  * brute force over the candidate points of the two programs with hard
    lines: the closest permitted point (LP2) and the least largest
    penetration of the soft lines within the hard region (LP3);
  * relations to the uncapped step: a cap too large to bind changes nothing
    (bit for bit), an uncapped class is unaffected by another class's cap;
  * FP64 central differences of the step's gradient with caps active.
"""
import itertools
import math

import numpy as np
import pytest

from paper_2008_11578_amd import scenarios

from test_oracle_lp import brute_lp2, line_circle, line_line, penetration, rand_lines

F32 = np.float32


def octagon_vertices(c, a_dt):
    k = np.arange(8)
    ang = (2 * k + 1) * math.pi / 8
    return np.asarray(c, float)[None, :] + a_dt * np.stack([np.cos(ang), np.sin(ang)], 1)


@pytest.mark.parametrize("v,vmax", [((1.0, 0.5), 2.0), ((0.0, 0.0), 1.5), ((3.0, -4.0), 2.5)])
def test_accel_lines_are_the_inscribed_octagon(oracle_mod, v, vmax):
    a, dt = 4.0, 0.1
    L = oracle_mod.accel_lines(v, vmax, a, dt)
    assert L.shape == (8, 4)
    sp = math.hypot(*v)
    c = np.array(v) * (vmax / sp if sp > vmax else 1.0)
    # the centre is strictly inside every edge, by a dt cos(pi/8)
    np.testing.assert_allclose(penetration(L, c), -a * dt * math.cos(math.pi / 8), rtol=1e-12)
    for vert in octagon_vertices(c, a * dt):
        assert abs(np.linalg.norm(vert - c) - a * dt) < 1e-12
        pen = penetration(L, vert)
        assert (np.abs(pen) < 1e-12).sum() == 2      # on exactly two edges
        assert pen.max() < 1e-12                     # inside all of them
    # points just outside the disc in the vertex directions are cut off
    for vert in octagon_vertices(c, a * dt * (1 + 1e-6)):
        assert penetration(L, vert).max() > 0
    assert oracle_mod.accel_lines(v, vmax, 0.0, dt).shape == (0, 4)


def _lone(v, pref, vmax, accel, dt=0.25):
    st = dict(px=np.zeros(1, F32), py=np.zeros(1, F32), vx=np.array([v[0]], F32),
              vy=np.array([v[1]], F32), pref_x=np.array([pref[0]], F32),
              pref_y=np.array([pref[1]], F32), radius=np.full(1, 0.3, F32),
              max_speed=np.full(1, vmax, F32), cls=np.ones(1, np.uint8))
    prm = scenarios.Params(dt=dt, pref_is_goal=0, accel=(0.0, accel))
    return st, prm


def test_lone_agent_closed_forms(oracle_mod):
    # a dt = 1: edge midpoint at cos(pi/8) along +x
    st, prm = _lone((0.0, 0.0), (10.0, 0.0), 20.0, 4.0)
    o = oracle_mod.step(st, prm)
    np.testing.assert_allclose([o["vx"][0], o["vy"][0]], [math.cos(math.pi / 8), 0.0],
                               atol=1e-12)
    assert o["status"][0] == 0
    # along a vertex direction: the vertex itself, at distance a dt
    ang = math.pi / 8
    st, prm = _lone((0.0, 0.0), (10 * math.cos(ang), 10 * math.sin(ang)), 20.0, 4.0)
    o = oracle_mod.step(st, prm)
    np.testing.assert_allclose([o["vx"][0], o["vy"][0]], [math.cos(ang), math.sin(ang)],
                               atol=1e-6)  # the desired direction is given in FP32
    # current velocity above the cap: the octagon sits about the clipped velocity
    st, prm = _lone((3.0, 0.0), (0.0, 0.0), 2.0, 2.0)
    o = oracle_mod.step(st, prm)
    np.testing.assert_allclose([o["vx"][0], o["vy"][0]],
                               [2.0 - 0.5 * math.cos(math.pi / 8), 0.0], atol=1e-12)
    # a desired velocity within reach is taken as it is
    st, prm = _lone((1.0, 1.0), (1.2, 0.9), 3.0, 4.0)
    o = oracle_mod.step(st, prm)
    np.testing.assert_allclose([o["vx"][0], o["vy"][0]], [float(F32(1.2)), float(F32(0.9))],
                               atol=0)


def brute_lp3_hard_value(soft, hard, vmax):
    """min over {|v| <= vmax, hard lines} of max_j delta_j(v) over the soft
    lines, by enumerating where the optimum of a convex piecewise-linear
    function over a convex region bounded by lines and a circle can sit."""
    n = np.stack([-soft[:, 3], soft[:, 2]], axis=1)
    eqs = []   # soft equalities as lines (q, d)
    for a, b in itertools.combinations(range(len(soft)), 2):
        g = n[a] - n[b]
        h = n[a] @ soft[a, 0:2] - n[b] @ soft[b, 0:2]
        gl = np.linalg.norm(g)
        if gl > 1e-12:
            q = g * h / (gl * gl)
            eqs.append(np.array([q[0], q[1], -g[1] / gl, g[0] / gl]))
    cands = [vmax * n[j] for j in range(len(soft))]
    for l in list(hard) + eqs:
        cands.extend(line_circle(l, vmax))
    for a, b in itertools.combinations(list(hard) + eqs, 2):
        p = line_line(a, b)
        if p is not None:
            cands.append(p)
    best = np.inf
    for c in cands:
        if np.linalg.norm(c) > vmax + 1e-9 or penetration(hard, c).max() > 1e-9:
            continue
        best = min(best, penetration(soft, c).max())
    return best


def test_lp_with_hard_lines_matches_brute_force(oracle_mod):
    rng = np.random.default_rng(808)
    n2 = n3 = hard_active = 0
    for it in range(2500):
        vmax = float(rng.uniform(0.5, 3.0))
        v = rng.uniform(-1.2, 1.2, 2) * vmax
        a_dt = float(rng.uniform(0.1, 1.5))
        hard = oracle_mod.accel_lines(v, vmax, a_dt, 1.0)
        sp = np.linalg.norm(v)
        c = v * (vmax / sp if sp > vmax else 1.0)
        m = int(rng.integers(1, 7))
        soft = rand_lines(rng, m)
        lines = np.concatenate([hard, soft])
        opt = rng.uniform(-3, 3, 2)
        res, fail = oracle_mod.lp_full_hard(lines, 8, vmax, opt, c)
        # hard lines and the speed cap always hold
        assert penetration(hard, res).max() <= 1e-9, it
        assert np.linalg.norm(res) <= vmax * (1 + 1e-9)
        assert fail >= 8, it            # the hard region always meets the disc
        if fail == len(lines):
            n2 += 1
            bf = brute_lp2(lines, vmax, opt)
            assert bf is not None
            assert np.linalg.norm(res - bf) <= 1e-9 * max(1.0, vmax), (it, res, bf)
        else:
            n3 += 1
            hard_active += bool(np.abs(penetration(hard, res)).min() < 1e-9)
            t_or = penetration(soft, res).max()
            t_bf = brute_lp3_hard_value(soft, hard, vmax)
            assert abs(t_or - t_bf) <= 1e-8, (it, t_or, t_bf)
    assert n2 > 500 and n3 > 500, (n2, n3)
    assert hard_active > 200, hard_active   # the least-penetration answer sits on a hard edge


def _crowd(seed, n=1500, side=40.0, n_veh=150):
    sc = scenarios.random_state(n, side, seed=seed, n_vehicles=n_veh,
                                params=scenarios.Params(dt=0.1, neighbor_dist=5.0,
                                                        max_neighbors=10))
    return {k: getattr(sc, k) for k in ("px", "py", "vx", "vy", "pref_x", "pref_y", "radius",
                                         "max_speed", "cls")}, sc.params


def test_cap_too_large_to_bind_changes_nothing(oracle_mod):
    import dataclasses
    st, prm = _crowd(5)
    o0 = oracle_mod.step(st, prm)
    o1 = oracle_mod.step(st, dataclasses.replace(prm, accel=(1e6, 1e6)))
    for k in ("vx", "vy", "px", "py", "status"):
        np.testing.assert_array_equal(o0[k], o1[k])


def test_vehicle_cap_leaves_pedestrians_and_bounds_vehicles(oracle_mod):
    import dataclasses
    st, prm = _crowd(6)
    a = 3.0
    o0 = oracle_mod.step(st, prm)
    o1 = oracle_mod.step(st, dataclasses.replace(prm, accel=(0.0, a)))
    ped = st["cls"] == 0
    np.testing.assert_array_equal(o0["vx"][ped], o1["vx"][ped])
    np.testing.assert_array_equal(o0["vy"][ped], o1["vy"][ped])
    veh = ~ped
    v = np.stack([st["vx"], st["vy"]], 1).astype(np.float64)[veh]
    vmax = st["max_speed"].astype(np.float64)[veh]
    sp = np.linalg.norm(v, axis=1)
    c = v * np.where(sp > vmax, vmax / np.maximum(sp, 1e-300), 1.0)[:, None]
    dv = np.stack([o1["vx"][veh], o1["vy"][veh]], 1) - c
    dt = float(F32(prm.dt))
    assert (np.linalg.norm(dv, axis=1) <= a * dt * (1 + 1e-12)).all()
    # and the cap binds for a good share of them (the test is not vacuous)
    changed = np.hypot(o1["vx"][veh] - o0["vx"][veh], o1["vy"][veh] - o0["vy"][veh]) > 1e-6
    assert changed.mean() > 0.3


def test_capped_step_gradient_matches_central_differences(oracle_mod):
    sc = scenarios.random_state(160, 14.0, seed=9, n_vehicles=40,
                                params=scenarios.Params(dt=0.1, neighbor_dist=5.0,
                                                        max_neighbors=10, pref_is_goal=0,
                                                        accel=(2.0, 3.0)))
    st = {k: np.asarray(getattr(sc, k), np.float64) for k in
          ("px", "py", "vx", "vy", "pref_x", "pref_y", "radius", "max_speed")}
    st["cls"] = sc.cls
    prm = sc.params
    n = len(st["px"])
    rng = np.random.default_rng(12)
    cot = {k: rng.normal(size=n) for k in ("px", "py", "vx", "vy")}
    g = oracle_mod.step_vjp(st, prm, cot["px"], cot["py"], cot["vx"], cot["vy"],
                            double_state=True)

    def loss(s):
        o = oracle_mod.rollout(s, prm, 1)
        return sum(float(np.dot(cot[k], o[k])) for k in ("px", "py", "vx", "vy")), o["trace"]

    base, tr0 = loss(st)
    h = 1e-6
    checked = skipped = 0
    fields = [("vx", "g_vx"), ("vy", "g_vy"), ("px", "g_px"), ("py", "g_py"),
              ("pref_x", "g_pref_x"), ("pref_y", "g_pref_y")]
    trial = 0
    while checked < 40 and trial < 150:
        f, gk = fields[trial % len(fields)]
        trial += 1
        i = int(rng.integers(0, n))
        sp = {k: v.copy() for k, v in st.items()}
        sm = {k: v.copy() for k, v in st.items()}
        sp[f][i] += h
        sm[f][i] -= h
        lp, trp = loss(sp)
        lm, trm = loss(sm)
        if trp != tr0 or trm != tr0:
            skipped += 1
            continue
        fd = (lp - lm) / (2 * h)
        assert abs(g[gk][i] - fd) <= 1e-5 * max(1.0, abs(fd)), (f, i, g[gk][i], fd)
        checked += 1
    assert checked >= 40
