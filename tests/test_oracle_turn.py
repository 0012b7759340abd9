"""Pins of the oracle's turn-rate limit (Sec. 5: non-holonomic vehicles add
linear constraints of their own motion to the same LP).

Reading under test: a vehicle moves along its heading, the direction of its
current velocity, and turns it by at most w dt per step, so the new velocity
lies in the wedge of half-angle phi = min(w dt, pi/2) about that heading,
apex at the origin; the wedge's two sides are hard lines (after any
acceleration lines), never relaxed by the least-penetration fallback.  At
rest there is no heading and no wedge.

Sources of truth, none of them the oracle itself:
  * the geometry of the wedge, from rotation matrices: both sides through
    the origin, the rays at +-phi from the heading on them, directions just
    inside phi permitted and just outside cut off;
  * closed forms for a lone agent (a desired velocity outside the wedge is
    projected onto the nearer side's ray, or onto the apex when it points
    away from both; inside it is taken as it is);
  * brute force over the candidate points of the programs with hard lines
    (closest permitted point; least largest penetration of the soft lines
    within the hard region), with and without acceleration lines;
  * relations to the uncapped step on a crowd: pedestrians without a cap are
    unchanged bit for bit, every capped vehicle ends inside its wedge, and
    the cap binds for many of them;
  * FP64 central differences of the step's gradient with the wedges active.
"""
import dataclasses
import math

import numpy as np
import pytest

from paper_2008_11578_amd import scenarios

from test_oracle_accel import brute_lp3_hard_value
from test_oracle_lp import brute_lp2, penetration, rand_lines

F32 = np.float32


def rot(a):
    return np.array([[math.cos(a), -math.sin(a)], [math.sin(a), math.cos(a)]])


@pytest.mark.parametrize("v,turn,dt", [((1.0, 0.0), 0.5, 0.1), ((-0.3, 2.0), 1.0, 0.25),
                                       ((3.0, -4.0), 20.0, 0.1), ((0.1, 0.1), 2.0, 0.5)])
def test_turn_lines_are_the_heading_wedge(oracle_mod, v, turn, dt):
    L = oracle_mod.turn_lines(v, turn, dt)
    assert L.shape == (2, 4)
    np.testing.assert_array_equal(L[:, 0:2], 0.0)                # through the origin
    np.testing.assert_allclose(np.linalg.norm(L[:, 2:4], axis=1), 1.0, rtol=1e-15)
    h = np.asarray(v) / np.linalg.norm(v)
    phi = min(turn * dt, math.pi / 2)
    for s in (0.5, 1.0, 3.0):
        # the heading is permitted, strictly unless the wedge is a half-plane
        assert penetration(L, s * h).max() <= -s * math.sin(phi) * (1 - 1e-12)
        for sign in (1, -1):
            ray = rot(sign * phi) @ h
            pen = penetration(L, s * ray)
            assert abs(pen).min() < 1e-12 and pen.max() < 1e-12   # on a side, inside both
            assert penetration(L, s * rot(sign * phi * (1 - 1e-6)) @ h).max() < 0
            if phi < math.pi / 2:
                assert penetration(L, s * rot(sign * phi * (1 + 1e-6)) @ h).max() > 0
    assert oracle_mod.turn_lines(v, 0.0, dt).shape == (0, 4)
    assert oracle_mod.turn_lines((0.0, 0.0), turn, dt).shape == (0, 4)


def _lone(v, pref, vmax, turn, dt=0.1, accel=0.0):
    st = dict(px=np.zeros(1, F32), py=np.zeros(1, F32), vx=np.array([v[0]], F32),
              vy=np.array([v[1]], F32), pref_x=np.array([pref[0]], F32),
              pref_y=np.array([pref[1]], F32), radius=np.full(1, 0.3, F32),
              max_speed=np.full(1, vmax, F32), cls=np.ones(1, np.uint8))
    prm = scenarios.Params(dt=dt, pref_is_goal=0, turn=(0.0, turn), accel=(0.0, accel))
    return st, prm


def test_lone_agent_closed_forms(oracle_mod):
    phi = float(F32(2.0)) * float(F32(0.1))
    # heading east, desired north: the left side's ray, (v_pref . r_L) r_L
    st, prm = _lone((1.0, 0.0), (0.0, 2.0), 3.0, 2.0)
    o = oracle_mod.step(st, prm)
    np.testing.assert_allclose([o["vx"][0], o["vy"][0]],
                               2.0 * math.sin(phi) * np.array([math.cos(phi), math.sin(phi)]),
                               atol=1e-12)
    assert o["status"][0] == 0
    # desired south-east, outside: the right side's ray
    st, prm = _lone((1.0, 0.0), (1.0, -2.0), 3.0, 2.0)
    o = oracle_mod.step(st, prm)
    r = np.array([math.cos(phi), -math.sin(phi)])
    np.testing.assert_allclose([o["vx"][0], o["vy"][0]], (np.array([1.0, -2.0]) @ r) * r,
                               atol=1e-12)
    # desired backwards: away from both sides, the apex
    st, prm = _lone((1.0, 0.0), (-2.0, 0.3), 3.0, 2.0)
    o = oracle_mod.step(st, prm)
    np.testing.assert_allclose([o["vx"][0], o["vy"][0]], [0.0, 0.0], atol=1e-12)
    # inside the wedge: taken as it is
    st, prm = _lone((1.0, 1.0), (1.5, 1.4), 3.0, 2.0)
    o = oracle_mod.step(st, prm)
    np.testing.assert_array_equal([o["vx"][0], o["vy"][0]], [float(F32(1.5)), float(F32(1.4))])
    # at rest: no heading, no wedge
    st, prm = _lone((0.0, 0.0), (-2.0, 0.3), 3.0, 2.0)
    o = oracle_mod.step(st, prm)
    np.testing.assert_array_equal([o["vx"][0], o["vy"][0]], [float(F32(-2.0)), float(F32(0.3))])
    # w dt beyond a right angle: the half-plane ahead of the heading
    st, prm = _lone((0.0, 2.0), (-1.0, -1.5), 3.0, 50.0)
    o = oracle_mod.step(st, prm)
    np.testing.assert_allclose([o["vx"][0], o["vy"][0]], [-1.0, 0.0], atol=1e-12)


def test_lp_with_heading_lines_matches_brute_force(oracle_mod):
    rng = np.random.default_rng(909)
    n2 = n3 = hard_active = 0
    for it in range(2500):
        vmax = float(rng.uniform(0.5, 3.0))
        v = rng.uniform(-1.2, 1.2, 2) * vmax
        turn_dt = float(rng.uniform(0.02, 2.0))
        with_acc = it % 2 == 1
        hard = oracle_mod.turn_lines(v, turn_dt, 1.0)
        if with_acc:
            hard = np.concatenate([oracle_mod.accel_lines(v, vmax, float(rng.uniform(0.1, 1.5)),
                                                          1.0), hard])
        sp = np.linalg.norm(v)
        c = v * (vmax / sp if sp > vmax else 1.0)
        m = int(rng.integers(1, 7))
        soft = rand_lines(rng, m)
        lines = np.concatenate([hard, soft])
        nh = len(hard)
        opt = rng.uniform(-3, 3, 2)
        res, fail = oracle_mod.lp_full_hard(lines, nh, vmax, opt, c)
        assert penetration(hard, res).max() <= 1e-9, it
        assert np.linalg.norm(res) <= vmax * (1 + 1e-9)
        assert fail >= nh, it           # the hard region always meets the disc
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
    assert hard_active > 200, hard_active


def _crowd(seed, n=1500, side=40.0, n_veh=150):
    sc = scenarios.random_state(n, side, seed=seed, n_vehicles=n_veh,
                                params=scenarios.Params(dt=0.1, neighbor_dist=5.0,
                                                        max_neighbors=10))
    return {k: getattr(sc, k) for k in ("px", "py", "vx", "vy", "pref_x", "pref_y", "radius",
                                         "max_speed", "cls")}, sc.params


def test_vehicle_turn_cap_leaves_pedestrians_and_bounds_vehicles(oracle_mod):
    st, prm = _crowd(16)
    turn = 1.5
    o0 = oracle_mod.step(st, prm)
    o1 = oracle_mod.step(st, dataclasses.replace(prm, turn=(0.0, turn)))
    ped = st["cls"] == 0
    for k in ("vx", "vy", "px", "py", "status"):
        np.testing.assert_array_equal(o0[k][ped], o1[k][ped])
    veh = ~ped
    v0 = np.stack([st["vx"], st["vy"]], 1).astype(np.float64)[veh]
    v1 = np.stack([o1["vx"], o1["vy"]], 1)[veh]
    phi = float(F32(turn)) * float(F32(prm.dt))
    moving = np.linalg.norm(v0, axis=1) > 0
    h = v0[moving] / np.linalg.norm(v0[moving], axis=1)[:, None]
    w = v1[moving]
    sp = np.linalg.norm(w, axis=1)
    ang = np.arctan2(h[:, 0] * w[:, 1] - h[:, 1] * w[:, 0], (h * w).sum(1))
    assert (np.abs(ang[sp > 1e-9]) <= phi * (1 + 1e-9) + 1e-12).all()
    changed = np.hypot(o1["vx"][veh] - o0["vx"][veh], o1["vy"][veh] - o0["vy"][veh]) > 1e-6
    assert changed.mean() > 0.3


def test_turn_capped_step_gradient_matches_central_differences(oracle_mod):
    """Derivatives of the step with respect to the velocities of vehicles
    whose new velocity sits on a side of their wedge (the heading, and so
    the side, turns with the velocity), against central differences."""
    sc = scenarios.random_state(160, 14.0, seed=19, n_vehicles=40,
                                params=scenarios.Params(dt=0.1, neighbor_dist=5.0,
                                                        max_neighbors=10, pref_is_goal=0,
                                                        turn=(0.0, 2.0)))
    st = {k: np.asarray(getattr(sc, k), np.float64) for k in
          ("px", "py", "vx", "vy", "pref_x", "pref_y", "radius", "max_speed")}
    st["cls"] = sc.cls
    prm = sc.params
    n = len(st["px"])
    o = oracle_mod.step(st, prm)
    on_side = [i for i in np.flatnonzero(sc.cls == 1)
               if np.abs(penetration(oracle_mod.turn_lines((st["vx"][i], st["vy"][i]), 2.0,
                                                           float(F32(0.1))),
                                     np.array([o["vx"][i], o["vy"][i]]))).min() < 1e-9]
    assert len(on_side) >= 8, len(on_side)
    rng = np.random.default_rng(22)
    cot = {k: rng.normal(size=n) for k in ("px", "py", "vx", "vy")}
    g = oracle_mod.step_vjp(st, prm, cot["px"], cot["py"], cot["vx"], cot["vy"],
                            double_state=True)

    def loss(s):
        o = oracle_mod.rollout(s, prm, 1)
        return sum(float(np.dot(cot[k], o[k])) for k in ("px", "py", "vx", "vy")), o["trace"]

    base, tr0 = loss(st)
    h = 1e-6
    checked = 0
    for i in on_side:
        for f, gk in (("vx", "g_vx"), ("vy", "g_vy")):
            sp = {k: v.copy() for k, v in st.items()}
            sm = {k: v.copy() for k, v in st.items()}
            sp[f][i] += h
            sm[f][i] -= h
            lp, trp = loss(sp)
            lm, trm = loss(sm)
            if trp != tr0 or trm != tr0:
                continue
            fd = (lp - lm) / (2 * h)
            assert abs(g[gk][i] - fd) <= 1e-5 * max(1.0, abs(fd)), (f, i, g[gk][i], fd)
            # the side's turn with the heading shows in the derivative
            checked += 1
    assert checked >= 12, checked
