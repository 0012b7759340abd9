"""Pins of the lifecycle oracle (agents leave at their goal, enter at clear
spawn points; Sec. 4, first experiment) by exact closed cases."""
import numpy as np

F32 = np.float32


def _agents(px, py, gx=None, gy=None, r=0.3, s=1.5):
    n = len(px)
    return dict(px=np.asarray(px, F32), py=np.asarray(py, F32), vx=np.zeros(n, F32),
                vy=np.zeros(n, F32),
                pref_x=np.asarray(gx if gx is not None else px, F32),
                pref_y=np.asarray(gy if gy is not None else py, F32),
                radius=np.full(n, r, F32), max_speed=np.full(n, s, F32),
                cls=np.zeros(n, np.uint8))


def test_arrival_boundary_is_inclusive(oracle_mod):
    # 3-4-5 triangle in exact binary values: |g - p| = 1.25 exactly
    r_on = F32(1.25)
    r_in = np.nextafter(r_on, F32(0))
    st = _agents([0.0, 0.0, 10.0], [0.0, 0.0, 10.0], [0.75, 0.75, 10.0], [1.0, 1.0, 10.0])
    st["radius"] = np.array([r_on, r_in, 0.3], F32)
    np.testing.assert_array_equal(oracle_mod.arrived(st), [1, 0, 1])


def test_remove_arrived_keeps_order(oracle_mod):
    rng = np.random.default_rng(0)
    n = 1000
    st = _agents(rng.uniform(0, 50, n), rng.uniform(0, 50, n))
    near = rng.random(n) < 0.3
    st["pref_x"] = np.where(near, st["px"] + F32(0.1), st["px"] + F32(5.0)).astype(F32)
    out = oracle_mod.remove_arrived(st)
    keep = ~near
    assert out["px"].shape[0] == int(keep.sum())
    np.testing.assert_array_equal(out["px"], st["px"][keep])
    np.testing.assert_array_equal(out["old_to_new"][keep], np.arange(int(keep.sum())))
    assert (out["old_to_new"][near] == -1).all()


def test_spawn_on_a_line_takes_every_third(oracle_mod):
    # D = (r + r) + T (s + s) = 0.5 + 0.5 * 2 = 1.5; spacing 0.5 -> distance 1.5
    # (exactly D, allowed) first reached three places on
    empty = _agents([], [])
    x = np.arange(30) * 0.5
    cand = dict(px=x, py=np.zeros(30), radius=np.full(30, 0.25), max_speed=np.full(30, 1.0))
    acc = oracle_mod.spawn(empty, cand, 0.5)
    np.testing.assert_array_equal(np.nonzero(acc)[0], np.arange(0, 30, 3))
    # spacing 0.625: ceil(1.5 / 0.625) = 3 as well; spacing 0.75: every second
    cand["px"] = np.arange(30) * 0.625
    np.testing.assert_array_equal(np.nonzero(oracle_mod.spawn(empty, cand, 0.5))[0],
                                  np.arange(0, 30, 3))
    cand["px"] = np.arange(30) * 0.75
    np.testing.assert_array_equal(np.nonzero(oracle_mod.spawn(empty, cand, 0.5))[0],
                                  np.arange(0, 30, 2))


def test_spawn_ring_around_an_agent(oracle_mod):
    # one agent at the origin (r 0.25, s 1); candidates (r 0.25, s 1), T = 1:
    # D = 0.5 + 2 = 2.5; on the ring of radius 2.5 every candidate is clear,
    # on the ring of radius 2.5 - 2^-20 none is (exact binary coordinates)
    agent = _agents([0.0], [0.0], r=0.25, s=1.0)
    for rho, expect in ((2.5, 1), (2.5 - 2.0 ** -20, 0)):
        pts = np.array([(rho, 0), (0, rho), (-rho, 0), (0, -rho)])
        # the ring points are far apart (3.5 > D), so they never block each other
        cand = dict(px=pts[:, 0], py=pts[:, 1], radius=np.full(4, 0.25), max_speed=np.ones(4))
        np.testing.assert_array_equal(oracle_mod.spawn(agent, cand, 1.0), [expect] * 4)
    # 3-4-5: candidate at (1.5, 2.0) is exactly 2.5 away
    cand = dict(px=[1.5], py=[2.0], radius=[0.25], max_speed=[1.0])
    assert oracle_mod.spawn(agent, cand, 1.0)[0] == 1
    cand["px"] = [np.nextafter(F32(1.5), F32(0))]
    assert oracle_mod.spawn(agent, cand, 1.0)[0] == 0


def test_spawn_zero_window_is_plain_overlap(oracle_mod):
    # T = 0: candidates are rejected exactly when their discs overlap someone
    agent = _agents([0.0], [0.0], r=0.5, s=9.0)
    cand = dict(px=[1.0, 0.96875], py=[0.0, 0.0], radius=[0.5, 0.5], max_speed=[9.0, 9.0])
    np.testing.assert_array_equal(oracle_mod.spawn(agent, cand, 0.0), [1, 0])


def test_spawn_is_greedy_and_maximal(oracle_mod):
    """Random case: the accepted set is pairwise clear and clear of every
    agent; every rejected candidate is blocked by an agent or by an earlier
    accepted candidate (the greedy rule in the given order)."""
    rng = np.random.default_rng(1)
    st = _agents(rng.uniform(0, 40, 300), rng.uniform(0, 40, 300))
    nc = 400
    cand = dict(px=rng.uniform(0, 40, nc).astype(F32), py=rng.uniform(0, 40, nc).astype(F32),
                radius=np.where(rng.random(nc) < 0.1, 1.5, 0.3).astype(F32),
                max_speed=np.where(rng.random(nc) < 0.1, 6.0, 1.5).astype(F32))
    T = F32(0.5)
    acc = oracle_mod.spawn(st, cand, T).astype(bool)

    def close(ax, ay, ar, as_, bx, by, br, bs):
        f = lambda v: np.asarray(v, np.float64)  # noqa: E731
        d = (f(ar) + f(br)) + f(T) * (f(as_) + f(bs))
        return (f(bx) - f(ax)) ** 2 + (f(by) - f(ay)) ** 2 < d * d

    for c in range(nc):
        blocked_agent = close(cand["px"][c], cand["py"][c], cand["radius"][c], cand["max_speed"][c],
                              st["px"], st["py"], st["radius"], st["max_speed"]).any()
        earlier = np.nonzero(acc[:c])[0]
        blocked_cand = close(cand["px"][c], cand["py"][c], cand["radius"][c], cand["max_speed"][c],
                             cand["px"][earlier], cand["py"][earlier], cand["radius"][earlier],
                             cand["max_speed"][earlier]).any()
        assert acc[c] == (not blocked_agent and not blocked_cand), c
    assert 0 < acc.sum() < nc


def test_overlap_stats_closed_forms(oracle_mod):
    """Two discs at distance d (exact binary values): one overlapping pair
    exactly when d < r_1 + r_2 (touching is not overlapping), clearance
    d - (r_1 + r_2); pairs beyond the reach count for nothing; fewer than two
    agents give no pair and an infinite clearance."""
    for f in (oracle_mod.overlap_stats, oracle_mod.overlap_stats_tree):
        for d, pairs in ((0.5, 1), (0.75, 0), (1.0, 0)):
            st = _agents([0.0, d], [0.0, 0.0])
            st["radius"] = np.array([0.25, 0.5], F32)
            got = f(st, 2.0)
            assert got["pairs"] == pairs and got["agents"] == 2 * pairs
            assert got["min_clearance"] == d - 0.75
        # a third agent 3 m away is outside a 2 m reach
        st = _agents([0.0, 1.0, 4.0], [0.0, 0.0, 0.0])
        st["radius"] = np.array([0.25, 0.5, 0.25], F32)
        got = f(st, 2.0)
        assert got["pairs"] == 0 and got["min_clearance"] == 0.25
        for m in (0, 1):
            got = f(_agents([0.0] * m, [0.0] * m), 2.0)
            assert got["pairs"] == 0 and got["agents"] == 0 and np.isinf(got["min_clearance"])


def test_overlap_stats_lattice(oracle_mod):
    """k x k lattice of spacing 1 m, radius 0.625 m: lattice neighbours
    overlap (1.25 > 1), diagonal ones do not (1.25 < sqrt 2), so there are
    2 k (k - 1) pairs, every agent is in one, and the clearance is -0.25."""
    k = 30
    gx, gy = np.meshgrid(np.arange(k, dtype=F32), np.arange(k, dtype=F32))
    st = _agents(gx.ravel(), gy.ravel(), r=0.625)
    for f in (oracle_mod.overlap_stats, oracle_mod.overlap_stats_tree):
        got = f(st, 3.0)
        assert got["pairs"] == 2 * k * (k - 1)
        assert got["agents"] == k * k
        assert got["min_clearance"] == -0.25


def test_overlap_stats_tree_equals_all_pairs(oracle_mod):
    """The k-d tree listing and the all-pairs loop agree exactly on random
    crowds with mixed radii, including pairs at the reach boundary."""
    rng = np.random.default_rng(5)
    for n, side, reach in ((2000, 40.0, 3.0), (3000, 25.0, 1.0), (500, 5.0, 0.5)):
        st = _agents(rng.uniform(0, side, n), rng.uniform(0, side, n))
        st["radius"] = np.where(rng.random(n) < 0.1, 1.5, 0.3).astype(F32)
        # a pair exactly at the reach (not counted) and one just inside it
        st["px"][:4] = np.array([0.0, reach, 100.0, 100.0 + np.nextafter(F32(reach), F32(0))], F32)
        st["py"][:4] = np.array([-50.0, -50.0, -50.0, -50.0], F32)
        a = oracle_mod.overlap_stats(st, reach)
        b = oracle_mod.overlap_stats_tree(st, reach)
        assert a == b
        assert a["pairs"] > 0
