"""GPU parity: the HIP path against the FP64 oracle, through the C ABI.

Neighbour lists must match bit for bit; one-step velocities from identical
FP32 states must agree within 1e-4 m/s for every well-conditioned agent (see
tests/parity.py for how conditioning is decided and bounded).
"""
import numpy as np
import pytest

import oracle
from paper_2008_11578_amd import scenarios

from parity import as_dict, compare_step, gpu_neighbors, gpu_step

pytestmark = pytest.mark.gpu


def _print(*a):
    print(*a, flush=True)


def _knn_exact(sc, params=None):
    params = params or sc.params
    st = as_dict(sc)
    nb, cn = gpu_neighbors(st, params)
    onb, ocn = oracle.knn(st["px"], st["py"], params.neighbor_dist, params.max_neighbors)
    np.testing.assert_array_equal(cn, ocn)
    np.testing.assert_array_equal(nb, onb)
    return cn


def test_knn_c1():
    sc = scenarios.c1_plain()
    _print("knn c1", sc.n)
    _knn_exact(sc)


@pytest.mark.parametrize("cell_frac", [1.0, 0.5, 0.34, 2.0])
def test_knn_cell_sizes(cell_frac):
    sc = scenarios.uniform_square(5000, 60.0, seed=21, n_vehicles=100)
    p = scenarios.Params(neighbor_dist=5.0, max_neighbors=16, cell_size=5.0 * cell_frac)
    _print("knn cell size", p.cell_size)
    _knn_exact(sc, p)


@pytest.mark.parametrize("k", [1, 4, 7, 10, 13, 20, 25, 32])
def test_knn_all_capacities(k):
    sc = scenarios.uniform_square(3000, 30.0, seed=k)
    p = scenarios.Params(neighbor_dist=4.0, max_neighbors=k)
    _print("knn k", k)
    cn = _knn_exact(sc, p)
    assert cn.max() == k


def test_knn_exact_ties_lattice():
    g = np.arange(40, dtype=np.float64)
    X, Y = np.meshgrid(g, g)
    perm = np.random.default_rng(3).permutation(1600)
    st = dict(px=X.ravel()[perm].astype(np.float32), py=Y.ravel()[perm].astype(np.float32))
    n = 1600
    for k in ("vx", "vy", "pref_x", "pref_y"):
        st[k] = np.zeros(n, np.float32)
    st["radius"] = np.full(n, 0.3, np.float32)
    st["max_speed"] = np.full(n, 1.5, np.float32)
    st["cls"] = np.zeros(n, np.uint8)
    p = scenarios.Params(neighbor_dist=2.5, max_neighbors=12)
    nb, cn = gpu_neighbors(st, p)
    onb, ocn = oracle.knn(st["px"], st["py"], 2.5, 12)
    np.testing.assert_array_equal(nb, onb)


def test_knn_c2_full():
    sc = scenarios.c2_mixed()
    _print("knn c2", sc.n)
    _knn_exact(sc)


def test_knn_c3_full():
    sc = scenarios.c3_crossing()
    _print("knn c3", sc.n)
    _knn_exact(sc)


def test_step_c1_all_agents():
    sc = scenarios.c1_plain()
    rep, g, o = compare_step(sc, sc.params, require_all=True)
    _print("step c1", rep)
    assert rep["n_bad"] == 0


def test_step_c1_trajectory_resync():
    # advance the GPU 20 steps; at each step re-run one step of both sides
    # from the GPU's FP32 state and compare (trajectories themselves diverge
    # chaotically between FP32 and FP64, so they are never compared)
    sc = scenarios.c1_plain()
    st = as_dict(sc)
    for t in range(sc.steps):
        rep, g, o = compare_step(st, sc.params)
        if t % 5 == 0:
            _print("c1 step", t, rep)
        st = dict(st)
        for k in ("px", "py", "vx", "vy"):
            st[k] = g[k]


def test_step_c2_mixed():
    sc = scenarios.c2_mixed()
    rep, g, o = compare_step(sc, sc.params)
    _print("step c2", rep)


def test_step_random_velocities_mixed():
    sc = scenarios.random_state(20000, 120.0, seed=8, n_vehicles=1000,
                                params=scenarios.Params(dt=0.05, neighbor_dist=5.0,
                                                        max_neighbors=16))
    rep, g, o = compare_step(sc, sc.params)
    _print("step random mixed", rep)


def test_step_dense_crossing_small():
    sc = scenarios.c3_crossing(side_count=128)
    st = as_dict(sc)
    rep, g, o = compare_step(st, sc.params)
    _print("step crossing 16k t=0", rep)


def _kept_run_checks(sc, params, targets, label, want_lp3=True):
    """Steps the scene the way the throughput measurement steps it (one
    workspace kept across steps, so every step after the first narrows its
    counting pass by the previous K-th neighbour distances).  At each target
    state the step is taken through orca_step_nbr, which also exports the
    neighbour lists this step selected: the lists must equal the oracle's
    exact lists bit for bit and every agent must meet the velocity contract.
    The checked step continues the run."""
    import torch
    from paper_2008_11578_amd import orca
    state = orca.State.from_arrays(sc)
    nxt = state.clone()
    ws = orca.Workspace(state.n)
    status = torch.zeros(state.n, dtype=torch.uint8, device="cuda")
    done = 0
    for target in targets:
        while done < target:
            orca.step(state, params, ws, out=nxt, status=status)
            state, nxt = nxt, state
            done += 1
        torch.cuda.synchronize()
        snap = state.to_numpy()
        _, nb, cn = orca.step_nbr(state, params, ws, out=nxt, status=status)
        torch.cuda.synchronize()
        onb, ocn = oracle.knn(snap["px"], snap["py"], params.neighbor_dist,
                              params.max_neighbors)
        np.testing.assert_array_equal(cn.cpu().numpy(), ocn)
        np.testing.assert_array_equal(nb.cpu().numpy(), onb)
        g = {k: getattr(nxt, k).cpu().numpy() for k in ("px", "py", "vx", "vy")}
        g["status"] = status.cpu().numpy()
        rep, _, _ = compare_step(snap, params, gpu=g)
        _print(label, "after", target, "steps: lists exact;", rep)
        if want_lp3:
            assert rep["lp3_gpu"] > 0
        state, nxt = nxt, state
        done += 1


def test_step_c3_full_in_bench_configuration():
    """The 1,048,576-agent dense crossing with 0.6 m cells, stepped as
    measured: the neighbour lists the step selected with its kept distances
    and every agent's velocity, against the oracle, at the steps that open
    (after 10 steps) and close (after 110) the timed window and two in
    between.  After 27 steps a pair touches to within 5e-10 m, which FP32
    takes for an overlap."""
    import dataclasses
    sc = scenarios.c3_crossing()
    params = dataclasses.replace(sc.params, cell_size=0.6)
    _kept_run_checks(sc, params, (10, 27, 60, 110), "step c3 1M")


def test_step_c2_kept_workspace_resync():
    """The mixed crowd (65,536 pedestrians, 1,024 vehicles) over its whole
    200-step run with one kept workspace: the step's own lists and every
    agent's velocity at the start, the middle and the end."""
    sc = scenarios.c2_mixed()
    _kept_run_checks(sc, sc.params, (0, 100, 200), "step c2")


def test_step_vehicle_share_half_kept_workspace():
    """The mixed geometry with half of the 66,560 agents vehicles (nearly
    every agent on the least-penetration fallback): lists and velocities at
    the first step and after 20 kept-workspace steps."""
    sc = scenarios.c2_vehicle_share(0.5)
    _kept_run_checks(sc, sc.params, (0, 20), "step vehicle share 0.5")


def test_step_nbr_equals_step():
    """orca_step_nbr takes the same step as orca_step (outputs, status and
    the distances kept for the next step), bit for bit, on a kept workspace."""
    import torch
    from paper_2008_11578_amd import orca
    sc = scenarios.random_state(30000, 100.0, seed=14, n_vehicles=600)
    st = orca.State.from_arrays(sc)
    ws = orca.Workspace(st.n)
    for _ in range(3):
        orca.step(st, sc.params, ws, out=st)
    ws2 = orca.Workspace(st.n)
    ws2.buf.copy_(ws.buf)
    s1 = torch.zeros(st.n, dtype=torch.uint8, device="cuda")
    s2 = torch.zeros_like(s1)
    a = orca.step(st, sc.params, ws, status=s1)
    b, nb, cn = orca.step_nbr(st, sc.params, ws2, status=s2)
    torch.cuda.synchronize()
    for k in ("px", "py", "vx", "vy"):
        assert torch.equal(getattr(a, k), getattr(b, k)), k
    assert torch.equal(s1, s2)
    # what the workspace carries to the next step (the kept neighbour
    # distances, its last region) is the same; the cell-ordered copy is not
    # compared, since the order of agents inside one cell follows the order
    # of the counting pass's atomic increments and differs between runs
    assert torch.equal(_kept_distances(ws, st.n), _kept_distances(ws2, st.n))


def _kept_distances(ws, n):
    """The workspace's last region: each agent's K-th neighbour distance
    kept for the next step (float32, caller order)."""
    import torch
    region = (4 * n + 255) // 256 * 256
    return ws.buf[ws.nbytes - region:ws.nbytes - region + 4 * n].view(torch.float32)


def test_kept_distances_change_no_result_full_size():
    """The measured 1M crossing stepped with a workspace kept across steps
    (counting pass narrowed by the previous K-th neighbour distances) equals,
    bit for bit, a step from the same state with a fresh workspace (whole
    neighbour circle), at states spread over the measured window."""
    import dataclasses
    import torch
    from paper_2008_11578_amd import orca
    sc = scenarios.c3_crossing()
    params = dataclasses.replace(sc.params, cell_size=0.6)
    state = orca.State.from_arrays(sc)
    nxt = state.clone()
    fresh = state.clone()
    ws = orca.Workspace(state.n)
    checks = (10, 27, 28, 60, 109)
    for t in range(110):
        if t in checks:
            orca.step(state, params, orca.Workspace(state.n), out=fresh)
        orca.step(state, params, ws, out=nxt)
        if t in checks:
            torch.cuda.synchronize()
            for k in ("px", "py", "vx", "vy"):
                assert torch.equal(getattr(nxt, k), getattr(fresh, k)), (t, k)
        state, nxt = nxt, state


def test_step_deterministic_and_inplace():
    import torch
    from paper_2008_11578_amd import orca
    sc = scenarios.random_state(30000, 100.0, seed=4, n_vehicles=300)
    st = orca.State.from_arrays(sc)
    ws = orca.Workspace(st.n)
    a = orca.step(st, sc.params, ws)
    b = orca.step(st, sc.params, ws)
    torch.cuda.synchronize()
    for k in ("px", "py", "vx", "vy"):
        assert torch.equal(getattr(a, k), getattr(b, k)), k
    c = st.clone()
    orca.step(c, sc.params, ws, out=c)
    torch.cuda.synchronize()
    for k in ("px", "py", "vx", "vy"):
        assert torch.equal(getattr(a, k), getattr(c, k)), k


def test_step_independent_of_kept_neighbour_distances():
    """The workspace keeps each agent's K-th neighbour distance to narrow the
    next counting pass.  Stale values (a denser crowd, a sparser crowd, a
    different state of the same crowd) must change nothing: every output is
    bit-identical to a step on a fresh workspace."""
    import torch
    from paper_2008_11578_amd import orca
    sc = scenarios.random_state(30000, 100.0, seed=5, n_vehicles=300)
    st = orca.State.from_arrays(sc)
    fresh = orca.step(st, sc.params, orca.Workspace(st.n))
    for side in (40.0, 400.0, 100.0):  # too small, too large, similar distances
        other = scenarios.random_state(30000, side, seed=6, n_vehicles=300)
        ws = orca.Workspace(st.n)
        o = orca.State.from_arrays(other)
        for _ in range(2):
            orca.step(o, other.params, ws, out=o)
        got = orca.step(st, sc.params, ws)
        got2 = orca.step(st, sc.params, ws)  # now with its own distances
        torch.cuda.synchronize()
        for k in ("px", "py", "vx", "vy"):
            assert torch.equal(getattr(fresh, k), getattr(got, k)), (side, k)
            assert torch.equal(getattr(fresh, k), getattr(got2, k)), (side, k)


def test_step_edge_cases():
    p = scenarios.Params(dt=0.1, neighbor_dist=5.0, max_neighbors=10, pref_is_goal=0)
    # single agent: desired velocity clipped to the cap
    st = dict(px=np.float32([1.0]), py=np.float32([2.0]), vx=np.float32([0]), vy=np.float32([0]),
              pref_x=np.float32([3.0]), pref_y=np.float32([4.0]), radius=np.float32([0.3]),
              max_speed=np.float32([1.5]), cls=np.uint8([0]))
    g = gpu_step(st, p)
    np.testing.assert_allclose([g["vx"][0], g["vy"][0]], [0.9, 1.2], atol=1e-6)
    # overlapping pair and a symmetric squeeze
    st = dict(px=np.float32([0, 0.5, -0.5]), py=np.float32([0, 0, 0]), vx=np.zeros(3, np.float32),
              vy=np.zeros(3, np.float32), pref_x=np.zeros(3, np.float32),
              pref_y=np.float32([0.7, 0, 0]), radius=np.full(3, 0.3, np.float32),
              max_speed=np.full(3, 1.5, np.float32), cls=np.zeros(3, np.uint8))
    g = gpu_step(st, p)
    o = oracle.step(st, p)
    np.testing.assert_allclose(g["vx"], o["vx"], atol=1e-5)
    np.testing.assert_allclose(g["vy"], o["vy"], atol=1e-5)
    assert g["status"][0] == 1
    # all agents on one vertical line (zero-width bounding box) and coincident agents
    n = 300
    st = dict(px=np.full(n, 7.0, np.float32), py=np.linspace(0, 50, n).astype(np.float32),
              vx=np.zeros(n, np.float32), vy=np.zeros(n, np.float32),
              pref_x=np.full(n, 0.5, np.float32), pref_y=np.zeros(n, np.float32),
              radius=np.full(n, 0.3, np.float32), max_speed=np.full(n, 1.5, np.float32),
              cls=np.zeros(n, np.uint8))
    st["py"][10] = st["py"][11]
    rep, g, o = compare_step(st, p)
    _print("line", rep)
    # n = 0 is a no-op
    from paper_2008_11578_amd import orca
    import torch
    e = orca.State.from_arrays({k: np.zeros(0, np.uint8 if k == "cls" else np.float32)
                                for k in orca.STATE_FIELDS})
    orca.step(e, p, orca.Workspace(0))
    torch.cuda.synchronize()


def test_step_large_coordinates_and_small_workspace():
    import torch
    from paper_2008_11578_amd import orca
    sc = scenarios.uniform_square(4000, 80.0, seed=12)
    st = as_dict(sc)
    st = dict(st)
    st["px"] = (st["px"].astype(np.float64) + 5000.0).astype(np.float32)
    # a workspace with very few cells forces the device to enlarge the cells
    s = orca.State.from_arrays(st)
    ws = orca.Workspace(s.n, max_cells=16)
    stat = torch.zeros(s.n, dtype=torch.uint8, device="cuda")
    out = orca.step(s, sc.params, ws, status=stat)
    torch.cuda.synchronize()
    g = {k: getattr(out, k).cpu().numpy() for k in ("px", "py", "vx", "vy")}
    g["status"] = stat.cpu().numpy()
    rep, _, _ = compare_step(st, sc.params, gpu=g)
    _print("large coordinates, 16 cells", rep)
    nb, cn = orca.build_grid(s, sc.params, ws)
    onb, ocn = oracle.knn(st["px"], st["py"], sc.params.neighbor_dist, sc.params.max_neighbors)
    np.testing.assert_array_equal(nb.cpu().numpy(), onb)
