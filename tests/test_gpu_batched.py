"""Batched form on the GPU: every scene of a batch must equal the single-scene
step on that scene alone, bit for bit (same kernels, same neighbour lists),
in both launch modes; the batch agrees with the FP64 oracle scene by scene;
graph replays equal eager steps."""
import dataclasses

import numpy as np
import pytest

import oracle
from paper_2008_11578_amd import scenarios

from parity import V_TOL, as_dict, compare_step

pytestmark = pytest.mark.gpu


def _batch(sizes, seed=0, vehicles=0.05, cell_size=0.0):
    parts, prm = [], []
    for s, n in enumerate(sizes):
        p = scenarios.Params(dt=0.05, neighbor_dist=5.0, max_neighbors=16 if s % 3 else 10,
                             cell_size=cell_size)
        side = max(np.sqrt(n / 0.5), 5.0)
        parts.append(scenarios.random_state(n, side, seed=seed + s, n_vehicles=int(vehicles * n),
                                            params=p))
        prm.append(p)
    off = np.zeros(len(parts) + 1, np.int32)
    off[1:] = np.cumsum([p.n for p in parts])
    cat = {k: np.concatenate([getattr(p, k) for p in parts]) for k in parts[0].arrays()}
    return parts, prm, off, cat


@pytest.mark.parametrize("mode", [0, 1])
def test_batched_equals_single_scene_steps(mode):
    import torch
    from paper_2008_11578_amd import orca
    sizes = [64, 1, 300, 2000, 77, 5000, 130, 0, 900]
    parts, prm, off, cat = _batch(sizes, seed=10)
    st = orca.State.from_arrays(cat)
    ws = orca.Workspace(st.n, n_scenes=len(sizes))
    b = orca.Batch(off, prm, mode=mode)
    status = torch.zeros(st.n, dtype=torch.uint8, device="cuda")
    out = orca.step_batched(st, b, ws, status=status)
    torch.cuda.synchronize()
    assert int(b.error.item()) == 0
    for s, part in enumerate(parts):
        if part.n == 0:
            continue
        sp = orca.State.from_arrays(part)
        st1 = torch.zeros(part.n, dtype=torch.uint8, device="cuda")
        o1 = orca.step(sp, prm[s], orca.Workspace(part.n), status=st1)
        torch.cuda.synchronize()
        a, z = off[s], off[s + 1]
        for k in ("px", "py", "vx", "vy"):
            assert torch.equal(getattr(out, k)[a:z], getattr(o1, k)), (s, k)
        assert torch.equal(status[a:z], st1), s


def _batch_result(out, status):
    g = {k: getattr(out, k).cpu().numpy() for k in ("px", "py", "vx", "vy")}
    g["status"] = status.cpu().numpy()
    return g


def _contract_per_scene(cat, off, prm, g, scenes, label, max_ill_frac=0.01):
    """The full parity contract (tests/parity.py) on the given scenes of a
    batch result g; the share of ill-conditioned agents is bounded over the
    scenes together (a scene of a few hundred agents can hold a few)."""
    n_ill = n_all = 0
    for s in scenes:
        a, z = int(off[s]), int(off[s + 1])
        if z == a:
            continue
        part = {k: v[a:z] for k, v in cat.items()}
        rep, _, _ = compare_step(part, prm[s], gpu={k: v[a:z] for k, v in g.items()},
                                 max_ill_frac=1.0)
        print(" ", label, "scene", int(s), rep, flush=True)
        n_ill += rep.get("n_ill", 0)
        n_all += rep["n"]
    assert n_ill <= max_ill_frac * max(n_all, 1), (n_ill, n_all)


def test_batched_matches_oracle_per_scene():
    import torch
    from paper_2008_11578_amd import orca
    sizes = [64, 500, 3000, 128, 1500]
    parts, prm, off, cat = _batch(sizes, seed=20)
    st = orca.State.from_arrays(cat)
    status = torch.zeros(st.n, dtype=torch.uint8, device="cuda")
    out = orca.step_batched(st, orca.Batch(off, prm), orca.Workspace(st.n, n_scenes=len(sizes)),
                            status=status)
    torch.cuda.synchronize()
    g = _batch_result(out, status)
    # the oracle's batched form equals its per-scene steps ...
    ob = oracle.step_batched(cat, off, prm)
    # ... and every scene of the GPU batch meets the contract agent by agent
    _contract_per_scene(cat, off, prm, g, range(len(sizes)), "batch of 5")
    for s in range(len(sizes)):
        a, z = int(off[s]), int(off[s + 1])
        o = oracle.step({k: v[a:z] for k, v in cat.items()}, prm[s])
        np.testing.assert_array_equal(ob["vx"][a:z], o["vx"])
        np.testing.assert_array_equal(ob["vy"][a:z], o["vy"])


def test_batched_c4_shape_runs_and_flags_nothing():
    import torch
    from paper_2008_11578_amd import orca
    sc = scenarios.c4_batched(n_scenes=64)
    st = orca.State.from_arrays(sc)
    b = orca.Batch(sc.scene_off, sc.scene_params)
    status = torch.zeros(st.n, dtype=torch.uint8, device="cuda")
    out = orca.step_batched(st, b, orca.Workspace(st.n, n_scenes=64), status=status)
    torch.cuda.synchronize()
    assert int(b.error.item()) == 0
    assert torch.isfinite(out.vx).all() and torch.isfinite(out.px).all()
    # three scenes (the first, a middle and the last) under the full contract
    _contract_per_scene(as_dict(sc), sc.scene_off, sc.scene_params, _batch_result(out, status),
                        (0, 31, 63), "c4 x64")


def _c4_full_check(sc, prm, st, g, label):
    """Every agent of a 512-scene batch result g (from state st) against the
    oracle's batched step; the full contract on every scene that holds an
    agent outside the tolerance, on the three largest scenes and on three
    others."""
    S = len(prm)
    cat = {k: v for k, v in st.items()}
    ob = oracle.step_batched(cat, sc.scene_off, prm)
    dv = np.hypot(g["vx"] - ob["vx"], g["vy"] - ob["vy"])
    print(" ", label, "oracle: max dv", float(dv.max()), "over tolerance",
          int(np.sum(dv > V_TOL)), flush=True)
    # agents outside the tolerance are rare, and each of them is put to the
    # contract below (ill-conditioned, and then holding a valid answer)
    assert np.mean(dv > V_TOL) < 1e-3
    sizes = np.diff(sc.scene_off)
    outside = np.searchsorted(sc.scene_off, np.nonzero(dv > V_TOL)[0], side="right") - 1
    sample = sorted(set(np.argsort(sizes)[-3:].tolist() + [0, S // 2, S - 1] + outside.tolist()))
    # the scenes start from random velocities with 5% vehicles, mostly on the
    # least-penetration fallback; a small scene can hold 1-2% agents whose
    # oracle answer FP32-sized perturbations move (for the single-scene
    # workloads the bound is 1%)
    _contract_per_scene(cat, sc.scene_off, prm, g, sample, label, max_ill_frac=0.02)


@pytest.mark.parametrize("block", [64, 256])
def test_batched_c4_full_in_measured_configuration(block):
    """All 512 scenes (5,559,168 agents) of the batched workload, in the launch
    configurations the autotuner chooses between at this size (cells of
    R_n / 2, the persistent form, capacity 16): every agent against the
    oracle, every scene bit for bit against its own plain step, and the full
    parity contract on the largest scenes and a few small ones."""
    import torch
    from paper_2008_11578_amd import orca
    sc = scenarios.c4_batched()
    S = len(sc.scene_params)
    prm = [dataclasses.replace(p, cell_size=0.5 * p.neighbor_dist) for p in sc.scene_params]
    st = orca.State.from_arrays(sc)
    b = orca.Batch(sc.scene_off, prm, mode=0, block=block, k_tile=16)
    status = torch.zeros(st.n, dtype=torch.uint8, device="cuda")
    out = orca.step_batched(st, b, orca.Workspace(st.n, n_scenes=S), status=status)
    torch.cuda.synchronize()
    assert int(b.error.item()) == 0
    g = {k: getattr(out, k).cpu().numpy() for k in ("px", "py", "vx", "vy")}
    g["status"] = status.cpu().numpy()
    print("c4 full", S, "scenes", st.n, "agents, block", block, flush=True)

    cat = as_dict(sc)

    # every scene equals its plain step
    for s in range(S):
        a, z = int(sc.scene_off[s]), int(sc.scene_off[s + 1])
        sp = orca.State(**{k: getattr(st, k)[a:z] for k in orca.STATE_FIELDS})
        st1 = torch.zeros(z - a, dtype=torch.uint8, device="cuda")
        o1 = orca.step(sp, prm[s], orca.Workspace(z - a), status=st1)
        torch.cuda.synchronize()
        for k in ("px", "py", "vx", "vy"):
            assert torch.equal(getattr(out, k)[a:z], getattr(o1, k)), (s, k)
        assert torch.equal(status[a:z], st1), s

    # every agent against the oracle, the full contract where it is needed
    _c4_full_check(sc, prm, cat, g, f"c4 full block {block}")


def test_batched_c4_graph_resync():
    """The 512-scene batch advanced by a captured 50-step graph in the
    measured launch configuration (cells of R_n / 2, persistent form, 64
    lanes, capacity 16, one workspace kept across steps): after 0, 50 and 100
    steps, one batched step from the graph's state with the kept workspace,
    every agent against the oracle (trajectories are never compared: FP32
    and FP64 separate chaotically, so both sides restart from the GPU's
    state)."""
    import torch
    from paper_2008_11578_amd import orca
    sc = scenarios.c4_batched()
    S = len(sc.scene_params)
    prm = [dataclasses.replace(p, cell_size=0.5 * p.neighbor_dist) for p in sc.scene_params]
    b = orca.Batch(sc.scene_off, prm, mode=0, block=64, k_tile=16)
    a = orca.State.from_arrays(sc)
    z = a.clone()
    ws = orca.Workspace(a.n, n_scenes=S)
    status = torch.zeros(a.n, dtype=torch.uint8, device="cuda")
    stream = torch.cuda.Stream()
    stream.wait_stream(torch.cuda.current_stream())
    graph = torch.cuda.CUDAGraph()
    with torch.cuda.stream(stream):
        with torch.cuda.graph(graph, stream=stream):
            x, y = a, z
            for _ in range(50):
                orca.step_batched(x, b, ws, out=y)
                x, y = y, x
    torch.cuda.synchronize()
    assert x is a  # an even number of steps ends where it started
    for done in (0, 50, 100):
        if done:
            graph.replay()
            torch.cuda.synchronize()
        snap = a.to_numpy()
        out = orca.step_batched(a, b, ws, out=z, status=status)
        torch.cuda.synchronize()
        assert int(b.error.item()) == 0
        _c4_full_check(sc, prm, snap, _batch_result(out, status), f"c4 graph after {done}")


def test_batched_kept_distances_change_no_result_full_size():
    """All 512 scenes stepped 30 times with a workspace kept across steps (as
    the measured graph does) equal, bit for bit, batched steps from the same
    states with a fresh workspace, at several of those steps."""
    import torch
    from paper_2008_11578_amd import orca
    sc = scenarios.c4_batched()
    S = len(sc.scene_params)
    prm = [dataclasses.replace(p, cell_size=0.5 * p.neighbor_dist) for p in sc.scene_params]
    b = orca.Batch(sc.scene_off, prm, mode=0, block=64, k_tile=16)
    state = orca.State.from_arrays(sc)
    nxt = state.clone()
    fresh = state.clone()
    ws = orca.Workspace(state.n, n_scenes=S)
    checks = (1, 5, 15, 29)
    for t in range(30):
        if t in checks:
            orca.step_batched(state, b, orca.Workspace(state.n, n_scenes=S), out=fresh)
        orca.step_batched(state, b, ws, out=nxt)
        if t in checks:
            torch.cuda.synchronize()
            assert int(b.error.item()) == 0
            for k in ("px", "py", "vx", "vy"):
                assert torch.equal(getattr(nxt, k), getattr(fresh, k)), (t, k)
        state, nxt = nxt, state


def test_batched_error_flag_on_bad_offsets():
    import torch
    from paper_2008_11578_amd import orca
    parts, prm, off, cat = _batch([100, 100, 100], seed=30)
    bad = off.copy()
    bad[1], bad[2] = 150, 120          # not ascending
    st = orca.State.from_arrays(cat)
    b = orca.Batch(bad, prm)
    orca.step_batched(st, b, orca.Workspace(st.n, n_scenes=3))
    torch.cuda.synchronize()
    assert int(b.error.item()) == 1
    prm2 = [dataclasses.replace(prm[0], dt=-1.0)] + prm[1:]
    b2 = orca.Batch(off, prm2)
    orca.step_batched(st, b2, orca.Workspace(st.n, n_scenes=3))
    torch.cuda.synchronize()
    assert int(b2.error.item()) == 1


def test_graph_replay_equals_eager():
    import torch
    from paper_2008_11578_amd import orca
    parts, prm, off, cat = _batch([400, 1200, 64, 3000], seed=40)
    n = int(off[-1])
    b = orca.Batch(off, prm)
    ws = orca.Workspace(n, n_scenes=len(prm))
    steps = 6
    # eager reference: `steps` ping-pong steps
    e0 = orca.State.from_arrays(cat)
    e1 = e0.clone()
    for t in range(steps):
        orca.step_batched(e0, b, ws, out=e1)
        e0, e1 = e1, e0
    torch.cuda.synchronize()
    ref = {k: getattr(e0, k).clone() for k in ("px", "py", "vx", "vy")}
    # captured: the same loop recorded once into a graph
    g0 = orca.State.from_arrays(cat)
    g1 = g0.clone()
    init = {k: getattr(g0, k).clone() for k in ("px", "py", "vx", "vy")}
    orca.step_batched(g0, b, ws, out=g1)       # warm-up outside capture
    torch.cuda.synchronize()
    for k in init:
        getattr(g0, k).copy_(init[k])
    stream = torch.cuda.Stream()
    stream.wait_stream(torch.cuda.current_stream())
    graph = torch.cuda.CUDAGraph()
    with torch.cuda.stream(stream):
        with torch.cuda.graph(graph, stream=stream):
            a, c = g0, g1
            for t in range(steps):
                orca.step_batched(a, b, ws, out=c)
                a, c = c, a
    torch.cuda.synchronize()
    final = a
    for rep in range(3):
        for k in init:
            getattr(g0, k).copy_(init[k])
        torch.cuda.synchronize()
        graph.replay()
        torch.cuda.synchronize()
        for k in ref:
            assert torch.equal(getattr(final, k), ref[k]), (rep, k)
        # eager work between replays
        orca.step_batched(e0, b, ws, out=e1)
        torch.cuda.synchronize()


def test_batched_per_scene_responsibility_matches_plain_steps():
    """Scenes that differ only in f (including sums other than 1) step exactly
    as the plain step does with each table."""
    import dataclasses
    import torch
    from paper_2008_11578_amd import orca, sweeps
    sc = scenarios.random_state(3000, 60.0, seed=21, n_vehicles=150)
    tables = [sweeps.table(0.5, 1.0, 0.0, 0.5), sweeps.table(0.5, 0.5, 0.5, 0.5),
              sweeps.table(0.25, 0.0, 0.0, 0.25), sweeps.table(1.0, 1.0, 1.0, 1.0)]
    S, n = len(tables), sc.n
    cat = {k: np.concatenate([getattr(sc, k)] * S) for k in sc.arrays()}
    off = np.arange(S + 1, dtype=np.int32) * n
    prm = [dataclasses.replace(sc.params, f=t) for t in tables]
    st = orca.State.from_arrays(cat)
    out = orca.step_batched(st, orca.Batch(off, prm), orca.Workspace(st.n, n_scenes=S))
    torch.cuda.synchronize()
    for s in range(S):
        o1 = orca.step(orca.State.from_arrays(sc), prm[s], orca.Workspace(n))
        torch.cuda.synchronize()
        for k in ("vx", "vy"):
            assert torch.equal(getattr(out, k)[s * n:(s + 1) * n], getattr(o1, k)), (s, k)
    # the tables really differ in effect
    assert not torch.equal(out.vx[:n], out.vx[n:2 * n])


def test_batched_per_scene_responsibility_matches_oracle():
    """Oracle parity for each table, sums other than 1 included."""
    import dataclasses
    from paper_2008_11578_amd import sweeps
    sc = scenarios.random_state(2000, 50.0, seed=22, n_vehicles=100)
    for t in (sweeps.table(0.25, 0.75, 0.75, 0.25), sweeps.table(1.0, 1.0, 1.0, 1.0)):
        compare_step(as_dict(sc), dataclasses.replace(sc.params, f=t))


def test_responsibility_sweep_head_on():
    """Isolated head-on pedestrian-vehicle encounters under four tables.
    f_{p|v} + f_{v|p} = 1 (either side takes all, or equal shares): no pair
    ever overlaps by more than rounding (with equal shares the discs end up
    touching, 1e-5 m deep).  Both zero: nobody turns, every velocity stays exactly as it
    was, and every pair collides.  With f_{p|v} = 0 the pedestrian's
    preferred velocity lies on its own half-plane's boundary, so it walks on
    unchanged."""
    from paper_2008_11578_amd import scenarios as scn, sweeps
    sc = scn.head_on_pairs()
    tabs = [sweeps.table(0.5, 0.0, 1.0, 0.5), sweeps.table(0.5, 0.5, 0.5, 0.5),
            sweeps.table(0.5, 0.0, 0.0, 0.5), sweeps.table(0.5, 1.0, 0.0, 0.5)]
    res = sweeps.run(tabs, sc, steps=sc.steps, reach=3.0)
    print([(r["f"], r["min_clearance"], r["worst_overlap_pairs"], r["mean_speed_ped"],
            r["mean_speed_veh"]) for r in res])
    vehicle_all, shared, nobody, ped_all = res
    for r in (vehicle_all, shared, ped_all):
        assert r["min_clearance"] > -1e-4
    assert vehicle_all["worst_overlap_pairs"] == 0
    assert nobody["worst_overlap_pairs"] == 16 and nobody["min_clearance"] < -1.0
    assert nobody["mean_speed_ped"] == 1.5 and nobody["mean_speed_veh"] == 6.0
    assert vehicle_all["mean_speed_ped"] == 1.5
    assert all(r["lp3_share"] >= 0 for r in res)


def test_responsibility_sweep_crowd_runs():
    """A mixed crowd under two tables: the sweep driver's statistics are
    well formed."""
    from paper_2008_11578_amd import scenarios as scn, sweeps
    sc = scn.uniform_square(1500, 45.0, seed=23, n_vehicles=75,
                            params=scn.Params(dt=0.05, neighbor_dist=5.0, max_neighbors=16))
    res = sweeps.run([sweeps.table(0.5, 1.0, 0.0, 0.5), sweeps.table(0.5, 0.0, 0.0, 0.5)], sc,
                     steps=20)
    for r in res:
        assert 0 <= r["lp3_share"] <= 1
        assert 0 <= r["final_overlap_pairs"] <= r["worst_overlap_pairs"]
        assert r["worst_overlap_agents"] <= sc.n and np.isfinite(r["min_clearance"])
        assert 0 < r["mean_speed_ped"] <= 1.5 + 1e-6 and 0 < r["mean_speed_veh"] <= 6 + 1e-5


@pytest.mark.parametrize("mode", [0, 1])
@pytest.mark.parametrize("block,k_tile", [(64, 0), (256, 0), (128, 24), (256, 32)])
def test_batched_block_and_tile_equal_single_scene_steps(mode, block, k_tile):
    """Lanes per workgroup and the compiled neighbour capacity are
    performance choices only: every scene still equals its plain step bit
    for bit."""
    import torch
    from paper_2008_11578_amd import orca
    sizes = [300, 1, 2000, 64, 900]
    parts, prm, off, cat = _batch(sizes, seed=33)
    st = orca.State.from_arrays(cat)
    b = orca.Batch(off, prm, mode=mode, block=block, k_tile=k_tile)
    out = orca.step_batched(st, b, orca.Workspace(st.n, n_scenes=len(sizes)))
    torch.cuda.synchronize()
    assert int(b.error.item()) == 0
    for s, p in enumerate(parts):
        if p.n == 0:
            continue
        o1 = orca.step(orca.State.from_arrays(p), prm[s], orca.Workspace(p.n))
        torch.cuda.synchronize()
        for k in ("vx", "vy", "px", "py"):
            assert torch.equal(getattr(out, k)[off[s]:off[s + 1]], getattr(o1, k)), (s, k)


def test_autotuner_picks_a_valid_configuration_and_caches_it(tmp_path, monkeypatch):
    from paper_2008_11578_amd import autotune, orca
    monkeypatch.setenv("ORCA_AUTOTUNE_CACHE", str(tmp_path / "tune.json"))
    sizes = [500, 3000, 64, 1200]
    parts, prm, off, cat = _batch(sizes, seed=44)
    st = orca.State.from_arrays(cat)
    ws = orca.Workspace(st.n, n_scenes=len(sizes))
    r = autotune.tune_batched(st, off, prm, ws, reps=1)
    assert r["factor"] in autotune.FACTORS and r["mode"] in autotune.MODES
    assert r["block"] in autotune.BLOCKS
    assert r["k_tile"] in autotune.K_TILES and r["k_tile"] >= max(p.max_neighbors for p in prm)
    assert not r["cached"] and len(r["timings"]) >= len(autotune.FACTORS) + 2
    r2 = autotune.tune_batched(st, off, prm, ws, reps=1)
    assert r2["cached"] and r2["block"] == r["block"] and r2["k_tile"] == r["k_tile"]


@pytest.mark.parametrize("mode", [0, 1])
@pytest.mark.parametrize("block", [64, 256])
def test_batched_lp3_cache_changes_no_result(mode, block):
    """The batched kernel caches LP3's sub-problem boundaries in the LDS
    columns of lanes of the same wavefront that run no LP3; a lane finds no
    such column when most of its wavefront runs LP3.  A jammed scene (most
    agents in LP3, so many lanes go without), a sparse one (few in LP3, every
    LP3 lane cached) and one in between must each equal the single-scene
    step, which never caches, bit for bit, and so must the status bytes."""
    import torch
    from paper_2008_11578_amd import orca
    p = scenarios.Params(dt=0.05, neighbor_dist=5.0, max_neighbors=16)
    parts = [scenarios.random_state(3000, np.sqrt(3000 / 3.0), seed=91, n_vehicles=150, params=p),
             scenarios.random_state(1500, np.sqrt(1500 / 0.05), seed=92, params=p),
             scenarios.random_state(2200, np.sqrt(2200 / 0.6), seed=93, n_vehicles=110, params=p)]
    off = np.zeros(len(parts) + 1, np.int32)
    off[1:] = np.cumsum([q.n for q in parts])
    cat = {k: np.concatenate([getattr(q, k) for q in parts]) for k in parts[0].arrays()}
    st = orca.State.from_arrays(cat)
    b = orca.Batch(off, [p] * len(parts), mode=mode, block=block, k_tile=16)
    status = torch.zeros(st.n, dtype=torch.uint8, device="cuda")
    out = orca.step_batched(st, b, orca.Workspace(st.n, n_scenes=len(parts)), status=status)
    torch.cuda.synchronize()
    assert int(b.error.item()) == 0
    share = [float(status[off[s]:off[s + 1]].float().mean().item()) for s in range(len(parts))]
    _share = ", ".join(f"{x:.3f}" for x in share)
    print(f"mode {mode} block {block}: LP3 share per scene {_share}", flush=True)
    assert share[0] > 0.6 and share[1] < 0.2
    for s, q in enumerate(parts):
        st1 = orca.State.from_arrays(q)
        status1 = torch.zeros(q.n, dtype=torch.uint8, device="cuda")
        o1 = orca.step(st1, p, orca.Workspace(q.n), status=status1)
        torch.cuda.synchronize()
        for k in ("vx", "vy", "px", "py"):
            assert torch.equal(getattr(out, k)[off[s]:off[s + 1]], getattr(o1, k)), (s, k)
        assert torch.equal(status[off[s]:off[s + 1]], status1), s
