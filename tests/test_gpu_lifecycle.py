"""GPU lifecycle entry points (orca_remove_arrived, orca_spawn) against the
oracle: decisions, counts and the written agents bit for bit."""
import numpy as np
import pytest

import oracle

pytestmark = pytest.mark.gpu

F32 = np.float32
FIELDS = ("px", "py", "vx", "vy", "pref_x", "pref_y", "radius", "max_speed", "cls")


def _crowd(rng, n, side, veh=0.05):
    v = rng.random(n) < veh
    return dict(px=rng.uniform(0, side, n).astype(F32), py=rng.uniform(0, side, n).astype(F32),
                vx=rng.normal(0, 1, n).astype(F32), vy=rng.normal(0, 1, n).astype(F32),
                pref_x=rng.uniform(0, side, n).astype(F32),
                pref_y=rng.uniform(0, side, n).astype(F32),
                radius=np.where(v, 1.5, 0.3).astype(F32),
                max_speed=np.where(v, 6.0, 1.5).astype(F32), cls=v.astype(np.uint8))


def _state(arrays, cap=None):
    import torch
    from paper_2008_11578_amd import orca
    n = len(arrays["px"])
    cap = n if cap is None else cap
    kw = {}
    for k in FIELDS:
        t = torch.zeros(cap, dtype=torch.uint8 if k == "cls" else torch.float32, device="cuda")
        if n:
            t[:n] = torch.as_tensor(arrays[k]).cuda()
        kw[k] = t
    return orca.State(**kw)


@pytest.mark.parametrize("n", [0, 1, 257, 100_000])
def test_remove_arrived_matches_oracle(n):
    import torch
    from paper_2008_11578_amd import orca
    rng = np.random.default_rng(n)
    a = _crowd(rng, n, 200.0)
    near = rng.random(n) < 0.3
    a["pref_x"] = np.where(near, a["px"] + rng.uniform(-0.4, 0.4, n), a["pref_x"]).astype(F32)
    a["pref_y"] = np.where(near, a["py"], a["pref_y"]).astype(F32)
    if n > 2:
        # the boundary |g - p| = r exactly (3-4-5 in binary values) and one ulp inside
        a["px"][:2] = 0.0
        a["py"][:2] = 0.0
        a["pref_x"][:2] = 0.75
        a["pref_y"][:2] = 1.0
        a["radius"][0] = F32(1.25)
        a["radius"][1] = np.nextafter(F32(1.25), F32(0))
    st = _state(a)
    out = _state({k: v[:0] for k, v in a.items()}, cap=max(n, 1))
    o2n = torch.empty(n, dtype=torch.int32, device="cuda")
    ws = orca.LifecycleWorkspace(n)
    cnt = orca.remove_arrived(st, out, ws, old_to_new=o2n if n else None)
    torch.cuda.synchronize()
    ref = oracle.remove_arrived(a)
    m = int(cnt.item())
    assert m == ref["px"].shape[0]
    for k in FIELDS:
        np.testing.assert_array_equal(getattr(out, k)[:m].cpu().numpy(), ref[k])
    if n:
        np.testing.assert_array_equal(o2n.cpu().numpy(), ref["old_to_new"])
    if n > 2:
        assert ref["old_to_new"][0] == -1 and ref["old_to_new"][1] == 0


def _spawn_case(n, nc, side, t_clear, seed, cand_side=None):
    import torch
    from paper_2008_11578_amd import orca
    rng = np.random.default_rng(seed)
    a = _crowd(rng, n, side)
    c = _crowd(rng, nc, cand_side if cand_side is not None else side, veh=0.1)
    c["vx"][:] = 0
    c["vy"][:] = 0
    st = _state(a, cap=n + nc)
    cand = _state(c)
    ws = orca.LifecycleWorkspace(n, nc)
    acc = torch.empty(nc, dtype=torch.uint8, device="cuda")
    tot = orca.spawn(st, n, cand, t_clear, ws, accepted=acc if nc else None)
    torch.cuda.synchronize()
    ref = oracle.spawn(a, c, t_clear)
    total = int(tot.item())
    assert total == n + int(ref.sum())
    if nc:
        np.testing.assert_array_equal(acc.cpu().numpy(), ref)
    keep = ref.astype(bool)
    for k in FIELDS:
        got = getattr(st, k).cpu().numpy()
        np.testing.assert_array_equal(got[:n], a[k])
        np.testing.assert_array_equal(got[n:total], c[k][keep])
    return ref


@pytest.mark.parametrize("n,nc,side", [(5000, 3000, 120.0), (0, 500, 40.0), (2000, 0, 40.0),
                                       (1, 1, 5.0), (20_000, 16384, 600.0)])
def test_spawn_matches_oracle(n, nc, side):
    ref = _spawn_case(n, nc, side, 0.5, seed=n + nc)
    if nc > 10:
        assert 0 < ref.sum() < nc


def test_spawn_crowded_candidates_overflow_lists():
    """Candidates packed into a small square: most conflict with more earlier
    candidates than the per-candidate list holds, so the exhaustive path of
    the decision rounds runs."""
    ref = _spawn_case(200, 3000, 60.0, 0.5, seed=11, cand_side=6.0)
    assert 0 < ref.sum() < 100


def test_spawn_line_closed_form():
    """Equal candidates on a line at spacing D/3: every third one enters."""
    import torch
    from paper_2008_11578_amd import orca
    nc = 300
    c = dict(px=(np.arange(nc) * 0.5).astype(F32), py=np.zeros(nc, F32), vx=np.zeros(nc, F32),
             vy=np.zeros(nc, F32), pref_x=np.zeros(nc, F32), pref_y=np.zeros(nc, F32),
             radius=np.full(nc, 0.25, F32), max_speed=np.ones(nc, F32),
             cls=np.zeros(nc, np.uint8))
    st = _state({k: v[:0] for k, v in c.items()}, cap=nc)
    ws = orca.LifecycleWorkspace(0, nc)
    acc = torch.empty(nc, dtype=torch.uint8, device="cuda")
    tot = orca.spawn(st, 0, _state(c), 0.5, ws, accepted=acc)
    torch.cuda.synchronize()
    np.testing.assert_array_equal(np.nonzero(acc.cpu().numpy())[0], np.arange(0, nc, 3))
    assert int(tot.item()) == 100


@pytest.mark.parametrize("n,side", [(0, 10.0), (2, 1.0), (3000, 30.0), (50_000, 200.0)])
def test_overlap_stats_matches_oracle(n, side):
    import torch
    from paper_2008_11578_amd import orca
    rng = np.random.default_rng(n + 7)
    a = _crowd(rng, n, side)
    st = _state(a)
    ws = orca.OverlapWorkspace(n)
    out = orca.overlap_stats(st, 3.0, ws)
    torch.cuda.synchronize()
    got = out.cpu().numpy()
    if n > 5000:
        # brute force on a slice keeps the oracle fast; the GPU runs on the slice too
        a = {k: v[:5000] for k, v in a.items()}
        st = _state(a)
        got = orca.overlap_stats(st, 3.0, orca.OverlapWorkspace(5000)).cpu().numpy()
    ref = oracle.overlap_stats(a, 3.0)
    assert int(got[0]) == ref["pairs"] and int(got[1]) == ref["agents"]
    if np.isinf(ref["min_clearance"]):
        assert np.isinf(got[2])
    else:
        assert abs(got[2] - ref["min_clearance"]) <= 1e-12
    if n >= 3000:
        assert ref["pairs"] > 0


@pytest.mark.parametrize("kind", ["2way", "4way"])
def test_crossing_run_conserves_agents(kind):
    """A small crossing with spawning and removal runs to the end: every
    group spawns its quota, everyone who entered leaves at the goal, and the
    per-step population always equals spawned minus arrived."""
    from paper_2008_11578_amd import crossing
    cfg = crossing.CrossingConfig(kind=kind, per_group=120, side=30.0, strip=5.0, proposals=16,
                                  t_clear=0.5, max_steps=1500, seed=3)
    r = crossing.run(cfg)
    G = 2 if kind == "2way" else 4
    assert r["spawned"] == G * 120
    assert r["arrived"] == r["spawned"] and r["remaining"] == 0
    for row in r["rows"]:
        assert row["agents"] >= row["arrived"] >= 0
    assert sum(row["arrived"] for row in r["rows"]) == r["arrived"]
    print(kind, r["steps"], "steps; lp3 share", round(r["lp3_share"], 4), "max overlap pairs",
          r["max_overlap_pairs"], "min clearance", r["min_clearance"])


def test_extensions_full_size_measured_configuration():
    """The three calls as the throughput measurement makes them on the
    1,048,576-agent dense crossing: removal with one agent in ten on its goal,
    16,384 spawn candidates uniform over the 700 m square with a 1 s window,
    and the overlap statistics within 1 m; decisions, counts and written
    agents against the oracle, bit for bit."""
    import torch
    from paper_2008_11578_amd import orca, scenarios
    sc = scenarios.c3_crossing()
    n = sc.n
    rng = np.random.default_rng(17)
    arr = dict(sc.arrays())
    done = rng.random(n) < 0.1
    arr["pref_x"] = np.where(done, arr["px"], arr["pref_x"]).astype(F32)
    arr["pref_y"] = np.where(done, arr["py"], arr["pref_y"]).astype(F32)
    st = orca.State.from_arrays(arr)
    out = st.clone()
    o2n = torch.empty(n, dtype=torch.int32, device="cuda")
    lws = orca.LifecycleWorkspace(n, orca.SPAWN_MAX)
    kept = int(orca.remove_arrived(st, out, lws, old_to_new=o2n).item())
    ref = oracle.remove_arrived(arr)
    print("remove: kept", kept, "of", n, flush=True)
    assert kept == ref["px"].shape[0]
    for k in FIELDS:
        np.testing.assert_array_equal(getattr(out, k)[:kept].cpu().numpy(), ref[k])
    np.testing.assert_array_equal(o2n.cpu().numpy(), ref["old_to_new"])

    nc = orca.SPAWN_MAX
    side = 700.0
    cand = {k: np.zeros(nc, F32) for k in FIELDS if k != "cls"}
    cand["px"] = rng.uniform(0, side, nc).astype(F32)
    cand["py"] = rng.uniform(0, side, nc).astype(F32)
    cand["pref_x"] = rng.uniform(0, side, nc).astype(F32)
    cand["pref_y"] = rng.uniform(0, side, nc).astype(F32)
    cand["radius"] = np.full(nc, 0.3, F32)
    cand["max_speed"] = np.full(nc, 1.5, F32)
    cand["cls"] = np.zeros(nc, np.uint8)
    big = orca.State(**{k: torch.cat([getattr(st, k), torch.zeros(nc, dtype=getattr(st, k).dtype,
                                                                  device="cuda")])
                        for k in orca.STATE_FIELDS})
    acc = torch.empty(nc, dtype=torch.uint8, device="cuda")
    tot = int(orca.spawn(big, n, orca.State.from_arrays(cand), 1.0, lws, accepted=acc).item())
    ref_acc = oracle.spawn(arr, cand, 1.0)
    print("spawn: accepted", tot - n, "of", nc, flush=True)
    np.testing.assert_array_equal(acc.cpu().numpy(), ref_acc)
    assert tot == n + int(ref_acc.sum())
    keep = ref_acc.astype(bool)
    for k in FIELDS:
        np.testing.assert_array_equal(getattr(big, k)[n:tot].cpu().numpy(), cand[k][keep])

    # as measured, and with radii grown by 1.6 so that many pairs overlap
    grown = dict(arr)
    grown["radius"] = (arr["radius"] * F32(1.6)).astype(F32)
    for a in (arr, grown):
        got = orca.overlap_stats(orca.State.from_arrays(a), 1.0,
                                 orca.OverlapWorkspace(n)).cpu().numpy()
        ref = oracle.overlap_stats_tree(a, 1.0)
        print("overlap:", got.tolist(), ref, flush=True)
        assert int(got[0]) == ref["pairs"] and int(got[1]) == ref["agents"]
        assert abs(got[2] - ref["min_clearance"]) <= 1e-12
    assert ref["pairs"] > 0
