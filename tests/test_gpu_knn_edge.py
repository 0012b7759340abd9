"""Neighbour selection at the edge of the counted circle, on the GPU.

Candidates whose FP64 squared distance lies a few 1e-8 (relative) below
R_n^2 -- so that it rounds to R_n^2 in FP32 -- are the ones whose fixed-point
sort key sits at its top value.  Crowds are built around agents with one or
several such candidates, both with fewer than k agents in range (the sorted
set is every candidate) and with the k-th neighbour among them (the last
histogram bin decides), and the lists must equal the oracle's bit for bit:
from orca_build_grid, and from the step itself (orca_step_nbr) on a fresh and
on a kept workspace.  The CPU side of this is tests/test_sort_key.py.
"""
import numpy as np
import pytest

import oracle
from paper_2008_11578_amd import scenarios

from parity import compare_step

pytestmark = pytest.mark.gpu


def boundary_point(xi, yi, rn, angle, rel=5e-8):
    """An FP32 point whose FP64 key to the FP32 point (xi, yi) lies in
    [rn^2 (1 - rel), rn^2) and rounds to FP32(rn^2)."""
    xi, yi = np.float32(xi), np.float32(yi)
    r2 = np.float64(np.float32(rn)) ** 2
    c = np.float32(xi + rn * np.cos(angle))
    d = np.float32(yi + rn * np.sin(angle))
    k = np.arange(-2500, 2501)
    X = (np.float64(c) + k * np.float64(np.spacing(c))).astype(np.float32)
    Y = (np.float64(d) + k * np.float64(np.spacing(d))).astype(np.float32)
    dx = X.astype(np.float64) - np.float64(xi)
    dy = Y.astype(np.float64) - np.float64(yi)
    key = dx[:, None] * dx[:, None] + dy[None, :] * dy[None, :]
    ok = (key < r2) & (key >= r2 * (1 - rel)) & (key.astype(np.float32) == np.float32(r2))
    a, b = np.nonzero(ok)
    assert a.size, (xi, yi, rn, angle)
    j = np.argmin(np.abs(a - 2500) + np.abs(b - 2500))
    return X[a[j]], Y[b[j]]


def edge_crowd(rn, n_edge, n_near, seed):
    """Agents 0 and 1 each with n_edge candidates on the edge of their
    circle and n_near well inside it, among 400 agents elsewhere."""
    rng = np.random.default_rng(seed)
    px, py = [], []
    for cx, cy in ((10.0, 10.0), (31.0, 12.0)):
        px.append(cx)
        py.append(cy)
    for a, (cx, cy) in enumerate(((10.0, 10.0), (31.0, 12.0))):
        for t in range(n_edge):
            x, y = boundary_point(cx, cy, rn, 0.4 + 2 * np.pi * t / n_edge + 0.1 * a)
            px.append(x)
            py.append(y)
        for t in range(n_near):
            ang = rng.uniform(0, 2 * np.pi)
            r = rng.uniform(0.7, 0.6 * rn)
            px.append(cx + r * np.cos(ang))
            py.append(cy + r * np.sin(ang))
    m = 400
    px += list(rng.uniform(0.0, 60.0, m))
    py += list(rng.uniform(30.0, 60.0, m))
    n = len(px)
    perm = rng.permutation(n)  # caller order unrelated to the construction
    st = {"px": np.float32(px)[perm], "py": np.float32(py)[perm]}
    st["vx"] = rng.uniform(-1, 1, n).astype(np.float32)
    st["vy"] = rng.uniform(-1, 1, n).astype(np.float32)
    st["pref_x"] = rng.uniform(0, 60, n).astype(np.float32)
    st["pref_y"] = rng.uniform(0, 60, n).astype(np.float32)
    st["radius"] = np.full(n, 0.25, np.float32)
    st["max_speed"] = np.full(n, 1.5, np.float32)
    st["cls"] = np.zeros(n, np.uint8)
    return st, np.argsort(perm)[:2]


CASES = [  # (R_n, k, edge candidates, inner candidates)
    # one edge candidate and the k-th neighbour in the last bin: its key
    # alone at the top of the fixed-point range
    (3.0, 10, 1, 9),
    (5.0, 4, 1, 3),
    (5.0, 20, 1, 10),
    # one edge candidate and fewer than k in range: every candidate is sorted
    (3.0, 16, 1, 3),
    (3.0, 1, 1, 0),
    # several edge candidates, equal at the top of the range: exact ties of
    # the fixed-point key, resolved by the FP64 keys and the indices
    (3.0, 10, 8, 3),
    (5.0, 20, 9, 5),
]


@pytest.mark.parametrize("rn,k,n_edge,n_near", CASES)
def test_edge_candidates_bit_exact(rn, k, n_edge, n_near):
    import torch
    from paper_2008_11578_amd import orca
    st, centres = edge_crowd(rn, n_edge, n_near, seed=int(rn * 10 + k))
    p = scenarios.Params(dt=0.1, neighbor_dist=rn, max_neighbors=k, pref_is_goal=1)
    print("edge case", rn, k, n_edge, n_near, "agents", st["px"].size, flush=True)
    onb, ocn = oracle.knn(st["px"], st["py"], rn, k)
    # the constructed agents do see their edge candidates
    assert (ocn[centres] == min(k, n_edge + n_near)).all()
    s = orca.State.from_arrays(st)
    ws = orca.Workspace(s.n)
    nb, cn = orca.build_grid(s, p, ws)
    torch.cuda.synchronize()
    np.testing.assert_array_equal(cn.cpu().numpy(), ocn)
    np.testing.assert_array_equal(nb.cpu().numpy(), onb)
    # the step's own lists, on a fresh workspace and then on the kept one
    ws2 = orca.Workspace(s.n)
    cur = s
    for t in range(3):
        snap = cur.to_numpy()
        nxt, nb2, cn2 = orca.step_nbr(cur, p, ws2)
        torch.cuda.synchronize()
        onb2, ocn2 = oracle.knn(snap["px"], snap["py"], rn, k)
        np.testing.assert_array_equal(cn2.cpu().numpy(), ocn2)
        np.testing.assert_array_equal(nb2.cpu().numpy(), onb2)
        cur = nxt
    rep, _, _ = compare_step(st, p)
    print("  step", rep, flush=True)


@pytest.mark.parametrize("n", [32768, 32769])
def test_lists_on_both_sides_of_the_fused_grid_setup(n):
    """Crowds of up to 32,768 agents (at most 128 partial bounding boxes)
    form the grid geometry inside the counting kernel; one agent more takes
    the separate setup kernel.  Both give the oracle's neighbour lists bit
    for bit, from orca_build_grid and from the step's own selection."""
    import torch
    from paper_2008_11578_amd import orca
    sc = scenarios.random_state(n, float(np.sqrt(n / 0.8)), seed=n % 97,
                                params=scenarios.Params(dt=0.1, neighbor_dist=3.0,
                                                        max_neighbors=12))
    st = {k: getattr(sc, k) for k in sc.arrays()}
    p = sc.params
    onb, ocn = oracle.knn(st["px"], st["py"], p.neighbor_dist, p.max_neighbors)
    s = orca.State.from_arrays(st)
    nb, cn = orca.build_grid(s, p, orca.Workspace(s.n))
    _, nb2, cn2 = orca.step_nbr(s, p, orca.Workspace(s.n))
    torch.cuda.synchronize()
    for a, b in ((cn, ocn), (nb, onb), (cn2, ocn), (nb2, onb)):
        np.testing.assert_array_equal(a.cpu().numpy(), b)
