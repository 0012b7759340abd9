"""Responsibility-matrix sweeps over batched scenes (the autonomous-vehicle
designer's question of Sec. 3.1 and Sec. 5: how much of the avoidance each
class should take on).

Every scene of the batch holds the same mixed crowd and differs only in its
responsibility table f (per-scene parameters of `orca_step_batched`), so one
batched launch per step advances all settings of the sweep together.  Each
scene then reports its overlapping pairs and agents and its smallest
clearance (`orca_overlap_stats`), the share of agents on the
least-penetration fallback, and the mean speed of each class.

Reading: the avoidance guarantee of a pair needs f_{A|B} + f_{B|A} = 1 when
the current relative velocity is outside the velocity obstacle and >= 1
when inside, so settings with a sum other than 1 are exactly where overlaps
are expected to appear.
"""
from __future__ import annotations

import dataclasses
from typing import Dict, List, Sequence, Tuple

import numpy as np
import torch

from . import orca, scenarios

FTable = Tuple[Tuple[float, float], Tuple[float, float]]


def table(f_pp: float, f_pv: float, f_vp: float, f_vv: float) -> FTable:
    """f[self][other] with 0 = pedestrian, 1 = vehicle."""
    return ((f_pp, f_pv), (f_vp, f_vv))


def run(tables: Sequence[FTable], scene: scenarios.Scenario, steps: int = 100,
        reach: float = 3.0) -> List[Dict[str, object]]:
    """Advances one copy of `scene` per responsibility table for `steps`
    batched steps; returns per-table statistics (worst overlap over the run,
    final overlap, smallest clearance, LP3 share, mean class speeds)."""
    S = len(tables)
    n = scene.n
    arrays = scene.arrays()
    cat = {k: np.concatenate([arrays[k]] * S) for k in arrays}
    off = np.arange(S + 1, dtype=np.int32) * n
    params = [dataclasses.replace(scene.params, f=t) for t in tables]
    st = orca.State.from_arrays(cat)
    nxt = st.clone()
    ws = orca.Workspace(st.n, n_scenes=S)
    batch = orca.Batch(off, params)
    status = torch.zeros(st.n, dtype=torch.uint8, device="cuda")
    ov_ws = orca.OverlapWorkspace(n)
    worst = np.zeros((S, 2))
    clear = np.full(S, np.inf)
    lp3 = np.zeros(S)
    for _ in range(steps):
        orca.step_batched(st, batch, ws, out=nxt, status=status)
        st, nxt = nxt, st
        for s in range(S):
            a, z = s * n, (s + 1) * n
            view = orca.State(**{k: getattr(st, k)[a:z] for k in orca.STATE_FIELDS})
            o = orca.overlap_stats(view, reach, ov_ws).cpu().numpy()
            worst[s] = np.maximum(worst[s], o[:2])
            clear[s] = min(clear[s], o[2])
        lp3 += status.view(S, n).float().mean(dim=1).cpu().numpy()
    if int(batch.error.item()) != 0:
        raise RuntimeError("batched step flagged an invalid scene")
    cls = torch.as_tensor(arrays["cls"]).cuda().bool()
    out = []
    for s, t in enumerate(tables):
        a, z = s * n, (s + 1) * n
        sp = torch.hypot(st.vx[a:z], st.vy[a:z])
        final = orca.overlap_stats(orca.State(**{k: getattr(st, k)[a:z]
                                                  for k in orca.STATE_FIELDS}),
                                   reach, ov_ws).cpu().numpy()
        out.append({"f": t, "pair_sums": (t[0][1] + t[1][0], 2 * t[0][0], 2 * t[1][1]),
                    "worst_overlap_pairs": int(worst[s, 0]),
                    "worst_overlap_agents": int(worst[s, 1]),
                    "final_overlap_pairs": int(final[0]),
                    "min_clearance": float(clear[s]),
                    "lp3_share": float(lp3[s] / max(steps, 1)),
                    "mean_speed_ped": float(sp[~cls].mean().item()) if (~cls).any() else None,
                    "mean_speed_veh": float(sp[cls].mean().item()) if cls.any() else None})
    return out
