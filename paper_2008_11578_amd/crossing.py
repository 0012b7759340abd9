"""Crossing experiments with spawning and removal (Sec. 4, first experiment).

Groups of pedestrians (and optionally vehicles) enter in start regions at
points that stay clear of everyone for `t_clear` seconds, walk to a goal in
the matching end region and leave once they reach it; the run ends when
every group has spawned its quota and everyone has left (or at `max_steps`).
Two-way: a left and a right group cross each other; four-way: plus a bottom
and a top group.  Each step records the population, the share of agents on
the least-penetration fallback, the overlapping pairs and agents, and the
smallest clearance (`orca_overlap_stats`), and the arrivals.

Random spawn proposals are drawn on the host from a seeded generator and
passed to `orca_spawn` as candidates; everything else runs on the device.
"""
from __future__ import annotations

import dataclasses
from typing import Dict, List, Optional

import numpy as np
import torch

from . import orca
from .scenarios import Params

STATE_FIELDS = orca.STATE_FIELDS


@dataclasses.dataclass
class CrossingConfig:
    kind: str = "4way"            # "2way" or "4way"
    per_group: int = 2500         # agents each group spawns in total
    side: float = 100.0           # square arena [0, side]^2
    strip: float = 10.0           # depth of the start and end regions
    proposals: int = 64           # spawn candidates per group per step
    t_clear: float = 1.0          # spawn clearance window [s]
    vehicle_share: float = 0.0    # share of vehicles among the spawned agents
    max_steps: int = 2000
    seed: int = 0
    params: Params = dataclasses.field(default_factory=lambda: Params(
        dt=0.1, time_horizon=2.0, neighbor_dist=5.0, max_neighbors=10, pref_is_goal=1))


def _regions(cfg: CrossingConfig):
    """(start box, end box) per group; boxes are (x0, y0, x1, y1)."""
    s, w = cfg.side, cfg.strip
    left, right = (0.0, 0.0, w, s), (s - w, 0.0, s, s)
    bottom, top = (0.0, 0.0, s, w), (0.0, s - w, s, s)
    groups = [(left, right), (right, left)]
    if cfg.kind == "4way":
        groups += [(bottom, top), (top, bottom)]
    elif cfg.kind != "2way":
        raise ValueError("kind must be '2way' or '4way'")
    return groups


def _proposals(rng, cfg: CrossingConfig, start, end, m):
    x = rng.uniform(start[0], start[2], m)
    y = rng.uniform(start[1], start[3], m)
    gx = rng.uniform(end[0], end[2], m)
    gy = rng.uniform(end[1], end[3], m)
    veh = rng.random(m) < cfg.vehicle_share
    return dict(px=x.astype(np.float32), py=y.astype(np.float32), vx=np.zeros(m, np.float32),
                vy=np.zeros(m, np.float32), pref_x=gx.astype(np.float32),
                pref_y=gy.astype(np.float32),
                radius=np.where(veh, 1.5, 0.3).astype(np.float32),
                max_speed=np.where(veh, 6.0, 1.5).astype(np.float32),
                cls=veh.astype(np.uint8))


def _buffers(cap: int, device="cuda") -> orca.State:
    return orca.State(**{k: torch.zeros(cap, dtype=torch.uint8 if k == "cls" else torch.float32,
                                        device=device) for k in STATE_FIELDS})


def _view(st: orca.State, n: int) -> orca.State:
    return orca.State(**{k: getattr(st, k)[:n] for k in STATE_FIELDS})


def run(cfg: CrossingConfig, record: bool = True) -> Dict[str, object]:
    """Runs one crossing experiment; returns totals and (with record) the
    per-step statistics."""
    rng = np.random.default_rng(cfg.seed)
    groups = _regions(cfg)
    G = len(groups)
    cap = G * cfg.per_group
    a, b = _buffers(cap), _buffers(cap)
    status = torch.zeros(cap, dtype=torch.uint8, device="cuda")
    n_cand_max = G * cfg.proposals
    life_ws = orca.LifecycleWorkspace(cap, n_cand_max)
    step_ws = orca.Workspace(cap)
    ov_ws = orca.OverlapWorkspace(cap)
    reach = max(cfg.params.neighbor_dist, 3.0)
    quota = [cfg.per_group] * G
    n = 0
    spawned = arrived = 0
    rows: List[dict] = []
    lp3_steps = 0.0
    agent_steps = 0
    pending = None  # (accepted flags, owners) of the last spawn, read with the step's results
    for t in range(cfg.max_steps):
        # spawn: every group still owing agents proposes candidates
        props, owner = [], []
        for g, (start, end) in enumerate(groups):
            if quota[g] > 0:
                m = min(cfg.proposals, quota[g])
                props.append(_proposals(rng, cfg, start, end, m))
                owner.append(np.full(m, g))
        if props:
            cand_np = {k: np.concatenate([p[k] for p in props]) for k in STATE_FIELDS}
            cand = orca.State.from_arrays(cand_np)
            acc = torch.empty(cand.n, dtype=torch.uint8, device="cuda")
            tot = orca.spawn(a, n, cand, cfg.t_clear, life_ws, accepted=acc)
            n = int(tot.item())  # the one synchronisation before the step
            pending = (acc, np.concatenate(owner))
        else:
            pending = None
        if n == 0 and not any(q > 0 for q in quota):
            break
        # one ORCA step of everyone present, in place, then the statistics,
        # the removal and the spawn decisions, all read back in one copy
        cur = _view(a, n)
        parts = []
        if n > 0:
            orca.step(cur, cfg.params, step_ws, out=cur, status=status[:n])
            parts.append(orca.overlap_stats(cur, reach, ov_ws))
            parts.append(status[:n].sum(dtype=torch.float64).reshape(1))
            parts.append(orca.remove_arrived(cur, _view(b, n), life_ws).to(torch.float64))
        if pending is not None:
            parts.append(pending[0].to(torch.float64))
        packed = torch.cat(parts).cpu().numpy() if parts else np.zeros(0)
        if n > 0:
            stats, lp3_n, left = packed[:3], float(packed[3]), int(packed[4])
            lp3 = lp3_n / n
            lp3_steps += lp3_n
            agent_steps += n
            rest = packed[5:]
        else:
            stats = np.array([0.0, 0.0, np.inf])
            lp3, left = 0.0, 0
            rest = packed
        if pending is not None:
            acc_h = rest.astype(bool)
            own = pending[1]
            for g in range(G):
                quota[g] -= int(acc_h[own == g].sum())
            spawned += int(acc_h.sum())
        arrived += n - left
        a, b = b, a
        if record:
            rows.append({"step": t, "agents": n, "arrived": n - left, "lp3_share": lp3,
                         "overlap_pairs": int(stats[0]), "overlap_agents": int(stats[1]),
                         "min_clearance": float(stats[2])})
        n = left
        if n == 0 and not any(q > 0 for q in quota):
            break
    return {"kind": cfg.kind, "groups": G, "per_group": cfg.per_group, "spawned": spawned,
            "arrived": arrived, "remaining": n, "steps": len(rows) if record else t + 1,
            "agent_steps": agent_steps,
            "lp3_share": lp3_steps / max(agent_steps, 1),
            "max_overlap_pairs": max((r["overlap_pairs"] for r in rows), default=0),
            "min_clearance": min((r["min_clearance"] for r in rows), default=float("inf")),
            "rows": rows if record else None}
