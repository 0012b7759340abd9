"""Seeded synthetic crowd scenarios (inputs only, no method arithmetic).

This module is the single source of inputs for both the GPU path and the
FP64 oracle.  It draws positions, goals, radii, speed caps and agent classes
with NumPy's PCG64 generator and returns them as FP32 structure-of-arrays in
caller order.  It contains none of the ORCA / linear-programming arithmetic.

The paper describes its workloads only in prose (Sec. 4: start and end
regions, spawn without overlap, goals on the opposite side, 2-way and 4-way
crossings, pedestrians and vehicles sharing one space, person-vehicle
responsibility 1/0).  The five recipes below are synthetic stand-ins with
those shapes; their exact sizes and parameters are stated with each function.

Agent classes: 0 = pedestrian, 1 = vehicle.  The responsibility table is
indexed ``f[class_of_self][class_of_other]`` (Sec. 3.1: person-person 1/2,
car-car 1/2, person-car 1, car-person 0).
"""
from __future__ import annotations

import dataclasses
import math
from typing import Dict, List, Optional

import numpy as np

PEDESTRIAN = 0
VEHICLE = 1

# Responsibility values used in the paper's experiments (Sec. 3.1, Sec. 4).
F_PAPER = ((0.5, 1.0), (0.0, 0.5))


@dataclasses.dataclass
class Params:
    """Per-scene simulation parameters (mirrors ``orca_params`` in orca.h)."""

    dt: float = 0.1
    time_horizon: float = 2.0
    neighbor_dist: float = 5.0
    cell_size: float = 0.0          # 0 selects the library default (= neighbor_dist)
    max_neighbors: int = 10
    pref_is_goal: int = 1           # 1: pref_x/pref_y hold goals; 0: they hold v_pref
    f: tuple = F_PAPER
    par_eps: float = 1e-5
    accel: tuple = (0.0, 0.0)      # acceleration cap per class [m/s^2]; 0 = none
    turn: tuple = (0.0, 0.0)       # turn-rate cap per class [rad/s]; 0 = none

    def as_dict(self) -> dict:
        return dataclasses.asdict(self)


@dataclasses.dataclass
class Scenario:
    """FP32 SoA agent state in caller order plus its parameters."""

    name: str
    params: Params
    px: np.ndarray
    py: np.ndarray
    vx: np.ndarray
    vy: np.ndarray
    pref_x: np.ndarray
    pref_y: np.ndarray
    radius: np.ndarray
    max_speed: np.ndarray
    cls: np.ndarray
    steps: int = 1
    # batched form: scene_off[S+1] (int32) and one Params per scene
    scene_off: Optional[np.ndarray] = None
    scene_params: Optional[List[Params]] = None
    # differentiable rollout: per-agent targets of the trajectory loss
    target_x: Optional[np.ndarray] = None
    target_y: Optional[np.ndarray] = None

    @property
    def n(self) -> int:
        return int(self.px.shape[0])

    def arrays(self) -> Dict[str, np.ndarray]:
        return {k: getattr(self, k) for k in
                ("px", "py", "vx", "vy", "pref_x", "pref_y", "radius",
                 "max_speed", "cls")}

    def copy(self) -> "Scenario":
        out = dataclasses.replace(self)
        for k, v in self.arrays().items():
            setattr(out, k, v.copy())
        return out


def _f32(a) -> np.ndarray:
    return np.ascontiguousarray(np.asarray(a, dtype=np.float64).astype(np.float32))


def _finish(name, params, px, py, gx, gy, radius, vmax, cls, steps, **extra):
    n = len(px)
    return Scenario(name=name, params=params, px=_f32(px), py=_f32(py),
                    vx=np.zeros(n, np.float32), vy=np.zeros(n, np.float32),
                    pref_x=_f32(gx), pref_y=_f32(gy), radius=_f32(radius),
                    max_speed=_f32(vmax), cls=np.ascontiguousarray(cls, dtype=np.uint8),
                    steps=steps, **extra)


def _perimeter_points(rng: np.random.Generator, count: int, side: float):
    """Uniform points on the boundary of the square [0, side]^2."""
    s = rng.uniform(0.0, 4.0 * side, size=count)
    edge = np.floor(s / side).astype(np.int64)
    t = s - edge * side
    x = np.where(edge == 0, t, np.where(edge == 1, side, np.where(edge == 2, side - t, 0.0)))
    y = np.where(edge == 0, 0.0, np.where(edge == 1, t, np.where(edge == 2, side, side - t)))
    return x, y


def uniform_square(n: int, side: float, seed: int, *, n_vehicles: int = 0,
                   params: Optional[Params] = None, steps: int = 1,
                   name: str = "uniform") -> Scenario:
    """Pedestrians (r 0.3 m, 1.5 m/s) and vehicles (r 1.5 m, 6 m/s) placed
    uniformly in [0, side]^2; pedestrian goals uniform in the square, vehicle
    goals uniform on its perimeter.  Vehicles are the last ``n_vehicles``
    agents."""
    rng = np.random.Generator(np.random.PCG64(seed))
    params = params or Params()
    n_ped = n - n_vehicles
    px = rng.uniform(0.0, side, size=n)
    py = rng.uniform(0.0, side, size=n)
    gx = rng.uniform(0.0, side, size=n)
    gy = rng.uniform(0.0, side, size=n)
    if n_vehicles:
        vx_, vy_ = _perimeter_points(rng, n_vehicles, side)
        gx[n_ped:] = vx_
        gy[n_ped:] = vy_
    radius = np.full(n, 0.3)
    vmax = np.full(n, 1.5)
    cls = np.zeros(n, np.uint8)
    radius[n_ped:] = 1.5
    vmax[n_ped:] = 6.0
    cls[n_ped:] = VEHICLE
    return _finish(name, params, px, py, gx, gy, radius, vmax, cls, steps)


def c1_plain(seed: int = 1) -> Scenario:
    """256 pedestrians in a 30 x 30 m square, goals in the same square;
    r 0.3 m, v_max 1.5 m/s, dt 0.1 s, tau 2 s, neighbour distance 5 m,
    at most 10 neighbours, 20 steps."""
    p = Params(dt=0.1, time_horizon=2.0, neighbor_dist=5.0, max_neighbors=10)
    return uniform_square(256, 30.0, seed, params=p, steps=20, name="c1_plain_256")


def c2_mixed(seed: int = 2) -> Scenario:
    """65,536 pedestrians + 1,024 vehicles uniform in 500 x 500 m; dt 0.05 s,
    tau 2 s, neighbour distance 5 m, at most 16 neighbours, 200 steps."""
    p = Params(dt=0.05, time_horizon=2.0, neighbor_dist=5.0, max_neighbors=16)
    return uniform_square(65536 + 1024, 500.0, seed, n_vehicles=1024, params=p,
                          steps=200, name="c2_mixed_66560")


def c2_vehicle_share(share: float, seed: int = 2) -> Scenario:
    """The mixed-crowd geometry (66,560 agents in 500 x 500 m, same
    parameters) with round(share * 66,560) of the agents vehicles."""
    n = 65536 + 1024
    nv = int(round(share * n))
    p = Params(dt=0.05, time_horizon=2.0, neighbor_dist=5.0, max_neighbors=16)
    return uniform_square(n, 500.0, seed, n_vehicles=nv, params=p, steps=200,
                          name=f"c2_vehicle_share_{share:g}")


def crossing(side_count: int, side: float, seed: int, *, jitter: float = 0.04,
             params: Optional[Params] = None, steps: int = 1,
             name: str = "crossing") -> Scenario:
    """Four-way crossing on a jittered square lattice.

    ``side_count``^2 pedestrians on a lattice of spacing side/side_count over
    [0, side]^2, each jittered by U(-jitter, +jitter) per axis.  The square is
    split by its diagonals into four groups (the triangle nearest each side);
    every agent's goal is its mirror image across the centre line parallel to
    its group's side, so the four flows cross everywhere."""
    rng = np.random.Generator(np.random.PCG64(seed))
    params = params or Params(neighbor_dist=3.0, max_neighbors=20)
    s = side / side_count
    idx = (np.arange(side_count) + 0.5) * s
    gx0, gy0 = np.meshgrid(idx, idx, indexing="xy")
    px = gx0.ravel() + rng.uniform(-jitter, jitter, size=side_count * side_count)
    py = gy0.ravel() + rng.uniform(-jitter, jitter, size=side_count * side_count)
    c = 0.5 * side
    horizontal = np.abs(px - c) > np.abs(py - c)   # left / right groups
    gx = np.where(horizontal, side - px, px)
    gy = np.where(horizontal, py, side - py)
    n = len(px)
    return _finish(name, params, px, py, gx, gy, np.full(n, 0.3), np.full(n, 1.5),
                   np.zeros(n, np.uint8), steps)


def head_on_pairs(pairs: int = 16, gap: float = 15.0, offset: float = 0.2,
                  spacing: float = 40.0) -> Scenario:
    """`pairs` isolated pedestrian-vehicle encounters: a pedestrian walking +x
    at 1.5 m/s and a vehicle driving -x at 6 m/s, `gap` metres apart with a
    lateral offset of `offset` (less than r_p + r_v, so without avoidance they
    collide).  Pairs are `spacing` metres apart, beyond each other's neighbour
    distance.  Preferred velocities equal the current ones (pref_is_goal = 0),
    so any change of velocity is avoidance."""
    k = np.arange(pairs, dtype=np.float64)
    px = np.stack([np.zeros(pairs), np.full(pairs, gap)], 1).ravel()
    py = np.stack([k * spacing, k * spacing + offset], 1).ravel()
    vx = np.tile([1.5, -6.0], pairs)
    n = 2 * pairs
    return Scenario(name="head_on_pairs", params=Params(dt=0.05, time_horizon=2.0,
                                                        neighbor_dist=10.0, max_neighbors=4,
                                                        pref_is_goal=0),
                    px=_f32(px), py=_f32(py), vx=_f32(vx), vy=np.zeros(n, np.float32),
                    pref_x=_f32(vx), pref_y=np.zeros(n, np.float32),
                    radius=_f32(np.tile([0.3, 1.5], pairs)),
                    max_speed=_f32(np.tile([1.5, 6.0], pairs)),
                    cls=np.tile(np.array([0, 1], np.uint8), pairs), steps=80)


def c3_crossing(seed: int = 3, side_count: int = 1024) -> Scenario:
    """1,048,576 pedestrians, four crossing flows in 700 x 700 m (about
    2.14 agents/m^2); r 0.3 m, v_max 1.5 m/s, dt 0.1 s, tau 2 s, neighbour
    distance 3 m, at most 20 neighbours, 100 steps."""
    p = Params(dt=0.1, time_horizon=2.0, neighbor_dist=3.0, max_neighbors=20)
    side = 700.0 * side_count / 1024.0
    return crossing(side_count, side, seed, params=p, steps=100,
                    name=f"c3_crossing_{side_count * side_count}")


def c4_batched(seed: int = 4, n_scenes: int = 512, lo: int = 64, hi: int = 65536) -> Scenario:
    """512 independent scenes with agent counts log-uniform in [64, 65,536],
    5% vehicles per scene, square side sized for 0.5 agents/m^2; per-scene
    parameters as the mixed workload (dt 0.05 s, tau 2 s, 5 m, 16 neighbours).
    Scenes are concatenated in caller order; ``scene_off`` delimits them."""
    rng = np.random.Generator(np.random.PCG64(seed))
    sizes = np.rint(np.exp(rng.uniform(math.log(lo), math.log(hi), size=n_scenes))).astype(np.int64)
    sub_seeds = rng.integers(0, 2**31 - 1, size=n_scenes)
    parts = []
    plist = []
    for s in range(n_scenes):
        n_s = int(sizes[s])
        n_veh = int(round(0.05 * n_s))
        side = math.sqrt(n_s / 0.5)
        p = Params(dt=0.05, time_horizon=2.0, neighbor_dist=5.0, max_neighbors=16)
        parts.append(uniform_square(n_s, side, int(sub_seeds[s]), n_vehicles=n_veh, params=p))
        plist.append(p)
    off = np.zeros(n_scenes + 1, np.int32)
    off[1:] = np.cumsum(sizes)
    cat = {k: np.concatenate([getattr(sc, k) for sc in parts]) for k in parts[0].arrays()}
    return Scenario(name=f"c4_batched_{n_scenes}x", params=plist[0], steps=100,
                    scene_off=off, scene_params=plist, **cat)


def c5_rollout(seed: int = 5, n: int = 16384, side: float = 240.0,
               speed: float = 1.4) -> Scenario:
    """Differentiable rollout: 16,384 pedestrians uniform in 240 x 240 m,
    v_pref = `speed` toward a uniform goal (held constant), targets of the
    loss drawn from an independent stream; v_max 1.5 m/s, dt 0.1 s, tau 2 s,
    5 m, 10 neighbours, 50 steps.  The desired speed sits below the cap: at
    |v_pref| = v_max the speed-disc projection has a kink in v_pref, which
    central differences would straddle."""
    rng = np.random.Generator(np.random.PCG64(seed))
    px = rng.uniform(0.0, side, size=n)
    py = rng.uniform(0.0, side, size=n)
    gx = rng.uniform(0.0, side, size=n)
    gy = rng.uniform(0.0, side, size=n)
    ang = np.arctan2(gy - py, gx - px)
    vpx = speed * np.cos(ang)
    vpy = speed * np.sin(ang)
    trng = np.random.Generator(np.random.PCG64(seed + 1000))
    tx = trng.uniform(0.0, side, size=n)
    ty = trng.uniform(0.0, side, size=n)
    p = Params(dt=0.1, time_horizon=2.0, neighbor_dist=5.0, max_neighbors=10, pref_is_goal=0)
    return _finish(f"c5_rollout_{n}", p, px, py, vpx, vpy, np.full(n, 0.3), np.full(n, 1.5),
                   np.zeros(n, np.uint8), 50, target_x=_f32(tx), target_y=_f32(ty))


def random_state(n: int, side: float, seed: int, *, n_vehicles: int = 0,
                 params: Optional[Params] = None, vel_scale: float = 1.0) -> Scenario:
    """Uniform positions with random current velocities (|v| up to
    ``vel_scale`` x v_max), used to test one step from a non-rest state."""
    sc = uniform_square(n, side, seed, n_vehicles=n_vehicles, params=params)
    rng = np.random.Generator(np.random.PCG64(seed + 7919))
    ang = rng.uniform(0.0, 2 * math.pi, size=n)
    mag = rng.uniform(0.0, vel_scale, size=n) * sc.max_speed.astype(np.float64)
    sc.vx = _f32(mag * np.cos(ang))
    sc.vy = _f32(mag * np.sin(ang))
    return sc


CONFIGS = {
    "c1": c1_plain,
    "c2": c2_mixed,
    "c3": c3_crossing,
    "c4": c4_batched,
    "c5": c5_rollout,
}
