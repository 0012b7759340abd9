#!/usr/bin/env python3
"""Throughput of the ORCA step on one MI355X.

Workload: the dense four-way crossing, 1,048,576 pedestrians on a jittered
lattice over 700 m x 700 m (about 2.14 agents/m^2), neighbour distance 3 m,
at most 20 neighbours, dt 0.1 s, tau 2 s; synthetic, seeded.  One step is
the whole path: grid build, exact k-nearest neighbours, ORCA half-planes,
one LP per agent with the least-penetration fallback, and the update.

    python bench.py [--gpus 1] [--steps K] [--warmup W]

Prints one JSON line.  `value` is agent-steps per second with the state
resident in HBM; `roofline` reports the fused step kernel against the
vector-ALU peak; `cpu_baseline` is the FP64 oracle timed on this host's
cores on a short sample of the same workload.
"""
from __future__ import annotations

import argparse
import ctypes
import dataclasses
import hashlib
import json
import os
import re
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

# MI355X: 256 CUs x 4 SIMD x 16 lanes at 2.4 GHz = 3.93e13 VALU lane-ops/s
# (non-packed FP32 / FP64 rate; FP32 vector 157.3 TFLOP/s counts an FMA as
# two flops and a packed op as two lanes).
VALU_PEAK_TOPS = 256 * 64 * 2.4e9 / 1e12
HBM_PEAK_GBS = 8000.0

# Algorithmic VALU lane-operations per unit of work counted by the oracle
# (a quarter-rate sqrt/reciprocal counts 4).  Units, in order of the oracle's
# work counters: candidate examined in the 3x3 stencil of R_n cells,
# in-range candidate, half-plane built, LP2 line checked, LP2 line re-solved,
# LP2 inner iteration, LP3 used, LP3 line re-solved, LP3 boundary line
# built, LP3 boundary line checked, LP3 boundary line re-solved, LP3 inner
# iteration.
OP_COST = (10, 0, 65, 4, 20, 15, 0, 10, 20, 4, 20, 15)
# Algorithmic HBM bytes per agent-step of the fused step kernel: read
# px, py, vx, vy, radius (cell-ordered copy), pref_x, pref_y, max_speed, class
# (33 B), write px, py, vx, vy (16 B).
STEP_BYTES_PER_AGENT = 49
# Algorithmic HBM bytes per agent-step of the adjoint kernel: the forward
# recomputation's 33 B read, the cotangents of (p', v') read (16 B), the
# cotangents of (p, v) and of pref written (24 B), the tau term (4 B), and
# three neighbour edges of 20 B written (60 B).
ADJ_BYTES_PER_AGENT = 33 + 16 + 24 + 4 + 60
# Algorithmic VALU lane-ops of the adjoint beyond its forward recomputation:
# the VJP of every half-plane through its frozen branch (twice the forward
# half-plane, 2 x 65) and the VJP of the LP's active set (a 2x2 solve and its
# transpose, 40 per agent).
ADJ_OPS_PER_NEIGHBOR = 130
ADJ_OPS_PER_AGENT = 40


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def source_hash(files=("step.hip", "orca_device.h", "orca_internal.h")) -> str:
    """Hash of a kernel's source files (comments removed and whitespace
    collapsed, so that only a change of code invalidates the committed
    counter summaries); by default the step kernel's."""
    h = hashlib.sha256()
    for f in files:
        with open(os.path.join(ROOT, "paper_2008_11578_amd", "csrc", f)) as fh:
            code = re.sub(r"/\*.*?\*/", "", fh.read(), flags=re.S)
        code = re.sub(r"//[^\n]*", "", code)
        # whitespace-insensitive, so that comments of another length leave it
        code = " ".join(code.split())
        h.update(code.encode())
    return h.hexdigest()[:16]


def traffic_from_profile(kernel_hash: str):
    """HBM bytes per launch of the step kernel from the committed rocprofv3
    counter summary, or None when missing or taken on other kernel source."""
    path = os.path.join(ROOT, "profiles", "k_step_c3_1M_hbm_traffic.md")
    if not os.path.exists(path):
        return None
    txt = open(path).read()
    mh = re.search(r"source_hash:\s*([0-9a-f]+)", txt)
    mb = re.search(r"traffic_bytes_per_launch:\s*([0-9.eE+]+)", txt)
    if not mh or not mb or mh.group(1) != kernel_hash:
        return None

    def num(key):
        m = re.search(key + r":\s*([0-9.eE+]+)", txt)
        return float(m.group(1)) if m else None

    # raw counters beside the calibrated bytes: the scale comes from a plain
    # streaming copy, which need not hold for the step's 16-byte gathers
    return {"bytes": float(mb.group(1)), "fetch_kib": num("fetch_kib_per_launch"),
            "write_kib": num("write_kib_per_launch"),
            "scale": {"fetch": num("fetch_scale"), "write": num("write_scale")}}


def valu_from_profile(kernel_hash: str):
    """VALU busy and lane utilisation (percent) of the step kernel from the
    committed rocprofv3 counter summary, or None when missing or taken on
    other kernel source."""
    path = os.path.join(ROOT, "profiles", "k_step_c3_1M_valu.md")
    if not os.path.exists(path):
        return None
    txt = open(path).read()
    mh = re.search(r"source_hash:\s*([0-9a-f]+)", txt)
    mb = re.search(r"valu_busy_pct:\s*([0-9.eE+]+)", txt)
    mu = re.search(r"valu_utilization_pct:\s*([0-9.eE+]+)", txt)
    mi = re.search(r"valu_insts_per_launch:\s*([0-9.eE+]+)", txt)
    if not mh or not mb or not mu or not mi or mh.group(1) != kernel_hash:
        return None
    return {"valu_busy_pct": float(mb.group(1)), "valu_utilization_pct": float(mu.group(1)),
            "valu_insts_per_launch": float(mi.group(1))}


class HipEvents:
    """Raw hipEvent_t handles from the HIP runtime torch has loaded."""

    def __init__(self):
        self.hip = ctypes.CDLL("libamdhip64.so.7")
        self.hip.hipEventCreate.argtypes = [ctypes.POINTER(ctypes.c_void_p)]
        self.hip.hipEventElapsedTime.argtypes = [ctypes.POINTER(ctypes.c_float),
                                                 ctypes.c_void_p, ctypes.c_void_p]
        self.hip.hipEventDestroy.argtypes = [ctypes.c_void_p]
        self.events = []

    def create(self) -> int:
        e = ctypes.c_void_p()
        rc = self.hip.hipEventCreate(ctypes.byref(e))
        if rc != 0:
            raise RuntimeError(f"hipEventCreate failed ({rc})")
        self.events.append(e.value)
        return e.value

    def elapsed_ms(self, a: int, b: int) -> float:
        ms = ctypes.c_float()
        rc = self.hip.hipEventElapsedTime(ctypes.byref(ms), ctypes.c_void_p(a), ctypes.c_void_p(b))
        if rc != 0:
            raise RuntimeError(f"hipEventElapsedTime failed ({rc})")
        return ms.value

    def close(self):
        for e in self.events:
            self.hip.hipEventDestroy(ctypes.c_void_p(e))
        self.events = []


def algorithmic_ops(work) -> float:
    import numpy as np
    return float((work.astype(np.float64) * np.asarray(OP_COST, np.float64)[None, :]).sum())


def cpu_model() -> str:
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(state_start, state_end, params, n, steps, steps_1t=2):
    """Times the FP64 oracle on this host: `steps` oracle steps from the
    state that opens the timed GPU window, plus one from the state that
    closes it, on all threads; then `steps_1t` steps on one thread.  Also
    returns the oracle's work counters on both states."""
    import numpy as np
    import oracle
    oracle.build(force=False)
    threads = oracle.set_threads(oracle_threads())
    t0 = time.perf_counter()
    st = dict(state_start)
    w_start = None
    for s in range(steps):
        o = oracle.step(st, params, want_work=(s == 0))
        if s == 0:
            w_start = o["work"]
        st = dict(st)
        for k in ("px", "py", "vx", "vy"):
            st[k] = o[k].astype(np.float32)
    o_end = oracle.step(state_end, params, want_work=True)
    elapsed = time.perf_counter() - t0
    rate = n * (steps + 1) / elapsed
    rate_1t = None
    if steps_1t > 0:
        oracle.set_threads(1)
        try:
            t1 = time.perf_counter()
            st = dict(state_start)
            for _ in range(steps_1t):
                o = oracle.step(st, params)
                st = dict(st)
                for k in ("px", "py", "vx", "vy"):
                    st[k] = o[k].astype(np.float32)
            rate_1t = n * steps_1t / (time.perf_counter() - t1)
        finally:
            oracle.set_threads(threads)
    return rate, elapsed, threads, w_start, o_end["work"], rate_1t


def oracle_ops(states, params):
    """Average algorithmic lane-ops per step launch over the given states
    (the oracle's work counters x OP_COST), with the mean in-range neighbour
    count and the LP3 share."""
    import numpy as np
    import oracle
    oracle.build(force=False)
    ops, nb, lp3 = [], [], []
    for st in states:
        w = oracle.step(st, params, want_work=True)["work"]
        ops.append(algorithmic_ops(w))
        nb.append(float(w[:, 2].mean()))
        lp3.append(float(w[:, 6].mean()))
    return float(np.mean(ops)), float(np.mean(nb)), float(np.mean(lp3))


def oracle_rate(state0, params, n, steps, threads=0):
    """The FP64 oracle stepped `steps` times from state0 (each step's FP32
    rounding fed back, as the GPU state is) on `threads` host threads (0:
    all); returns (agent-steps/s, seconds, threads used)."""
    import numpy as np
    import oracle
    oracle.build(force=False)
    full = oracle_threads()
    used = oracle.set_threads(threads if threads > 0 else full)
    try:
        st = dict(state0)
        t0 = time.perf_counter()
        for _ in range(steps):
            o = oracle.step(st, params)
            st = dict(st)
            for k in ("px", "py", "vx", "vy"):
                st[k] = o[k].astype(np.float32)
        el = time.perf_counter() - t0
    finally:
        oracle.set_threads(full)
    return n * steps / el, el, used


_FULL_THREADS = []


def oracle_threads() -> int:
    """The oracle's default (all host threads) OpenMP thread count."""
    if not _FULL_THREADS:
        import oracle
        _FULL_THREADS.append(oracle.set_threads(0))
    return _FULL_THREADS[0]


def alu_roofline(ops, k_ms, n, bytes_per_agent, kernel, **extra):
    """Roofline object of a step-type kernel: algorithmic lane-ops per launch
    over its measured duration against the vector-ALU peak, with the
    algorithmic HBM rate against the HBM peak beside it."""
    achieved = ops / (k_ms * 1e-3) / 1e12
    hbm = bytes_per_agent * n / (k_ms * 1e-3) / 1e9
    out = {"bound": "alu", "achieved": achieved, "peak": VALU_PEAK_TOPS, "unit": "Top/s",
           "frac": achieved / VALU_PEAK_TOPS, "traffic": None, "kernel": kernel,
           "kernel_ms": k_ms, "ops_per_launch": ops,
           "hbm_algorithmic_GBs": hbm, "hbm_frac": hbm / HBM_PEAK_GBS,
           "hbm_peak_GBs": HBM_PEAK_GBS}
    out.update(extra)
    return out


def run_plain(sc, params, steps, warmup):
    """Steps one scene `warmup` + `steps` times through orca_step_ex on one
    workspace kept across steps (HIP events around the grid build and the
    step kernel of every timed step).  Returns the wall time, the mean event
    times, the LP3 share of the last step and the states opening and closing
    the timed window."""
    import numpy as np
    import torch
    from paper_2008_11578_amd import orca
    n = sc.n
    state = orca.State.from_arrays(sc)
    nxt = state.clone()
    ws = orca.Workspace(n)
    status = torch.zeros(n, dtype=torch.uint8, device="cuda")
    for _ in range(warmup):
        orca.step(state, params, ws, out=nxt, status=status)
        state, nxt = nxt, state
    torch.cuda.synchronize()
    out = {"start": state.to_numpy()}
    hip = HipEvents()
    # events are created before the timed region
    pre = [(hip.create(), hip.create(), hip.create()) for _ in range(steps)]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for s in range(steps):
        orca.step(state, params, ws, out=nxt, status=status, events=pre[s])
        state, nxt = nxt, state
    torch.cuda.synchronize()
    out["wall"] = time.perf_counter() - t0
    out["grid_ms"] = float(np.mean([hip.elapsed_ms(a, b) for a, b, c in pre]))
    out["k_ms"] = float(np.mean([hip.elapsed_ms(b, c) for a, b, c in pre]))
    hip.close()
    out["lp3_share"] = float(status.float().mean().item())
    out["end"] = state.to_numpy()
    return out


def bench_config_leg(name, sc, params, steps, cpu_1t_steps, cpu=True):
    """One plain configuration run for its whole step count from its seeded
    initial state (after an untimed warm-up run on a copy), with the step
    kernel's roofline and the oracle timed on the same step count."""
    from paper_2008_11578_amd import orca
    n = sc.n
    warm = run_plain(sc, params, min(steps, 5), 0)  # code objects, caches
    del warm
    r = run_plain(sc, params, steps, 0)
    value = n * steps / r["wall"]
    leg = {"workload": sc.name, "agents": n, "steps": steps, "value": value,
           "unit": "agent-steps/s", "ms_per_step": r["wall"] * 1e3 / steps,
           "grid_ms": r["grid_ms"], "step_kernel_ms": r["k_ms"], "lp3_share_end": r["lp3_share"]}
    if cpu:
        ops, nbr, lp3 = oracle_ops([r["start"], r["end"]], params)
        leg["roofline"] = alu_roofline(ops, r["k_ms"], n, STEP_BYTES_PER_AGENT,
                                       f"k_step<{params.max_neighbors}>",
                                       mean_neighbors=nbr, oracle_lp3_share=lp3)
        rate, el, th = oracle_rate(r["start"], params, n, steps)
        rate1, el1, _ = oracle_rate(r["start"], params, n, cpu_1t_steps, threads=1)
        leg["cpu_baseline"] = {
            "value": rate, "unit": "agent-steps/s", "cores": th, "kind": "oracle",
            "sample": f"the whole {steps}-step run from the same initial state ({el:.2f} s); "
                      f"single thread: {cpu_1t_steps} steps ({el1:.2f} s)",
            "single_thread_value": rate1, "nproc": os.cpu_count(), "cpu_model": cpu_model(),
            "speedup": value / rate}
    log(f"[bench] {name}: {n} agents x {steps} steps, {leg['ms_per_step']:.3f} ms/step, "
        f"step kernel {r['k_ms']:.3f} ms, {value:.3e} agent-steps/s"
        + (f", oracle {leg['cpu_baseline']['value']:.3e} ({leg['cpu_baseline']['cores']} threads),"
           f" roofline frac {leg['roofline']['frac']:.3f}" if cpu else ""))
    return leg


def grid_kernels_from_profile(n, n_cells, grid_ms):
    """HBM fractions of the grid-build kernels of the measured workload:
    algorithmic bytes per launch (n agents, n_cells cells) over each
    kernel's average duration from the committed rocprofv3 kernel trace of
    the same command, while the grid source is the one it was taken on; and
    the whole build's bytes over the live HIP-event time of the build."""
    per_kernel = {
        # read px, py; clear the histogram
        "k_bbox_partial": 8 * n + 4 * n_cells,
        # read px, py; write cell and rank; histogram counts read and written
        "k_cell_count": 16 * n + 8 * n_cells,
        # read the histogram
        "k_scan_reduce": 4 * n_cells,
        # read the histogram, write the cell starts
        "k_scan_apply": 8 * n_cells,
        # read cell, rank, start[cell], px, py, radius, vx, vy, class; write two float4
        "k_scatter": 33 * n + 32 * n,
    }
    total = sum(per_kernel.values())
    out = {"algorithmic_bytes": total, "grid_ms": grid_ms,
           "hbm_frac_whole_build": total / (grid_ms * 1e-3) / 1e9 / HBM_PEAK_GBS,
           "cells": n_cells, "kernels": None}
    path = os.path.join(ROOT, "profiles", "k_step_c3_1M_kernel_stats.md")
    if not os.path.exists(path):
        return out
    txt = open(path).read()
    mh = re.search(r"grid_source_hash:\s*([0-9a-f]+)", txt)
    if not mh or mh.group(1) != source_hash(("grid.hip", "orca_internal.h")):
        return out
    ks = {}
    for name, b in per_kernel.items():
        m = re.search(r"\|\s*" + name + r"\s*\|\s*(\d+)\s*\|\s*([0-9.]+)\s*\|", txt)
        if m:
            us = float(m.group(2))
            ks[name] = {"bytes": b, "avg_us": us, "GBs": b / (us * 1e-6) / 1e9,
                        "hbm_frac": b / (us * 1e-6) / 1e9 / HBM_PEAK_GBS}
    out["kernels"] = ks
    return out


def capture_loop(step_fn, a, b, steps):
    """Records `steps` ping-pong steps a->b->a... into one HIP graph; returns
    (graph, final state)."""
    import torch
    stream = torch.cuda.Stream()
    stream.wait_stream(torch.cuda.current_stream())
    graph = torch.cuda.CUDAGraph()
    with torch.cuda.stream(stream):
        with torch.cuda.graph(graph, stream=stream):
            x, y = a, b
            for _ in range(steps):
                step_fn(x, y)
                x, y = y, x
    torch.cuda.synchronize()
    return graph, x


def bench_batched(steps: int, cpu: bool = True):
    """512 uneven scenes (about 5.6M agents) per step: the autotuned batched
    step captured as a `steps`-step graph, against 512 sequential single-scene
    steps captured as a graph.  The persistent step kernel's duration comes
    from HIP events around it over eager steps after the graph; its roofline
    takes the oracle's work counters on the states opening and closing the
    timed graph; the oracle's batched step is timed beside it."""
    import numpy as np
    import torch
    from paper_2008_11578_amd import autotune, orca, scenarios
    sc = scenarios.c4_batched()
    S = len(sc.scene_params)
    n = sc.n
    st = orca.State.from_arrays(sc)
    nxt = st.clone()
    ws = orca.Workspace(n, n_scenes=S)
    tuned = autotune.tune_batched(st, sc.scene_off, sc.scene_params, ws, reps=3, use_cache=False)
    batch = orca.Batch(sc.scene_off, tuned["params"], mode=tuned["mode"], block=tuned["block"],
                       k_tile=tuned["k_tile"])
    graph, _ = capture_loop(lambda x, y: orca.step_batched(x, batch, ws, out=y), st, nxt, steps)
    graph.replay()
    torch.cuda.synchronize()
    snap_start = st.to_numpy() if cpu else None
    t0 = time.perf_counter()
    graph.replay()
    torch.cuda.synchronize()
    ms = (time.perf_counter() - t0) * 1e3 / steps
    snap_end = st.to_numpy() if cpu else None
    assert int(batch.error.item()) == 0
    # the step kernel alone: HIP events around it over eager steps
    hip = HipEvents()
    k_steps = 10
    pre = [(hip.create(), hip.create(), hip.create()) for _ in range(k_steps)]
    a, b = st, nxt
    for e in pre:
        orca.step_batched(a, batch, ws, out=b, events=e)
        a, b = b, a
    torch.cuda.synchronize()
    k_ms = float(np.mean([hip.elapsed_ms(e[1], e[2]) for e in pre]))
    g_ms = float(np.mean([hip.elapsed_ms(e[0], e[1]) for e in pre]))
    hip.close()
    # per-scene baseline: one orca_step per scene, sequentially, in a graph
    parts = []
    for s in range(S):
        a, z = int(sc.scene_off[s]), int(sc.scene_off[s + 1])
        parts.append((orca.State(**{k: getattr(st, k)[a:z] for k in orca.STATE_FIELDS}),
                      orca.State(**{k: getattr(nxt, k)[a:z] for k in orca.STATE_FIELDS}),
                      orca.Workspace(z - a), tuned["params"][s]))

    def per_scene(x_is_st):
        for xs, ys, wss, p in parts:
            if x_is_st:
                orca.step(xs, p, wss, out=ys)
            else:
                orca.step(ys, p, wss, out=xs)

    per_scene(True)
    torch.cuda.synchronize()
    stream = torch.cuda.Stream()
    stream.wait_stream(torch.cuda.current_stream())
    g2 = torch.cuda.CUDAGraph()
    with torch.cuda.stream(stream):
        with torch.cuda.graph(g2, stream=stream):
            per_scene(True)
            per_scene(False)
    torch.cuda.synchronize()
    g2.replay()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    g2.replay()
    torch.cuda.synchronize()
    ms_ps = (time.perf_counter() - t0) * 1e3 / 2
    log(f"[bench] batched {S} scenes, {n} agents: {ms:.3f} ms/step (graph of {steps}), "
        f"step kernel {k_ms:.3f} ms, per-scene {ms_ps:.3f} ms/step, tuned factor "
        f"{tuned['factor']:.3f} mode {tuned['mode']} block {tuned['block']} "
        f"k tile {tuned['k_tile']}")
    out = {"metric": "scene-steps/s (512 uneven scenes, one batched step per graph node set)",
           "scenes": S, "agents": n, "ms_per_step": ms,
           "scene_steps_per_s": S / (ms * 1e-3), "agent_steps_per_s": n / (ms * 1e-3),
           "grid_ms": g_ms, "step_kernel_ms": k_ms,
           "per_scene_ms_per_step": ms_ps, "speedup_vs_per_scene": ms_ps / ms,
           "graph_steps": steps, "tuned": {"cell_factor": tuned["factor"],
                                            "mode": tuned["mode"], "block": tuned["block"],
                                            "k_tile": tuned["k_tile"]}}
    if cpu:
        import oracle
        oracle.build(force=False)
        prm = tuned["params"]
        ops = []
        for snap in (snap_start, snap_end):
            w = oracle.step_batched(snap, sc.scene_off, prm, want_work=True)["work"]
            ops.append(algorithmic_ops(w))
        k_max = max(p.max_neighbors for p in prm)
        out["roofline"] = alu_roofline(float(np.mean(ops)), k_ms, n, STEP_BYTES_PER_AGENT,
                                       f"k_step_batched<{tuned['k_tile'] or k_max}>")
        full = oracle_threads()
        oracle.set_threads(full)
        reps = 3
        t0 = time.perf_counter()
        cur = dict(snap_start)
        for _ in range(reps):
            o = oracle.step_batched(cur, sc.scene_off, prm)
            cur = dict(cur)
            for k in ("px", "py", "vx", "vy"):
                cur[k] = o[k].astype(np.float32)
        el = time.perf_counter() - t0
        # one thread: one step of the first 128 scenes (a bounded sample)
        s1 = 128
        n1 = int(sc.scene_off[s1])
        part = {k: v[:n1] for k, v in snap_start.items()}
        oracle.set_threads(1)
        try:
            t1 = time.perf_counter()
            oracle.step_batched(part, sc.scene_off[:s1 + 1], prm[:s1])
            el1 = time.perf_counter() - t1
        finally:
            oracle.set_threads(full)
        rate = n * reps / el
        out["cpu_baseline"] = {
            "value": rate, "unit": "agent-steps/s", "cores": full, "kind": "oracle",
            "sample": f"{reps} batched oracle steps of all {S} scenes from the state opening the "
                      f"timed graph ({el:.1f} s); single thread: one step of the first {s1} "
                      f"scenes ({n1} agents, {el1:.2f} s)",
            "single_thread_value": n1 / el1, "nproc": os.cpu_count(), "cpu_model": cpu_model(),
            "speedup": (n / (ms * 1e-3)) / rate}
        log(f"[bench] batched oracle {rate:.3e} agent-steps/s on {full} threads; roofline frac "
            f"{out['roofline']['frac']:.3f}")
    return out


def bench_vehicle_share(steps: int = 100, warmup: int = 10, cpu: bool = True):
    """Agent-steps/s of the mixed-crowd geometry (66,560 agents) at vehicle
    shares 0, 1.5, 5 and 50 %: pedestrians and vehicles take the same
    instructions, so the rate per unit of work should not depend on the
    share.  Per share: the step kernel's time (HIP events), the oracle's
    algorithmic lane-ops per launch on the states opening and closing the
    timed steps, and the lane-ops per second this gives."""
    from paper_2008_11578_amd import scenarios
    rates, per = {}, {}
    for share in (0.0, 0.015, 0.05, 0.5):
        sc = scenarios.c2_vehicle_share(share)
        r = run_plain(sc, sc.params, steps, warmup)
        key = f"{share:g}"
        rates[key] = sc.n * steps / r["wall"]
        d = {"agent_steps_per_s": rates[key], "step_kernel_ms": r["k_ms"],
             "lp3_share_end": r["lp3_share"]}
        if cpu:
            ops, nbr, lp3 = oracle_ops([r["start"], r["end"]], sc.params)
            d.update(ops_per_agent_step=ops / sc.n, oracle_lp3_share=lp3,
                     lane_ops_Tps=ops / (r["k_ms"] * 1e-3) / 1e12,
                     frac=ops / (r["k_ms"] * 1e-3) / 1e12 / VALU_PEAK_TOPS)
        per[key] = d
    lo, hi = min(rates.values()), max(rates.values())
    out = {"metric": "agent-steps/s, 66,560 agents, by vehicle share", "steps": steps,
           "rates": rates, "spread": hi / lo - 1.0, "per_share": per}
    if cpu:
        f = [d["lane_ops_Tps"] for d in per.values()]
        out["work_rate_spread"] = max(f) / min(f) - 1.0
    log("[bench] vehicle share " + ", ".join(
        f"{k}: {v['agent_steps_per_s']:.3e} agent-steps/s"
        + (f" ({v['ops_per_agent_step']:.0f} ops/agent-step, {v['lane_ops_Tps']:.2f} Top/s)"
           if cpu else "") for k, v in per.items()))
    return out


def bench_extensions(reps: int = 20):
    """The rows beyond the plain step, on the dense crossing's 1,048,576
    agents: leaving at the goal (orca_remove_arrived, a stable compaction,
    against HBM), entering (orca_spawn with 16,384 candidates), the overlap
    statistics (orca_overlap_stats) and the step with acceleration caps and
    with turn-rate caps against the same step without them.  HIP events on the library's
    stream (torch's current stream) around `reps` calls."""
    import dataclasses
    import numpy as np
    import torch
    from paper_2008_11578_amd import orca, scenarios

    def timed(fn, k=reps):
        fn()
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(k):
            fn()
        e1.record()
        torch.cuda.synchronize()
        return e0.elapsed_time(e1) / k

    sc = scenarios.c3_crossing()
    n = sc.n
    arr = sc.arrays()
    # one agent in ten stands on its goal, so removal keeps nine in ten
    rng = np.random.default_rng(17)
    done = rng.random(n) < 0.1
    arr = dict(arr)
    arr["pref_x"] = np.where(done, arr["px"], arr["pref_x"]).astype(np.float32)
    arr["pref_y"] = np.where(done, arr["py"], arr["pref_y"]).astype(np.float32)
    st = orca.State.from_arrays(arr)
    out = st.clone()
    o2n = torch.empty(n, dtype=torch.int32, device="cuda")
    lws = orca.LifecycleWorkspace(n, orca.SPAWN_MAX)
    kept = int(orca.remove_arrived(st, out, lws, old_to_new=o2n).item())
    rm_ms = timed(lambda: orca.remove_arrived(st, out, lws, old_to_new=o2n))
    # read 9 fields (33 B) of every agent, write them for the survivors and
    # the old-to-new index of every agent
    rm_bytes = 33 * n + 33 * kept + 4 * n
    rm = {"ms": rm_ms, "agents": n, "kept": kept, "algorithmic_bytes": rm_bytes,
          "GBs": rm_bytes / (rm_ms * 1e-3) / 1e9,
          "hbm_frac": rm_bytes / (rm_ms * 1e-3) / 1e9 / HBM_PEAK_GBS}

    # spawning: 16,384 candidates uniform over the square against everyone
    nc = orca.SPAWN_MAX
    side = 700.0
    cand = {k: np.zeros(nc, np.float32) for k in orca.STATE_FIELDS if k != "cls"}
    cand["px"] = rng.uniform(0, side, nc).astype(np.float32)
    cand["py"] = rng.uniform(0, side, nc).astype(np.float32)
    cand["pref_x"] = rng.uniform(0, side, nc).astype(np.float32)
    cand["pref_y"] = rng.uniform(0, side, nc).astype(np.float32)
    cand["radius"] = np.full(nc, 0.3, np.float32)
    cand["max_speed"] = np.full(nc, 1.5, np.float32)
    cand["cls"] = np.zeros(nc, np.uint8)
    cst = orca.State.from_arrays(cand)
    big = orca.State(**{k: torch.cat([getattr(st, k), torch.zeros(nc, dtype=getattr(st, k).dtype,
                                                                  device="cuda")])
                        for k in orca.STATE_FIELDS})
    acc = torch.empty(nc, dtype=torch.uint8, device="cuda")
    tot = int(orca.spawn(big, n, cst, 1.0, lws, accepted=acc).item())
    sp_ms = timed(lambda: orca.spawn(big, n, cst, 1.0, lws, accepted=acc))
    sp = {"ms": sp_ms, "agents": n, "candidates": nc, "accepted": tot - n,
          "candidates_per_s": nc / (sp_ms * 1e-3)}

    # overlap statistics over pairs closer than 1 m (twice the largest radius)
    ows = orca.OverlapWorkspace(n)
    ores = orca.overlap_stats(st, 1.0, ows).cpu().numpy()
    ov_ms = timed(lambda: orca.overlap_stats(st, 1.0, ows))
    ov = {"ms": ov_ms, "agents": n, "reach": 1.0, "pairs": int(ores[0]),
          "agents_per_s": n / (ov_ms * 1e-3)}

    # the dense crossing's step with acceleration caps (2 m/s^2 for everyone)
    # and with turn-rate caps (1 rad/s for everyone)
    params = dataclasses.replace(sc.params, cell_size=0.6)
    capped = dataclasses.replace(params, accel=(2.0, 2.0))
    turned = dataclasses.replace(params, turn=(1.0, 1.0))
    res = {}
    for name, p in (("uncapped", params), ("capped", capped), ("turned", turned)):
        a = orca.State.from_arrays(sc)
        b = a.clone()
        ws = orca.Workspace(n)
        for _ in range(5):
            orca.step(a, p, ws, out=b)
            a, b = b, a

        def two():
            orca.step(a, p, ws, out=b)
            orca.step(b, p, ws, out=a)

        res[name] = timed(two, k=10) / 2
    ac = {"ms_per_step_capped": res["capped"], "ms_per_step_uncapped": res["uncapped"],
          "agent_steps_per_s_capped": n / (res["capped"] * 1e-3),
          "ratio": res["capped"] / res["uncapped"]}
    tu = {"ms_per_step_turn_capped": res["turned"], "ms_per_step_uncapped": res["uncapped"],
          "agent_steps_per_s_turn_capped": n / (res["turned"] * 1e-3),
          "ratio": res["turned"] / res["uncapped"]}
    log(f"[bench] extensions: remove {rm_ms:.3f} ms ({rm['GBs']:.0f} GB/s), spawn {sp_ms:.3f} ms, "
        f"overlap {ov_ms:.3f} ms, capped step {res['capped']:.3f} ms, turn-capped step "
        f"{res['turned']:.3f} ms vs {res['uncapped']:.3f}")
    return {"metric": "ms per call on the 1,048,576-agent dense crossing",
            "remove_arrived": rm, "spawn": sp, "overlap_stats": ov, "accel_step": ac,
            "turn_step": tu}


def bench_crossing():
    """The paper's first experiment shape run end to end: two-way and
    four-way crossings of 2,500 agents per group in a 100 m square with
    spawning at clear points, stepping, overlap statistics and removal at the
    goal every step, until everyone has arrived.  Reports the wall time per
    step (host synchronisation included), the agent-steps/s this gives, the
    flow of arrivals, the LP3 share and the overlaps."""
    import torch
    from paper_2008_11578_amd import crossing
    out = {}
    for kind in ("2way", "4way"):
        cfg = crossing.CrossingConfig(kind=kind, per_group=2500, side=100.0, strip=10.0,
                                      proposals=64, t_clear=1.0, max_steps=5000, seed=11)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        r = crossing.run(cfg, record=True)
        torch.cuda.synchronize()
        el = time.perf_counter() - t0
        dt = float(cfg.params.dt)
        out[kind] = {"agents": r["spawned"], "arrived": r["arrived"], "steps": r["steps"],
                     "agent_steps": r["agent_steps"], "wall_s": el,
                     "ms_per_step": el / max(r["steps"], 1) * 1e3,
                     "agent_steps_per_s": r["agent_steps"] / el,
                     "arrivals_per_sim_s": r["arrived"] / (r["steps"] * dt),
                     "lp3_share": r["lp3_share"], "max_overlap_pairs": r["max_overlap_pairs"],
                     "min_clearance_m": r["min_clearance"]}
        log(f"[bench] crossing {kind}: {r['spawned']} agents, {r['steps']} steps in {el:.2f} s, "
            f"lp3 {r['lp3_share']:.3f}, max overlap pairs {r['max_overlap_pairs']}")
    return {"metric": "crossings with spawning and removal, 2,500 agents per group", **out}


def bench_sweep():
    """A responsibility sweep: six tables f over 512 isolated head-on
    pedestrian-vehicle encounters (1,024 agents), as six scenes of one
    batched step, 80 steps; per table the pairs that ever overlap, the
    smallest clearance, the LP3 share and the final mean speeds, and the
    time per batched step of the whole sweep."""
    import torch
    from paper_2008_11578_amd import scenarios, sweeps
    sc = scenarios.head_on_pairs(pairs=512)
    tables = [sweeps.table(0.5, 1.0, 0.0, 0.5), sweeps.table(0.5, 0.5, 0.5, 0.5),
              sweeps.table(0.5, 0.75, 0.25, 0.5), sweeps.table(0.5, 0.0, 1.0, 0.5),
              sweeps.table(0.5, 0.25, 0.25, 0.5), sweeps.table(0.5, 0.0, 0.0, 0.5)]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    res = sweeps.run(tables, sc, steps=sc.steps, reach=3.0)
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    log(f"[bench] sweep {len(tables)} tables x {sc.n} agents x {sc.steps} steps: {el:.2f} s")
    return {"metric": "responsibility sweep, six tables as six scenes of one batched step",
            "scene": "512 isolated head-on pedestrian-vehicle pairs", "agents_per_table": sc.n,
            "steps": sc.steps, "wall_s": el, "ms_per_step": el / sc.steps * 1e3,
            "tables": [{k: (list(map(list, v)) if k == "f" else v) for k, v in r.items()}
                       for r in res]}


def bench_adjoint(reps: int = 3, cpu: bool = True):
    """Differentiable rollout: 16,384 agents, 50 steps, checkpoints every 10:
    forward rollout, then the backward pass (segment replays and
    orca_step_backward), timed with HIP events.  The per-agent adjoint
    kernel is timed alone (events around it) over the backward steps of the
    rollout's own trajectory; the oracle's gradient of the same rollout
    (forward, then its one-step VJPs chained backwards) is timed beside it."""
    import numpy as np
    import torch
    from paper_2008_11578_amd import orca, rollout, scenarios
    sc = scenarios.c5_rollout()
    p = sc.params
    n, steps = sc.n, sc.steps
    st0 = orca.State.from_arrays(sc)
    tx = torch.as_tensor(sc.target_x).cuda()
    ty = torch.as_tensor(sc.target_y).cuda()

    def once():
        vpx = st0.pref_x.clone().requires_grad_(True)
        vpy = st0.pref_y.clone().requires_grad_(True)
        # a host scalar: the forward reads it without a device synchronisation
        tau = torch.tensor(float(np.float32(p.time_horizon)), requires_grad=True)
        e0, e1, e2 = (torch.cuda.Event(enable_timing=True) for _ in range(3))
        e0.record()
        px, py = rollout.rollout(vpx, vpy, tau, st0, p, steps=steps, ckpt=10)
        loss = rollout.trajectory_loss(px, py, tx, ty)
        e1.record()
        loss.backward()
        e2.record()
        torch.cuda.synchronize()
        return e0.elapsed_time(e1), e1.elapsed_time(e2), float(loss.item()), float(tau.grad.item())

    once()
    runs = [once() for _ in range(reps)]
    fwd = float(np.median([r[0] for r in runs]))
    bwd = float(np.median([r[1] for r in runs]))
    # the same rollout captured in HIP graphs (forward; backward with its
    # segment replays): replays with the desired velocities and the loss's
    # cotangents as inputs
    rg = rollout.RolloutGraph(st0, p, float(np.float32(p.time_horizon)), steps=steps, ckpt=10)
    gtimes = []
    for _ in range(reps + 1):
        e0, e1, e2 = (torch.cuda.Event(enable_timing=True) for _ in range(3))
        e0.record()
        gx, gy = rg.forward(st0.pref_x, st0.pref_y)
        e1.record()
        cx = (2.0 / n) * (gx - tx)
        cy = (2.0 / n) * (gy - ty)
        rg.g_px.copy_(cx)
        rg.g_py.copy_(cy)
        rg.g_bwd.replay()
        e2.record()
        torch.cuda.synchronize()
        gtimes.append((e0.elapsed_time(e1), e1.elapsed_time(e2)))
    rg.backward(cx, cy)  # the replayed segments end where the forward went
    fwd_g = float(np.median([t[0] for t in gtimes[1:]]))
    bwd_g = float(np.median([t[1] for t in gtimes[1:]]))
    # the adjoint kernel alone over the rollout's trajectory
    import dataclasses
    pv = dataclasses.replace(p, pref_is_goal=0)
    s, s2 = st0.clone(), st0.clone()
    ws = orca.Workspace(n)
    states = []
    for _ in range(steps):
        states.append(s.clone())
        orca.step(s, pv, ws, out=s2)
        s, s2 = s2, s
    wsb = orca.Workspace(n, backward=True)
    gen = torch.Generator(device="cuda").manual_seed(9)
    g = [torch.randn(n, device="cuda", generator=gen) for _ in range(4)]
    gpr = [torch.zeros(n, device="cuda") for _ in range(2)]
    gt = torch.zeros(1, device="cuda")
    out4 = tuple(torch.empty(n, device="cuda") for _ in range(4))
    hip = HipEvents()
    pre = [(hip.create(), hip.create(), hip.create()) for _ in range(steps)]
    for t in range(steps - 1, -1, -1):
        orca.step_backward(states[t], pv, wsb, *g, gpr[0], gpr[1], gt, out=out4, events=pre[t])
    torch.cuda.synchronize()
    k_ms = float(np.mean([hip.elapsed_ms(e[1], e[2]) for e in pre]))
    hip.close()
    log(f"[bench] adjoint {n} agents x {steps} steps: forward {fwd:.2f} ms, backward {bwd:.2f} ms, "
        f"adjoint kernel {k_ms * 1e3:.1f} us; captured: forward {fwd_g:.2f} ms, "
        f"backward {bwd_g:.2f} ms")
    out = {"metric": "agent-steps/s of a differentiable rollout (forward + backward)",
           "agents": n, "steps": steps, "checkpoint_every": 10, "forward_ms": fwd,
           "backward_ms": bwd, "adjoint_kernel_ms": k_ms,
           "agent_steps_per_s": n * steps / ((fwd + bwd) * 1e-3),
           "backward_agent_steps_per_s": n * steps / (bwd * 1e-3),
           "captured": {"forward_ms": fwd_g, "backward_ms": bwd_g,
                        "agent_steps_per_s": n * steps / ((fwd_g + bwd_g) * 1e-3)},
           "loss": runs[-1][2], "dL_dtau": runs[-1][3]}
    if cpu:
        import oracle
        oracle.build(force=False)
        snaps = [states[0].to_numpy(), states[-1].to_numpy()]
        ops = []
        for snap in snaps:
            w = oracle.step(snap, pv, want_work=True)["work"]
            ops.append(algorithmic_ops(w) + ADJ_OPS_PER_NEIGHBOR * float(w[:, 2].sum())
                       + ADJ_OPS_PER_AGENT * n)
        out["roofline"] = alu_roofline(float(np.mean(ops)), k_ms, n, ADJ_BYTES_PER_AGENT,
                                       f"k_adjoint<{p.max_neighbors}>")
        st = {k: np.array(getattr(sc, k), dtype=np.uint8 if k == "cls" else np.float64)
              for k in ("px", "py", "vx", "vy", "pref_x", "pref_y", "radius", "max_speed", "cls")}
        full = oracle_threads()
        oracle.set_threads(full)
        t0 = time.perf_counter()
        oracle.rollout_grad(st, p, steps, sc.target_x, sc.target_y)
        el = time.perf_counter() - t0
        steps1 = 5
        oracle.set_threads(1)
        try:
            t1 = time.perf_counter()
            oracle.rollout_grad(st, p, steps1, sc.target_x, sc.target_y)
            el1 = time.perf_counter() - t1
        finally:
            oracle.set_threads(full)
        rate = n * steps / el
        out["cpu_baseline"] = {
            "value": rate, "unit": "agent-steps/s (forward + backward)", "cores": full,
            "kind": "oracle",
            "sample": f"the oracle's gradient of the whole {steps}-step rollout (FP64 forward, "
                      f"then its one-step VJPs chained backwards, {el:.2f} s); single thread: "
                      f"a {steps1}-step rollout's gradient ({el1:.2f} s)",
            "single_thread_value": n * steps1 / el1, "nproc": os.cpu_count(),
            "cpu_model": cpu_model(), "speedup": out["agent_steps_per_s"] / rate}
        log(f"[bench] adjoint oracle {rate:.3e} agent-steps/s on {full} threads; adjoint kernel "
            f"roofline frac {out['roofline']['frac']:.3f}")
    return out


def main(argv=None):
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawTextHelpFormatter)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=100)
    ap.add_argument("--warmup", type=int, default=10)
    ap.add_argument("--cpu-steps", type=int, default=40,
                    help="oracle steps in the CPU-baseline sample (0 disables it)")
    ap.add_argument("--side", type=int, default=1024,
                    help="lattice side of the crossing workload (1024 -> 1,048,576 agents)")
    ap.add_argument("--cell-size", type=float, default=0.6,
                    help="grid cell size in m (0.6 = R_n/5, the fastest of a sweep over "
                         "{3, 2, 1.5, 1, 0.75, 0.6, 0.5} m for this workload; 0 = library "
                         "default R_n)")
    ap.add_argument("--batched-steps", type=int, default=100,
                    help="graph-captured steps of the 512-scene batched form (0 skips it)")
    ap.add_argument("--no-adjoint", dest="adjoint", action="store_false",
                    help="skip the differentiable-rollout leg")
    ap.add_argument("--no-sweep", dest="sweep", action="store_false",
                    help="skip the responsibility sweep")
    ap.add_argument("--no-crossing", dest="crossing", action="store_false",
                    help="skip the crossing runs with spawning and removal")
    ap.add_argument("--no-extensions", dest="extensions", action="store_false",
                    help="skip the lifecycle / overlap / acceleration-cap leg")
    ap.add_argument("--no-vehicle-share", dest="vehicle_share", action="store_false",
                    help="skip the vehicle-share sweep of the mixed crowd")
    ap.add_argument("--no-legs", dest="legs", action="store_false",
                    help="skip the 256-agent and mixed-crowd configuration runs")
    ap.add_argument("--calibrate-gather", type=int, default=0, metavar="MIB",
                    help="only gather MIB of 16-byte records 5 times in a locally shuffled "
                         "order (FETCH_SIZE calibration for the step's gathers)")
    ap.add_argument("--calibrate-copy", type=int, default=0, metavar="MIB",
                    help="only run a plain device copy of MIB MiB (5 times) and exit: the "
                         "reference kernel for scaling HBM counters")
    args = ap.parse_args(argv)

    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print(f"bench.py measures one GPU only; --gpus {args.gpus} (WORLD_SIZE={world}) is not "
              "supported: the library steps a scene on one GPU (sharding by scenes or by spatial "
              "slabs is a design, not an implemented path)", file=sys.stderr)
        return 2

    import numpy as np
    import torch

    from paper_2008_11578_amd import orca, scenarios

    if not torch.cuda.is_available():
        print("bench.py needs a GPU", file=sys.stderr)
        return 2
    torch.cuda.set_device(0)
    if args.calibrate_copy > 0:
        a = torch.empty(args.calibrate_copy << 18, dtype=torch.float32, device="cuda").fill_(1.0)
        b = torch.empty_like(a)
        for _ in range(5):
            b.copy_(a)
        torch.cuda.synchronize()
        log(f"[bench] copied {args.calibrate_copy} MiB 5 times")
        return 0
    if args.calibrate_gather > 0:
        # 16-byte records read in an order shuffled within windows of 4096
        # records (every cache line is used whole, as the step's candidate
        # rows use theirs), 32-bit indices, written in order
        m = args.calibrate_gather << 16
        src = torch.ones((m, 4), dtype=torch.float32, device="cuda")
        g = torch.Generator(device="cpu").manual_seed(5)
        win = 4096
        perm = torch.cat([torch.randperm(win, generator=g) + w for w in range(0, m, win)])
        idx = perm.to(torch.int32).cuda()
        dst = torch.empty_like(src)
        for _ in range(5):
            torch.index_select(src, 0, idx, out=dst)
        torch.cuda.synchronize()
        log(f"[bench] gathered {args.calibrate_gather} MiB 5 times ({m} records, "
            f"{m * 16 + m * 4} bytes read per gather)")
        return 0
    sc = scenarios.c3_crossing(side_count=args.side)
    n = sc.n
    params = dataclasses.replace(sc.params, cell_size=args.cell_size)
    log(f"[bench] workload {sc.name}: n={n}, k={params.max_neighbors}, R_n={params.neighbor_dist}")
    r = run_plain(sc, params, args.steps, args.warmup)
    snap_start, snap_end = r["start"], r["end"]
    wall, g_ms, k_ms, lp3_share = r["wall"], r["grid_ms"], r["k_ms"], r["lp3_share"]
    ms_per_step = wall * 1e3 / args.steps
    value = n * args.steps / wall
    log(f"[bench] {args.steps} steps: {ms_per_step:.3f} ms/step, grid {g_ms:.3f} ms, "
        f"step kernel {k_ms:.3f} ms, LP3 share at end {lp3_share:.3f}")

    # the grid geometry of the state closing the timed window (cells used)
    st_end = orca.State.from_arrays(snap_end)
    wsg = orca.Workspace(n)
    orca.build_grid(st_end, params, wsg, want_neighbors=False)
    torch.cuda.synchronize()
    meta = wsg.buf[:64].cpu().numpy()
    n_cells = int(meta[28:32].view(np.int32)[0])  # GridMeta.n_cells
    grid = grid_kernels_from_profile(n, n_cells, g_ms)
    del wsg, st_end

    cpu = None
    ops_per_launch = None
    if args.cpu_steps > 0:
        rate, el, threads, w0, w1, rate_1t = cpu_baseline(snap_start, snap_end, params, n,
                                                           args.cpu_steps)
        ops_per_launch = 0.5 * (algorithmic_ops(w0) + algorithmic_ops(w1))
        cpu = {"value": rate, "unit": "agent-steps/s", "cores": threads, "kind": "oracle",
               "sample": f"{args.cpu_steps} FP64 oracle steps from the state opening the timed "
                         f"GPU window plus 1 from the state closing it, {n} agents "
                         f"({el:.1f} s); single-thread rate from 2 steps of the same state",
               "single_thread_value": rate_1t, "nproc": os.cpu_count(),
               "cpu_model": cpu_model(), "speedup": value / rate}
        log(f"[bench] oracle: {rate:.3e} agent-steps/s on {threads} threads ({el:.1f} s), "
            f"{rate_1t:.3e} on 1 thread")

    roof = None
    if ops_per_launch is not None:
        kh = source_hash()
        roof = alu_roofline(ops_per_launch, k_ms, n, STEP_BYTES_PER_AGENT,
                            f"k_step<{params.max_neighbors}>", source_hash=kh)
        traffic = traffic_from_profile(kh)
        if traffic:
            roof.update(traffic=traffic["bytes"], traffic_raw_fetch_kib=traffic["fetch_kib"],
                        traffic_raw_write_kib=traffic["write_kib"],
                        traffic_scale=traffic["scale"],
                        hbm_measured_GBs=traffic["bytes"] / (k_ms * 1e-3) / 1e9,
                        hbm_measured_frac=traffic["bytes"] / (k_ms * 1e-3) / 1e9 / HBM_PEAK_GBS)
        valu = valu_from_profile(kh)
        if valu:
            # lane-ops the hardware executed (active lanes of every VALU
            # instruction) per second, against the same peak
            executed = (valu["valu_insts_per_launch"] * 64 * valu["valu_utilization_pct"] / 100
                        / (k_ms * 1e-3) / 1e12)
            roof.update(valu, executed_lane_ops_Tps=executed,
                        executed_frac=executed / VALU_PEAK_TOPS)

    legs = None
    if args.legs:
        c1 = scenarios.c1_plain()
        c2 = scenarios.c2_mixed()
        legs = {"c1": bench_config_leg("c1", c1, c1.params, c1.steps, c1.steps,
                                       cpu=args.cpu_steps > 0),
                "c2": bench_config_leg("c2", c2, c2.params, c2.steps, 10,
                                       cpu=args.cpu_steps > 0)}
    cpu_on = args.cpu_steps > 0
    batched = bench_batched(args.batched_steps, cpu=cpu_on) if args.batched_steps > 0 else None
    adjoint = bench_adjoint(cpu=cpu_on) if args.adjoint else None
    vshare = bench_vehicle_share(cpu=cpu_on) if args.vehicle_share else None
    ext = bench_extensions() if args.extensions else None
    cross = bench_crossing() if args.crossing else None
    sweep = bench_sweep() if args.sweep else None

    out = {
        "metric": "agent-steps/sec at 1M agents (ORCA+LP); batched & adjoint steps/sec",
        "value": value,
        "unit": "agent-steps/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_per_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": f"dense four-way crossing, {n} pedestrians, 700 m square, "
                               f"R_n 3 m, k 20, dt 0.1 s, tau 2 s",
                   "agents": n, "max_neighbors": params.max_neighbors,
                   "cell_size": params.cell_size,
                   "grid_ms": g_ms, "step_kernel_ms": k_ms, "lp3_share_end": lp3_share},
        "roofline": roof,
        "cpu_baseline": cpu,
        "grid_kernels": grid,
        "legs": legs,
        "batched": batched,
        "adjoint": adjoint,
        "vehicle_share": vshare,
        "extensions": ext,
        "crossing": cross,
        "sweep": sweep,
    }
    print(json.dumps(out), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
