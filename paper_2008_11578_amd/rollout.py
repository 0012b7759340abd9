"""Differentiable ORCA rollouts (the adjoint form of the step).

`Rollout` is a torch.autograd.Function: its forward runs `steps` ORCA steps
(orca_step) from a given state with per-agent desired velocities v_pref
(held constant) and a shared look-ahead tau, and returns the final
positions; its backward re-runs the forward from checkpoints saved every
`ckpt` steps and chains orca_step_backward through each segment in reverse,
returning the gradients with respect to v_pref and tau.  All work runs in
the library's kernels; checkpoints are plain device copies of (px, py, vx, vy).
"""
from __future__ import annotations

import dataclasses
from typing import Tuple

import torch

from . import orca


class Rollout(torch.autograd.Function):
    @staticmethod
    def forward(ctx, v_pref_x, v_pref_y, tau, state0: orca.State, params, steps: int, ckpt: int):
        # the step's scalar parameters travel by value to the kernels, so tau
        # is read on the host once per rollout: no synchronisation when it
        # is a host tensor (its gradient is then returned on the host), one
        # when it lives on the device
        p = dataclasses.replace(params, time_horizon=float(tau.detach().reshape(()).item()),
                                pref_is_goal=0)
        ctx.tau_device = tau.device
        n = state0.n
        st = state0.clone()
        st.pref_x = v_pref_x.detach().contiguous().clone()
        st.pref_y = v_pref_y.detach().contiguous().clone()
        nxt = st.clone()
        ws = orca.Workspace(n)
        ckpts = []
        for t in range(steps):
            if t % ckpt == 0:
                ckpts.append(tuple(getattr(st, k).clone() for k in ("px", "py", "vx", "vy")))
            orca.step(st, p, ws, out=nxt)
            st, nxt = nxt, st
        ctx.p = p
        ctx.steps = steps
        ctx.ckpt = ckpt
        ctx.ckpts = ckpts
        ctx.base = st.clone()  # pref/radius/speed/class arrays for the replays
        return st.px.clone(), st.py.clone()

    @staticmethod
    def backward(ctx, g_px, g_py):
        p, steps, ckpt = ctx.p, ctx.steps, ctx.ckpt
        base = ctx.base
        n = base.n
        dev = base.px.device
        gpx = (g_px if g_px is not None else torch.zeros(n, device=dev)).contiguous().clone()
        gpy = (g_py if g_py is not None else torch.zeros(n, device=dev)).contiguous().clone()
        gvx = torch.zeros(n, dtype=torch.float32, device=dev)
        gvy = torch.zeros(n, dtype=torch.float32, device=dev)
        g_prx = torch.zeros(n, dtype=torch.float32, device=dev)
        g_pry = torch.zeros(n, dtype=torch.float32, device=dev)
        g_tau = torch.zeros(1, dtype=torch.float32, device=dev)
        ws = orca.Workspace(n)
        wsb = orca.Workspace(n, backward=True)
        n_seg = len(ctx.ckpts)
        # each replayed segment must end exactly where the forward pass went
        # (the next checkpoint, or the final state): the gradient then belongs
        # to the forward trajectory.  Mismatches are counted on the device and
        # checked once at the end.
        mismatch = torch.zeros((), dtype=torch.int64, device=dev)
        ends = [tuple(getattr(base, k) for k in ("px", "py", "vx", "vy"))]
        for seg in range(n_seg - 1, -1, -1):
            t0 = seg * ckpt
            t1 = min(t0 + ckpt, steps)
            st = base.clone()
            for k, v in zip(("px", "py", "vx", "vy"), ctx.ckpts[seg]):
                getattr(st, k).copy_(v)
            states = []
            nxt = st.clone()
            for t in range(t0, t1):
                states.append(st.clone())
                orca.step(st, p, ws, out=nxt)
                st, nxt = nxt, st
            want = ends[0] if seg == n_seg - 1 else ctx.ckpts[seg + 1]
            for k, v in zip(("px", "py", "vx", "vy"), want):
                mismatch += (getattr(st, k) != v).sum()
            for t in range(t1 - 1, t0 - 1, -1):
                orca.step_backward(states[t - t0], p, wsb, gpx, gpy, gvx, gvy, g_prx, g_pry,
                                   g_tau, out=(gpx, gpy, gvx, gvy))
        if int(mismatch.item()) != 0:
            raise RuntimeError("rollout backward: a replayed segment left the forward trajectory "
                               f"({int(mismatch.item())} differing values)")
        return g_prx, g_pry, g_tau.reshape(()).to(ctx.tau_device), None, None, None, None


def rollout(v_pref_x: torch.Tensor, v_pref_y: torch.Tensor, tau: torch.Tensor,
            state0: orca.State, params, steps: int = 50, ckpt: int = 10) -> Tuple[torch.Tensor, torch.Tensor]:
    """Final positions after `steps` ORCA steps; differentiable w.r.t. the
    per-agent desired velocities and the shared look-ahead tau."""
    return Rollout.apply(v_pref_x, v_pref_y, tau, state0, params, steps, ckpt)


def trajectory_loss(px: torch.Tensor, py: torch.Tensor, target_x: torch.Tensor,
                    target_y: torch.Tensor) -> torch.Tensor:
    """Mean squared distance of the final positions to their targets."""
    return ((px - target_x) ** 2 + (py - target_y) ** 2).mean()


class RolloutGraph:
    """A rollout captured in two HIP graphs (forward; backward with its
    segment replays) for one initial state, step count, checkpoint interval
    and tau, so that a replay takes new desired velocities and cotangents
    without re-launching the ~10 kernels of every step one by one.  The
    step's scalar parameters (tau among them) are baked into the graphs.

    The arithmetic is the eager Rollout's, kernel for kernel, so replays
    equal it bit for bit.  The check that every replayed segment ends where
    the forward went runs eagerly after the backward replay (a reduction
    inside the graph could record memory-set nodes)."""

    def __init__(self, state0: orca.State, params, tau: float, steps: int = 50, ckpt: int = 10):
        self.p = dataclasses.replace(params, time_horizon=float(tau), pref_is_goal=0)
        self.steps, self.ckpt = steps, ckpt
        n = self.n = state0.n
        dev = state0.px.device
        f32 = dict(dtype=torch.float32, device=dev)
        # static inputs
        self.base = state0.clone()
        self.v_pref_x = torch.zeros(n, **f32)
        self.v_pref_y = torch.zeros(n, **f32)
        self.g_px = torch.zeros(n, **f32)
        self.g_py = torch.zeros(n, **f32)
        # static working state, checkpoints and outputs
        self.st = state0.clone()
        self.nxt = state0.clone()
        self.n_seg = (steps + ckpt - 1) // ckpt
        self.ckpts = [tuple(torch.zeros(n, **f32) for _ in range(4)) for _ in range(self.n_seg)]
        self.final = tuple(torch.zeros(n, **f32) for _ in range(4))
        self.ends = [tuple(torch.zeros(n, **f32) for _ in range(4)) for _ in range(self.n_seg)]
        self.g_prx = torch.zeros(n, **f32)
        self.g_pry = torch.zeros(n, **f32)
        self.g_tau = torch.zeros(1, **f32)
        self.ws = orca.Workspace(n)
        self.wsb = orca.Workspace(n, backward=True)
        self.seg = [(self.base.clone(), self.base.clone()) for _ in range(ckpt)]
        self.cot = tuple(torch.zeros(n, **f32) for _ in range(4))
        # one eager pass of each part loads the code objects, then capture
        self._forward()
        self._backward()
        torch.cuda.synchronize()
        self.g_fwd = self._capture(self._forward)
        self.g_bwd = self._capture(self._backward)

    @staticmethod
    def _capture(fn):
        stream = torch.cuda.Stream()
        stream.wait_stream(torch.cuda.current_stream())
        graph = torch.cuda.CUDAGraph()
        with torch.cuda.stream(stream):
            with torch.cuda.graph(graph, stream=stream):
                fn()
        torch.cuda.synchronize()
        return graph

    def _forward(self):
        st, nxt = self.st, self.nxt
        for k in ("px", "py", "vx", "vy"):
            getattr(st, k).copy_(getattr(self.base, k))
        st.pref_x.copy_(self.v_pref_x)
        st.pref_y.copy_(self.v_pref_y)
        nxt.pref_x.copy_(self.v_pref_x)
        nxt.pref_y.copy_(self.v_pref_y)
        for t in range(self.steps):
            if t % self.ckpt == 0:
                for dst, k in zip(self.ckpts[t // self.ckpt], ("px", "py", "vx", "vy")):
                    dst.copy_(getattr(st, k))
            orca.step(st, self.p, self.ws, out=nxt)
            st, nxt = nxt, st
        for dst, k in zip(self.final, ("px", "py", "vx", "vy")):
            dst.copy_(getattr(st, k))

    def _backward(self):
        gpx, gpy, gvx, gvy = self.cot
        gpx.copy_(self.g_px)
        gpy.copy_(self.g_py)
        gvx.fill_(0.0)
        gvy.fill_(0.0)
        self.g_prx.fill_(0.0)
        self.g_pry.fill_(0.0)
        self.g_tau.fill_(0.0)
        for seg in range(self.n_seg - 1, -1, -1):
            t0 = seg * self.ckpt
            t1 = min(t0 + self.ckpt, self.steps)
            states = []
            for t in range(t0, t1):
                s, nx = self.seg[t - t0]
                if t == t0:
                    for k, v in zip(("px", "py", "vx", "vy"), self.ckpts[seg]):
                        getattr(s, k).copy_(v)
                for k in ("pref_x", "pref_y"):
                    getattr(s, k).copy_(getattr(self.st, k))
                if t + 1 < t1:
                    orca.step(s, self.p, self.ws, out=self.seg[t - t0 + 1][0])
                else:
                    orca.step(s, self.p, self.ws, out=nx)
                    for dst, k in zip(self.ends[seg], ("px", "py", "vx", "vy")):
                        dst.copy_(getattr(nx, k))
                states.append(s)
            for t in range(t1 - 1, t0 - 1, -1):
                orca.step_backward(states[t - t0], self.p, self.wsb, gpx, gpy, gvx, gvy,
                                   self.g_prx, self.g_pry, self.g_tau, out=(gpx, gpy, gvx, gvy))

    def forward(self, v_pref_x: torch.Tensor, v_pref_y: torch.Tensor):
        """Final positions for these desired velocities (static outputs)."""
        self.v_pref_x.copy_(v_pref_x)
        self.v_pref_y.copy_(v_pref_y)
        self.g_fwd.replay()
        return self.final[0], self.final[1]

    def backward(self, g_px: torch.Tensor, g_py: torch.Tensor):
        """Gradients (v_pref_x, v_pref_y, tau) of <g_px, px> + <g_py, py>
        for the last forward replay (static outputs)."""
        self.g_px.copy_(g_px)
        self.g_py.copy_(g_py)
        self.g_bwd.replay()
        bad = 0
        for seg in range(self.n_seg):
            want = self.final if seg == self.n_seg - 1 else self.ckpts[seg + 1]
            for a, b in zip(self.ends[seg], want):
                bad += int((a != b).sum().item())
        if bad:
            raise RuntimeError("rollout graph: a replayed segment left the forward trajectory "
                               f"({bad} differing values)")
        return self.g_prx, self.g_pry, self.g_tau.reshape(())
