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
