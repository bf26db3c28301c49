"""Differentiable rollouts of the MHD step for torch.autograd.

`Rollout` advances (cons, bface) by a fixed number of steps of a fixed dt
with the library's step and, in backward, runs the library's hand-written
reverse mode (athmhd_step_vjp) step by step from the last step to the first.
Memory follows step checkpointing: the forward pass keeps the state at the
start of every segment of `seg` steps (ceil(nsteps / ncheck) with ncheck
checkpoints, sqrt(nsteps) by default); backward recomputes the states inside
one segment at a time from its checkpoint (keeping each step's stage inputs,
so the reverse steps do not recompute them), so at most ncheck + seg states
(and their stage inputs) are held.  `Prim2Cons` is prim -> cons with its reverse mode (athmhd_prim2cons_vjp),
so gradients can be taken with respect to primitive variables.

Both functions only sequence library calls: every arithmetic step runs in
the HIP kernels of libathmhd.
"""
from __future__ import annotations

import math

import torch


class Rollout(torch.autograd.Function):
    """(cons_0, bface_0) -> (cons_N, bface_N) after nsteps steps of size dt.

    apply(cons0, bface0, solver, dt, nsteps, ncheck=None)"""

    @staticmethod
    def forward(ctx, cons0, bface0, solver, dt, nsteps, ncheck=None):
        nsteps = int(nsteps)
        if ncheck is None:
            ncheck = max(1, int(math.isqrt(max(nsteps, 1))))
        seg = max(1, -(-nsteps // int(ncheck)))
        c = cons0.detach().clone()
        b = bface0.detach().clone()
        checkpoints = []
        for s in range(nsteps):
            if s % seg == 0:
                checkpoints.append((s, c.clone(), b.clone()))
            solver.step(c, b, dt)
        ctx.solver, ctx.dt, ctx.nsteps, ctx.seg = solver, float(dt), nsteps, seg
        ctx.checkpoints = checkpoints
        return c, b

    @staticmethod
    def backward(ctx, g_cons, g_bface):
        solver, dt, seg = ctx.solver, ctx.dt, ctx.seg
        like_c, like_b = ctx.checkpoints[0][1], ctx.checkpoints[0][2]
        gc = torch.zeros_like(like_c) if g_cons is None else g_cons.detach().clone().contiguous()
        gb = torch.zeros_like(like_b) if g_bface is None else g_bface.detach().clone().contiguous()
        for s0, c0, b0 in reversed(ctx.checkpoints):
            s1 = min(s0 + seg, ctx.nsteps)
            # recompute the segment, keeping every step's start state and its
            # stage inputs (so the reverse step does not recompute them)
            states = []
            c, b = c0.clone(), b0.clone()
            for q in range(s0, s1):
                cs, bs = c.clone(), b.clone()
                st = None
                if q < s1 - 1:  # the last step's stages are recomputed by step_vjp
                    if solver.extra_stages:
                        st = solver.stages_like(c)
                        solver.step_stages(c, b, dt, st)
                    else:
                        solver.step(c, b, dt)
                states.append((cs, bs, st))
            for cs, bs, st in reversed(states):
                solver.step_vjp(cs, bs, dt, gc, gb, out_cons=gc, out_bface=gb, stages=st)
            del states
        ctx.checkpoints = None
        return gc, gb, None, None, None, None


class Prim2Cons(torch.autograd.Function):
    """cons = prim2cons(prim, bface); apply(prim, bface, solver)."""

    @staticmethod
    def forward(ctx, prim, bface, solver):
        ctx.save_for_backward(prim, bface)
        ctx.solver = solver
        return solver.prim2cons(prim.detach(), bface.detach())

    @staticmethod
    def backward(ctx, g_cons):
        prim, bface = ctx.saved_tensors
        g_cons = g_cons.detach().contiguous()
        g_bface = torch.zeros_like(bface)
        g_prim = ctx.solver.prim2cons_vjp(prim.detach(), bface.detach(), g_cons, g_bface)
        return g_prim, g_bface, None
