"""torch.autograd.Function around the library's hand-written adjoint.

``NuObjective.apply(theta_w, theta0, cavity, nsteps, avg_last, ckpt_every)``
returns J, the mean hot-wall Nusselt number (Eqs. 18-19) over the last
``avg_last`` of ``nsteps`` steps of ``cavity`` started at rest with the
temperature field ``theta0`` and hot-wall profile ``theta_w``.  Its backward
is dmrt_adjoint_backward: recompute from checkpoints plus the adjoint step
kernel on the GPU; the tensors cross the C ABI as host float64 arrays.

A cavity stores one forward run.  When another objective's forward (or a
call that changes the cavity's wall or initial field) has replaced it by
the time this objective's backward runs, the backward first repeats this
objective's forward (the step is deterministic, so it reproduces J bitwise)
and then differentiates it; the cavity is left holding this objective's
wall, initial field and final state.
"""
from __future__ import annotations

import numpy as np
import torch


class NuObjective(torch.autograd.Function):
    @staticmethod
    def forward(ctx, theta_w, theta0, cavity, nsteps, avg_last, ckpt_every=500):
        tw = np.ascontiguousarray(theta_w.detach().to("cpu", torch.float64).numpy())
        t0 = np.ascontiguousarray(theta0.detach().to("cpu", torch.float64).numpy())
        cavity.set_hot_wall(tw)
        cavity.set_theta(t0)
        J = cavity.adjoint_forward(nsteps, avg_last, ckpt_every)
        ctx.cavity = cavity
        ctx.run = (tw, t0, nsteps, avg_last, ckpt_every, J)
        ctx.gen = cavity.adjoint_generation()
        ctx.shapes = (theta_w.shape, theta0.shape)
        ctx.devices = (theta_w.device, theta0.device)
        ctx.dtypes = (theta_w.dtype, theta0.dtype)
        return torch.tensor(J, dtype=torch.float64)

    @staticmethod
    def backward(ctx, grad_out):
        c = ctx.cavity
        if c.adjoint_generation() != ctx.gen:
            tw, t0, nsteps, avg_last, ckpt_every, J = ctx.run
            c.set_hot_wall(tw)
            c.set_theta(t0)
            J2 = c.adjoint_forward(nsteps, avg_last, ckpt_every)
            if J2 != J:
                raise RuntimeError(f"repeated forward gave J = {J2!r}, not {J!r}")
            ctx.gen = c.adjoint_generation()
        gw, g0 = c.adjoint_backward()
        s = float(grad_out)
        # gradients in the inputs' own dtype and device (computed in FP64)
        gw_t = torch.from_numpy(np.ascontiguousarray(gw * s)).reshape(ctx.shapes[0]).to(
            device=ctx.devices[0], dtype=ctx.dtypes[0])
        g0_t = torch.from_numpy(np.ascontiguousarray(g0 * s)).reshape(ctx.shapes[1]).to(
            device=ctx.devices[1], dtype=ctx.dtypes[1])
        return gw_t, g0_t, None, None, None, None


def nu_objective(theta_w, theta0, cavity, nsteps, avg_last, ckpt_every=500):
    return NuObjective.apply(theta_w, theta0, cavity, nsteps, avg_last, ckpt_every)
