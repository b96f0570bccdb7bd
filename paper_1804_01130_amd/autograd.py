"""Differentiable multi-step advection: a torch.autograd.Function over the C interface.

Forward: n steps of iso_advect_step, keeping the state every ``checkpoint_every`` steps.
Backward: for each segment, last first, the states are recomputed from its checkpoint with
traced steps (keeping the intermediates the adjoint needs), then iso_advect_step_adjoint runs
backwards through the segment.  Memory is one state per checkpoint plus one segment of
intermediates.  Gradients flow to the initial state and to every step's face fluxes; the cell
velocities and time step are held fixed.
"""
from __future__ import annotations

import torch


def _trace_buffers(n_cells, n_faces, device):
    f64 = dict(dtype=torch.float64, device=device)
    return {"vert_alpha": torch.empty(8 * n_cells, **f64), "kind": torch.empty(n_cells, dtype=torch.int32,
                                                                                device=device),
            "iso": torch.empty(n_cells, **f64), "dV": torch.empty(n_faces, **f64),
            "alpha_raw": torch.empty(n_cells, **f64)}


class _Advect(torch.autograd.Function):
    @staticmethod
    def forward(ctx, alpha0, phis, plan, Us, dt, n_steps, every):
        a = alpha0.detach().clone(memory_format=torch.contiguous_format)  # never the caller's storage
        b = torch.empty_like(a)
        checkpoints = {0: a.clone()}
        for n in range(n_steps):
            plan.step(a, phis[n], Us[n], dt, out=b)
            a, b = b, a
            if (n + 1) % every == 0 and n + 1 < n_steps:
                checkpoints[n + 1] = a.clone()
        ctx.plan, ctx.dt, ctx.n_steps, ctx.every = plan, dt, n_steps, every
        ctx.checkpoints = checkpoints
        ctx.save_for_backward(phis, Us)
        return a.clone()

    @staticmethod
    def backward(ctx, abar_out):
        phis, Us = ctx.saved_tensors
        plan, dt, n_steps, every = ctx.plan, ctx.dt, ctx.n_steps, ctx.every
        n_cells, n_faces = plan.mesh.n_cells, plan.mesh.n_faces
        abar = abar_out.detach().contiguous().clone()
        phibar = torch.zeros_like(phis)
        tmp_a = torch.empty_like(abar)
        starts = sorted(ctx.checkpoints)
        for s0 in reversed(starts):
            s1 = min(s0 + every, n_steps)
            # recompute the segment's states and intermediates
            states, traces = [ctx.checkpoints[s0]], []
            a = ctx.checkpoints[s0]
            for n in range(s0, s1):
                tr = _trace_buffers(n_cells, n_faces, abar.device)
                out = torch.empty_like(a)
                plan.step(a, phis[n], Us[n], dt, out=out, trace=tr)
                traces.append(tr)
                states.append(out)
                a = out
            for n in range(s1 - 1, s0 - 1, -1):
                k = n - s0
                plan.adjoint(states[k], phis[n], Us[n], dt, abar, trace=traces[k], alpha_bar=tmp_a,
                             phi_bar=phibar[n])
                abar, tmp_a = tmp_a, abar
        return abar, phibar, None, None, None, None, None


def advect(alpha0, phis, plan, Us, dt, n_steps=None, checkpoint_every=10):
    """alpha after n_steps steps from alpha0 with fluxes phis[n] and velocities Us[n] (device tensors,
    float64, shapes [n_steps, n_faces] and [n_steps, 3 n_cells]); differentiable in alpha0 and phis."""
    n_steps = phis.shape[0] if n_steps is None else n_steps
    return _Advect.apply(alpha0, phis, plan, Us, float(dt), int(n_steps), int(checkpoint_every))
