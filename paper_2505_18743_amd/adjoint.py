"""Gradients of point observations of the free surface with respect to the
per-cell Manning coefficients and bed offsets, through the HIP step adjoint
(sw_step_record / sw_vjp_step), as a torch.autograd.Function with
checkpointed recomputation.

Forward: ``nsteps`` fixed-dt steps from ``state0``; the state is kept every
``checkpoint_every`` steps; returns the free surface at the points after each
step, [nsteps, G].  Backward: segments are walked in reverse; each is
recomputed from its checkpoint with its stage states recorded on the device,
then its steps are reversed with sw_vjp_step, adding the observation adjoint of
each step to the state adjoint before that step's reverse pass.
"""
from __future__ import annotations

import numpy as np
import torch


class PointObservation:
    """value_g = sum_j phi[g, j] zeta[cell[g], j] on a context's nodal layout."""

    def __init__(self, cells, phi, n_dofs_per_cell, device):
        cells = np.asarray(cells, dtype=np.int64)
        self.G = len(cells)
        self.np_ = n_dofs_per_cell
        self.cells = torch.as_tensor(cells, device=device)
        self.phi = torch.as_tensor(np.asarray(phi, dtype=np.float64), device=device)
        # adjoint scatter without colliding indices: gauges grouped by cell
        uniq, inv = np.unique(cells, return_inverse=True)
        self.ucells = torch.as_tensor(uniq, device=device)
        grp = np.zeros((len(uniq), self.G))
        grp[inv, np.arange(self.G)] = 1.0
        self.group = torch.as_tensor(grp, device=device)

    def values(self, zeta):
        return (zeta.view(-1, self.np_)[self.cells] * self.phi).sum(1)

    def add_adjoint(self, zeta_bar, gvals):
        contrib = self.group @ (gvals[:, None] * self.phi)          # [U, NP]
        zeta_bar.view(-1, self.np_).index_add_(0, self.ucells, contrib)


class ObservedRun(torch.autograd.Function):
    @staticmethod
    def forward(ctx, nman, dbed, solver, state0, t0, dt, nsteps, obs, checkpoint_every):
        solver.set_manning(nman.detach())
        solver.set_bed_offset(dbed.detach())
        solver.set_state(*[x.detach() for x in state0[:3]])
        solver.set_time(t0)
        out = torch.empty(nsteps, obs.G, dtype=torch.float64, device=solver.dev)
        ckpt = {}
        for n in range(nsteps):
            if n % checkpoint_every == 0:
                ckpt[n] = torch.stack(solver.get_state()[:3], 0)
            solver.step(dt)
            out[n] = obs.values(solver.get_state()[0])
        ctx.solver, ctx.t0, ctx.dt, ctx.nsteps, ctx.obs, ctx.C = solver, t0, dt, nsteps, obs, checkpoint_every
        ctx.ckpt = ckpt
        return out

    @staticmethod
    def backward(ctx, gout):
        s, dt, C, obs = ctx.solver, ctx.dt, ctx.C, ctx.obs
        KN = s.n_dofs
        ns = s.n_stages()
        sbar = torch.zeros(3, KN, dtype=torch.float64, device=s.dev)
        nbar = torch.zeros(s.n_cells, dtype=torch.float64, device=s.dev)
        dbar = torch.zeros(s.n_cells, dtype=torch.float64, device=s.dev)
        stages = torch.empty(min(C, ctx.nsteps), ns, 3, KN, dtype=torch.float64, device=s.dev)
        gout = gout.contiguous()
        for start in reversed(range(0, ctx.nsteps, C)):
            seg = min(C, ctx.nsteps - start)
            st = ctx.ckpt[start]
            s.set_state(st[0], st[1], st[2])
            s.set_time(ctx.t0 + start * dt)
            for i in range(seg):
                s.step_record(dt, stages[i])
            for i in reversed(range(seg)):
                n = start + i
                obs.add_adjoint(sbar[0], gout[n])
                s.vjp_step(stages[i], ctx.t0 + n * dt, dt, sbar, nbar, dbar)
        ctx.ckpt = None
        # the step adjoint is exact only in the all-wet regime; a stage state
        # outside it is flagged on the device and raises here
        s.sync()
        return nbar, dbar, None, None, None, None, None, None, None


def observed_run(solver, nman, dbed, state0, t0, dt, nsteps, obs, checkpoint_every=20):
    """Differentiable free-surface observations [nsteps, G] (see module doc)."""
    return ObservedRun.apply(nman, dbed, solver, state0, t0, dt, nsteps, obs, checkpoint_every)
