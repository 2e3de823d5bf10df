"""A velocity-Verlet trajectory as a differentiable torch function.

    xT, UT = trajectory(sim, x0, v0, eps, sig, t_q, dt)

runs sim.n_steps steps of mdx_integrate_step from (x0, v0) with the per-type
LJ parameters eps, sig and the charges q + t_q * dq, and returns the final
positions unwrapped by the image counters ([3, N] float32) and the final
potential energy (float64 scalar). Its backward runs the library's reverse
pass (mdx_adjoint_begin, then mdx_adjoint_segment per segment from the last
to the first) from checkpoints saved every sim.checkpoint_every steps:
gradients with respect to x0, v0, eps, sig, t_q and dt of whatever loss is
built on (xT, UT). Every step of the forward and of the reverse pass runs in
the library's kernels; this module saves and restores checkpoints and
marshals arguments.
"""
from __future__ import annotations

import numpy as np
import torch

from . import mdx


class Simulation:
    """A context plus what a differentiable run needs: the base charges, the
    charge direction dq, the number of steps and the checkpoint spacing."""

    def __init__(self, system, n_steps: int, checkpoint_every: int = 10, charge_direction=None,
                 device="cuda:0", **desc_overrides):
        self.system = system
        self.n_steps = int(n_steps)
        self.checkpoint_every = int(checkpoint_every)
        self.device = torch.device(device)
        desc, self._keep = mdx.desc_from_system(system, **desc_overrides)
        self.stream = torch.cuda.current_stream(self.device)
        self.ctx = mdx.create(desc, self.stream.cuda_stream)
        self.n = int(system.n_atoms)
        self.n_types = len(system.type_sigma)
        self.q0 = np.asarray(system.charge, np.float32).copy()
        self.dq = (np.zeros(self.n, np.float32) if charge_direction is None
                   else np.asarray(charge_direction, np.float32).copy())
        mdx.set_charge_direction(self.ctx, self.dq)

    def close(self):
        if self.ctx:
            mdx.destroy(self.ctx)
            self.ctx = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def segments(self):
        k, out, done = self.checkpoint_every, [], 0
        while done < self.n_steps:
            out.append(min(k, self.n_steps - done))
            done += out[-1]
        return out

    def set_parameters(self, eps, sig, t_q):
        q = self.q0 + np.float32(float(t_q)) * self.dq
        mdx.set_parameters(self.ctx, sig.detach().cpu().numpy(), eps.detach().cpu().numpy(), q)


class _Trajectory(torch.autograd.Function):
    @staticmethod
    def forward(fctx, sim, x0, v0, eps, sig, t_q, dt):
        dtf = float(dt)
        sim.set_parameters(eps, sig, t_q)
        ctx = sim.ctx
        pos = x0.detach().contiguous().clone()
        vel = v0.detach().contiguous().clone()
        force = torch.zeros_like(pos)
        mdx.reset_images(ctx)
        mdx.build_neighbors(ctx, pos)
        mdx.compute_nonbonded(ctx, pos, force)
        if sim.system.pme_grid[0]:
            mdx.compute_pme(ctx, pos, force)
        saves = []
        for k in sim.segments():
            state = torch.empty(mdx.state_size(ctx), dtype=torch.uint8, device=pos.device)
            mdx.save_state(ctx, state)
            saves.append((k, state, pos.clone(), vel.clone(), force.clone()))
            mdx.integrate_step(ctx, pos, vel, force, k, dtf)
        xT = torch.empty_like(pos)
        mdx.get_unwrapped(ctx, pos, xT)
        e_nb = torch.zeros(6, dtype=torch.float64, device=pos.device)
        e_rec = torch.zeros(1, dtype=torch.float64, device=pos.device)
        scratch = torch.zeros_like(pos)
        mdx.compute_nonbonded(ctx, pos, scratch, e_nb)
        if sim.system.pme_grid[0]:
            mdx.compute_pme(ctx, pos, scratch, e_rec)
        UT = e_nb.sum() + e_rec.sum()
        fctx.sim = sim
        fctx.saves = saves
        fctx.dt = dtf
        fctx.final = (pos, force)
        return xT, UT

    @staticmethod
    def backward(fctx, gx, gU):
        sim = fctx.sim
        ctx = sim.ctx
        pos, force = fctx.final
        dev = pos.device
        gx = (torch.zeros_like(pos) if gx is None else gx.detach().float().contiguous())
        gU = (torch.zeros(1, dtype=torch.float64, device=dev) if gU is None
              else gU.detach().to(torch.float64).reshape(1).contiguous())
        q = torch.empty_like(pos)
        p = torch.empty_like(pos)
        grad = torch.zeros(2 * sim.n_types + 2, dtype=torch.float64, device=dev)
        mdx.adjoint_begin(ctx, pos, force, gx, gU, q, p, grad)
        for s in range(len(fctx.saves) - 1, -1, -1):
            k, state, xs, vs, fs = fctx.saves[s]
            mdx.load_state(ctx, state)
            mdx.adjoint_segment(ctx, xs, vs, fs, k, fctx.dt, s == 0, q, p, grad)
        T = sim.n_types
        return (None, q, p, grad[:T].float(), grad[T:2 * T].float(), grad[2 * T].float(),
                grad[2 * T + 1].float())


def trajectory(sim: Simulation, x0, v0, eps, sig, t_q, dt):
    """(x_T unwrapped, U(x_T)); differentiable in every tensor argument."""
    return _Trajectory.apply(sim, x0, v0, eps, sig, t_q, dt)
