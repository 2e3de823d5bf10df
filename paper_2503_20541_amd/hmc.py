"""Differentiable Hamiltonian Monte Carlo tuning (the paper's Sec. IV).

A proposal of Hamiltonian Monte Carlo samples velocities from the
Maxwell-Boltzmann distribution of the current masses, runs velocity Verlet,
and is accepted with probability min(1, exp(-(E' - E)/kT)), E = U + K. The
paper tunes the time step, the trajectory length and the masses by the
gradient of the expected squared jump distance of the positions, weighted
over every step l of the trajectory:

    L_HMC = (1/R) sum_i sum_{l=1}^{L_q} w_l alpha_{i,l} / l |x_{i,l} - x_{i,0}|^2

(R replicas; w_l the folded-normal density N_F(l; mu_L, sigma_L), alpha_{i,l}
the acceptance probability of stopping at step l, L_q the 0.999 quantile of
N_F(mu_L, sigma_L)); the time step is a folded normal N_F(mu_dt, 0.01 mu_dt),
reparameterised as |mu_dt (1 + 0.01 eps)|.

`proposal(sim, x0, v0, m, dt, n)` is the differentiable trajectory: its
outputs are the unwrapped positions, the velocities and the potential energy
of every state 0..n, and its backward runs the library's reverse pass as
one-step segments with each state's loss terms injected between them
(mdx_adjoint_inject), so the gradients reach x0, v0, the masses (through the
dynamics; the sampled velocities and the kinetic energy depend on them in
torch) and dt. Every step of the forward and reverse pass runs in the
library's kernels; this module assembles the objective from their outputs.
`HMCTuner` runs the tuning: gradient steps on mu_dt, mu_L and a mass
repartitioning with the total mass fixed, and the chains' Metropolis moves.
"""
from __future__ import annotations

import math

import torch

from . import mdx


def folded_normal_pdf(x, mu, sigma):
    """N_F(x; mu, sigma), the density of |N(mu, sigma^2)| on x > 0."""
    c = 1.0 / math.sqrt(2.0 * math.pi * sigma * sigma)
    return c * (torch.exp(-(x - mu) ** 2 / (2 * sigma * sigma)) +
                torch.exp(-(x + mu) ** 2 / (2 * sigma * sigma)))


def folded_normal_quantile(mu: float, sigma: float, q: float = 0.999) -> float:
    """x with P(|N(mu, sigma^2)| <= x) = q, by bisection."""
    cdf = lambda x: 0.5 * (math.erf((x - mu) / (sigma * math.sqrt(2))) +
                           math.erf((x + mu) / (sigma * math.sqrt(2))))
    lo, hi = 0.0, abs(mu) + 20.0 * sigma
    for _ in range(200):
        mid = 0.5 * (lo + hi)
        if cdf(mid) < q:
            lo = mid
        else:
            hi = mid
    return hi


class _Proposal(torch.autograd.Function):
    @staticmethod
    def forward(fctx, sim, x0, v0, m, dt, n_steps):
        ctx = sim.ctx
        dtf = float(dt)
        mdx.set_masses(ctx, m.detach().cpu().numpy())
        dev = x0.device
        pos = x0.detach().contiguous().clone()
        vel = v0.detach().contiguous().clone()
        force = torch.zeros_like(pos)
        X = torch.empty((n_steps + 1,) + tuple(pos.shape), dtype=pos.dtype, device=dev)
        V = torch.empty_like(X)
        E = torch.zeros((n_steps + 1, mdx.MDX_N_ENERGY), dtype=torch.float64, device=dev)
        mdx.reset_images(ctx)
        mdx.build_neighbors(ctx, pos)
        mdx.compute_nonbonded(ctx, pos, force, E[0, :6])
        if sim.system.pme_grid[0]:
            mdx.compute_pme(ctx, pos, force, E[0, 6:7])
        X[0] = pos
        V[0] = vel
        saves = []
        for k in range(n_steps):
            state = torch.empty(mdx.state_size(ctx), dtype=torch.uint8, device=dev)
            mdx.save_state(ctx, state)
            saves.append((state, pos.clone(), vel.clone(), force.clone()))
            mdx.integrate_step(ctx, pos, vel, force, 1, dtf, E[k + 1])
            mdx.get_unwrapped(ctx, pos, X[k + 1])
            V[k + 1] = vel
        saves.append((None, pos.clone(), vel.clone(), force.clone()))
        fctx.sim = sim
        fctx.saves = saves
        fctx.dt = dtf
        U = E[:, :7].sum(dim=1)          # potential energy of every state
        return X, V, U

    @staticmethod
    def backward(fctx, gX, gV, gU):
        sim = fctx.sim
        ctx = sim.ctx
        saves = fctx.saves
        n_steps = len(saves) - 1
        x_end = saves[-1][1]
        dev = x_end.device
        q = torch.zeros_like(x_end)
        p = torch.zeros_like(x_end)
        grad = torch.zeros(2 * sim.n_types + 2, dtype=torch.float64, device=dev)
        gmass = torch.zeros(sim.n, dtype=torch.float64, device=dev)
        gX = (torch.zeros((n_steps + 1,) + tuple(x_end.shape), dtype=x_end.dtype, device=dev)
              if gX is None else gX.detach().float().contiguous())
        gV = None if gV is None else gV.detach().float().contiguous()
        gU = None if gU is None else gU.detach().to(torch.float64).contiguous()

        def inject(k):
            f = saves[k][3]
            mdx.adjoint_inject(ctx, f, gX[k], None if gV is None else gV[k],
                               None if gU is None else gU[k:k + 1], q, p)

        for k in range(n_steps, 0, -1):
            inject(k)
            state, xs, vs, fs = saves[k - 1]
            mdx.load_state(ctx, state)
            mdx.adjoint_segment(ctx, xs, vs, fs, 1, fctx.dt, True, q, p, grad, last=True,
                                grad_mass=gmass)
        inject(0)
        T = sim.n_types
        return None, q, p, gmass.float(), grad[2 * T + 1].float(), None


def proposal(sim, x0, v0, m, dt, n_steps: int):
    """(X [n+1, 3, N] unwrapped positions, V [n+1, 3, N], U [n+1] float64)."""
    return _Proposal.apply(sim, x0, v0, m, dt, int(n_steps))


def esjd_loss(sims, x0s, m, mu_dt, mu_L, xi_v, xi_dt, kT, sigma_dt_rel=0.01, sigma_L=1.0):
    """The step-weighted ESJD objective L_HMC over the replicas `sims` from
    positions x0s (one [3, N] tensor each). m: per-atom masses [N]; mu_dt,
    mu_L: scalar tensors; xi_v [R][3, N] and xi_dt [R]: the standard normals
    the proposals draw (velocities v0 = sqrt(kT accel / m) xi_v, time step
    |mu_dt (1 + sigma_dt_rel xi_dt)|). Returns (loss, per-replica details)."""
    accel = float(sims[0].system.accel)
    L_q = int(math.ceil(folded_normal_quantile(float(mu_L.detach()), sigma_L)))
    ell = torch.arange(1, L_q + 1, dtype=torch.float64, device=m.device)
    w = folded_normal_pdf(ell, mu_L.double(), sigma_L)
    total = 0.0
    info = []
    for i, sim in enumerate(sims):
        v0 = torch.sqrt(kT * accel / m)[None, :] * xi_v[i]
        dt = torch.abs(mu_dt * (1.0 + sigma_dt_rel * xi_dt[i]))
        X, V, U = proposal(sim, x0s[i], v0, m, dt, L_q)
        K = 0.5 * (m.double()[None, None, :] * V.double() ** 2).sum(dim=(1, 2)) / accel
        Etot = U + K
        alpha = torch.clamp(torch.exp(-(Etot[1:] - Etot[0]) / kT), max=1.0)
        jump = ((X[1:].double() - X[0].double()) ** 2).sum(dim=(1, 2))
        total = total + (w * alpha / ell * jump).sum()
        info.append(dict(alpha=alpha.detach(), jump=jump.detach(), dt=float(dt.detach()),
                         positions=X.detach()))
    return total / len(sims), dict(L_q=L_q, replicas=info)


class HMCTuner:
    """Tunes the HMC proposal by gradient ascent on L_HMC (Sec. IV).

    R chains of `system` (one library context each) start from its
    positions. Each iteration draws the chains' velocity and time-step
    normals from a seeded generator and evaluates L_HMC and its gradient with
    respect to mu_dt, mu_L and one log-scale per mass group: m_i = m0_i
    exp(theta_g(i)), rescaled so that the total mass stays that of m0 (a
    change of the total mass is a change of the time step). It then takes an
    Adam step towards a larger L_HMC and moves every chain. The proposal is
    the state after l steps, l drawn from the weights w_l of L_HMC (the folded
    normal N_F(mu_L, sigma_L) at l = 1..L_q, normalised), accepted with its
    probability alpha_{i,l}. The chains run one after another, each on its own
    context; all force and reverse-pass work runs in the library's kernels.
    """

    def __init__(self, system, n_chains: int, kT: float, mu_dt: float, mu_L: float, mass_groups,
                 lr=(0.01, 0.2, 0.01), seed: int = 0, device="cuda:0"):
        import numpy as np
        from .trajectory import Simulation
        self.dev = torch.device(device)
        self.sims = [Simulation(system, 1, 1, device=device) for _ in range(n_chains)]
        self.n = int(system.n_atoms)
        self.kT = float(kT)
        self.box = torch.as_tensor(np.asarray(system.box, np.float32), device=self.dev)[:, None]
        self.x = [torch.from_numpy(np.asarray(system.pos, np.float32).copy()).to(self.dev)
                  for _ in range(n_chains)]
        self.m0 = torch.from_numpy(np.asarray(system.mass, np.float64)).to(self.dev)
        self.groups = torch.as_tensor(np.asarray(mass_groups), dtype=torch.long, device=self.dev)
        n_groups = int(self.groups.max()) + 1
        f64 = dict(dtype=torch.float64, device=self.dev)
        self.mu_dt = torch.tensor(float(mu_dt), requires_grad=True, **f64)
        self.mu_L = torch.tensor(float(mu_L), requires_grad=True, **f64)
        self.theta = torch.zeros(n_groups, requires_grad=True, **f64)
        self.opt = torch.optim.Adam([{"params": [self.mu_dt], "lr": lr[0]},
                                     {"params": [self.mu_L], "lr": lr[1]},
                                     {"params": [self.theta], "lr": lr[2]}])
        self.rng = np.random.Generator(np.random.PCG64(seed))

    def masses(self):
        """Per-atom masses (float64, differentiable in theta), total fixed."""
        m = self.m0 * torch.exp(self.theta[self.groups])
        return m * (self.m0.sum() / m.sum())

    def _wrap(self, x):
        w = torch.remainder(x, self.box)
        return torch.where(w >= self.box, w - self.box, w).contiguous()

    def step(self):
        """One iteration; returns the objective before the update, the
        parameters after it and the chains' acceptances."""
        R = len(self.sims)
        xi_v = [torch.from_numpy(self.rng.standard_normal((3, self.n)).astype("float32"))
                .to(self.dev) for _ in range(R)]
        xi_dt = [float(z) for z in self.rng.standard_normal(R)]
        m = self.masses()
        mu_L0 = float(self.mu_L.detach())
        loss, info = esjd_loss(self.sims, self.x, m.float(), self.mu_dt, self.mu_L, xi_v, xi_dt,
                               self.kT)
        self.opt.zero_grad()
        (-loss).backward()
        self.opt.step()
        with torch.no_grad():
            self.mu_dt.clamp_(min=1e-3)
            self.mu_L.clamp_(min=1.0)
        # chain moves: l from the weights of L_HMC, accepted with alpha_{i,l}
        L_q = info["L_q"]
        ell = torch.arange(1, L_q + 1, dtype=torch.float64)
        w = folded_normal_pdf(ell, mu_L0, 1.0).numpy()
        w = w / w.sum()
        accepted = []
        for i, r in enumerate(info["replicas"]):
            l = int(self.rng.choice(L_q, p=w)) + 1
            ok = bool(self.rng.random() < float(r["alpha"][l - 1]))
            if ok:
                self.x[i] = self._wrap(r["positions"][l])
            accepted.append(ok)
        return dict(loss=float(loss.detach()), mu_dt=float(self.mu_dt.detach()),
                    mu_L=float(self.mu_L.detach()),
                    group_masses=self.group_masses(), acceptance=sum(accepted) / R, L_q=L_q)

    def group_masses(self):
        """The current mass of one atom of each group (the first of the group)."""
        m = self.masses().detach()
        out = []
        for g in range(int(self.groups.max()) + 1):
            idx = torch.nonzero(self.groups == g)[0, 0]
            out.append(float(m[idx]))
        return out

    def close(self):
        for s in self.sims:
            s.close()
