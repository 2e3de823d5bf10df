"""GPU: the step-weighted ESJD objective of Hamiltonian Monte Carlo tuning
(paper_2503_20541_amd.hmc over mdx_integrate_step, mdx_adjoint_segment and
mdx_adjoint_inject) and its gradients with respect to the mean time step,
the mean trajectory length and the masses against the FP64 oracle
(oracle/hmc.py) and the closed form of free particles."""

import numpy as np
import pytest

import synth
from oracle import adjoint, hmc as ohmc
from helpers import announce

pytestmark = pytest.mark.gpu

KT = 0.0019872041 * 300.0


def _gpu(s, x0s, xi_v, xi_dt, mu_dt, mu_L, kT, mdir):
    import torch
    from paper_2503_20541_amd import hmc, trajectory as tj
    dev = torch.device("cuda:0")
    sims = [tj.Simulation(s, 1, 1) for _ in x0s]
    try:
        m = torch.from_numpy(s.mass.astype(np.float32)).to(dev).requires_grad_(True)
        mdt = torch.tensor(mu_dt, dtype=torch.float64, device=dev, requires_grad=True)
        mL = torch.tensor(mu_L, dtype=torch.float64, device=dev, requires_grad=True)
        X0 = [torch.from_numpy(x.astype(np.float32)).to(dev) for x in x0s]
        XI = [torch.from_numpy(x.astype(np.float32)).to(dev) for x in xi_v]
        loss, info = hmc.esjd_loss(sims, X0, m, mdt, mL, XI, [float(z) for z in xi_dt], kT)
        loss.backward()
        torch.cuda.synchronize()
        flags = [hmc.mdx.get_status(sim.ctx) for sim in sims]
        return dict(loss=float(loss.detach()), mu_dt=float(mdt.grad), mu_L=float(mL.grad),
                    mass_dir=float((m.grad.double().cpu().numpy() * mdir).sum()),
                    L_q=info["L_q"], flags=flags,
                    alpha=[r["alpha"].cpu().numpy() for r in info["replicas"]])
    finally:
        for sim in sims:
            sim.close()


@pytest.mark.parametrize("mu_dt", [1.0, 2.0])
def test_water_esjd_gradients_match_the_fp64_oracle(mu_dt):
    s = synth.config_system("water375")
    rng = np.random.default_rng(5)
    R, mu_L = 2, 5.0
    xi_v = [rng.standard_normal((3, s.n_atoms)) for _ in range(R)]
    xi_dt = rng.standard_normal(R)
    x0s = [s.pos.astype(np.float64) for _ in range(R)]
    # repartitioning: one unit from O to each of its H (total mass fixed)
    mdir = np.where(s.atom_type == 0, -2.0, 1.0)
    announce(f"hmc esjd water375 R={R} mu_dt={mu_dt} mu_L={mu_L}")
    g = _gpu(s, x0s, xi_v, xi_dt, mu_dt, mu_L, KT, mdir)
    assert g["flags"] == [0] * R
    # the oracle draws the same velocities from the float32 normals the GPU got
    xi32 = [x.astype(np.float32).astype(np.float64) for x in xi_v]
    ff = adjoint.ForceField(s)
    ref = ohmc.gradients(ff, x0s, s.mass.astype(np.float64), mu_dt, mu_L, xi32, xi_dt, KT,
                         mdir)
    assert g["L_q"] == ref["L_q"]
    # scales: the derivative of the objective when every proposal is accepted
    # (dL/dmu_dt = 2 L / mu_dt; the mass direction moves |L| / m per unit),
    # against which the acceptance terms cancel
    scale = {"loss": abs(ref["loss"]), "mu_L": abs(ref["mu_L"]),
             "mu_dt": max(abs(ref["mu_dt"]), 2 * ref["loss"] / mu_dt),
             "mass_dir": max(abs(ref["mass_dir"]), ref["loss"] / float(s.mass.min()))}
    for k in scale:
        print(f"{k}: gpu {g[k]:.9g} oracle {ref[k]:.9g} "
              f"err/scale {abs(g[k] - ref[k]) / scale[k]:.2e}", flush=True)
    print("alpha", [np.round(a, 4).tolist() for a in g["alpha"]], flush=True)
    for k in scale:
        assert abs(g[k] - ref[k]) <= 2e-3 * scale[k], (k, g[k], ref[k])


def test_free_particles_closed_form():
    # no forces: alpha = 1 and x_l - x_0 = l dt v0, so the objective and its
    # derivatives are sums over the sampled velocities in closed form
    s = synth.random_box(100, [12.0, 12.0, 12.0], 2.0, 0.5, 3, charged=False)
    s.type_epsilon[:] = 0.0
    R = 3
    rng = np.random.default_rng(2)
    xi_v = [rng.standard_normal((3, s.n_atoms)) for _ in range(R)]
    xi_dt = rng.standard_normal(R)
    x0s = [s.pos.astype(np.float64)] * R
    kT, c = 1.3, float(s.accel)
    mu_dt, mu_L = 0.02, 6.0
    mdir = rng.standard_normal(s.n_atoms)
    announce("hmc esjd free particles closed form")
    g = _gpu(s, x0s, xi_v, xi_dt, mu_dt, mu_L, kT, mdir)
    m = s.mass.astype(np.float32).astype(np.float64)
    ell = np.arange(1, g["L_q"] + 1)
    W = (ohmc.folded_normal_pdf(ell, mu_L, 1.0) * ell).sum()
    a = np.array([1.0 + 0.01 * z for z in xi_dt])
    xi32 = [x.astype(np.float32).astype(np.float64) for x in xi_v]
    S = np.array([(kT * c / m[None, :] * xi * xi).sum() for xi in xi32])
    dS = np.array([(-kT * c / m[None, :] ** 2 * xi * xi * mdir[None, :]).sum() for xi in xi32])
    L = W * (mu_dt ** 2 * a ** 2 * S).sum() / R
    dL_dt = W * (2 * mu_dt * a ** 2 * S).sum() / R
    dL_m = W * (mu_dt ** 2 * a ** 2 * dS).sum() / R
    print(f"loss {g['loss']:.9g} / {L:.9g}  dt {g['mu_dt']:.9g} / {dL_dt:.9g}  "
          f"m {g['mass_dir']:.9g} / {dL_m:.9g}", flush=True)
    assert all(np.all(al == 1.0) for al in g["alpha"])
    # float32 positions: the jumps carry rounding of the positions (~1e-6)
    assert abs(g["loss"] - L) <= 1e-4 * L
    assert abs(g["mu_dt"] - dL_dt) <= 1e-4 * dL_dt
    assert abs(g["mass_dir"] - dL_m) <= 1e-4 * abs(L) / m.min()
    # mu_L enters through the weights only
    dW = (ohmc.folded_normal_pdf(ell, mu_L + 1e-6, 1.0) * ell).sum() - \
         (ohmc.folded_normal_pdf(ell, mu_L - 1e-6, 1.0) * ell).sum()
    assert abs(g["mu_L"] - L / W * dW / 2e-6) <= 1e-4 * abs(L / W * dW / 2e-6)


def _tune(seed, iters=2):
    import torch
    from paper_2503_20541_amd import hmc
    s = synth.config_system("water375")
    groups = np.where(s.atom_type == 0, 0, 1)
    t = hmc.HMCTuner(s, 2, KT, 1.0, 5.0, groups, lr=(0.01, 0.2, 0.01), seed=seed)
    try:
        x_start = [x.clone() for x in t.x]
        out = [t.step() for _ in range(iters)]
        m = t.masses().detach().cpu().numpy()
        x = [xi.cpu().numpy() for xi in t.x]
        flags = [hmc.mdx.get_status(sim.ctx) for sim in t.sims]
        theta = t.theta.detach().cpu().numpy()
        torch.cuda.synchronize()
        return s, out, m, x, [xs.cpu().numpy() for xs in x_start], flags, theta
    finally:
        t.close()


def test_tuner_steps_keep_the_total_mass_and_repeat():
    # two iterations of gradient ascent on L_HMC with the chains' Metropolis
    # moves: the total mass stays fixed, Adam's first steps have the size of
    # the learning rate (the gradients were finite and non-zero), the chains
    # stay in the box, and a second tuner with the same seed repeats the
    # first bit for bit
    announce("hmc tuner water375 two chains two iterations")
    s, out, m, x, x0, flags, theta = _tune(7)
    assert flags == [0, 0]
    m0 = s.mass.astype(np.float64)
    assert abs(m.sum() - m0.sum()) <= 1e-12 * m0.sum()
    first = out[0]
    # Adam's first step is lr g / (|g| + 1e-8)
    assert abs(abs(first["mu_dt"] - 1.0) - 0.01) <= 1e-4 * 0.01
    assert abs(abs(first["mu_L"] - 5.0) - 0.2) <= 1e-4 * 0.2
    assert np.all(np.isfinite(theta)) and np.all(theta != 0.0)
    for xi in x:
        assert np.all((xi >= 0.0) & (xi < s.box[:, None]))
    for r in out:
        assert np.isfinite(r["loss"]) and r["loss"] > 0.0
    s2, out2, m2, x2, _, _, _ = _tune(7)
    assert out2 == out
    assert np.array_equal(m2, m)
    for a, b in zip(x, x2):
        assert np.array_equal(a, b)
