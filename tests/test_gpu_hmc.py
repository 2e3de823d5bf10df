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
