"""GPU parity for the reaction-field Coulomb variant (Eq. 8): forces, energies
and virial against the FP64 oracle, dynamics, and its argument checks.
Bars as for the Ewald path (1e-5 relative RMS forces, 1e-6 energies)."""
import math

import numpy as np
import pytest

import synth
from oracle import forcefield
from helpers import announce, gpu_context, rel_rms

pytestmark = pytest.mark.gpu

F_TOL = 1e-5
E_TOL = 1e-6


def rf_system(name, eps_s):
    s = synth.config_system(name)
    s.rf_epsilon = eps_s
    s.ewald_delta = 0.0
    s.pme_grid = (0, 0, 0)
    return s


@pytest.mark.parametrize("options", [0, 1], ids=["full", "half"])
@pytest.mark.parametrize("eps_s", [78.5, math.inf], ids=["eps78", "conducting"])
@pytest.mark.parametrize("name", ["water375", "water9k"])
def test_reaction_field_parity(name, eps_s, options):
    import torch
    s = rf_system(name, eps_s)
    announce(f"reaction field {name} eps_s={eps_s} options={options}")
    with gpu_context(s, options=options) as (mdx, ctx, t):
        mdx.build_neighbors(ctx, t["pos"])
        mdx.compute_nonbonded(ctx, t["pos"], t["force"], t["e_nb"])
        W = torch.zeros(9, dtype=torch.float64, device="cuda:0")
        f2 = torch.zeros_like(t["force"])
        mdx.compute_nonbonded(ctx, t["pos"], f2, None, W)
        torch.cuda.synchronize()
        assert mdx.get_status(ctx) == 0
        F = t["force"].cpu().numpy()
        E = t["e_nb"].cpu().numpy()
        W = W.cpu().numpy().reshape(3, 3)
    ref = forcefield.nonbonded_terms(s)
    assert rel_rms(F, ref["F"]) < F_TOL
    Eref = ref["E"]
    scale = abs(Eref.sum())
    assert Eref[2] == 0.0 and Eref[3] == 0.0
    for k in range(6):
        assert abs(E[k] - Eref[k]) <= E_TOL * max(abs(Eref[k]), scale), (k, E[k], Eref[k])
    wmax = np.abs(np.diag(ref["W"])).max()
    assert np.abs(W - ref["W"]).max() <= 1e-5 * wmax


def test_reaction_field_dynamics_conserve_energy():
    # conducting limit: the pair energy and force both vanish at r_c, so
    # velocity Verlet keeps the total energy to the integration error
    import torch
    s = rf_system("water9k", math.inf)
    n_steps = 60
    announce("reaction field water9k dynamics")
    with gpu_context(s) as (mdx, ctx, t):
        mdx.build_neighbors(ctx, t["pos"])
        mdx.compute_nonbonded(ctx, t["pos"], t["force"])
        en = torch.zeros((n_steps, mdx.MDX_N_ENERGY), dtype=torch.float64, device="cuda:0")
        mdx.integrate_step(ctx, t["pos"], t["vel"], t["force"], n_steps, 0.5, en)
        torch.cuda.synchronize()
        assert mdx.get_status(ctx) == 0
        E = en.cpu().numpy()
        F_end = t["force"].cpu().numpy().astype(np.float64)
        pos = t["pos"].cpu().numpy()
    assert np.all(E[:, 2] == 0.0) and np.all(E[:, 3] == 0.0) and np.all(E[:, 6] == 0.0)
    etot = E.sum(axis=1)
    assert np.abs(etot - etot[0]).max() < 0.02 * E[:, 7].mean()
    # the force left behind is the oracle's at the final positions
    s2 = s.copy()
    s2.pos = pos
    ref = forcefield.nonbonded_terms(s2)
    assert rel_rms(F_end, ref["F"]) < F_TOL


def test_reaction_field_argument_checks():
    import paper_2503_20541_amd as mdx
    s = rf_system("water375", 78.5)
    for bad in (dict(ewald_delta=5e-4), dict(pme_grid=(16, 16, 16)), dict(rf_epsilon=-1.0),
                dict(rf_epsilon=float("nan"))):
        desc, keep = mdx.desc_from_system(s, **bad)
        with pytest.raises(mdx.MdxError) as e:
            mdx.create(desc)
        assert e.value.code == mdx.MDX_E_INVALID, bad
