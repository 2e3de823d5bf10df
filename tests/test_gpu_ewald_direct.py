"""GPU parity: the direct reciprocal Ewald sum (mdx_compute_ewald_direct)
against the oracle's direct sum, and against smooth PME at the same alpha."""
import numpy as np
import pytest

import synth
from oracle import ewald, forcefield
from helpers import announce, gpu_context, rel_rms

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("name,n_max", [("water375", 8), ("water375", 3), ("water9k", 5)])
def test_direct_ewald_matches_oracle(name, n_max):
    import torch
    s = synth.config_system(name)
    announce(f"direct Ewald {name} n_max={n_max}")
    with gpu_context(s) as (mdx, ctx, t):
        e = torch.zeros(1, dtype=torch.float64, device="cuda:0")
        mdx.compute_ewald_direct(ctx, t["pos"], t["force"], e, n_max)
        torch.cuda.synchronize()
        F = t["force"].cpu().numpy()
        E = float(e.cpu()[0])
    a = forcefield.alpha(s)
    Eref, Fref = ewald.reciprocal_direct(s.pos.astype(np.float64), s.charge, s.box, a,
                                         s.coulomb_k, n_max)
    assert abs(E - Eref) <= 1e-9 * abs(Eref), (E, Eref)
    assert rel_rms(F, Fref) < 1e-6


def test_direct_ewald_agrees_with_pme_and_accumulates():
    import torch
    s = synth.config_system("water375")
    announce("direct Ewald vs PME water375")
    with gpu_context(s) as (mdx, ctx, t):
        mdx.build_neighbors(ctx, t["pos"])
        e_pme = torch.zeros(1, dtype=torch.float64, device="cuda:0")
        f_pme = torch.zeros_like(t["force"])
        mdx.compute_pme(ctx, t["pos"], f_pme, e_pme)
        e_dir = torch.zeros(1, dtype=torch.float64, device="cuda:0")
        f_dir = torch.full_like(t["force"], 1.0)
        mdx.compute_ewald_direct(ctx, t["pos"], f_dir, e_dir, 10)
        torch.cuda.synchronize()
        f_dir = f_dir.cpu().numpy() - 1.0        # accumulated onto ones
        Ep, Ed = float(e_pme.cpu()[0]), float(e_dir.cpu()[0])
        Fp = f_pme.cpu().numpy()
        with pytest.raises(mdx.MdxError):
            mdx.compute_ewald_direct(ctx, t["pos"], t["force"], None, 0)
    # the two GPU paths differ by the SPME discretisation error of this coarse
    # grid (0.7 % here), exactly as the oracle's SPME and direct sums do
    a = forcefield.alpha(s)
    p64 = s.pos.astype(np.float64)
    E_spme = forcefield.pme_terms(s)["E"]
    E_dir, F_dir_ref = ewald.reciprocal_direct(p64, s.charge, s.box, a, s.coulomb_k, 10)
    assert abs((Ep - Ed) - (E_spme - E_dir)) <= 1e-6 * abs(E_dir), (Ep - Ed, E_spme - E_dir)
    assert rel_rms(f_dir, F_dir_ref) < 1e-6
