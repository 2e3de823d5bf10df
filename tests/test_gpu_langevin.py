"""GPU: Langevin dynamics (BAOAB with Philox4x64-10 normals) through
mdx_set_langevin + mdx_integrate_step against the FP64 oracle."""
import numpy as np
import pytest

import synth
from oracle import forcefield, integrate
from helpers import announce, gpu_context

pytestmark = pytest.mark.gpu


def _dev(a, b, box):
    d = a - b
    d -= box[:, None] * np.round(d / box[:, None])
    return float(np.sqrt((d * d).mean()))


def test_langevin_trajectory_tracks_oracle():
    import torch
    s = synth.config_system("lj1k")
    n_steps, kT, gamma, seed = 60, 1.0, 2.0, 20240601
    announce("langevin lj1k 60 steps")
    with gpu_context(s) as (mdx, ctx, t):
        mdx.build_neighbors(ctx, t["pos"])
        mdx.compute_nonbonded(ctx, t["pos"], t["force"])
        mdx.set_langevin(ctx, kT, gamma, seed)
        mdx.integrate_step(ctx, t["pos"], t["vel"], t["force"], n_steps, float(s.dt))
        torch.cuda.synchronize()
        assert mdx.get_status(ctx) == 0
        x_gpu = t["pos"].cpu().numpy().astype(np.float64)
        v_gpu = t["vel"].cpu().numpy().astype(np.float64)
    F = lambda p: forcefield.total_forces_fp64(s, p)[1]
    box = s.box.astype(np.float64)
    ref = integrate.langevin_baoab(s.pos, s.vel, s.mass, s.box, F, float(s.dt), n_steps,
                                   float(s.accel), kT, gamma, seed)
    # how far float32-sized perturbations of the start carry in the oracle
    rng = np.random.default_rng(3)
    p2 = s.pos.astype(np.float64) * (1.0 + 6e-8 * rng.standard_normal(s.pos.shape))
    pert = integrate.langevin_baoab(p2, s.vel, s.mass, s.box, F, float(s.dt), n_steps,
                                    float(s.accel), kT, gamma, seed)
    d_gpu = _dev(x_gpu, ref["pos"], box)
    d_ref = _dev(pert["pos"], ref["pos"], box)
    assert d_gpu <= 10 * max(d_ref, 1e-6), (d_gpu, d_ref)
    assert np.sqrt(((v_gpu - ref["vel"]) ** 2).mean()) < 1e-3 * np.sqrt((ref["vel"] ** 2).mean())


def test_langevin_thermostat_reaches_the_target_temperature():
    # without forces the Ornstein-Uhlenbeck step is exact: from rest the
    # kinetic temperature relaxes to T with no time-step bias
    import torch
    s = synth.random_box(20000, [40.0, 40.0, 40.0], 2.0, 0.5, 9)
    s.type_epsilon[:] = 0.0
    s.charge[:] = 0.0
    s.vel[:] = 0.0
    kT, gamma, dt, n_steps = 1.5, 0.5, 0.02, 400
    announce("langevin free particles thermostat")
    with gpu_context(s) as (mdx, ctx, t):
        mdx.build_neighbors(ctx, t["pos"])
        mdx.compute_nonbonded(ctx, t["pos"], t["force"])
        mdx.set_langevin(ctx, kT, gamma, 77)
        en = torch.zeros((n_steps, mdx.MDX_N_ENERGY), dtype=torch.float64, device="cuda:0")
        mdx.integrate_step(ctx, t["pos"], t["vel"], t["force"], n_steps, dt, en)
        torch.cuda.synchronize()
        assert mdx.get_status(ctx) == 0
        ke = en.cpu().numpy()[:, 7]
    kin_T = 2.0 * ke / (3 * s.n_atoms)           # in units of kT (k_B = 1)
    # the kinetic energy relaxes with time constant 1/(2 gamma) = 50 steps:
    # from step 300 on the deficit is below e^-6
    assert abs(kin_T[300:].mean() / kT - 1.0) < 0.015, kin_T[300:].mean()
    assert kin_T[0] < 0.1 * kT


def test_langevin_is_reproducible_across_calls():
    import torch
    s = synth.config_system("water375")
    out = []
    for chunks in ([20], [3, 17], [1] * 20):
        with gpu_context(s) as (mdx, ctx, t):
            mdx.build_neighbors(ctx, t["pos"])
            mdx.compute_nonbonded(ctx, t["pos"], t["force"])
            mdx.compute_pme(ctx, t["pos"], t["force"])
            mdx.set_langevin(ctx, 0.6, 0.05, 12345)
            for k in chunks:
                mdx.integrate_step(ctx, t["pos"], t["vel"], t["force"], k, 0.5)
            torch.cuda.synchronize()
            out.append((t["pos"].cpu().numpy(), t["vel"].cpu().numpy()))
    for p, v in out[1:]:
        assert np.array_equal(p, out[0][0]) and np.array_equal(v, out[0][1])


def test_langevin_argument_checks():
    import paper_2503_20541_amd as mdx
    s = synth.config_system("water375")
    with gpu_context(s) as (m, ctx, t):
        for kT, gamma in ((-1.0, 0.1), (1.0, -0.1), (float("nan"), 0.1), (1.0, float("inf"))):
            with pytest.raises(m.MdxError) as e:
                m.set_langevin(ctx, kT, gamma, 1)
            assert e.value.code == m.MDX_E_INVALID
        m.set_langevin(ctx, 0.6, 0.0, 1)   # gamma = 0: velocity Verlet again
    with gpu_context(s, options=mdx.MDX_OPT_KAHAN_VV) as (m, ctx, t):
        with pytest.raises(m.MdxError) as e:
            m.set_langevin(ctx, 0.6, 0.1, 1)
        assert e.value.code == m.MDX_E_UNSUPPORTED


def test_paper_protocol_reaction_field_langevin_water():
    # the paper's scaling protocol on a small box: reaction field, Langevin at
    # 300 K with gamma = 0.1 / fs, dt = 0.5 fs; the thermostat holds the
    # temperature while the lattice start relaxes
    import math
    import torch
    s = synth.config_system("water9k")
    s.rf_epsilon, s.ewald_delta, s.pme_grid = 78.5, 0.0, (0, 0, 0)
    n_steps = 300
    announce("reaction field + Langevin water9k")
    with gpu_context(s) as (mdx, ctx, t):
        mdx.build_neighbors(ctx, t["pos"])
        mdx.compute_nonbonded(ctx, t["pos"], t["force"])
        mdx.set_langevin(ctx, float(s.boltzmann) * 300.0, 0.1, 99)
        en = torch.zeros((n_steps, mdx.MDX_N_ENERGY), dtype=torch.float64, device="cuda:0")
        mdx.integrate_step(ctx, t["pos"], t["vel"], t["force"], n_steps, 0.5, en)
        torch.cuda.synchronize()
        assert mdx.get_status(ctx) == 0
        E = en.cpu().numpy()
    assert np.all(np.isfinite(E)) and np.all(E[:, 6] == 0.0) and np.all(E[:, 3] == 0.0)
    temp = 2.0 * E[:, 7] / (3 * s.n_atoms * float(s.boltzmann))
    assert abs(temp[150:].mean() / 300.0 - 1.0) < 0.06, temp[150:].mean()
