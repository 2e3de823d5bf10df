"""GPU: rigid water (SHAKE positions + RATTLE velocities) through
mdx_set_rigid_water + mdx_integrate_step against the FP64 constraint oracle."""
import math

import numpy as np
import pytest

import synth
from oracle import constraints, forcefield
from helpers import announce, gpu_context

pytestmark = pytest.mark.gpu

W = synth.systems.WATER
D_OH = W["bond_r0"]
D_HH = 2.0 * D_OH * math.sin(math.radians(W["angle_theta0_deg"]) / 2.0)


def rigid_rf_water(name, coulomb="rf", flexible_terms=False):
    s = synth.config_system(name)
    if not flexible_terms:
        s.bond_k[:] = 0.0
        s.angle_k[:] = 0.0
    if coulomb == "rf":
        s.rf_epsilon, s.ewald_delta, s.pme_grid = math.inf, 0.0, (0, 0, 0)
    mols = np.arange(s.n_atoms, dtype=np.int32).reshape(-1, 3)
    return s, mols


def _dists(x, box, mols):
    L = np.asarray(box, np.float64)[:, None]
    out = []
    for a, b in constraints._pairs(mols):
        d = x[:, a] - x[:, b]
        d -= L * np.round(d / L)
        out.append(np.sqrt((d * d).sum(axis=0)))
    return out


def _dev(a, b, box):
    d = a - b
    d -= box[:, None] * np.round(d / box[:, None])
    return float(np.sqrt((d * d).mean()))


@pytest.mark.parametrize("coulomb,part", [("rf", False), ("pme", False), ("rf", True)])
def test_rigid_water_tracks_the_rattle_oracle(coulomb, part):
    # with PME the intramolecular pairs carry the Ewald exclusion correction;
    # part: only every other molecule rigid, the others flexible (bond and
    # angle terms on, dt = 0.5 fs), which takes the library's other opening
    # path (positions before the drift copied aside)
    import torch
    s, mols = rigid_rf_water("water375", coulomb, flexible_terms=part)
    if part:
        mols = mols[::2].copy()
    # start from velocities that already satisfy the constraints (the library
    # projects after each closing kick, the oracle also before the first step)
    s.vel = constraints.rattle_velocities(s.pos, s.vel, s.mass, s.box, mols).astype(np.float32)
    n_steps, dt = (40, 0.5) if part else (30, 2.0)
    announce(f"rigid water375 ({coulomb}, part={part}) {n_steps} steps at {dt} fs")
    with gpu_context(s) as (mdx, ctx, t):
        mdx.build_neighbors(ctx, t["pos"])
        mdx.compute_nonbonded(ctx, t["pos"], t["force"])
        if coulomb == "pme":
            mdx.compute_pme(ctx, t["pos"], t["force"])
        mdx.set_rigid_water(ctx, mols, D_OH, D_HH)
        en = torch.zeros((n_steps, mdx.MDX_N_ENERGY), dtype=torch.float64, device="cuda:0")
        mdx.integrate_step(ctx, t["pos"], t["vel"], t["force"], n_steps, dt, en)
        torch.cuda.synchronize()
        assert mdx.get_status(ctx) == 0
        x_gpu = t["pos"].cpu().numpy().astype(np.float64)
        v_gpu = t["vel"].cpu().numpy().astype(np.float64)
        ke_gpu = float(en[-1, mdx.MDX_ENERGY_KINETIC].item())
    for d, ref in zip(_dists(x_gpu, s.box, mols), (D_OH, D_OH, D_HH)):
        assert np.abs(d / ref - 1.0).max() < 1e-5
    m64 = s.mass.astype(np.float64)
    kin = lambda v: 0.5 * float((m64[None, :] * v * v).sum()) / float(s.accel)
    # the kinetic energy slot is that of the projected velocities the call returns
    assert abs(ke_gpu - kin(v_gpu)) <= 1e-9 * kin(v_gpu), (ke_gpu, kin(v_gpu))
    F = lambda p: forcefield.total_forces_fp64(s, p)[1]
    box = s.box.astype(np.float64)
    ref = constraints.velocity_verlet_rattle(s.pos, s.vel, s.mass, s.box, F, dt, n_steps,
                                             float(s.accel), mols, D_OH, D_HH)
    # and close to the oracle's (the unprojected kinetic energy sat 1.7-2 % above)
    assert abs(ke_gpu - kin(ref["vel"])) < 2e-3 * kin(ref["vel"]), (ke_gpu, kin(ref["vel"]))
    # the same scheme with the state rounded to float32 after every step:
    # how far float32 storage alone carries the trajectory from the FP64 one
    m = s.mass.astype(np.float64)
    L = box[:, None]
    acc = float(s.accel)
    x32 = s.pos.astype(np.float64)
    v32 = constraints.rattle_velocities(x32, s.vel, m, box, mols)
    F32 = F(x32)
    for _ in range(n_steps):
        v32 = v32 + 0.5 * dt * acc * F32 / m[None, :]
        y = x32 + dt * v32
        y2, _ = constraints.shake(x32, y, m, box, mols, D_OH, D_HH)
        v32 = v32 + (y2 - y) / dt
        x32 = (y2 - L * np.floor(y2 / L)).astype(np.float32).astype(np.float64)
        F32 = F(x32)
        v32 = v32 + 0.5 * dt * acc * F32 / m[None, :]
        v32 = constraints.rattle_velocities(x32, v32, m, box, mols)
        v32 = v32.astype(np.float32).astype(np.float64)
    d_gpu = _dev(x_gpu, ref["pos"], box)
    d_f32 = _dev(x32, ref["pos"], box)
    assert d_gpu <= 10 * max(d_f32, 1e-6), (d_gpu, d_f32)


def test_rigid_water_conserves_energy_at_two_femtoseconds():
    import torch
    s, mols = rigid_rf_water("water9k")
    n_steps = 100
    announce("rigid water9k 100 steps at 2 fs")
    with gpu_context(s) as (mdx, ctx, t):
        mdx.build_neighbors(ctx, t["pos"])
        mdx.compute_nonbonded(ctx, t["pos"], t["force"])
        mdx.set_rigid_water(ctx, mols, D_OH, D_HH)
        en = torch.zeros((n_steps, mdx.MDX_N_ENERGY), dtype=torch.float64, device="cuda:0")
        mdx.integrate_step(ctx, t["pos"], t["vel"], t["force"], n_steps, 2.0, en)
        torch.cuda.synchronize()
        assert mdx.get_status(ctx) == 0
        E = en.cpu().numpy()
        x = t["pos"].cpu().numpy().astype(np.float64)
    for d, ref in zip(_dists(x, s.box, mols), (D_OH, D_OH, D_HH)):
        assert np.abs(d / ref - 1.0).max() < 1e-5
    etot = E.sum(axis=1)
    drift = np.abs(etot - etot[0]).max() / E[:, 7].mean()
    print(f"rigid water9k 2 fs: max |E - E0| / <KE> = {drift:.3e}", flush=True)
    assert drift < 0.01      # 7.3e-3 measured with the projected kinetic energy


def test_rigid_water_split_calls_match_one_call_bitwise():
    import torch
    s, mols = rigid_rf_water("water9k", "pme")
    n_steps = 24
    out = []
    for chunks in ([n_steps], [5, 7, 1, n_steps - 13]):
        announce(f"rigid water9k {n_steps} steps in calls of {chunks}")
        with gpu_context(s) as (mdx, ctx, t):
            mdx.build_neighbors(ctx, t["pos"])
            mdx.compute_nonbonded(ctx, t["pos"], t["force"])
            mdx.compute_pme(ctx, t["pos"], t["force"])
            mdx.set_rigid_water(ctx, mols, D_OH, D_HH)
            for k in chunks:
                mdx.integrate_step(ctx, t["pos"], t["vel"], t["force"], k, 2.0)
            torch.cuda.synchronize()
            assert mdx.get_status(ctx) == 0      # MDX_FLAG_CONSTRAINT stays clear too
            out.append((t["pos"].cpu().numpy(), t["vel"].cpu().numpy()))
    for a, b in zip(out[0], out[1]):
        assert np.array_equal(a, b)


def test_rigid_water_argument_checks():
    s, mols = rigid_rf_water("water375")
    with gpu_context(s) as (m, ctx, t):
        for bad in (np.array([[0, 1, s.n_atoms]]), np.array([[0, 1, 1]]), np.array([[-1, 1, 2]])):
            with pytest.raises(m.MdxError) as e:
                m.set_rigid_water(ctx, bad, D_OH, D_HH)
            assert e.value.code == m.MDX_E_INVALID
        with pytest.raises(m.MdxError) as e:
            m.set_rigid_water(ctx, mols, -1.0, D_HH)
        assert e.value.code == m.MDX_E_INVALID
        m.set_rigid_water(ctx, mols, D_OH, D_HH)
        with pytest.raises(m.MdxError) as e:
            m.set_langevin(ctx, 0.6, 0.1, 1)
        assert e.value.code == m.MDX_E_UNSUPPORTED
        m.set_rigid_water(ctx, mols[:0], D_OH, D_HH)   # off again
        m.set_langevin(ctx, 0.6, 0.1, 1)


def test_settle_step_matches_the_closed_form_oracle():
    # one rigid step from an exactly constrained start: the GPU's SETTLE
    # positions against the oracle's closed form of the same drift
    import torch
    s, mols = rigid_rf_water("water375")
    x0, _ = constraints.shake(s.pos.astype(np.float64), s.pos.astype(np.float64), s.mass, s.box,
                              mols, D_OH, D_HH)
    s.pos = (x0 - s.box[:, None] * np.floor(x0 / s.box[:, None])).astype(np.float32)
    s.vel = constraints.rattle_velocities(s.pos, s.vel, s.mass, s.box, mols).astype(np.float32)
    dt = 2.0
    announce("settle one step water375")
    with gpu_context(s) as (mdx, ctx, t):
        mdx.build_neighbors(ctx, t["pos"])
        mdx.compute_nonbonded(ctx, t["pos"], t["force"])
        F = t["force"].cpu().numpy().astype(np.float64)
        mdx.set_rigid_water(ctx, mols, D_OH, D_HH)
        mdx.integrate_step(ctx, t["pos"], t["vel"], t["force"], 1, dt)
        torch.cuda.synchronize()
        assert mdx.get_status(ctx) == 0
        x_gpu = t["pos"].cpu().numpy().astype(np.float64)
    x = s.pos.astype(np.float64)
    m = s.mass.astype(np.float64)
    y = x + dt * (s.vel.astype(np.float64) + 0.5 * dt * float(s.accel) * F / m[None, :])
    ref = constraints.settle(x, y, m, s.box, mols, D_OH, D_HH)
    L = s.box.astype(np.float64)[:, None]
    d = x_gpu - ref
    d -= L * np.round(d / L)
    assert np.abs(d).max() < 2e-5, np.abs(d).max()


def test_unequal_hydrogen_masses_take_the_iterative_path():
    import torch
    s, mols = rigid_rf_water("water375")
    s.mass[mols[:, 1]] = 2.014           # one deuterium per molecule: no closed form
    s.vel = constraints.rattle_velocities(s.pos, s.vel, s.mass, s.box, mols).astype(np.float32)
    announce("rigid water375 with HDO (SHAKE)")
    with gpu_context(s) as (mdx, ctx, t):
        mdx.build_neighbors(ctx, t["pos"])
        mdx.compute_nonbonded(ctx, t["pos"], t["force"])
        mdx.set_rigid_water(ctx, mols, D_OH, D_HH)
        mdx.integrate_step(ctx, t["pos"], t["vel"], t["force"], 20, 2.0)
        torch.cuda.synchronize()
        assert mdx.get_status(ctx) == 0
        x = t["pos"].cpu().numpy().astype(np.float64)
    for d, ref in zip(_dists(x, s.box, mols), (D_OH, D_OH, D_HH)):
        assert np.abs(d / ref - 1.0).max() < 1e-5
