"""Benchmark of the force-evaluation hot path on one MI355X.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--no-cpu-baseline]

One step = one velocity-Verlet step of the 96,000-atom water box (32,000
flexible 3-site waters, L = 98.6 A, r_c = 9 A, r_g = 2.25 A, PME 100^3,
order 4, dt = 1 fs): half kick + drift, the r_g/2 validity test (list rebuilt
every 10 steps and whenever it fails), LJ + real-space Ewald pair kernel,
exclusion/bonded terms, smooth PME (spread, FFTs, influence multiply,
gather) and the closing half kick. Inputs are resident in HBM before timing.

The seeded lattice start is far from equilibrium: without a thermostat it
heats to about 750 K within a few hundred femtoseconds. Before the warm-up
the box is brought to 300 K (the paper's water temperature) by 3000 steps
with the velocities rescaled every 100 steps; this input preparation is not
timed, and the temperature at the start and end of the timed run is
reported. --equilibrate 0 times the run from the lattice start instead.

Prints one JSON line: ns/day (value), pair-interactions/s, the pair kernel's
roofline fraction (its launch durations from HIP events that its own dispatch
records on the context's stream) and the CPU oracle timed on a bounded sample (rank 0, N = 1).
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

WORKLOAD = "water96k"
METRIC = "ns/day & pair-interactions/s, 96k-atom PME water; fwd+adjoint vs plain fwd"

# Per-unit work of the pair kernel (VALU lane-operations): ~55 per interacting
# unique pair, ~8 per listed unique pair beyond r_c (distance test only).
OPS_PER_INTERACTING = 55.0
OPS_PER_LISTED_ONLY = 8.0
# FP32 VALU issue peak without packed math: 256 CU x 64 lanes x 2.4 GHz.
VALU_PEAK_T = 256 * 64 * 2.4e9 / 1e12
# HBM bytes per pair-kernel launch from rocprofv3 FETCH_SIZE / WRITE_SIZE
# passes, scaled by the same counters on a plain copy of known size
# (profiles/pair_kernel_counters_water96k.md); set to None when the kernel
# changes until the counters are taken again.
PAIR_TRAFFIC_BYTES = 61.5e6
PAIR_TRAFFIC_COMMIT = "f9aef80"     # the commit whose k_pair the counters measured
# Whole-step floors of the 96,000-atom water step (the method's compulsory
# work per step: 199 MB of HBM traffic -- fused integrate 6.1 MB, pair kernel
# per-atom I/O plus a 4-byte-per-pair Verlet list 118 MB, PME 56 MB, list
# build amortised over 10 steps 12 MB -- and 1.2e9 FP32 VALU lane operations):
# 24.9 us at 8 TB/s, 30.5 us at the non-packed VALU issue rate.
STEP_HBM_BYTES = 199e6
STEP_VALU_OPS = 1.2e9
HBM_PEAK_BPS = 8.0e12


def parse():
    p = argparse.ArgumentParser()
    p.add_argument("--gpus", type=int, default=1)
    p.add_argument("--steps", type=int, default=1000)
    p.add_argument("--warmup", type=int, default=100)
    p.add_argument("--no-cpu-baseline", action="store_true")
    p.add_argument("--no-batch", action="store_true",
                   help="skip the 256-replica batch against sequential replicas timing")
    p.add_argument("--no-hmc", action="store_true",
                   help="skip the HMC tuning measurement")
    p.add_argument("--no-adjoint", action="store_true",
                   help="skip the forward+adjoint against plain forward timing (9k water)")
    p.add_argument("--equilibrate", type=int, default=3000,
                   help="steps of velocity-rescaled equilibration to 300 K before the warm-up "
                        "(0: start the timed run from the lattice start, which heats up)")
    p.add_argument("--cpu-only", action="store_true", help=argparse.SUPPRESS)
    p.add_argument("--half-list", action="store_true",
                   help="run the benchmark with MDX_OPT_HALF_LIST (each pair once, float "
                        "atomics: forces not bitwise reproducible) instead of the default list")
    p.add_argument("--sweep", action="store_true",
                   help="instead of the benchmark: time per step against system size for "
                        "water boxes with reaction-field and with PME electrostatics (one "
                        "JSON line per box and method)")
    p.add_argument("--sweep-protocols", default="rf,pme,rf_langevin_paper,rf_rigid_2fs",
                   help="comma-separated protocols of --sweep")
    p.add_argument("--sweep-molecules", type=int, nargs="*", default=None,
                   help="only these box sizes (water molecules) in --sweep")
    p.add_argument("--ewald-direct", action="store_true",
                   help="instead of the benchmark: time the direct reciprocal Ewald sum "
                        "(converged to 1e-8 in the Gaussian factor) against SPME for the "
                        "9,000- and 96,000-atom water boxes (one JSON line each)")
    p.add_argument("--copy-probe", type=int, default=0, metavar="MIB",
                   help="only copy a MIB-sized float32 buffer 10 times (calibrates the "
                        "FETCH_SIZE / WRITE_SIZE counters against known traffic) and exit")
    return p.parse_args()


def pair_counts():
    path = os.path.join(ROOT, "tests", "golden", "pair_counts.json")
    with open(path) as f:
        return json.load(f)[WORKLOAD]


def temperature(sys_, vel, n_rigid=0):
    """Instantaneous temperature from the device velocities: 3N degrees of
    freedom, less three per rigid molecule and three for the conserved
    momentum when molecules are rigid."""
    import torch
    m = torch.from_numpy(sys_.mass.astype("float64")).to(vel.device)
    ke = 0.5 * float((m[None, :] * vel.double() ** 2).sum()) / float(sys_.accel)
    dof = 3 * sys_.n_atoms - (3 * n_rigid + 3 if n_rigid else 0)
    return 2.0 * ke / (dof * float(sys_.boltzmann))


_POOL_SYS = None      # the system the pool's workers sum pair terms of (fork start)


def _pair_chunk(bounds):
    """Interaction test and pair terms of one slice of the listed pairs (pool
    worker)."""
    import numpy as np
    from oracle import forcefield, neighbors, nonbonded
    s, pairs = _POOL_SYS
    lo, hi = bounds
    chunk = pairs[lo:hi]
    inter = chunk[neighbors.interacting(s.pos, s.box, s.r_cut, s.r_ghost, chunk)]
    pt = nonbonded.pair_terms(s.pos.astype(np.float64), s.box, inter, s.atom_type,
                              s.type_sigma, s.type_epsilon, s.charge, forcefield.alpha(s),
                              s.coulomb_k, r_cut=float(s.r_cut), switch_r=float(s.switch_r))
    return pt["F"], len(inter)


def _oracle_step_seconds(sys_, reps, cores):
    """The untuned oracle: one list build (amortised over the rebuild cadence)
    and `reps` force evaluations (nonbonded + SPME when the system has a grid)
    with their velocity-Verlet updates. cores > 1: the pair sum, which
    dominates, is split into `cores` slices of the interacting pairs summed by
    a process pool; the rest stays in one process."""
    import multiprocessing as mp
    import numpy as np
    from oracle import forcefield, neighbors

    global _POOL_SYS
    t0 = time.perf_counter()
    pairs = forcefield.neighbor_list(sys_)
    t_list = time.perf_counter() - t0
    n_int = 0
    pool = None
    if cores > 1:     # pool start-up is not timed
        _POOL_SYS = (sys_, pairs)
        pool = mp.get_context("fork").Pool(cores)
        edges = np.linspace(0, len(pairs), cores + 1).astype(int)
        chunks = list(zip(edges[:-1], edges[1:]))
    t1 = time.perf_counter()
    try:
        for _ in range(reps):
            if pool is None:
                nb = forcefield.nonbonded_terms(sys_, pairs=pairs)
                F = nb["F"]
                n_int = nb["n_interacting"]
            else:
                # the pair terms in the pool, the exclusion, bonded and self
                # terms through the oracle with an empty pair list
                parts = pool.map(_pair_chunk, chunks)
                nb = forcefield.nonbonded_terms(sys_, pairs=pairs[:0])
                F = nb["F"] + sum(p[0] for p in parts)
                n_int = sum(p[1] for p in parts)
            if sum(sys_.pme_grid) > 0:
                F = F + forcefield.pme_terms(sys_)["F"]
            x = sys_.pos.astype(np.float64)
            v = sys_.vel.astype(np.float64)
            m = sys_.mass.astype(np.float64)
            v = v + 0.5 * sys_.dt * sys_.accel * F / m[None, :]
            x = x + sys_.dt * v
    finally:
        if pool is not None:
            pool.close()
            pool.join()
        _POOL_SYS = None
    t2 = time.perf_counter()
    t_step = t_list / sys_.rebuild_every + (t2 - t1) / reps
    return t_step, n_int, t_list + (t2 - t1)


def cpu_baseline(sys_, names=("lj1k", "water9k")):
    """The oracle on a bounded sample of the workload, on 1 core (the headline
    value: NumPy element-wise work is single-threaded) and on all the host's
    cores (pair sum in a process pool), for the 96,000-atom box and the two
    smaller configurations."""
    import synth
    cores_all = max(1, min(len(os.sched_getaffinity(0)), 16))
    t1c, n_int, cpu_s = _oracle_step_seconds(sys_, 2, 1)
    tall, _, cpu_all = _oracle_step_seconds(sys_, 2, cores_all)
    out = dict(value=0.0864 * sys_.dt / t1c, unit="ns/day", cores=1, kind="oracle",
               sample=("one list build + two nonbonded+SPME force evaluations with VV updates "
                       "of the 96,000-atom water box's initial state (list build amortised "
                       f"over 10 steps); {cpu_s:.1f} s of CPU work"),
               seconds_per_step=t1c, pair_interactions_per_s=n_int / t1c,
               host_cores=len(os.sched_getaffinity(0)),
               all_cores={"cores": cores_all, "value": 0.0864 * sys_.dt / tall,
                          "seconds_per_step": tall, "pair_interactions_per_s": n_int / tall,
                          "wall_s": round(cpu_all, 1)},
               by_workload={})
    for name in names:
        s = synth.config_system(name)
        reps = 5 if s.n_atoms < 5000 else 2
        row = {}
        for cores in (1, cores_all):
            t, n, _ = _oracle_step_seconds(s, reps, cores)
            unit = "steps/s" if name == "lj1k" else "ns/day"
            val = 1.0 / t if name == "lj1k" else 0.0864 * s.dt / t
            row[f"cores_{cores}"] = {"value": val, "unit": unit, "seconds_per_step": t,
                                     "pair_interactions_per_s": n / t}
        out["by_workload"][name] = row
    return out


def copy_probe(mib):
    """A plain device-to-device copy of known size (reads and writes mib MiB
    per launch), used to scale the hardware byte counters."""
    import torch
    n = mib * (1 << 20) // 4
    src = torch.ones(n, dtype=torch.float32, device="cuda:0")
    dst = torch.empty_like(src)
    for _ in range(10):
        dst.copy_(src)
    torch.cuda.synchronize()
    print(json.dumps({"copy_probe_MiB": mib, "launches": 10}), flush=True)


# (molecules, PME grid) of the size sweep: water at 0.997 g/cm^3, box edge
# (29.91 A^3 per molecule)^(1/3), grid spacing about 1 A (no PME grid for the
# largest box, which runs the reaction-field protocols only)
SWEEP_BOXES = ((1000, 32), (4000, 48), (8000, 64), (27000, 96), (32000, 100), (64000, 128),
               (100000, 0))


def sweep(args):
    """Time per step against N for the same water model under up to four
    protocols: velocity Verlet with the reaction field (Eq. 8, eps_s = 78.5)
    and with SPME (the shape of the paper's RFA / PME scaling figure), both at
    r_c = 9 A, r_g = 2.25 A, dt = 1 fs; and the paper's own benchmark protocol
    (reaction field, Langevin dynamics at 300 K with gamma = 0.1 / fs,
    dt = 0.5 fs, r_c = 10 A, r_g = 2.5 A); and, as a fourth protocol, the
    reaction field with rigid water (SHAKE / RATTLE) at dt = 2 fs. Lists are
    rebuilt every 10 steps
    (and whenever an atom has moved more than r_g / 2); each run is brought to
    300 K for 1000 untimed steps first."""
    import math
    import numpy as np
    import torch
    import synth
    import paper_2503_20541_amd as mdx
    dev = torch.device("cuda:0")
    stream = torch.cuda.current_stream(dev)
    for n_mol, K in SWEEP_BOXES:
        if args.sweep_molecules and n_mol not in args.sweep_molecules:
            continue
        L = (n_mol * 29.91) ** (1.0 / 3.0)
        base = synth.water_box(n_mol, L, (max(K, 32),) * 3, 9.0, None, 5e-4, 11,
                               n_steps=1000, name=f"water{3 * n_mol}")
        for method in args.sweep_protocols.split(","):
            if method == "pme" and K == 0:
                continue
            s = base.copy()
            dt, gamma, n_rigid = float(s.dt), 0.0, 0
            if method != "pme":
                s.rf_epsilon, s.ewald_delta, s.pme_grid = 78.5, 0.0, (0, 0, 0)
            if method == "rf_langevin_paper":
                s.r_cut, s.r_ghost = s.r_cut.__class__(10.0), s.r_ghost.__class__(2.5)
                dt, gamma = 0.5, 0.1
            if method == "rf_rigid_2fs":
                dt = 2.0
            desc, keep = mdx.desc_from_system(s)
            ctx = mdx.create(desc, stream.cuda_stream)
            pos = torch.from_numpy(s.pos.copy()).to(dev)
            vel = torch.from_numpy(s.vel.copy()).to(dev)
            force = torch.zeros_like(pos)
            mdx.build_neighbors(ctx, pos)
            mdx.compute_nonbonded(ctx, pos, force)
            if method == "pme":
                mdx.compute_pme(ctx, pos, force)
            if method == "rf_rigid_2fs":
                w = synth.systems.WATER
                d_oh = float(w["bond_r0"])
                d_hh = 2.0 * d_oh * math.sin(math.radians(w["angle_theta0_deg"]) / 2.0)
                n_rigid = s.n_atoms // 3
                mdx.set_rigid_water(ctx, np.arange(s.n_atoms, dtype=np.int32).reshape(-1, 3),
                                    d_oh, d_hh)
            for _ in range(10):
                mdx.integrate_step(ctx, pos, vel, force, 100, dt)
                vel.mul_((300.0 / temperature(s, vel, n_rigid)) ** 0.5)
            if gamma > 0:
                mdx.set_langevin(ctx, float(s.boltzmann) * 300.0, gamma, 2025)
            mdx.integrate_step(ctx, pos, vel, force, args.warmup, dt)
            b0 = mdx.get_info(ctx).n_builds
            start = torch.cuda.Event(enable_timing=True)
            stop = torch.cuda.Event(enable_timing=True)
            torch.cuda.synchronize()
            start.record(stream)
            mdx.integrate_step(ctx, pos, vel, force, args.steps, dt)
            stop.record(stream)
            torch.cuda.synchronize()
            ms = start.elapsed_time(stop) / args.steps
            builds = mdx.get_info(ctx).n_builds - b0
            flags = mdx.get_status(ctx)
            t_end = temperature(s, vel, n_rigid)
            mdx.destroy(ctx)
            print(json.dumps({"sweep": "time_per_step_vs_n", "protocol": method,
                              "n_atoms": s.n_atoms, "box_A": round(L, 2),
                              "pme_grid": K if method == "pme" else None,
                              "r_cut_A": float(s.r_cut), "dt_fs": dt, "langevin_gamma": gamma,
                              "steps": args.steps, "ms_per_step": round(ms, 5),
                              "ns_per_day": round(0.0864 * dt * 1e3 / ms, 3),
                              "list_builds": builds, "temperature_K_end": round(t_end, 1),
                              "status_flags": flags}), flush=True)


def ewald_direct_vs_pme():
    """Reciprocal energy and time of one evaluation by the direct sum and by
    SPME at the configured grid, same alpha: the direct sum's n_max makes the
    Gaussian factor exp(-pi^2 m^2/alpha^2) fall below 1e-8 at the cube face."""
    import math
    import torch
    import synth
    import paper_2503_20541_amd as mdx
    from oracle import forcefield
    dev = torch.device("cuda:0")
    stream = torch.cuda.current_stream(dev)
    for name in ("water9k", "water96k"):
        s = synth.config_system(name)
        a = forcefield.alpha(s)
        L = float(max(s.box))
        n_max = int(math.ceil(L * a * math.sqrt(math.log(1e8)) / math.pi))
        desc, keep = mdx.desc_from_system(s)
        ctx = mdx.create(desc, stream.cuda_stream)
        pos = torch.from_numpy(s.pos.copy()).to(dev)
        mdx.build_neighbors(ctx, pos)
        out = {}
        for method in ("pme", "direct"):
            e = torch.zeros(1, dtype=torch.float64, device=dev)
            f = torch.zeros_like(pos)
            call = (lambda: mdx.compute_pme(ctx, pos, f, e)) if method == "pme" else \
                (lambda: mdx.compute_ewald_direct(ctx, pos, f, e, n_max))
            call()
            f.zero_()                 # the forces accumulate: count the timed calls only
            torch.cuda.synchronize()
            t0 = torch.cuda.Event(enable_timing=True)
            t1 = torch.cuda.Event(enable_timing=True)
            reps = 20 if method == "pme" else 3
            t0.record(stream)
            for _ in range(reps):
                call()
            t1.record(stream)
            torch.cuda.synchronize()
            out[method] = (t0.elapsed_time(t1) / reps, float(e.cpu()[0]), f.cpu().numpy() / reps)
        mdx.destroy(ctx)
        import numpy as np
        fd, fp = out["direct"][2], out["pme"][2]
        print(json.dumps({"ewald_direct_vs_pme": name, "n_atoms": s.n_atoms,
                          "pme_grid": list(s.pme_grid), "direct_n_max": n_max,
                          "direct_vectors": ((2 * n_max + 1) ** 3 - 1) // 2,
                          "ms_pme": round(out["pme"][0], 4), "ms_direct": round(out["direct"][0], 3),
                          "E_rec_pme": out["pme"][1], "E_rec_direct": out["direct"][1],
                          "pme_energy_rel_error": abs(out["pme"][1] / out["direct"][1] - 1.0),
                          "pme_force_rel_rms_error": float(np.sqrt(((fp - fd) ** 2).sum()
                                                                   / (fd ** 2).sum()))}),
              flush=True)


def adjoint_ratio(reps=5):
    """The metric's second half on the 9,000-atom water box: 100 velocity-
    Verlet steps of 1 fs as a plain forward (mdx_integrate_step) against the
    differentiable forward with checkpoints every 10 steps plus its reverse
    pass (loss U(x_T)/N + MSD; gradients with respect to x0, v0, eps, sigma,
    the O charge and dt), both timed with events on the context's stream,
    median of `reps`."""
    import numpy as np
    import torch
    import synth
    import paper_2503_20541_amd as mdx
    from paper_2503_20541_amd import trajectory as tj
    s = synth.config_system("water9k")
    n_steps, every, dt = 100, 10, 1.0
    dev = torch.device("cuda:0")
    dq = np.where(s.atom_type == 0, 1.0, -0.5).astype(np.float32)
    sim = tj.Simulation(s, n_steps, every, charge_direction=dq)
    stream = sim.stream
    try:
        def timed(fn):
            out = []
            for _ in range(reps + 1):
                a = torch.cuda.Event(enable_timing=True)
                b = torch.cuda.Event(enable_timing=True)
                torch.cuda.synchronize()
                a.record(stream)
                fn()
                b.record(stream)
                torch.cuda.synchronize()
                out.append(a.elapsed_time(b))
            return float(np.median(out[1:]))      # the first is a warm-up

        pos = torch.from_numpy(s.pos.copy()).to(dev)
        vel = torch.from_numpy(s.vel.copy()).to(dev)
        force = torch.zeros_like(pos)

        def plain():
            pos.copy_(torch.from_numpy(s.pos))
            vel.copy_(torch.from_numpy(s.vel))
            mdx.build_neighbors(sim.ctx, pos)
            mdx.compute_nonbonded(sim.ctx, pos, force)
            mdx.compute_pme(sim.ctx, pos, force)
            mdx.integrate_step(sim.ctx, pos, vel, force, n_steps, dt)

        def fwd_adj():
            x0 = torch.from_numpy(s.pos.copy()).to(dev).requires_grad_(True)
            v0 = torch.from_numpy(s.vel.copy()).to(dev).requires_grad_(True)
            eps = torch.from_numpy(s.type_epsilon.copy()).to(dev).requires_grad_(True)
            sig = torch.from_numpy(s.type_sigma.copy()).to(dev).requires_grad_(True)
            tq = torch.zeros((), device=dev, requires_grad=True)
            dtt = torch.tensor(dt, device=dev, requires_grad=True)
            xT, UT = tj.trajectory(sim, x0, v0, eps, sig, tq, dtt)
            L = UT / s.n_atoms + ((xT.double() - x0.double()) ** 2).sum() / s.n_atoms
            L.backward()

        t_fwd = timed(plain)
        t_adj = timed(fwd_adj)
        flags = mdx.get_status(sim.ctx)
    finally:
        sim.close()
    return {"workload": "water9k: 3,000 flexible waters, PME 48^3, 100 steps of 1 fs, "
                        "checkpoints every 10 steps, loss U(x_T)/N + MSD",
            "ms_per_step_fwd": round(t_fwd / n_steps, 5),
            "ms_per_step_fwd_adjoint": round(t_adj / n_steps, 5),
            "ratio": round(t_adj / t_fwd, 3), "repetitions": reps, "status_flags": flags}


def hmc_tuning(iters=8, chains=10):
    """Differentiable HMC tuning (the paper's Sec. IV) on the 9,000-atom water
    box equilibrated at 300 K: `chains` chains (the paper's R = 10) from the paper's untuned
    parameters (dt 0.5 fs, L = 10, no mass repartitioning), O and H masses as
    two shared groups with the total mass fixed. Each iteration evaluates
    L_HMC over every chain's proposal (forward steps with the state saved
    after each), its reverse pass, an Adam step and the chains' Metropolis
    moves. Timed on the host around whole iterations (the iteration
    synchronises to read the acceptances)."""
    import numpy as np
    import torch
    import synth
    import paper_2503_20541_amd as mdx
    from paper_2503_20541_amd import hmc
    s = synth.config_system("water9k")
    kT = 0.0019872041 * 300.0
    # the chains start from a 300 K liquid: 2,000 Langevin steps of 1 fs
    # (gamma 0.1 / fs) from the synthetic lattice start
    dev = torch.device("cuda:0")
    stream = torch.cuda.current_stream(dev)
    desc, keep = mdx.desc_from_system(s)
    ctx = mdx.create(desc, stream.cuda_stream)
    try:
        pos = torch.from_numpy(s.pos.copy()).to(dev)
        vel = torch.from_numpy(s.vel.copy()).to(dev)
        force = torch.zeros_like(pos)
        mdx.build_neighbors(ctx, pos)
        mdx.compute_nonbonded(ctx, pos, force)
        mdx.compute_pme(ctx, pos, force)
        mdx.set_langevin(ctx, kT, 0.1, 20541)
        mdx.integrate_step(ctx, pos, vel, force, 2000, 1.0)
        torch.cuda.synchronize()
        eq_flags = mdx.get_status(ctx)
        s = s.copy()
        s.pos = pos.cpu().numpy()
    finally:
        mdx.destroy(ctx)
    groups = np.where(s.atom_type == 0, 0, 1)
    t = hmc.HMCTuner(s, chains, kT, 0.5, 10.0, groups, seed=20541)
    try:
        t.step()                      # warm-up (library set-up, first allocations)
        torch.cuda.synchronize()
        hist, steps = [], 0
        t0 = time.perf_counter()
        for _ in range(iters):
            r = t.step()
            hist.append(r)
            steps += chains * r["L_q"]
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        flags = eq_flags
        for sim in t.sims:
            flags |= mdx.get_status(sim.ctx)
    finally:
        t.close()
    return {"workload": "water9k: 3,000 flexible waters, PME 48^3, 300 K; %d chains, L_HMC over "
                        "L_q steps, gradients in mu_dt, mu_L and the O/H masses (total fixed)"
                        % chains,
            "iterations": iters, "ms_per_iteration": round(1e3 * dt / iters, 2),
            "trajectory_steps_per_s": round(steps / dt, 1),
            "loss": [round(h["loss"], 6) for h in hist],
            "mu_dt_fs": round(hist[-1]["mu_dt"], 4), "mu_L": round(hist[-1]["mu_L"], 3),
            "masses_O_H": [round(v, 4) for v in hist[-1]["group_masses"]],
            "acceptance": round(float(np.mean([h["acceptance"] for h in hist])), 3),
            "status_flags": flags}


def batch_throughput(steps=50):
    """Batched replicas: the 256-replica workload (even index LJ at reduced
    density 0.8, odd index flexible water, 500-20,000 atoms log-uniform, each
    with its own box and ~1 A PME grid) stepped together by mdx_batch_integrate
    (graph launches of 10-step chunks on one stream per replica), against the
    same replicas stepped one after another launch by launch. The column
    width and list-build mode of every replica come from mdx_autotune, run
    on one replica per kind and size quartile."""
    import numpy as np
    import torch
    import synth
    import paper_2503_20541_amd as mdx
    t0 = time.perf_counter()
    systems = synth.batch_replicas()
    t_gen = time.perf_counter() - t0
    dev = torch.device("cuda:0")
    stream = torch.cuda.current_stream(dev)
    sizes = np.array([s.n_atoms for s in systems])
    kind = np.array([0 if s.pme_grid[0] == 0 else 1 for s in systems])
    # autotune one representative per (kind, size quartile)
    tuned = {}
    for k in (0, 1):
        idx = np.where(kind == k)[0]
        q = np.quantile(sizes[idx], [0.25, 0.5, 0.75])
        for b in range(4):
            members = [i for i in idx if np.searchsorted(q, sizes[i]) == b]
            if not members:
                continue
            rep = members[len(members) // 2]
            desc, keep = mdx.desc_from_system(systems[rep])
            pos = torch.from_numpy(systems[rep].pos.copy()).to(dev)
            vel = torch.from_numpy(systems[rep].vel.copy()).to(dev)
            m, opt, _ = mdx.autotune(desc, pos, vel, float(systems[rep].dt), 10, stream.cuda_stream)
            for i in members:
                tuned[i] = (m, opt)
    ctxs, keep, T = [], [], []
    try:
        for i, s in enumerate(systems):
            m, opt = tuned[i]
            desc, kp = mdx.desc_from_system(s, cell_divisions=m, options=opt)
            keep.append(kp)
            ctx = mdx.create(desc, stream.cuda_stream)
            ctxs.append(ctx)
            t = dict(pos=torch.from_numpy(s.pos.copy()).to(dev),
                     vel=torch.from_numpy(s.vel.copy()).to(dev))
            t["force"] = torch.zeros_like(t["pos"])
            mdx.build_neighbors(ctx, t["pos"])
            mdx.compute_nonbonded(ctx, t["pos"], t["force"])
            if s.pme_grid[0]:
                mdx.compute_pme(ctx, t["pos"], t["force"])
            T.append(t)
        dts = [float(s.dt) for s in systems]
        P, V, F = ([t[k] for t in T] for k in ("pos", "vel", "force"))
        b = None

        def run_batch():
            mdx.batch_integrate(b, P, V, F, steps, dts, stream.cuda_stream)

        def run_sequential():
            for ctx, t, d in zip(ctxs, T, dts):
                mdx.integrate_step(ctx, t["pos"], t["vel"], t["force"], steps, d)

        def timed(fn):
            a = torch.cuda.Event(enable_timing=True)
            z = torch.cuda.Event(enable_timing=True)
            torch.cuda.synchronize()
            a.record(stream)
            fn()
            z.record(stream)
            torch.cuda.synchronize()
            return a.elapsed_time(z)

        # replicas side by side, each on its own stream: launch by launch,
        # then as graph launches of 10-step chunks; then one after another
        ms = {}
        for chunk in (0, 10):
            b = mdx.batch_create(ctxs, chunk)
            try:
                run_batch()               # warm-up (with a chunk: records each replica's)
                ms[chunk] = min(timed(run_batch) for _ in range(3))
            finally:
                mdx.batch_destroy(b)
        for ctx in ctxs:
            mdx.set_graph(ctx, 0)         # launch by launch again
        run_sequential()
        ms_seq = min(timed(run_sequential) for _ in range(3))
        ms_batch = min(ms.values())
        flags = 0
        for ctx in ctxs:
            flags |= mdx.get_status(ctx)
    finally:
        torch.cuda.synchronize()
        for ctx in ctxs:
            mdx.destroy(ctx)
    atom_steps = float(sizes.sum()) * steps
    return {"workload": "256 replicas, even LJ (rho* 0.8), odd water (0.0334 molecules/A^3), "
                        "500-20,000 atoms log-uniform, own box and ~1 A PME grid",
            "n_atoms_total": int(sizes.sum()), "steps": steps,
            "ms_batched": round(ms_batch, 3), "ms_sequential": round(ms_seq, 3),
            "ms_batched_streams": round(ms[0], 3), "ms_batched_graphs": round(ms[10], 3),
            "atom_steps_per_s_batched": atom_steps / (ms_batch * 1e-3),
            "atom_steps_per_s_sequential": atom_steps / (ms_seq * 1e-3),
            "speedup": round(ms_seq / ms_batch, 3),
            "autotuned": {"cell_divisions": sorted({int(v[0]) for v in tuned.values()}),
                          "cooperative_build": sum(1 for v in tuned.values() if v[1] & 2)},
            "input_generation_s": round(t_gen, 1), "status_flags": flags}


def main():
    args = parse()
    if args.copy_probe > 0:
        copy_probe(args.copy_probe)
        return
    if args.ewald_direct:
        ewald_direct_vs_pme()
        return
    if args.sweep:
        sweep(args)
        return
    if args.gpus != 1:
        print(f"bench.py measures one GPU only; --gpus {args.gpus} is not supported "
              "(the hot path runs on a single MI355X)", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import synth

    s = synth.config_system(WORKLOAD)
    counts = pair_counts()
    result = {"metric": METRIC, "unit": "ns/day", "higher_is_better": True, "n_gpus": 1,
              "steps": args.steps, "warmup": args.warmup, "scaling": "weak",
              "vs_baseline": None, "dtype": "f32", "data": "synthetic",
              "config": {"workload": ("water96k: 32,000 flexible 3-site waters (96,000 atoms), "
                                      "L=98.6 A, r_c=9 A, r_g=2.25 A, Ewald delta 5e-4, "
                                      "PME 100^3 order 4, dt=1 fs, list rebuilt every 10 steps"),
                         "n_atoms": s.n_atoms, "dt_fs": s.dt, "pme_grid": list(s.pme_grid),
                         "list": "half (each pair once)" if args.half_list else
                                 "full (each pair from both ends, deterministic)",
                         "parallelism": "single GPU"}}

    if not args.cpu_only:
        import torch
        import paper_2503_20541_amd as mdx

        dev = torch.device("cuda:0")
        stream = torch.cuda.current_stream(dev)
        desc, keep = mdx.desc_from_system(
            s, options=mdx.MDX_OPT_HALF_LIST if args.half_list else 0)
        ctx = mdx.create(desc, stream.cuda_stream)
        pos = torch.from_numpy(s.pos.copy()).to(dev)
        vel = torch.from_numpy(s.vel.copy()).to(dev)
        force = torch.zeros_like(pos)
        mdx.build_neighbors(ctx, pos)
        mdx.compute_nonbonded(ctx, pos, force)
        mdx.compute_pme(ctx, pos, force)
        # The synthetic lattice start is far from equilibrium and heats up as
        # its potential energy relaxes; optionally bring it to 300 K first by
        # rescaling the velocities every 100 steps (input preparation, not
        # timed).
        done = 0
        while done < args.equilibrate:
            k = min(100, args.equilibrate - done)
            mdx.integrate_step(ctx, pos, vel, force, k, s.dt)
            vel.mul_((300.0 / temperature(s, vel)) ** 0.5)
            done += k
        if args.warmup > 0:
            mdx.integrate_step(ctx, pos, vel, force, args.warmup, s.dt)
        torch.cuda.synchronize()
        flags0 = mdx.get_status(ctx)
        t_start = temperature(s, vel)
        builds0 = mdx.get_info(ctx).n_builds
        # only the pair kernel is bracketed by events inside the timed region
        # (every event record adds a small gap between kernels)
        mdx.set_timing(ctx, 1 << mdx.MDX_TIMING_PAIR)
        start = torch.cuda.Event(enable_timing=True)
        stop = torch.cuda.Event(enable_timing=True)
        torch.cuda.synchronize()
        start.record(stream)
        mdx.integrate_step(ctx, pos, vel, force, args.steps, s.dt)
        stop.record(stream)
        torch.cuda.synchronize()
        ms_total = start.elapsed_time(stop)
        pair_ms, pair_n = mdx.get_timing(ctx, mdx.MDX_TIMING_PAIR)
        mdx.set_timing(ctx, False)
        info = mdx.get_info(ctx)
        builds = info.n_builds - builds0
        t_end = temperature(s, vel)
        # diagnostic only, after the timed region: PME chain and build times
        mdx.set_timing(ctx, (1 << mdx.MDX_TIMING_PME) | (1 << mdx.MDX_TIMING_BUILD))
        mdx.integrate_step(ctx, pos, vel, force, min(args.steps, 100), s.dt)
        pme_ms, pme_n = mdx.get_timing(ctx, mdx.MDX_TIMING_PME)
        build_ms, build_n = mdx.get_timing(ctx, mdx.MDX_TIMING_BUILD)
        mdx.set_timing(ctx, False)
        # diagnostic only: the same steps as graph launches of 10-step chunks
        mdx.set_graph(ctx, 10)
        n_g = max(10, min(args.steps, 200) // 10 * 10)
        mdx.integrate_step(ctx, pos, vel, force, 10, s.dt)        # records the chunk
        g0 = torch.cuda.Event(enable_timing=True)
        g1 = torch.cuda.Event(enable_timing=True)
        torch.cuda.synchronize()
        g0.record(stream)
        mdx.integrate_step(ctx, pos, vel, force, n_g, s.dt)
        g1.record(stream)
        torch.cuda.synchronize()
        ms_graph = g0.elapsed_time(g1) / n_g
        mdx.set_graph(ctx, 0)
        flags = mdx.get_status(ctx) | flags0
        ok = bool(torch.isfinite(pos).all() and torch.isfinite(vel).all())
        mdx.destroy(ctx)

        ms_step = ms_total / args.steps
        steps_per_s = 1e3 / ms_step
        ns_day = steps_per_s * s.dt * 0.0864
        ops = (OPS_PER_INTERACTING * counts["interacting_pairs"]
               + OPS_PER_LISTED_ONLY * (counts["listed_pairs"] - counts["interacting_pairs"]))
        achieved = ops / (pair_ms * 1e-3) / 1e12
        t_hbm = STEP_HBM_BYTES / HBM_PEAK_BPS
        t_valu = STEP_VALU_OPS / (VALU_PEAK_T * 1e12)
        result.update({
            "value": round(ns_day, 3), "ms_per_step": round(ms_step, 5),
            # step time against the step's floors (compulsory HBM bytes; the
            # larger of the HBM and VALU floors)
            "hbm_frac_step": round(t_hbm / (ms_step * 1e-3), 4),
            "binding_roof_frac_step": round(max(t_hbm, t_valu) / (ms_step * 1e-3), 4),
            "step_floor_us": {"hbm": round(t_hbm * 1e6, 2), "valu": round(t_valu * 1e6, 2)},
            "pair_interactions_per_s": counts["interacting_pairs"] * steps_per_s,
            "status_flags": flags, "finite": ok,
            "equilibration_steps": args.equilibrate,
            "list_builds": builds, "temperature_K": [round(t_start, 1), round(t_end, 1)],
            "list_tiles": info.n_list_tiles, "list_entries": info.n_list_entries,
            "kernel_ms": {"pair": round(pair_ms, 5), "pme_chain_overlapped": round(pme_ms, 5),
                          "build_gated": round(build_ms, 5)},
            "graph_replay_ms_per_step": round(ms_graph, 5),
            "roofline": {"bound": "alu", "achieved": round(achieved, 3),
                         "peak": round(VALU_PEAK_T, 2), "unit": "TFLOP/s",
                         "frac": round(achieved / VALU_PEAK_T, 4), "traffic": PAIR_TRAFFIC_BYTES,
                         "traffic_measured_on": PAIR_TRAFFIC_COMMIT,
                         "kernel": "k_pair", "launches": pair_n,
                         "per_unit": f"{OPS_PER_INTERACTING:g} FP32 VALU ops per interacting "
                                     f"pair + {OPS_PER_LISTED_ONLY:g} per listed pair beyond r_c; "
                                     f"{counts['interacting_pairs']} + "
                                     f"{counts['listed_pairs'] - counts['interacting_pairs']} "
                                     "unique pairs per launch"},
        })
    if not args.cpu_only and not args.no_adjoint:
        result["adjoint"] = adjoint_ratio()
    if not args.cpu_only and not args.no_batch:
        result["batch"] = batch_throughput()
    if not args.cpu_only and not args.no_hmc:
        result["hmc"] = hmc_tuning()
    if not args.no_cpu_baseline:
        result["cpu_baseline"] = cpu_baseline(s)
    print(json.dumps(result), flush=True)
    # a run that raised a status flag (list or cell overflow, stale list) or
    # left non-finite coordinates measured something else: fail loudly
    if result.get("status_flags", 0) != 0 or result.get("finite") is False:
        print(f"bench: status flags {result.get('status_flags')}, finite "
              f"{result.get('finite')}: the measurement is not valid", file=sys.stderr, flush=True)
        sys.exit(3)


if __name__ == "__main__":
    main()
