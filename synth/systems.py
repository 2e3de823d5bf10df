"""Seeded synthetic systems: Lennard-Jones fluid and flexible 3-site water.

Every array the GPU path sees is generated in float64, rounded once to its
storage type (float32 / int32) and stored here; the oracle widens the same
rounded arrays to float64. Nothing here evaluates the model.

Workload shapes follow the paper's water-box benchmarks (TIP3P-shaped water at
~1 g/cm^3, 3-site charges, LJ on oxygen only, 9-10 A cutoff; Sec. III.A) and
the LJ fluid used for integrator checks.
"""
from __future__ import annotations

import dataclasses
import math

import numpy as np

# ---------------------------------------------------------------------------
# Unit systems (input constants, not method arithmetic).
#   real units: kcal/mol, Angstrom, amu, fs, elementary charge
#   coulomb_k  = 138.935456 kJ nm/(mol e^2) expressed in kcal A/(mol e^2)
#   accel      = converts (kcal/mol/A)/amu into A/fs^2
#   boltzmann  = kcal/(mol K)
# ---------------------------------------------------------------------------
REAL_UNITS = dict(coulomb_k=138.935456 * 10.0 / 4.184, accel=4.184e-4,
                  boltzmann=0.0019872041)
REDUCED_UNITS = dict(coulomb_k=1.0, accel=1.0, boltzmann=1.0)

# Water model (flexible 3-site, TIP3P-like charges and O-only LJ).
WATER = dict(q_O=-0.834, q_H=0.417, sigma_O=3.1507, eps_O=0.1521,
             bond_k=450.0, bond_r0=0.9572, angle_k=55.0,
             angle_theta0_deg=104.52, m_O=15.9994, m_H=1.008)

WATER_MOLECULE_DENSITY = 0.033383  # molecules / A^3 (about 0.998 g/cm^3)


@dataclasses.dataclass
class System:
    """A periodic system in the layout the C-ABI consumes.

    pos, vel: float32 [3, N] (structure of arrays); box: float32 [3].
    Per-atom charge/mass float32 [N], atom_type int32 [N]; per-type
    type_sigma/type_epsilon float32 [T].  Topology: exclusions int32 [E, 2],
    bonds int32 [B, 2] (+ bond_k, bond_r0), angles int32 [A, 3] as
    (end, vertex, end) (+ angle_k, angle_theta0 in radians).
    """
    name: str
    box: np.ndarray
    pos: np.ndarray
    vel: np.ndarray
    charge: np.ndarray
    mass: np.ndarray
    atom_type: np.ndarray
    type_sigma: np.ndarray
    type_epsilon: np.ndarray
    exclusions: np.ndarray
    bonds: np.ndarray
    bond_k: np.ndarray
    bond_r0: np.ndarray
    angles: np.ndarray
    angle_k: np.ndarray
    angle_theta0: np.ndarray
    r_cut: np.float32
    r_ghost: np.float32
    ewald_delta: float           # 0 -> no electrostatics
    pme_grid: tuple              # (0,0,0) -> no PME
    coulomb_k: float
    accel: float
    boltzmann: float
    dt: float
    n_steps: int
    rebuild_every: int
    switch_r: np.float32 = np.float32(0.0)   # <= 0: plain truncation
    rf_epsilon: float = 0.0      # > 0: reaction-field Coulomb with this eps_s (inf allowed)

    @property
    def n_atoms(self) -> int:
        return int(self.pos.shape[1])

    def copy(self) -> "System":
        return dataclasses.replace(
            self, **{f.name: (getattr(self, f.name).copy()
                              if isinstance(getattr(self, f.name), np.ndarray)
                              else getattr(self, f.name))
                     for f in dataclasses.fields(self)})


def _rng(config_index: int, stream: int) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(20541 + 10 * config_index + stream))


def _to_box_f32(x64: np.ndarray, box32: np.ndarray) -> np.ndarray:
    """Round positions to float32 inside [0, L) per dimension."""
    L = box32.astype(np.float64)[:, None]
    x = np.mod(x64, L)
    x32 = x.astype(np.float32)
    # rounding can land exactly on L; keep the half-open interval
    for d in range(3):
        row = x32[d]
        row[row >= box32[d]] = np.float32(0.0)
        row[row < 0] = np.float32(0.0)
    return x32


def _maxwell_boltzmann(rng, mass64, temperature, boltzmann, accel):
    """Velocities with per-component variance kB*T*accel/m; COM momentum removed."""
    sd = np.sqrt(boltzmann * temperature * accel / mass64)
    v = rng.standard_normal((3, mass64.size)) * sd[None, :]
    p = (v * mass64[None, :]).sum(axis=1) / mass64.sum()
    v -= p[:, None]
    return v.astype(np.float32)


# ---------------------------------------------------------------------------
# Lennard-Jones fluid
# ---------------------------------------------------------------------------
def lj_fluid(n_side: int = 10, density: float = 0.8, jitter: float = 0.1,
             r_cut: float = 2.5, r_ghost: float = 0.3, temperature: float = 1.0,
             config_index: int = 0, dt: float = 0.005, n_steps: int = 100,
             rebuild_every: int = 10, name: str = "lj") -> System:
    """Simple-cubic lattice of n_side^3 atoms at reduced density, sigma=eps=m=1."""
    n = n_side ** 3
    L64 = (n / density) ** (1.0 / 3.0)
    box = np.full(3, L64, dtype=np.float32)
    a = L64 / n_side
    idx = np.arange(n)
    ix, iy, iz = idx // (n_side * n_side), (idx // n_side) % n_side, idx % n_side
    sites = np.stack([(ix + 0.5) * a, (iy + 0.5) * a, (iz + 0.5) * a])
    rng = _rng(config_index, 0)
    sites = sites + rng.uniform(-jitter, jitter, size=sites.shape)
    pos = _to_box_f32(sites, box)
    mass = np.ones(n, dtype=np.float32)
    vel = _maxwell_boltzmann(_rng(config_index, 1), mass.astype(np.float64),
                             temperature, 1.0, 1.0)
    return System(
        name=name, box=box, pos=pos, vel=vel,
        charge=np.zeros(n, np.float32), mass=mass,
        atom_type=np.zeros(n, np.int32),
        type_sigma=np.array([1.0], np.float32), type_epsilon=np.array([1.0], np.float32),
        exclusions=np.zeros((0, 2), np.int32),
        bonds=np.zeros((0, 2), np.int32), bond_k=np.zeros(0, np.float32),
        bond_r0=np.zeros(0, np.float32),
        angles=np.zeros((0, 3), np.int32), angle_k=np.zeros(0, np.float32),
        angle_theta0=np.zeros(0, np.float32),
        r_cut=np.float32(r_cut), r_ghost=np.float32(r_ghost),
        ewald_delta=0.0, pme_grid=(0, 0, 0), dt=dt, n_steps=n_steps,
        rebuild_every=rebuild_every, **REDUCED_UNITS)


# ---------------------------------------------------------------------------
# Flexible 3-site water
# ---------------------------------------------------------------------------
def _random_rotations(rng, n):
    """Uniform random rotation matrices (Shoemake's quaternion method)."""
    u1, u2, u3 = rng.random(n), rng.random(n), rng.random(n)
    a = np.sqrt(1.0 - u1)
    b = np.sqrt(u1)
    qx, qy = a * np.sin(2 * np.pi * u2), a * np.cos(2 * np.pi * u2)
    qz, qw = b * np.sin(2 * np.pi * u3), b * np.cos(2 * np.pi * u3)
    R = np.empty((n, 3, 3))
    R[:, 0, 0] = 1 - 2 * (qy * qy + qz * qz)
    R[:, 0, 1] = 2 * (qx * qy - qz * qw)
    R[:, 0, 2] = 2 * (qx * qz + qy * qw)
    R[:, 1, 0] = 2 * (qx * qy + qz * qw)
    R[:, 1, 1] = 1 - 2 * (qx * qx + qz * qz)
    R[:, 1, 2] = 2 * (qy * qz - qx * qw)
    R[:, 2, 0] = 2 * (qx * qz - qy * qw)
    R[:, 2, 1] = 2 * (qy * qz + qx * qw)
    R[:, 2, 2] = 1 - 2 * (qx * qx + qy * qy)
    return R


def _molecule_atoms(O, R, r0, theta0):
    """O positions (n,3) and rotations (n,3,3) -> atoms (n,3,3) as O,H,H."""
    h = 0.5 * theta0
    body = np.array([[0.0, 0.0, 0.0],
                     [r0 * math.sin(h), 0.0, r0 * math.cos(h)],
                     [-r0 * math.sin(h), 0.0, r0 * math.cos(h)]])
    return O[:, None, :] + np.einsum("nab,kb->nka", R, body)


def water_box(n_mol: int, box_len: float, pme_grid=(48, 48, 48), r_cut: float = 9.0,
              r_ghost: float | None = None, ewald_delta: float = 5e-4,
              config_index: int = 1, temperature: float = 300.0, o_jitter: float = 0.3,
              min_intermolecular: float = 1.7, dt: float = 1.0, n_steps: int = 100,
              rebuild_every: int = 10, name: str = "water") -> System:
    """Water molecules on a jittered cubic lattice with random orientations.

    n_side^3 >= n_mol lattice sites; n_mol of them chosen by a seeded
    permutation and kept in lattice order. Orientations are resampled (at most
    100 rounds) until no intermolecular atom pair is closer than
    `min_intermolecular` (H carries no LJ and would otherwise collapse onto O).
    """
    from scipy.spatial import cKDTree  # input generation only

    W = WATER
    n_side = int(math.ceil(n_mol ** (1.0 / 3.0) - 1e-9))
    box = np.full(3, box_len, dtype=np.float32)
    L64 = float(box[0])
    a = L64 / n_side
    rng = _rng(config_index, 0)
    chosen = np.sort(rng.permutation(n_side ** 3)[:n_mol])
    ix, iy, iz = chosen // (n_side * n_side), (chosen // n_side) % n_side, chosen % n_side
    O = np.stack([(ix + 0.5) * a, (iy + 0.5) * a, (iz + 0.5) * a], axis=1)
    O = O + rng.uniform(-o_jitter, o_jitter, size=O.shape)
    theta0 = math.radians(W["angle_theta0_deg"])
    R = _random_rotations(rng, n_mol)
    for _ in range(100):
        atoms = _molecule_atoms(O, R, W["bond_r0"], theta0).reshape(-1, 3)
        tree = cKDTree(np.mod(atoms, L64), boxsize=L64)
        pairs = tree.query_pairs(min_intermolecular, output_type="ndarray")
        inter = pairs[(pairs[:, 0] // 3) != (pairs[:, 1] // 3)]
        if inter.size == 0:
            break
        bad = np.unique(inter // 3)
        R[bad] = _random_rotations(rng, bad.size)
    else:
        raise RuntimeError("water_box: could not resolve close contacts")
    atoms = _molecule_atoms(O, R, W["bond_r0"], theta0).reshape(-1, 3).T
    pos = _to_box_f32(atoms, box)

    n = 3 * n_mol
    is_O = (np.arange(n) % 3) == 0
    charge = np.where(is_O, W["q_O"], W["q_H"]).astype(np.float32)
    mass64 = np.where(is_O, W["m_O"], W["m_H"])
    atom_type = np.where(is_O, 0, 1).astype(np.int32)
    o = np.arange(n_mol, dtype=np.int32) * 3
    bonds = np.concatenate([np.stack([o, o + 1], 1), np.stack([o, o + 2], 1)])
    bonds = bonds[np.lexsort((bonds[:, 1], bonds[:, 0]))]
    exclusions = np.concatenate([bonds, np.stack([o + 1, o + 2], 1)])
    exclusions = exclusions[np.lexsort((exclusions[:, 1], exclusions[:, 0]))].astype(np.int32)
    angles = np.stack([o + 1, o, o + 2], 1).astype(np.int32)
    vel = _maxwell_boltzmann(_rng(config_index, 1), mass64, temperature,
                             REAL_UNITS["boltzmann"], REAL_UNITS["accel"])
    return System(
        name=name, box=box, pos=pos, vel=vel, charge=charge,
        mass=mass64.astype(np.float32), atom_type=atom_type,
        type_sigma=np.array([W["sigma_O"], 1.0], np.float32),
        type_epsilon=np.array([W["eps_O"], 0.0], np.float32),
        exclusions=exclusions, bonds=bonds.astype(np.int32),
        bond_k=np.full(len(bonds), W["bond_k"], np.float32),
        bond_r0=np.full(len(bonds), W["bond_r0"], np.float32),
        angles=angles, angle_k=np.full(n_mol, W["angle_k"], np.float32),
        angle_theta0=np.full(n_mol, theta0, np.float32),
        r_cut=np.float32(r_cut),
        r_ghost=np.float32(0.25 * r_cut if r_ghost is None else r_ghost),
        ewald_delta=ewald_delta, pme_grid=tuple(int(k) for k in pme_grid),
        dt=dt, n_steps=n_steps, rebuild_every=rebuild_every, **REAL_UNITS)


# ---------------------------------------------------------------------------
# Small random boxes for property tests
# ---------------------------------------------------------------------------
def random_box(n_atoms: int, box, r_cut: float, r_ghost: float, seed: int,
               n_types: int = 3, charged: bool = True, n_excl_per_atom: int = 1,
               pme_grid=(0, 0, 0), ewald_delta: float = 5e-4,
               min_dist: float = 0.0) -> System:
    """Uniform random atoms with random types, a neutral charge set and a few
    random exclusions between atoms of nearby index. Reduced-like units."""
    rng = np.random.Generator(np.random.PCG64(seed))
    box = np.asarray(box, dtype=np.float32).reshape(3)
    x = rng.random((3, n_atoms)) * box.astype(np.float64)[:, None]
    if min_dist > 0:
        from scipy.spatial import cKDTree
        for _ in range(200):
            pts = np.mod(x.T, box.astype(np.float64))
            tree = cKDTree(pts, boxsize=box.astype(np.float64))
            bad = np.unique(tree.query_pairs(min_dist, output_type="ndarray")[:, 1])
            if bad.size == 0:
                break
            x[:, bad] = rng.random((3, bad.size)) * box.astype(np.float64)[:, None]
    pos = _to_box_f32(x, box)
    atom_type = rng.integers(0, n_types, n_atoms).astype(np.int32)
    sig = rng.uniform(0.8, 1.2, n_types).astype(np.float32)
    eps = rng.uniform(0.5, 1.5, n_types).astype(np.float32)
    if charged:
        q = rng.uniform(-1, 1, n_atoms)
        q -= q.mean()
        charge = q.astype(np.float32)
    else:
        charge = np.zeros(n_atoms, np.float32)
    ex = []
    for i in range(n_atoms):
        for _ in range(n_excl_per_atom):
            j = int((i + rng.integers(1, 4)) % n_atoms)
            if j != i:
                ex.append((min(i, j), max(i, j)))
    ex = np.array(sorted(set(ex)), dtype=np.int32).reshape(-1, 2)
    mass = rng.uniform(1.0, 2.0, n_atoms).astype(np.float32)
    vel = _maxwell_boltzmann(np.random.Generator(np.random.PCG64(seed + 1)),
                             mass.astype(np.float64), 1.0, 1.0, 1.0)
    return System(
        name=f"random{n_atoms}", box=box, pos=pos, vel=vel, charge=charge, mass=mass,
        atom_type=atom_type, type_sigma=sig, type_epsilon=eps, exclusions=ex,
        bonds=np.zeros((0, 2), np.int32), bond_k=np.zeros(0, np.float32),
        bond_r0=np.zeros(0, np.float32), angles=np.zeros((0, 3), np.int32),
        angle_k=np.zeros(0, np.float32), angle_theta0=np.zeros(0, np.float32),
        r_cut=np.float32(r_cut), r_ghost=np.float32(r_ghost),
        ewald_delta=(ewald_delta if charged else 0.0), pme_grid=tuple(pme_grid),
        dt=0.002, n_steps=10, rebuild_every=10, **REDUCED_UNITS)


# ---------------------------------------------------------------------------
# Batched replicas
# ---------------------------------------------------------------------------
def lj_fluid_n(n_atoms: int, density: float = 0.8, seed_stream: int = 0, jitter: float = 0.1,
               r_cut: float = 2.5, r_ghost: float = 0.3, temperature: float = 1.0,
               dt: float = 0.005, name: str = "lj") -> System:
    """LJ fluid of any size: n_atoms of the n_side^3 >= n_atoms sites of a
    simple-cubic lattice at reduced density, chosen by a seeded permutation
    and kept in lattice order."""
    n_side = int(math.ceil(n_atoms ** (1.0 / 3.0) - 1e-9))
    L64 = (n_atoms / density) ** (1.0 / 3.0)
    a = L64 / n_side
    rng = np.random.Generator(np.random.PCG64(20541 + 30 + seed_stream))
    keep = np.sort(rng.permutation(n_side ** 3)[:n_atoms])
    ix, iy, iz = keep // (n_side * n_side), (keep // n_side) % n_side, keep % n_side
    sites = np.stack([(ix + 0.5) * a, (iy + 0.5) * a, (iz + 0.5) * a])
    sites = sites + rng.uniform(-jitter, jitter, size=sites.shape)
    box = np.full(3, L64, dtype=np.float32)
    s = lj_fluid(2, density, 0.0, r_cut, r_ghost, temperature, 0, dt, 10, 10, name)
    mass = np.ones(n_atoms, dtype=np.float32)
    return dataclasses.replace(
        s, box=box, pos=_to_box_f32(sites, box),
        vel=_maxwell_boltzmann(rng, mass.astype(np.float64), temperature, 1.0, 1.0),
        charge=np.zeros(n_atoms, np.float32), mass=mass,
        atom_type=np.zeros(n_atoms, np.int32))


def smooth_grid_size(n: int) -> int:
    """Smallest 2^a 3^b 5^c >= n (an FFT-friendly grid dimension)."""
    k = max(4, int(n))
    while True:
        m = k
        for p in (2, 3, 5):
            while m % p == 0:
                m //= p
        if m == 1:
            return k
        k += 1


def batch_replicas(n_rep: int = 256, n_min: int = 500, n_max: int = 20000,
                   water_min_atoms: int = 1143) -> list:
    """The batched-replica workload: even index an LJ fluid at reduced density
    0.8, odd index flexible water at 0.033383 molecules/A^3, sizes
    round(exp(U(ln n_min, ln n_max))); water sizes rounded to whole molecules
    and clamped to >= water_min_atoms (a smaller box is under twice the list
    radius, 2 (9 + 2.25) A); per-replica box and a PME grid of about 1 A
    spacing (the next 2^a 3^b 5^c)."""
    rng = np.random.Generator(np.random.PCG64(20541 + 30))
    sizes = np.rint(np.exp(rng.uniform(math.log(n_min), math.log(n_max), n_rep))).astype(int)
    out = []
    for r, n in enumerate(sizes):
        if r % 2 == 0:
            out.append(lj_fluid_n(int(n), 0.8, seed_stream=r, name=f"lj{n}_{r}"))
        else:
            n_mol = max(int(round(n / 3)), -(-water_min_atoms // 3))
            L = (n_mol / WATER_MOLECULE_DENSITY) ** (1.0 / 3.0)
            K = smooth_grid_size(int(math.ceil(L)))
            # little oxygen jitter: a size just above a lattice cube leaves ~2.7 A sites
            out.append(water_box(n_mol, L, (K, K, K), 9.0, None, 5e-4, 3, o_jitter=0.05,
                                 name=f"water{3 * n_mol}_{r}"))
    return out


# ---------------------------------------------------------------------------
# Named workload configurations
# ---------------------------------------------------------------------------
CONFIGS = {
    # LJ fluid, N=1000, rho*=0.8, cutoff 2.5 sigma, skin 0.3 sigma, 100 VV steps
    "lj1k": lambda: lj_fluid(10, 0.8, 0.1, 2.5, 0.3, 1.0, 0, 0.005, 100, 10, "lj1k"),
    # 3,000 waters (9,000 atoms), L=44.8 A, cutoff 9 A, PME 48^3
    "water9k": lambda: water_box(3000, 44.8, (48, 48, 48), 9.0, None, 5e-4, 1,
                                 name="water9k"),
    # 32,000 waters (96,000 atoms), L=98.6 A, cutoff 9 A, PME 100^3, dt 1 fs
    "water96k": lambda: water_box(32000, 98.6, (100, 100, 100), 9.0, None, 5e-4, 2,
                                  n_steps=1000, name="water96k"),
    # small water box for fast oracle-side tests (cutoff/skin scaled down)
    "water375": lambda: water_box(125, 15.54, (16, 16, 16), 6.0, 1.5, 5e-4, 7,
                                  name="water375"),
}


def config_system(name: str) -> System:
    return CONFIGS[name]()
