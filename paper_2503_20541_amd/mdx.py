"""ctypes binding of libmdx (the C ABI declared in include/mdx.h).

Argument marshalling only: every step of the force evaluation runs in the HIP
kernels of libmdx.so. Device buffers are passed as raw addresses (for torch
tensors, ``t.data_ptr()``), streams as ``hipStream_t`` handles
(``torch.cuda.current_stream().cuda_stream``).

Importing this module loads libmdx.so from the package directory. When the
library is missing or older than any of its sources it is built first with
hipcc (``build.ensure_built``); if that fails the import raises ImportError.
There is no fallback path.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libmdx.so")

from . import build as _build

try:
    _build.ensure_built()
except Exception as exc:          # no hipcc, or the sources do not compile
    raise ImportError(f"libmdx.so could not be built at {LIB_PATH}: {exc}") from exc
_lib = ctypes.CDLL(LIB_PATH)

# ---- constants mirrored from mdx.h ------------------------------------------
MDX_OK = 0
MDX_E_INVALID = -1
MDX_E_BOX_TOO_SMALL = -2
MDX_E_HIP = -3
MDX_E_CAPACITY = -4
MDX_E_NO_LIST = -5
MDX_E_NO_PME = -6
MDX_E_OUT_OF_MEMORY = -7
MDX_E_UNSUPPORTED = -8

MDX_FLAG_NL_OVERFLOW = 0x1
MDX_FLAG_NL_STALE = 0x2
MDX_FLAG_NONFINITE = 0x4
MDX_FLAG_OUT_OF_BOX = 0x8
MDX_FLAG_CELL_OVERFLOW = 0x10
MDX_FLAG_COLUMN_OVERFLOW = 0x20
MDX_FLAG_CONSTRAINT = 0x40

MDX_ENERGY_LJ = 0
MDX_ENERGY_COUL_DIR = 1
MDX_ENERGY_COUL_EXCL = 2
MDX_ENERGY_COUL_SELF = 3
MDX_ENERGY_BOND = 4
MDX_ENERGY_ANGLE = 5
MDX_ENERGY_COUL_REC = 6
MDX_ENERGY_KINETIC = 7
MDX_N_ENERGY = 8

MDX_OPT_HALF_LIST = 0x1
MDX_OPT_COOPERATIVE_BUILD = 0x2
MDX_OPT_KAHAN_VV = 0x4

MDX_TIMING_PAIR = 0
MDX_TIMING_PME = 1
MDX_TIMING_BUILD = 2

EXPORTED = ("mdx_error_string", "mdx_create", "mdx_destroy", "mdx_set_stream",
            "mdx_build_neighbors", "mdx_get_neighbor_pairs", "mdx_compute_nonbonded",
            "mdx_compute_pme", "mdx_integrate_step", "mdx_get_status", "mdx_get_info",
            "mdx_set_timing", "mdx_get_timing", "mdx_get_images", "mdx_set_langevin",
            "mdx_compute_ewald_direct", "mdx_set_rigid_water", "mdx_state_size",
            "mdx_save_state", "mdx_load_state", "mdx_compute_ewald_direct_noalloc",
            "mdx_ewald_direct_noalloc_bytes", "mdx_set_parameters", "mdx_set_charge_direction",
            "mdx_adjoint_begin", "mdx_adjoint_segment", "mdx_reset_images", "mdx_get_unwrapped",
            "mdx_set_graph", "mdx_set_masses", "mdx_adjoint_inject", "mdx_batch_create",
            "mdx_batch_integrate", "mdx_batch_destroy", "mdx_autotune")

_fp = ctypes.POINTER(ctypes.c_float)
_ip = ctypes.POINTER(ctypes.c_int32)


class SystemDesc(ctypes.Structure):
    _fields_ = [
        ("n_atoms", ctypes.c_int32), ("box", ctypes.c_float * 3),
        ("charge", _fp), ("mass", _fp), ("atom_type", _ip),
        ("n_types", ctypes.c_int32), ("type_sigma", _fp), ("type_epsilon", _fp),
        ("n_exclusions", ctypes.c_int32), ("exclusions", _ip),
        ("n_bonds", ctypes.c_int32), ("bonds", _ip), ("bond_k", _fp), ("bond_r0", _fp),
        ("n_angles", ctypes.c_int32), ("angles", _ip), ("angle_k", _fp),
        ("angle_theta0", _fp),
        ("r_cut", ctypes.c_float), ("r_ghost", ctypes.c_float), ("switch_r", ctypes.c_float),
        ("ewald_delta", ctypes.c_double), ("ewald_alpha", ctypes.c_double),
        ("pme_grid", ctypes.c_int32 * 3), ("pme_order", ctypes.c_int32),
        ("coulomb_k", ctypes.c_double), ("accel", ctypes.c_double),
        ("boltzmann", ctypes.c_double),
        ("cell_divisions", ctypes.c_int32), ("nl_capacity", ctypes.c_int32),
        ("rebuild_every", ctypes.c_int32), ("options", ctypes.c_uint32),
        ("rf_epsilon", ctypes.c_double),
    ]


class Info(ctypes.Structure):
    _fields_ = [
        ("n_atoms", ctypes.c_int32), ("cell_dims", ctypes.c_int32 * 3),
        ("cell_divisions", ctypes.c_int32), ("nl_capacity", ctypes.c_int32),
        ("pme_grid", ctypes.c_int32 * 3), ("pme_brick", ctypes.c_int32 * 3),
        ("alpha", ctypes.c_double), ("r_list", ctypes.c_double),
        ("n_list_entries", ctypes.c_int64), ("steps_taken", ctypes.c_int64),
        ("n_builds", ctypes.c_int64), ("n_list_tiles", ctypes.c_int64),
    ]


_vp = ctypes.c_void_p
_lib.mdx_error_string.restype = ctypes.c_char_p
_lib.mdx_error_string.argtypes = [ctypes.c_int]
_lib.mdx_create.argtypes = [ctypes.POINTER(_vp), ctypes.POINTER(SystemDesc), _vp]
_lib.mdx_destroy.argtypes = [_vp]
_lib.mdx_set_stream.argtypes = [_vp, _vp]
_lib.mdx_build_neighbors.argtypes = [_vp, _vp]
_lib.mdx_get_neighbor_pairs.argtypes = [_vp, _vp, ctypes.c_int64, ctypes.POINTER(ctypes.c_int64)]
_lib.mdx_compute_nonbonded.argtypes = [_vp, _vp, _vp, _vp, _vp]
_lib.mdx_compute_pme.argtypes = [_vp, _vp, _vp, _vp, _vp]
_lib.mdx_integrate_step.argtypes = [_vp, _vp, _vp, _vp, ctypes.c_int32, ctypes.c_float, _vp]
_lib.mdx_get_status.argtypes = [_vp, ctypes.POINTER(ctypes.c_uint32)]
_lib.mdx_get_images.argtypes = [_vp, _vp]
_lib.mdx_set_langevin.argtypes = [_vp, ctypes.c_double, ctypes.c_double, ctypes.c_uint64]
_lib.mdx_compute_ewald_direct.argtypes = [_vp, _vp, _vp, _vp, ctypes.c_int32]
_lib.mdx_compute_ewald_direct_noalloc.argtypes = [_vp, _vp, _vp, _vp, ctypes.c_int32]
_lib.mdx_ewald_direct_noalloc_bytes.argtypes = [ctypes.c_int32, ctypes.c_int32,
                                                ctypes.POINTER(ctypes.c_int64),
                                                ctypes.POINTER(ctypes.c_int64)]
_lib.mdx_set_rigid_water.argtypes = [_vp, _vp, ctypes.c_int32, ctypes.c_double, ctypes.c_double]
_lib.mdx_get_info.argtypes = [_vp, ctypes.POINTER(Info)]
_lib.mdx_state_size.argtypes = [_vp, ctypes.POINTER(ctypes.c_int64)]
_lib.mdx_save_state.argtypes = [_vp, _vp, ctypes.c_int64]
_lib.mdx_load_state.argtypes = [_vp, _vp, ctypes.c_int64]
_lib.mdx_set_parameters.argtypes = [_vp, _vp, _vp, _vp]
_lib.mdx_set_charge_direction.argtypes = [_vp, _vp]
_lib.mdx_adjoint_begin.argtypes = [_vp, _vp, _vp, _vp, _vp, _vp, _vp, _vp, _vp]
_lib.mdx_adjoint_segment.argtypes = [_vp, _vp, _vp, _vp, ctypes.c_int32, ctypes.c_float,
                                     ctypes.c_int32, _vp, _vp, _vp, _vp]
_lib.mdx_set_masses.argtypes = [_vp, _vp]
_lib.mdx_adjoint_inject.argtypes = [_vp, _vp, _vp, _vp, _vp, _vp, _vp]
_lib.mdx_reset_images.argtypes = [_vp]
_lib.mdx_set_graph.argtypes = [_vp, ctypes.c_int32]
_lib.mdx_batch_create.argtypes = [ctypes.POINTER(_vp), ctypes.POINTER(_vp), ctypes.c_int32,
                                  ctypes.c_int32]
_lib.mdx_batch_integrate.argtypes = [_vp, ctypes.POINTER(_vp), ctypes.POINTER(_vp),
                                     ctypes.POINTER(_vp), ctypes.c_int32,
                                     ctypes.POINTER(ctypes.c_float), _vp]
_lib.mdx_batch_destroy.argtypes = [_vp]
_lib.mdx_autotune.argtypes = [ctypes.POINTER(SystemDesc), _vp, _vp, ctypes.c_float,
                              ctypes.c_int32, _vp, ctypes.POINTER(ctypes.c_int32),
                              ctypes.POINTER(ctypes.c_uint32), ctypes.POINTER(ctypes.c_double)]
_lib.mdx_get_unwrapped.argtypes = [_vp, _vp, _vp]
_lib.mdx_set_timing.argtypes = [_vp, ctypes.c_int]
_lib.mdx_get_timing.argtypes = [_vp, ctypes.c_int, ctypes.POINTER(ctypes.c_double),
                                ctypes.POINTER(ctypes.c_int64)]
for _name in EXPORTED[1:]:
    getattr(_lib, _name).restype = ctypes.c_int


class MdxError(RuntimeError):
    def __init__(self, code: int, where: str):
        super().__init__(f"{where}: {error_string(code)} ({code})")
        self.code = code


def error_string(code: int) -> str:
    return _lib.mdx_error_string(int(code)).decode()


def _check(code: int, where: str) -> int:
    if code != MDX_OK:
        raise MdxError(code, where)
    return code


def _ptr(x) -> int | None:
    """Device/host address of a torch tensor, numpy array or int (None -> NULL)."""
    if x is None:
        return None
    if isinstance(x, int):
        return x
    if hasattr(x, "data_ptr"):
        return x.data_ptr()
    if isinstance(x, np.ndarray):
        return x.ctypes.data
    raise TypeError(f"cannot take the address of {type(x)}")


def make_desc(n_atoms, box, charge, mass, atom_type, type_sigma, type_epsilon,
              exclusions=None, bonds=None, bond_k=None, bond_r0=None, angles=None,
              angle_k=None, angle_theta0=None, r_cut=1.0, r_ghost=0.0, switch_r=0.0,
              ewald_delta=0.0, ewald_alpha=0.0, pme_grid=(0, 0, 0), pme_order=4,
              coulomb_k=1.0, accel=1.0, boltzmann=1.0, cell_divisions=0, nl_capacity=0,
              rebuild_every=10, options=0, rf_epsilon=0.0):
    """Fills an mdx_system_desc from host arrays. Returns (desc, keepalive)."""
    keep = []

    def arr(a, dt, shape=None):
        if a is None:
            return None
        a = np.ascontiguousarray(np.asarray(a, dtype=dt))
        if shape is not None:
            a = a.reshape(shape)
        keep.append(a)
        return a

    def p(a, ct):
        return a.ctypes.data_as(ctypes.POINTER(ct)) if a is not None and a.size else None

    ex = arr(exclusions if exclusions is not None else np.zeros((0, 2)), np.int32, (-1, 2))
    bo = arr(bonds if bonds is not None else np.zeros((0, 2)), np.int32, (-1, 2))
    an = arr(angles if angles is not None else np.zeros((0, 3)), np.int32, (-1, 3))
    d = SystemDesc()
    d.n_atoms = int(n_atoms)
    d.box[:] = [float(v) for v in np.asarray(box, np.float32).reshape(3)]
    d.charge = p(arr(charge, np.float32), ctypes.c_float)
    d.mass = p(arr(mass, np.float32), ctypes.c_float)
    d.atom_type = p(arr(atom_type, np.int32), ctypes.c_int32)
    ts = arr(type_sigma, np.float32)
    d.n_types = int(ts.size)
    d.type_sigma = p(ts, ctypes.c_float)
    d.type_epsilon = p(arr(type_epsilon, np.float32), ctypes.c_float)
    d.n_exclusions = int(len(ex))
    d.exclusions = p(ex, ctypes.c_int32)
    d.n_bonds = int(len(bo))
    d.bonds = p(bo, ctypes.c_int32)
    d.bond_k = p(arr(bond_k if bond_k is not None else [], np.float32), ctypes.c_float)
    d.bond_r0 = p(arr(bond_r0 if bond_r0 is not None else [], np.float32), ctypes.c_float)
    d.n_angles = int(len(an))
    d.angles = p(an, ctypes.c_int32)
    d.angle_k = p(arr(angle_k if angle_k is not None else [], np.float32), ctypes.c_float)
    d.angle_theta0 = p(arr(angle_theta0 if angle_theta0 is not None else [], np.float32),
                       ctypes.c_float)
    d.r_cut = float(r_cut)
    d.r_ghost = float(r_ghost)
    d.switch_r = float(switch_r)
    d.ewald_delta = float(ewald_delta)
    d.ewald_alpha = float(ewald_alpha)
    d.pme_grid[:] = [int(k) for k in pme_grid]
    d.pme_order = int(pme_order)
    d.coulomb_k = float(coulomb_k)
    d.accel = float(accel)
    d.boltzmann = float(boltzmann)
    d.cell_divisions = int(cell_divisions)
    d.nl_capacity = int(nl_capacity)
    d.rebuild_every = int(rebuild_every)
    d.options = int(options)
    d.rf_epsilon = float(rf_epsilon)
    return d, keep


def desc_from_system(sys, **overrides):
    """mdx_system_desc for an object carrying synth.System's fields."""
    kw = dict(n_atoms=sys.n_atoms, box=sys.box, charge=sys.charge, mass=sys.mass,
              atom_type=sys.atom_type, type_sigma=sys.type_sigma,
              type_epsilon=sys.type_epsilon, exclusions=sys.exclusions, bonds=sys.bonds,
              bond_k=sys.bond_k, bond_r0=sys.bond_r0, angles=sys.angles,
              angle_k=sys.angle_k, angle_theta0=sys.angle_theta0, r_cut=float(sys.r_cut),
              r_ghost=float(sys.r_ghost), switch_r=float(sys.switch_r),
              ewald_delta=float(sys.ewald_delta), pme_grid=tuple(sys.pme_grid),
              coulomb_k=float(sys.coulomb_k), accel=float(sys.accel),
              boltzmann=float(sys.boltzmann), rebuild_every=int(sys.rebuild_every),
              rf_epsilon=float(getattr(sys, "rf_epsilon", 0.0)))
    kw.update(overrides)
    return make_desc(**kw)


# ---- entry points (same names as the C ABI, without the prefix) -------------
def create(desc: SystemDesc, stream: int | None = None) -> int:
    h = _vp()
    _check(_lib.mdx_create(ctypes.byref(h), ctypes.byref(desc), stream), "mdx_create")
    return h.value


def destroy(ctx: int) -> None:
    _check(_lib.mdx_destroy(ctx), "mdx_destroy")


def set_stream(ctx: int, stream: int | None) -> None:
    _check(_lib.mdx_set_stream(ctx, stream), "mdx_set_stream")


def build_neighbors(ctx: int, pos) -> None:
    _check(_lib.mdx_build_neighbors(ctx, _ptr(pos)), "mdx_build_neighbors")


def get_neighbor_pairs(ctx: int) -> np.ndarray:
    n = ctypes.c_int64(0)
    rc = _lib.mdx_get_neighbor_pairs(ctx, None, 0, ctypes.byref(n))
    if rc not in (MDX_OK, MDX_E_CAPACITY):
        _check(rc, "mdx_get_neighbor_pairs")
    out = np.zeros((max(n.value, 1), 2), np.int32)
    _check(_lib.mdx_get_neighbor_pairs(ctx, out.ctypes.data, out.shape[0], ctypes.byref(n)),
           "mdx_get_neighbor_pairs")
    return out[:n.value]


def compute_nonbonded(ctx: int, pos, force, energy=None, virial=None) -> None:
    _check(_lib.mdx_compute_nonbonded(ctx, _ptr(pos), _ptr(force), _ptr(energy), _ptr(virial)),
           "mdx_compute_nonbonded")


def compute_pme(ctx: int, pos, force, energy=None, virial=None) -> None:
    _check(_lib.mdx_compute_pme(ctx, _ptr(pos), _ptr(force), _ptr(energy), _ptr(virial)),
           "mdx_compute_pme")


def integrate_step(ctx: int, pos, vel, force, n_steps: int, dt: float, energies=None) -> None:
    _check(_lib.mdx_integrate_step(ctx, _ptr(pos), _ptr(vel), _ptr(force), int(n_steps),
                                   float(dt), _ptr(energies)), "mdx_integrate_step")


def get_status(ctx: int) -> int:
    f = ctypes.c_uint32(0)
    _check(_lib.mdx_get_status(ctx, ctypes.byref(f)), "mdx_get_status")
    return int(f.value)


def compute_ewald_direct(ctx: int, pos, force, energy=None, n_max: int = 8) -> None:
    _check(_lib.mdx_compute_ewald_direct(ctx, _ptr(pos), _ptr(force), _ptr(energy), int(n_max)),
           "mdx_compute_ewald_direct")


def compute_ewald_direct_noalloc(ctx: int, pos, force, energy=None, n_max: int = 8) -> None:
    """compute_ewald_direct with the library's fixed scratch array (no allocation)."""
    _check(_lib.mdx_compute_ewald_direct_noalloc(ctx, _ptr(pos), _ptr(force), _ptr(energy),
                                                 int(n_max)),
           "mdx_compute_ewald_direct_noalloc")


def ewald_direct_noalloc_bytes(n_atoms: int, n_max: int):
    """(scratch bytes the no-allocation direct sum needs, the array's size)."""
    b = ctypes.c_int64(0)
    lim = ctypes.c_int64(0)
    _check(_lib.mdx_ewald_direct_noalloc_bytes(int(n_atoms), int(n_max), ctypes.byref(b),
                                               ctypes.byref(lim)),
           "mdx_ewald_direct_noalloc_bytes")
    return int(b.value), int(lim.value)


def set_rigid_water(ctx: int, mols, d_oh: float, d_hh: float) -> None:
    """Rigid water (RATTLE) for later integrate_step calls; mols: host int [M, 3]."""
    m = np.ascontiguousarray(np.asarray(mols, np.int32).reshape(-1, 3))
    _check(_lib.mdx_set_rigid_water(ctx, m.ctypes.data if m.size else None, int(len(m)),
                                    float(d_oh), float(d_hh)), "mdx_set_rigid_water")


def set_langevin(ctx: int, kT: float, gamma: float, seed: int) -> None:
    """Langevin (BAOAB) dynamics for later integrate_step calls; gamma = 0: VV."""
    _check(_lib.mdx_set_langevin(ctx, float(kT), float(gamma), int(seed) & ((1 << 64) - 1)),
           "mdx_set_langevin")


def get_images(ctx: int, img) -> None:
    """Copies the image counters (int32 [3][N] device tensor) into img."""
    _check(_lib.mdx_get_images(ctx, _ptr(img)), "mdx_get_images")


def state_size(ctx: int) -> int:
    n = ctypes.c_int64(0)
    _check(_lib.mdx_state_size(ctx, ctypes.byref(n)), "mdx_state_size")
    return int(n.value)


def save_state(ctx: int, state, capacity: int | None = None) -> None:
    """Writes the context's state into a device buffer (e.g. a uint8 tensor)."""
    cap = capacity if capacity is not None else state.numel() * state.element_size()
    _check(_lib.mdx_save_state(ctx, _ptr(state), int(cap)), "mdx_save_state")


def load_state(ctx: int, state, size: int | None = None) -> None:
    size = size if size is not None else state.numel() * state.element_size()
    _check(_lib.mdx_load_state(ctx, _ptr(state), int(size)), "mdx_load_state")


def _host_f32(a):
    if a is None:
        return None, None
    h = np.ascontiguousarray(np.asarray(a, dtype=np.float32))
    return h, h.ctypes.data


def set_parameters(ctx: int, type_sigma=None, type_epsilon=None, charge=None) -> None:
    """Host arrays (per type, per type, per atom); None leaves one unchanged."""
    s, sp = _host_f32(type_sigma)
    e, ep = _host_f32(type_epsilon)
    q, qp = _host_f32(charge)
    _check(_lib.mdx_set_parameters(ctx, sp, ep, qp), "mdx_set_parameters")


def set_charge_direction(ctx: int, dq) -> None:
    h, hp = _host_f32(dq)
    _check(_lib.mdx_set_charge_direction(ctx, hp), "mdx_set_charge_direction")


MDX_ADJ_FIRST = 0x1
MDX_ADJ_LAST = 0x2


def adjoint_begin(ctx: int, pos, force, gx, gU, q, p, grad, gv=None) -> None:
    _check(_lib.mdx_adjoint_begin(ctx, _ptr(pos), _ptr(force), _ptr(gx), _ptr(gv), _ptr(gU),
                                  _ptr(q), _ptr(p), _ptr(grad)), "mdx_adjoint_begin")


def adjoint_segment(ctx: int, x0, v0, f0, n_steps: int, dt: float, first: bool, q, p,
                    grad, last: bool = False, grad_mass=None) -> None:
    flags = (MDX_ADJ_FIRST if first else 0) | (MDX_ADJ_LAST if last else 0)
    _check(_lib.mdx_adjoint_segment(ctx, _ptr(x0), _ptr(v0), _ptr(f0), int(n_steps), float(dt),
                                    flags, _ptr(q), _ptr(p), _ptr(grad), _ptr(grad_mass)),
           "mdx_adjoint_segment")


def adjoint_inject(ctx: int, force, gx, gv, gU, q, p) -> None:
    _check(_lib.mdx_adjoint_inject(ctx, _ptr(force), _ptr(gx), _ptr(gv), _ptr(gU), _ptr(q),
                                   _ptr(p)), "mdx_adjoint_inject")


def set_masses(ctx: int, mass) -> None:
    h, hp = _host_f32(mass)
    _check(_lib.mdx_set_masses(ctx, hp), "mdx_set_masses")


def set_graph(ctx: int, chunk: int) -> None:
    """Replay integrate_step in chunk-step HIP graphs (0: launch by launch)."""
    _check(_lib.mdx_set_graph(ctx, int(chunk)), "mdx_set_graph")


def batch_create(ctxs, chunk: int) -> int:
    arr = (_vp * len(ctxs))(*ctxs)
    out = _vp()
    _check(_lib.mdx_batch_create(ctypes.byref(out), arr, len(ctxs), int(chunk)),
           "mdx_batch_create")
    return out.value


def batch_integrate(batch: int, pos, vel, force, n_steps: int, dt, stream) -> None:
    """pos, vel, force: sequences of device tensors (one per replica); dt:
    sequence of floats; stream: a hipStream_t handle."""
    n = len(pos)
    P = (_vp * n)(*[_ptr(t) for t in pos])
    V = (_vp * n)(*[_ptr(t) for t in vel])
    F = (_vp * n)(*[_ptr(t) for t in force])
    D = (ctypes.c_float * n)(*[float(d) for d in dt])
    _check(_lib.mdx_batch_integrate(batch, P, V, F, int(n_steps), D, stream),
           "mdx_batch_integrate")


def batch_destroy(batch: int) -> None:
    _check(_lib.mdx_batch_destroy(batch), "mdx_batch_destroy")


def autotune(desc, pos, vel, dt: float, steps: int, stream):
    """(cell_divisions, options, ms per step of the eight candidates)."""
    m = ctypes.c_int32(0)
    o = ctypes.c_uint32(0)
    ms = (ctypes.c_double * 8)()
    _check(_lib.mdx_autotune(ctypes.byref(desc), _ptr(pos), _ptr(vel), float(dt), int(steps),
                             stream, ctypes.byref(m), ctypes.byref(o), ms), "mdx_autotune")
    return int(m.value), int(o.value), list(ms)


def reset_images(ctx: int) -> None:
    _check(_lib.mdx_reset_images(ctx), "mdx_reset_images")


def get_unwrapped(ctx: int, pos, out) -> None:
    _check(_lib.mdx_get_unwrapped(ctx, _ptr(pos), _ptr(out)), "mdx_get_unwrapped")


def get_info(ctx: int) -> Info:
    info = Info()
    _check(_lib.mdx_get_info(ctx, ctypes.byref(info)), "mdx_get_info")
    return info


def set_timing(ctx: int, groups) -> None:
    """groups: True (all groups), False (none), or a bit mask of 1 << MDX_TIMING_*."""
    mask = 7 if groups is True else (0 if groups is False else int(groups))
    _check(_lib.mdx_set_timing(ctx, mask), "mdx_set_timing")


def get_timing(ctx: int, group: int):
    """(mean launch duration in ms, number of recorded launches)."""
    ms = ctypes.c_double(0.0)
    n = ctypes.c_int64(0)
    _check(_lib.mdx_get_timing(ctx, int(group), ctypes.byref(ms), ctypes.byref(n)),
           "mdx_get_timing")
    return ms.value, n.value


def library():
    """The loaded ctypes library (for symbol checks)."""
    return _lib
