"""Gradients of a velocity-Verlet trajectory loss, FP64 (the paper's premise,
Sec. I and Sec. IV: the simulation is differentiable end to end, so a loss
on a trajectory can be differentiated with respect to the force-field
parameters, the initial state and the time step).

TEST INFRASTRUCTURE ONLY (see oracle/__init__.py).

Loss (the reading of "mean final potential energy + MSD"):

    L = U(x_T) / N + (1/N) sum_i |x_T,i - x_0,i|^2

with unwrapped coordinates and the initial velocities held fixed. Parameters:
per-type LJ epsilon and sigma, and a scalar t that moves the charges along a
fixed direction, q(t) = q + t dq (for water, dq = 1 on O and -1/2 on H ties
q_H = -q_O / 2); the gradient with respect to t is the gradient with respect
to q_O.

Interaction set. A plain cutoff makes the loss discontinuous where a pair
crosses r_c; the gradient computed here is that of the frozen-set loss: the
pairs that interact at each step of the unperturbed run (r < r_c, excluded
pairs removed) are recorded and reused, so the loss is smooth and central
finite differences with the same sets converge to it.

Derivatives of the forces. `force_field` below evaluates U and F = -dU/dx
with complex-safe arithmetic (the minimum-image shift and the B-spline cell
are chosen from the real parts; no conjugates or absolute values), so a
directional derivative of F along u is Im F(x + i h u) / h to machine
precision (complex-step differentiation, Squire and Trapp 1998; Martins,
Sturdza and Alonso 2003). It is pinned to the plain oracle on real inputs.

Reverse recursion. One step of velocity Verlet (Sec. II.D.1) with
a(x) = c F(x) / m is

    v'      = v_n + (dt/2) a(x_n)
    x_{n+1} = x_n + dt v'
    v_{n+1} = v' + (dt/2) a(x_{n+1})

Given the adjoints (Xb, Vb) = (dL/dx_{n+1}, dL/dv_{n+1}) the chain rule
gives, in this order,

    xt  = Xb + (dt/2) J(x_{n+1})^T Vb           x_{n+1} feeds v_{n+1}
    vpb = Vb + dt xt                             v' feeds x_{n+1} and v_{n+1}
    Xb  = xt + (dt/2) J(x_n)^T vpb               x_n feeds x_{n+1} and v'
    Vb  = vpb
    theta_b += (dt/2) [da(x_{n+1})/dtheta]^T Vb_old + (dt/2) [da(x_n)/dtheta]^T vpb
    dt_b    += Vb_old . a_{n+1} / 2 + xt . v' + vpb . a_n / 2

with J = da/dx, so J^T w = c dF[w / m] (the Hessian is symmetric). The
recursion starts from Xb = dL/dx_T = -F(x_T)/N + 2 (x_T - x_0)/N, Vb = 0,
and the loss's direct dependence on x_0 (-2 (x_T - x_0)/N) is added at the
end.
"""
from __future__ import annotations

import math

import numpy as np
from scipy.special import erf, erfc

from . import pme as _pme

H_CS = 1e-30          # complex-step size (no cancellation, any tiny value works)


# ---------------------------------------------------------------------------
# Complex-safe force field
# ---------------------------------------------------------------------------
def _disp(pos, box, i, j):
    """x_j - x_i at the nearest image, the image chosen from the real part."""
    L = np.asarray(box, np.float64)[:, None]
    d = pos[:, j] - pos[:, i]
    return d - L * np.round(d.real / L)


def _acc(n, i, j, fj, dtype):
    F = np.zeros((3, n), dtype)
    for a in range(3):
        np.add.at(F[a], j, fj[a])
        np.subtract.at(F[a], i, fj[a])
    return F


def _bspline(n, w):
    """Cardinal B-spline M_n(w) by the recursion of the PME paragraph, with
    M_2 taken piecewise by the real part of w (analytic inside a cell)."""
    if n == 2:
        wr = np.real(w)
        return np.where((wr >= 0) & (wr < 1), w, np.where((wr >= 1) & (wr <= 2), 2.0 - w, 0.0))
    return (w * _bspline(n - 1, w) + (n - w) * _bspline(n - 1, w - 1.0)) / (n - 1)


def _dbspline(n, w):
    return _bspline(n - 1, w) - _bspline(n - 1, w - 1.0)


def _spme_cs(pos, q, box, grid, alpha, ke, G, order=4):
    """Smooth PME energy and forces, complex-safe: E = (k_e/2) sum_k Q phi with
    phi = K1 K2 K3 ifftn(G fftn(Q)) (for real Q this is the plain oracle's
    (k_e/2) sum_m G |Q^|^2, since G is real and even)."""
    n = pos.shape[1]
    dt = np.result_type(pos, q)
    L = np.asarray(box, np.float64)
    idx, w, dw = [], [], []
    for d in range(3):
        K = int(grid[d])
        u = K * pos[d] / L[d]
        k0 = np.floor(u.real)
        t = np.arange(order)
        arg = (u - k0)[:, None] + t[None, :]
        idx.append(((k0[:, None] - t[None, :]) % K).astype(np.int64))
        w.append(_bspline(order, arg))
        dw.append(_dbspline(order, arg) * (K / L[d]))
    Q = np.zeros(tuple(int(k) for k in grid), dt)
    for a in range(order):
        for b in range(order):
            for c in range(order):
                np.add.at(Q, (idx[0][:, a], idx[1][:, b], idx[2][:, c]),
                          q * w[0][:, a] * w[1][:, b] * w[2][:, c])
    # the convolution is a real linear map (G real and even): applied to the
    # real and imaginary parts separately, so the transform's rounding in one
    # part never leaks into the other (which would swamp the complex step)
    conv = lambda R: np.fft.ifftn(G * np.fft.fftn(R)).real * float(np.prod(grid))
    phi = conv(Q.real) + 1j * conv(Q.imag) if np.iscomplexobj(Q) else conv(Q)
    E = 0.5 * ke * (Q * phi).sum()
    F = np.zeros((3, n), dt)
    for a in range(order):
        for b in range(order):
            for c in range(order):
                p = phi[idx[0][:, a], idx[1][:, b], idx[2][:, c]]
                F[0] -= dw[0][:, a] * w[1][:, b] * w[2][:, c] * p
                F[1] -= w[0][:, a] * dw[1][:, b] * w[2][:, c] * p
                F[2] -= w[0][:, a] * w[1][:, b] * dw[2][:, c] * p
    return E, F * (ke * q)[None, :]


class ForceField:
    """The system's model (LJ with Lorentz-Berthelot mixing, Eqs. 4-5; real-
    space Ewald, Eq. 10; the erf exclusion correction; the self and
    neutralising terms, Eq. 12; harmonic bonds and angles, Eqs. 1-2; smooth
    PME) with the parameters as explicit arguments:
    eps, sig: per type; charge: per atom. Any of them, and the positions, may
    be complex."""

    def __init__(self, sys):
        from . import forcefield
        self.sys = sys
        self.n = int(sys.pos.shape[1])
        self.box = np.asarray(sys.box, np.float64)
        self.alpha = forcefield.alpha(sys)
        self.ke = float(sys.coulomb_k)
        self.r_cut = float(sys.r_cut)
        self.types = np.asarray(sys.atom_type, np.int64)
        self.ex = np.asarray(sys.exclusions, np.int64).reshape(-1, 2)
        self.bonds = np.asarray(sys.bonds, np.int64).reshape(-1, 2)
        self.bond_k = np.asarray(sys.bond_k, np.float64)
        self.bond_r0 = np.asarray(sys.bond_r0, np.float64)
        self.angles = np.asarray(sys.angles, np.int64).reshape(-1, 3)
        self.angle_k = np.asarray(sys.angle_k, np.float64)
        self.angle_t0 = np.asarray(sys.angle_theta0, np.float64)
        self.grid = tuple(int(k) for k in sys.pme_grid)
        self.has_pme = self.alpha > 0 and sum(self.grid) > 0
        if self.has_pme:
            self.G = _pme.influence(self.grid, self.box, self.alpha)[0]
        ex_keys = np.minimum(self.ex[:, 0], self.ex[:, 1]) * self.n + \
            np.maximum(self.ex[:, 0], self.ex[:, 1])
        self.ex_keys = np.unique(ex_keys)

    def params0(self):
        s = self.sys
        return dict(eps=np.asarray(s.type_epsilon, np.float64).copy(),
                    sig=np.asarray(s.type_sigma, np.float64).copy(),
                    charge=np.asarray(s.charge, np.float64).copy())

    def interacting_pairs(self, pos):
        """Non-excluded pairs i < j with r < r_c at real positions (FP64)."""
        from scipy.spatial import cKDTree
        p = np.mod(np.real(pos).T, self.box)
        tree = cKDTree(p, boxsize=self.box)
        pairs = tree.query_pairs(self.r_cut, output_type="ndarray")
        if len(pairs) == 0:
            return np.zeros((0, 2), np.int64)
        pairs = np.sort(pairs, axis=1).astype(np.int64)
        keys = pairs[:, 0] * self.n + pairs[:, 1]
        pairs = pairs[~np.isin(keys, self.ex_keys)]
        return pairs[np.lexsort((pairs[:, 1], pairs[:, 0]))]

    def __call__(self, pos, params, pairs):
        """(U, F [3, N]) at pos with the given interacting pairs."""
        n = self.n
        eps, sig, q = params["eps"], params["sig"], params["charge"]
        dt = np.result_type(pos, eps, sig, q)
        U = 0.0
        F = np.zeros((3, n), dt)
        a, ke = self.alpha, self.ke
        if len(pairs):
            i, j = pairs[:, 0], pairs[:, 1]
            d = _disp(pos, self.box, i, j)
            r2 = (d * d).sum(axis=0)
            r = np.sqrt(r2)
            ti, tj = self.types[i], self.types[j]
            sij = 0.5 * (sig[ti] + sig[tj])                   # Eq. 5
            eij = np.sqrt(eps[ti] * eps[tj])                  # Eq. 5
            s6 = (sij * sij / r2) ** 3
            U = U + (4.0 * eij * (s6 * s6 - s6)).sum()        # Eq. 4
            du = 4.0 * eij * (-12.0 * s6 * s6 + 6.0 * s6) / r
            if a > 0:
                qq = ke * q[i] * q[j]
                U = U + (qq * erfc(a * r) / r).sum()          # Eq. 10, n = 0
                du = du - qq * (erfc(a * r) / r2 +
                                2.0 * a / math.sqrt(math.pi) * np.exp(-a * a * r2) / r)
            F = F + _acc(n, i, j, d * (-du / r), dt)
        if a > 0 and len(self.ex):
            i, j = self.ex[:, 0], self.ex[:, 1]
            d = _disp(pos, self.box, i, j)
            r2 = (d * d).sum(axis=0)
            r = np.sqrt(r2)
            qq = ke * q[i] * q[j]
            U = U - (qq * erf(a * r) / r).sum()
            du = -qq * (2.0 * a / math.sqrt(math.pi) * np.exp(-a * a * r2) / r - erf(a * r) / r2)
            F = F + _acc(n, i, j, d * (-du / r), dt)
        if a > 0:
            V = float(np.prod(self.box))
            Qt = q.sum()
            U = U - ke * a / math.sqrt(math.pi) * (q * q).sum() \
                - ke * math.pi * Qt * Qt / (2.0 * V * a * a)  # Eq. 12 + background
        if len(self.bonds):
            i, j = self.bonds[:, 0], self.bonds[:, 1]
            d = _disp(pos, self.box, i, j)
            r = np.sqrt((d * d).sum(axis=0))
            U = U + (self.bond_k * (r - self.bond_r0) ** 2).sum()         # Eq. 1
            F = F + _acc(n, i, j, d * (-2.0 * self.bond_k * (r - self.bond_r0) / r), dt)
        if len(self.angles):
            i, j, l = self.angles[:, 0], self.angles[:, 1], self.angles[:, 2]
            A = _disp(pos, self.box, j, i)
            B = _disp(pos, self.box, j, l)
            ra = np.sqrt((A * A).sum(axis=0))
            rb = np.sqrt((B * B).sum(axis=0))
            ah, bh = A / ra, B / rb
            c = (ah * bh).sum(axis=0)
            th = np.arccos(c)
            U = U + (self.angle_k * (th - self.angle_t0) ** 2).sum()      # Eq. 2
            g = 2.0 * self.angle_k * (th - self.angle_t0) / np.sqrt(1.0 - c * c)
            Fi = g * (bh - c * ah) / ra
            Fl = g * (ah - c * bh) / rb
            for ax in range(3):
                np.add.at(F[ax], i, Fi[ax])
                np.add.at(F[ax], l, Fl[ax])
                np.subtract.at(F[ax], j, Fi[ax] + Fl[ax])
        if self.has_pme:
            Er, Fr = _spme_cs(pos, q, self.box, self.grid, a, ke, self.G)
            U = U + Er
            F = F + Fr
        return U, F

    # ---- derivatives by complex step ----
    def dforce(self, pos, params, pairs, u):
        """Directional derivative of F along u: d/de F(pos + e u) = -H u."""
        return np.imag(self(pos + 1j * H_CS * u, params, pairs)[1]) / H_CS

    def param_directions(self, dq):
        """The parameter directions: eps_t, then sig_t for every type, then the
        charge direction dq."""
        T = len(self.sys.type_epsilon)
        out = []
        for k in range(T):
            e = np.zeros(T)
            e[k] = 1.0
            out.append(("eps", e))
        for k in range(T):
            e = np.zeros(T)
            e[k] = 1.0
            out.append(("sig", e))
        out.append(("charge", np.asarray(dq, np.float64)))
        return out

    def dparams(self, pos, params, pairs, dq):
        """Per parameter direction: (dU/dtheta, dF/dtheta [3, N])."""
        out = []
        for name, e in self.param_directions(dq):
            p = dict(params)
            p[name] = params[name] + 1j * H_CS * e
            U, F = self(pos, p, pairs)
            out.append((np.imag(U) / H_CS, np.imag(F) / H_CS))
        return out


# ---------------------------------------------------------------------------
# Trajectory, loss and gradients
# ---------------------------------------------------------------------------
def trajectory(ff, params, x0, v0, dt, n_steps, pair_sets=None):
    """FP64 velocity Verlet from (x0, v0), unwrapped. pair_sets: the
    interacting pairs of every step (None: recorded from this run).
    Returns dict(x [T+1], vh [T] (half-step velocities), F [T+1], U_T,
    pair_sets)."""
    m = np.asarray(ff.sys.mass, np.float64)[None, :]
    c = float(ff.sys.accel)
    x = np.asarray(x0, np.float64).copy()
    v = np.asarray(v0, np.float64).copy()
    record = pair_sets is None
    sets = [] if record else pair_sets
    if record:
        sets.append(ff.interacting_pairs(x))
    U, F = ff(x, params, sets[0])
    xs, vhs, Fs = [x.copy()], [], [F]
    for s in range(n_steps):
        vh = v + 0.5 * dt * c * F / m
        x = x + dt * vh
        if record:
            sets.append(ff.interacting_pairs(x))
        U, F = ff(x, params, sets[s + 1])
        v = vh + 0.5 * dt * c * F / m
        xs.append(x.copy())
        vhs.append(vh)
        Fs.append(F)
    return dict(x=np.array(xs), vh=np.array(vhs), F=np.array(Fs), U_T=float(np.real(U)),
                v_T=v, pair_sets=sets)


def loss(tr, x0, n):
    d = tr["x"][-1] - np.asarray(x0, np.float64)
    return tr["U_T"] / n + float((d * d).sum()) / n


def gradients(ff, params, x0, v0, dt, n_steps, dq, tr=None):
    """dL/dx0 [3, N], dL/dv0 [3, N], dL/dtheta (eps_t..., sig_t..., t) and
    dL/d(dt), by the reverse recursion of the module docstring over the
    frozen interaction sets of the run. dL/deps_t is NaN for a type with
    eps_t = 0 (Lorentz-Berthelot's sqrt(eps_i eps_j) has no derivative
    there)."""
    if tr is None:
        tr = trajectory(ff, params, x0, v0, dt, n_steps)
    n = ff.n
    m = np.asarray(ff.sys.mass, np.float64)[None, :]
    c = float(ff.sys.accel)
    h = 0.5 * dt
    sets = tr["pair_sets"]
    xT, x0 = tr["x"][-1], np.asarray(x0, np.float64)
    acc = lambda F: c * F / m
    Jt = lambda k, w: c * ff.dforce(tr["x"][k], params, sets[k], w / m)
    dpar = lambda k: ff.dparams(tr["x"][k], params, sets[k], dq)
    # dL/dx_T, dL/dv_T, and the loss's direct parameter dependence (U_T / N)
    Xb = -tr["F"][-1] / n + 2.0 * (xT - x0) / n
    Vb = np.zeros_like(Xb)
    theta = np.array([dU / n for dU, _ in dpar(n_steps)])
    dtb = 0.0
    for s in range(n_steps - 1, -1, -1):
        a_next, a_now = acc(tr["F"][s + 1]), acc(tr["F"][s])
        xt = Xb + h * Jt(s + 1, Vb)
        theta += h * np.array([float((c * dF * Vb / m).sum()) for _, dF in dpar(s + 1)])
        dtb += 0.5 * float((Vb * a_next).sum())
        vpb = Vb + dt * xt
        dtb += float((xt * tr["vh"][s]).sum())
        Xb = xt + h * Jt(s, vpb)
        theta += h * np.array([float((c * dF * vpb / m).sum()) for _, dF in dpar(s)])
        dtb += 0.5 * float((vpb * a_now).sum())
        Vb = vpb
    Xb = Xb - 2.0 * (xT - x0) / n
    # LB mixing, sqrt(eps_i eps_j), has no derivative at eps_t = 0
    T = len(params["eps"])
    theta[:T] = np.where(np.real(params["eps"]) > 0, theta[:T], np.nan)
    return dict(x0=Xb, v0=Vb, theta=theta, dt=dtb, loss=loss(tr, x0, n), traj=tr)


def frozen_loss(ff, params, x0, v0, dt, n_steps, pair_sets):
    """The loss of a run that reuses the given interaction sets."""
    tr = trajectory(ff, params, x0, v0, dt, n_steps, pair_sets=pair_sets)
    return loss(tr, x0, ff.n)


def perturb(params, name, e, h):
    p = dict(params)
    p[name] = params[name] + h * e
    return p
