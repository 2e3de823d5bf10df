"""Smooth particle-mesh Ewald in float64 (paper Sec. II.A.2, PME paragraph,
which follows Essmann et al.'s smooth PME with recursively defined B-splines).

Steps, in order:
 1. scaled fractional coordinates u_d = K_d x_d / L_d;
 2. charge spreading Q(k) = sum_i q_i prod_d M_n(u_id - k_d) over the n
    grid points k_d = floor(u_id) - t (mod K_d), t = 0..n-1;
 3. forward 3D DFT Q^ = fftn(Q) (numpy.fft);
 4. influence function G(m) = B(m) C(m), with
      B(m) = prod_d |b_d(m_d)|^2,
      |b_d(m)|^-2 = |sum_{k=0}^{n-2} M_n(k+1) exp(2 pi i m k / K_d)|^2,
      C(m) = exp(-pi^2 |m'|^2 / alpha^2) / (pi V |m'|^2),  C(0) = 0,
    m'_d = m_d / L_d with m_d taken in (-K_d/2, K_d/2];
 5. E_rec = (k_e/2) sum_m G(m) |Q^(m)|^2;
 6. phi = K1 K2 K3 ifftn(G Q^) (real part), so E_rec = (k_e/2) sum_k Q(k) phi(k);
 7. F_i = -k_e sum_k dQ(k)/dx_i phi(k);
 8. virial W_ab = sum_m E(m) [delta_ab - 2 (1 + pi^2 |m'|^2/alpha^2) m'_a m'_b / |m'|^2].
"""
from __future__ import annotations

import numpy as np

from .bspline import M, dM


def bspline_moduli(K: int, order: int = 4):
    """|b(m)|^2 for m = 0..K-1."""
    m = np.arange(K)
    k = np.arange(order - 1)
    s = (M(order, k + 1.0)[None, :] * np.exp(2j * np.pi * np.outer(m, k) / K)).sum(axis=1)
    return 1.0 / np.abs(s) ** 2


def _signed_index(K):
    m = np.arange(K)
    return np.where(m <= K // 2, m, m - K)


def influence(grid, box, alpha, order=4):
    """G = B C on the full grid (axes x, y, z), plus the reciprocal vectors."""
    K = [int(k) for k in grid]
    L = np.asarray(box, np.float64)
    V = float(np.prod(L))
    mx = _signed_index(K[0]) / L[0]
    my = _signed_index(K[1]) / L[1]
    mz = _signed_index(K[2]) / L[2]
    MX, MY, MZ = np.meshgrid(mx, my, mz, indexing="ij")
    msq = MX ** 2 + MY ** 2 + MZ ** 2
    with np.errstate(divide="ignore", invalid="ignore"):
        C = np.exp(-np.pi ** 2 * msq / alpha ** 2) / (np.pi * V * msq)
    C[0, 0, 0] = 0.0
    B = (bspline_moduli(K[0], order)[:, None, None] * bspline_moduli(K[1], order)[None, :, None]
         * bspline_moduli(K[2], order)[None, None, :])
    return B * C, (MX, MY, MZ, msq)


def spline_weights(pos, box, grid, order=4):
    """Per atom and dimension: grid indices [3, N, order], M_n and dM_n/dx."""
    pos = np.asarray(pos, np.float64)
    L = np.asarray(box, np.float64)
    idx, w, dw = [], [], []
    for d in range(3):
        K = int(grid[d])
        u = K * pos[d] / L[d]
        k0 = np.floor(u)
        t = np.arange(order)
        arg = (u - k0)[:, None] + t[None, :]          # u - (k0 - t)
        idx.append(((k0[:, None] - t[None, :]) % K).astype(np.int64))
        w.append(M(order, arg))
        dw.append(dM(order, arg) * (K / L[d]))
    return idx, w, dw


def spread(pos, charge, box, grid, order=4):
    idx, w, _ = spline_weights(pos, box, grid, order)
    q = np.asarray(charge, np.float64)
    Q = np.zeros(tuple(int(k) for k in grid))
    for a in range(order):
        for b in range(order):
            for c in range(order):
                np.add.at(Q, (idx[0][:, a], idx[1][:, b], idx[2][:, c]),
                          q * w[0][:, a] * w[1][:, b] * w[2][:, c])
    return Q


def spme(pos, charge, box, grid, alpha, coulomb_k, order=4):
    """Returns dict(E, F [3,N], W [3,3], Q, phi)."""
    pos = np.asarray(pos, np.float64)
    q = np.asarray(charge, np.float64)
    Ktot = int(np.prod(grid))
    Q = spread(pos, q, box, grid, order)
    Qh = np.fft.fftn(Q)
    G, (MX, MY, MZ, msq) = influence(grid, box, alpha, order)
    Em = 0.5 * coulomb_k * G * np.abs(Qh) ** 2
    E = float(Em.sum())
    phi = np.fft.ifftn(G * Qh).real * Ktot
    idx, w, dw = spline_weights(pos, box, grid, order)
    F = np.zeros((3, pos.shape[1]))
    for a in range(order):
        for b in range(order):
            for c in range(order):
                p = phi[idx[0][:, a], idx[1][:, b], idx[2][:, c]]
                F[0] -= dw[0][:, a] * w[1][:, b] * w[2][:, c] * p
                F[1] -= w[0][:, a] * dw[1][:, b] * w[2][:, c] * p
                F[2] -= w[0][:, a] * w[1][:, b] * dw[2][:, c] * p
    F *= coulomb_k * q[None, :]
    mv = [MX, MY, MZ]
    W = np.zeros((3, 3))
    with np.errstate(divide="ignore", invalid="ignore"):
        fac = np.where(msq > 0, 2.0 * (1.0 + np.pi ** 2 * msq / alpha ** 2) / msq, 0.0)
    for a in range(3):
        for b in range(3):
            W[a, b] = float((Em * ((1.0 if a == b else 0.0) - fac * mv[a] * mv[b])).sum())
    return dict(E=E, F=F, W=W, Q=Q, phi=phi)
