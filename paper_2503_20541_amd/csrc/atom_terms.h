// Per-atom force terms shared by the stand-alone kernels and the fused
// integration kernels: bonded terms with the Ewald exclusion correction
// (Eqs. 1-2; the erf term removed for excluded pairs), and the PME force
// interpolation for one atom.
#pragma once

#include "mdx_internal.h"

namespace mdx {

struct BondedParams {
  float L[3], hL[3];
  double Ld[3];
  double alpha, two_a_sqrtpi, coulomb_k;
};

// Device pointers of the topology and per-atom charges (caller atom order).
struct Topology {
  const float* q;
  const int* ex_start;
  const int* ex_idx;
  const int* bonds;
  const float* bond_k;
  const float* bond_r0;
  const int* bt_start;
  const int* bt_idx;
  const int* angles;
  const float* angle_k;
  const float* angle_t0;
  const int* at_start;
  const int* at_idx;
};

// One term of each kind, the arithmetic only (member positions and parameters
// passed in). excl_term: -k_e q_a q_b erf(alpha r)/r for excluded partner b,
// in FP64 with the exact minimum-image displacement of the float32
// coordinates; adds the force on a to g, books the energy by the lower atom.
template <bool ENERGY, bool VIR>
__device__ __forceinline__ void excl_term(int a, int b, float xa, float ya, float za, float xb,
                                          float yb, float zb, double qa, float qb,
                                          const BondedParams& bp, double& gx, double& gy,
                                          double& gz, double& e_ex, double* w) {
  double d[3] = {(double)xb - (double)xa, (double)yb - (double)ya, (double)zb - (double)za};
  for (int t = 0; t < 3; ++t) {
    if (d[t] > 0.5 * bp.Ld[t]) d[t] -= bp.Ld[t];
    else if (d[t] < -0.5 * bp.Ld[t]) d[t] += bp.Ld[t];
  }
  double r2 = d[0] * d[0] + d[1] * d[1] + d[2] * d[2];
  double r = sqrt(r2);
  double ir = 1.0 / r;
  double qq = bp.coulomb_k * qa * (double)qb;
  double ar = bp.alpha * r;
  double erfv = erf(ar);
  double u = -qq * erfv * ir;
  // dU/dr = -qq (2a/sqrt(pi) exp(-a^2 r^2)/r - erf/r^2); force on a = dU/dr * d / r
  double dudr = -qq * (bp.two_a_sqrtpi * exp(-ar * ar) - erfv * ir) * ir;
  double s = dudr * ir;
  gx += s * d[0];
  gy += s * d[1];
  gz += s * d[2];
  if (ENERGY && a < b) e_ex += u;
  if (VIR && a < b) vir_add_dd(w, -s, d[0], d[1], d[2]);   // d (x) F_b, F_b = -s d
}

// Harmonic bond (i, j) with force constant k and length r0; the energy is
// booked by its first atom.
template <bool ENERGY, bool VIR>
__device__ __forceinline__ void bond_term(int a, int i, int j, float xi, float yi, float zi,
                                          float xj, float yj, float zj, float k, float r0,
                                          const BondedParams& bp, float& fx, float& fy,
                                          float& fz, double& e_b, double* w) {
  float dx = min_image(xi, xj, bp.L[0], bp.hL[0]);
  float dy = min_image(yi, yj, bp.L[1], bp.hL[1]);
  float dz = min_image(zi, zj, bp.L[2], bp.hL[2]);
  float r = sqrtf(dx * dx + dy * dy + dz * dz);
  float dr = r - r0;
  float g = -2.0f * k * dr / r;   // force on j = g * d
  float sgn = (a == j) ? 1.0f : -1.0f;
  fx += sgn * g * dx;
  fy += sgn * g * dy;
  fz += sgn * g * dz;
  if (ENERGY && a == i) e_b += (double)(k * dr * dr);
  if (VIR && a == i) vir_add_dd(w, (double)g, dx, dy, dz);   // d (x) F_j, F_j = g d
}

// Harmonic angle i-j-l (vertex j) with force constant k and rest angle t0;
// p holds the x, y, z of i, j, l; the energy is booked by the vertex.
template <bool ENERGY, bool VIR>
__device__ __forceinline__ void angle_term(int a, int i, int j, int l, const float p[9], float k,
                                           float t0, const BondedParams& bp, float& fx,
                                           float& fy, float& fz, double& e_a, double* w) {
  float ax = min_image(p[3], p[0], bp.L[0], bp.hL[0]);
  float ay = min_image(p[4], p[1], bp.L[1], bp.hL[1]);
  float az = min_image(p[5], p[2], bp.L[2], bp.hL[2]);
  float bx = min_image(p[3], p[6], bp.L[0], bp.hL[0]);
  float by = min_image(p[4], p[7], bp.L[1], bp.hL[1]);
  float bz = min_image(p[5], p[8], bp.L[2], bp.hL[2]);
  float ra = sqrtf(ax * ax + ay * ay + az * az);
  float rb = sqrtf(bx * bx + by * by + bz * bz);
  float ira = 1.0f / ra, irb = 1.0f / rb;
  float ahx = ax * ira, ahy = ay * ira, ahz = az * ira;
  float bhx = bx * irb, bhy = by * irb, bhz = bz * irb;
  float c = ahx * bhx + ahy * bhy + ahz * bhz;
  c = fminf(1.0f, fmaxf(-1.0f, c));
  float theta = acosf(c);
  float dth = theta - t0;
  float dU = 2.0f * k * dth;
  float s = sqrtf(fmaxf(1.0f - c * c, 1e-12f));
  float pre = dU / s;
  float fix = pre * (bhx - c * ahx) * ira, fiy = pre * (bhy - c * ahy) * ira,
        fiz = pre * (bhz - c * ahz) * ira;
  float flx = pre * (ahx - c * bhx) * irb, fly = pre * (ahy - c * bhy) * irb,
        flz = pre * (ahz - c * bhz) * irb;
  if (a == i) { fx += fix; fy += fiy; fz += fiz; }
  if (a == l) { fx += flx; fy += fly; fz += flz; }
  if (a == j) { fx -= fix + flx; fy -= fiy + fly; fz -= fiz + flz; }
  if (ENERGY && a == j) e_a += (double)(k * dth * dth);
  if (VIR && a == j) {
    // (r_i - r_j) (x) F_i + (r_l - r_j) (x) F_l, symmetrised
    w[0] += (double)ax * fix + (double)bx * flx;
    w[1] += (double)ay * fiy + (double)by * fly;
    w[2] += (double)az * fiz + (double)bz * flz;
    w[3] += 0.5 * ((double)ax * fiy + (double)bx * fly + (double)ay * fix + (double)by * flx);
    w[4] += 0.5 * ((double)ax * fiz + (double)bx * flz + (double)az * fix + (double)bz * flx);
    w[5] += 0.5 * ((double)ay * fiz + (double)by * flz + (double)az * fiy + (double)bz * fly);
  }
}

// The first exclusion, bond and angle of one part of atom a's lists (the
// terms whose index in the list is part modulo nparts), with their
// parameters and member positions. Each is a chain of dependent loads (list
// start, term index, members, member positions); fetching the three kinds'
// chains side by side, before any arithmetic, overlaps them. A water atom has
// at most two terms of a kind, so with four parts these are all its terms;
// terms_apply loops over any others.
struct AtomTerms {
  int e_lo, e_hi, b_lo, b_hi, g_lo, g_hi;   // first index of the part, list end
  float xa, ya, za, qa;
  int eb;                                  // exclusion partner (-1: none)
  float eq, ep[3];
  int bt, bi, bj;                          // bond (-1: none)
  float bk, br, bp6[6];
  int gt, gi, gj, gl;                      // angle (-1: none)
  float gk, g0, gp[9];
};

template <bool COUL>
__device__ __forceinline__ void terms_begin(AtomTerms& t, int a, const float* __restrict__ pos,
                                            int n, const Topology& tp, int part) {
  const unsigned ua = a, un = n;
  t.xa = ld32(pos, ua);
  t.ya = ld32(pos, un + ua);
  t.za = ld32(pos, 2 * un + ua);
  t.e_lo = t.e_hi = 0;
  if (COUL) {
    t.qa = ld32(tp.q, ua);
    t.e_lo = ld32(tp.ex_start, ua) + part;
    t.e_hi = ld32(tp.ex_start, ua + 1);
  }
  t.b_lo = ld32(tp.bt_start, ua) + part;
  t.b_hi = ld32(tp.bt_start, ua + 1);
  t.g_lo = ld32(tp.at_start, ua) + part;
  t.g_hi = ld32(tp.at_start, ua + 1);
}

// Branch-free: a part with no term of a kind still loads (term 0, atom a),
// and the index -1 marks it. The topology arrays hold at least one zero
// entry per member even when a kind has no terms, so these loads stay in
// bounds.
template <bool COUL>
__device__ __forceinline__ void terms_fetch(AtomTerms& t, int a, const float* __restrict__ pos,
                                            int n, const Topology& tp) {
  const bool he = COUL && t.e_lo < t.e_hi, hb = t.b_lo < t.b_hi, hg = t.g_lo < t.g_hi;
  const unsigned un = n;
  const int eb = COUL ? ld32(tp.ex_idx, he ? (unsigned)t.e_lo : 0u) : 0;
  const int bt = ld32(tp.bt_idx, hb ? (unsigned)t.b_lo : 0u);
  const int gt = ld32(tp.at_idx, hg ? (unsigned)t.g_lo : 0u);
  t.eb = he ? eb : -1;
  t.bt = hb ? bt : -1;
  t.gt = hg ? gt : -1;
  const unsigned e = he ? eb : a, b = hb ? bt : 0, g = hg ? gt : 0;
  if (COUL) {
    t.ep[0] = ld32(pos, e);
    t.ep[1] = ld32(pos, un + e);
    t.ep[2] = ld32(pos, 2 * un + e);
    t.eq = ld32(tp.q, e);
  }
  t.bi = ld32(tp.bonds, 2 * b);
  t.bj = ld32(tp.bonds, 2 * b + 1);
  t.bk = ld32(tp.bond_k, b);
  t.br = ld32(tp.bond_r0, b);
  t.gi = ld32(tp.angles, 3 * g);
  t.gj = ld32(tp.angles, 3 * g + 1);
  t.gl = ld32(tp.angles, 3 * g + 2);
  t.gk = ld32(tp.angle_k, g);
  t.g0 = ld32(tp.angle_t0, g);
  for (unsigned d = 0; d < 3; ++d) {
    t.bp6[d] = ld32(pos, d * un + t.bi);
    t.bp6[3 + d] = ld32(pos, d * un + t.bj);
  }
  for (unsigned d = 0; d < 3; ++d) {
    t.gp[d] = ld32(pos, d * un + t.gi);
    t.gp[3 + d] = ld32(pos, d * un + t.gj);
    t.gp[6 + d] = ld32(pos, d * un + t.gl);
  }
}

// Adds the part's terms in list order, kind by kind (exclusions summed in
// FP64 first, then bonds, then angles): the fetched first term of each kind,
// then the rest with their loads in the loop.
template <bool ENERGY, bool COUL, bool VIR>
__device__ __forceinline__ void terms_apply(const AtomTerms& t, int a,
                                            const float* __restrict__ pos, int n,
                                            const BondedParams& bp, const Topology& tp,
                                            float& fx, float& fy, float& fz, double& e_ex,
                                            double& e_b, double& e_a, int nparts, double* w) {
  if (COUL) {
    double gx = 0.0, gy = 0.0, gz = 0.0;
    const double qa = (double)t.qa;
    if (t.eb >= 0) {
      excl_term<ENERGY, VIR>(a, t.eb, t.xa, t.ya, t.za, t.ep[0], t.ep[1], t.ep[2], qa, t.eq, bp,
                             gx, gy, gz, e_ex, w);
      for (int k = t.e_lo + nparts; k < t.e_hi; k += nparts) {
        const int b = tp.ex_idx[k];
        excl_term<ENERGY, VIR>(a, b, t.xa, t.ya, t.za, pos[b], pos[n + b], pos[2 * n + b], qa,
                               tp.q[b], bp, gx, gy, gz, e_ex, w);
      }
    }
    fx += (float)gx;
    fy += (float)gy;
    fz += (float)gz;
  }
  if (t.bt >= 0) {
    bond_term<ENERGY, VIR>(a, t.bi, t.bj, t.bp6[0], t.bp6[1], t.bp6[2], t.bp6[3], t.bp6[4],
                           t.bp6[5], t.bk, t.br, bp, fx, fy, fz, e_b, w);
    for (int k = t.b_lo + nparts; k < t.b_hi; k += nparts) {
      const int b = tp.bt_idx[k];
      const int i = tp.bonds[2 * b], j = tp.bonds[2 * b + 1];
      bond_term<ENERGY, VIR>(a, i, j, pos[i], pos[n + i], pos[2 * n + i], pos[j], pos[n + j],
                             pos[2 * n + j], tp.bond_k[b], tp.bond_r0[b], bp, fx, fy, fz, e_b, w);
    }
  }
  if (t.gt >= 0) {
    angle_term<ENERGY, VIR>(a, t.gi, t.gj, t.gl, t.gp, t.gk, t.g0, bp, fx, fy, fz, e_a, w);
    for (int k = t.g_lo + nparts; k < t.g_hi; k += nparts) {
      const int g = tp.at_idx[k];
      const int i = tp.angles[3 * g], j = tp.angles[3 * g + 1], l = tp.angles[3 * g + 2];
      const float p[9] = {pos[i], pos[n + i], pos[2 * n + i], pos[j], pos[n + j],
                          pos[2 * n + j], pos[l], pos[n + l], pos[2 * n + l]};
      angle_term<ENERGY, VIR>(a, i, j, l, p, tp.angle_k[g], tp.angle_t0[g], bp, fx, fy, fz, e_a,
                              w);
    }
  }
}

// Adds to (fx, fy, fz) the force on caller atom a from its bonds, angles and
// (FP64) exclusion corrections (Eqs. 1-2 with the erf term of each excluded
// pair removed); books each term's energy once: an exclusion by its lower
// atom, a bond by its first atom, an angle by its vertex. With nparts > 1 the
// call handles only the terms whose index in the atom's lists is part modulo
// nparts (the callers sum the parts in a fixed order). With VIR, each term
// also adds its virial sum_k s_k (x) F_k (s_k: member positions relative to
// one member, minimum image) to w[6], booked like its energy.
template <bool ENERGY, bool COUL, bool VIR = false>
__device__ __forceinline__ void bonded_excl_atom(int a, const float* __restrict__ pos, int n,
                                                 const BondedParams& bp, const Topology& tp,
                                                 float& fx, float& fy, float& fz, double& e_ex,
                                                 double& e_b, double& e_a, int part = 0,
                                                 int nparts = 1, double* w = nullptr) {
  AtomTerms t;
  terms_begin<COUL>(t, a, pos, n, tp, part);
  terms_fetch<COUL>(t, a, pos, n, tp);
  terms_apply<ENERGY, COUL, VIR>(t, a, pos, n, bp, tp, fx, fy, fz, e_ex, e_b, e_a, nparts, w);
}

struct PmeParams {
  int K[3];
  int Kxh;
  int B[3];
  int nb[3];
  float s_hi[3], s_lo[3];   // K_d / L_d = s_hi + s_lo
  float Kf[3], invK[3];      // K_d and fl(1 / K_d) as floats
  float coulomb_k;
  double exp_fac;           // pi^2 / alpha^2
  double inv_piV;           // 1 / (pi V)
};

// Cubic B-spline weights M_4(f + t), t = 0..3, for fractional part f, and
// their derivatives with respect to u (uniform cubic basis written out).
__device__ __forceinline__ void spline4(float f, float th[4], float dth[4]) {
  float g = 1.0f - f;
  float f2 = f * f, f3 = f2 * f;
  const float s = 1.0f / 6.0f;
  th[0] = f3 * s;
  th[1] = (1.0f + 3.0f * f + 3.0f * f2 - 3.0f * f3) * s;
  th[2] = (4.0f - 6.0f * f2 + 3.0f * f3) * s;
  th[3] = g * g * g * s;
  dth[0] = 0.5f * f2;
  dth[1] = 0.5f * (1.0f + 2.0f * f - 3.0f * f2);
  dth[2] = 0.5f * (-4.0f * f + 3.0f * f2);
  dth[3] = -0.5f * g * g;
}

// u = x K/L split into integer base k0 in [0, K) and fraction f in [0, 1),
// with the scale carried as a float pair so f is accurate to ~1 ulp.
__device__ __forceinline__ void grid_coord(float x, float s_hi, float s_lo, int K, int& k0,
                                           float& f) {
  float u = x * s_hi;
  float kf = floorf(u);
  f = fmaf(x, s_hi, -kf) + x * s_lo;
  int k = (int)kf;
  if (f < 0.f) { f += 1.0f; --k; }
  if (f >= 1.0f) { f -= 1.0f; ++k; }
  if (f < 0.f) f = 0.f;
  k %= K;
  if (k < 0) k += K;
  k0 = k;
}

// The B-spline stencil of an atom: base grid point and the weights and their
// derivatives per axis.
struct PmeStencil {
  int k0[3];
  float th[3][4], dth[3][4];
};

__device__ __forceinline__ void pme_stencil(float4 p, const PmeParams& pp, PmeStencil& st) {
  const float xyz[3] = {p.x, p.y, p.z};
  for (int d = 0; d < 3; ++d) {
    float fr;
    grid_coord(xyz[d], pp.s_hi[d], pp.s_lo[d], pp.K[d], st.k0[d], fr);
    spline4(fr, st.th[d], st.dth[d]);
  }
}

// Entry t of a 4-vector by selects (t may vary per lane; indexing a
// register array by it would put the array in scratch memory).
__device__ __forceinline__ float pick4(const float w[4], int t) {
  return t == 0 ? w[0] : t == 1 ? w[1] : t == 2 ? w[2] : w[3];
}

// The 16 potential values of z plane t3 of the stencil, v[4 t2 + t1].
__device__ __forceinline__ void pme_plane_load(const PmeStencil& st, const float* __restrict__ phi,
                                               const PmeParams& pp, int t3, float v[16]) {
  // grid indices below 2^30 (K <= 1024 per axis)
  int z = st.k0[2] - t3;
  z += z < 0 ? pp.K[2] : 0;
  for (int t2 = 0; t2 < 4; ++t2) {
    int y = st.k0[1] - t2;
    y += y < 0 ? pp.K[1] : 0;
    const unsigned row = ((unsigned)z * pp.K[1] + y) * pp.K[0];
    for (int t1 = 0; t1 < 4; ++t1) {
      int x = st.k0[0] - t1;
      x += x < 0 ? pp.K[0] : 0;
      v[4 * t2 + t1] = ld32(phi, row + x);
    }
  }
}

// Adds one z plane's part of grad(theta) . phi to g; thz, dthz: the plane's
// z weight and its derivative.
__device__ __forceinline__ void pme_plane_add(const PmeStencil& st, const float v[16], float thz,
                                              float dthz, float& gx, float& gy, float& gz) {
  for (int t2 = 0; t2 < 4; ++t2) {
    float ayz = st.th[1][t2] * thz;
    float dyz = st.dth[1][t2] * thz;
    float ydz = st.th[1][t2] * dthz;
    for (int t1 = 0; t1 < 4; ++t1) {
      gx += st.dth[0][t1] * ayz * v[4 * t2 + t1];
      gy += st.th[0][t1] * dyz * v[4 * t2 + t1];
      gz += st.th[0][t1] * ydz * v[4 * t2 + t1];
    }
  }
}

// F = -k_e q g scaled from grid to box units, added to (fx, fy, fz).
__device__ __forceinline__ void pme_force_add(float4 p, const PmeParams& pp, float gx, float gy,
                                              float gz, float& fx, float& fy, float& fz) {
  float c = -pp.coulomb_k * p.w;
  fx += c * gx * (pp.s_hi[0] + pp.s_lo[0]);
  fy += c * gy * (pp.s_hi[1] + pp.s_lo[1]);
  fz += c * gz * (pp.s_hi[2] + pp.s_lo[2]);
}

// Reciprocal-space force on an atom at p (charge p.w):
// F = -k_e q sum_k grad(theta(u - k)) phi(k) over its 4x4x4 stencil; the
// z planes t3 = t3_first, t3_first + t3_step, ... < 4 of the stencil only.
__device__ __forceinline__ void pme_gather_atom(float4 p, const float* __restrict__ phi,
                                                const PmeParams& pp, float& fx, float& fy,
                                                float& fz, int t3_first = 0, int t3_step = 1) {
  PmeStencil st;
  pme_stencil(p, pp, st);
  float gx = 0.f, gy = 0.f, gz = 0.f;
  for (int t3 = t3_first; t3 < 4; t3 += t3_step) {
    float v[16];
    pme_plane_load(st, phi, pp, t3, v);
    pme_plane_add(st, v, pick4(st.th[2], t3), pick4(st.dth[2], t3), gx, gy, gz);
  }
  pme_force_add(p, pp, gx, gy, gz, fx, fy, fz);
}

// Host helpers filling the parameter structs from a context.
BondedParams make_bonded_params(const Ctx& c);
Topology make_topology(const Ctx& c);
PmeParams make_pme_params(const Ctx& c);

}  // namespace mdx
