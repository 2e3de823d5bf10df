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

// Adds to (fx, fy, fz) the force on caller atom a from its bonds, angles and
// (FP64) exclusion corrections; books each term's energy once: an exclusion
// by its lower atom, a bond by its first atom, an angle by its vertex. With
// nparts > 1 the call handles only the terms whose index in the atom's lists
// is part modulo nparts (the callers sum the parts in a fixed order).
// With VIR, each term also adds its virial sum_k s_k (x) F_k (s_k: member
// positions relative to one member, minimum image) to w[6], booked like its
// energy.
template <bool ENERGY, bool COUL, bool VIR = false>
__device__ __forceinline__ void bonded_excl_atom(int a, const float* __restrict__ pos, int n,
                                                 const BondedParams& bp, const Topology& tp,
                                                 float& fx, float& fy, float& fz, double& e_ex,
                                                 double& e_b, double& e_a, int part = 0,
                                                 int nparts = 1, double* w = nullptr) {
  float xa = pos[a], ya = pos[n + a], za = pos[2 * n + a];
  if (COUL) {
    // -k_e q_a q_b erf(alpha r)/r over excluded partners, in FP64 with the
    // exact minimum-image displacement of the float32 coordinates.
    double gx = 0.0, gy = 0.0, gz = 0.0;
    double qa = (double)tp.q[a];
    for (int k = tp.ex_start[a] + part; k < tp.ex_start[a + 1]; k += nparts) {
      int b = tp.ex_idx[k];
      double d[3] = {(double)pos[b] - (double)xa, (double)pos[n + b] - (double)ya,
                     (double)pos[2 * n + b] - (double)za};
      for (int t = 0; t < 3; ++t) {
        if (d[t] > 0.5 * bp.Ld[t]) d[t] -= bp.Ld[t];
        else if (d[t] < -0.5 * bp.Ld[t]) d[t] += bp.Ld[t];
      }
      double r2 = d[0] * d[0] + d[1] * d[1] + d[2] * d[2];
      double r = sqrt(r2);
      double qq = bp.coulomb_k * qa * (double)tp.q[b];
      double ar = bp.alpha * r;
      double erfv = erf(ar);
      double u = -qq * erfv / r;
      // dU/dr = -qq (2a/sqrt(pi) exp(-a^2 r^2)/r - erf/r^2); force on a = dU/dr * d / r
      double dudr = -qq * (bp.two_a_sqrtpi * exp(-ar * ar) / r - erfv / r2);
      double s = dudr / r;
      gx += s * d[0];
      gy += s * d[1];
      gz += s * d[2];
      if (ENERGY && a < b) e_ex += u;
      if (VIR && a < b) vir_add_dd(w, -s, d[0], d[1], d[2]);   // d (x) F_b, F_b = -s d
    }
    fx += (float)gx;
    fy += (float)gy;
    fz += (float)gz;
  }
  for (int k = tp.bt_start[a] + part; k < tp.bt_start[a + 1]; k += nparts) {
    int t = tp.bt_idx[k];
    int i = tp.bonds[2 * t], j = tp.bonds[2 * t + 1];
    float dx = min_image(pos[i], pos[j], bp.L[0], bp.hL[0]);
    float dy = min_image(pos[n + i], pos[n + j], bp.L[1], bp.hL[1]);
    float dz = min_image(pos[2 * n + i], pos[2 * n + j], bp.L[2], bp.hL[2]);
    float r = sqrtf(dx * dx + dy * dy + dz * dz);
    float dr = r - tp.bond_r0[t];
    float g = -2.0f * tp.bond_k[t] * dr / r;   // force on j = g * d
    float sgn = (a == j) ? 1.0f : -1.0f;
    fx += sgn * g * dx;
    fy += sgn * g * dy;
    fz += sgn * g * dz;
    if (ENERGY && a == i) e_b += (double)(tp.bond_k[t] * dr * dr);
    if (VIR && a == i) vir_add_dd(w, (double)g, dx, dy, dz);   // d (x) F_j, F_j = g d
  }
  for (int k = tp.at_start[a] + part; k < tp.at_start[a + 1]; k += nparts) {
    int t = tp.at_idx[k];
    int i = tp.angles[3 * t], j = tp.angles[3 * t + 1], l = tp.angles[3 * t + 2];
    float ax = min_image(pos[j], pos[i], bp.L[0], bp.hL[0]);
    float ay = min_image(pos[n + j], pos[n + i], bp.L[1], bp.hL[1]);
    float az = min_image(pos[2 * n + j], pos[2 * n + i], bp.L[2], bp.hL[2]);
    float bx = min_image(pos[j], pos[l], bp.L[0], bp.hL[0]);
    float by = min_image(pos[n + j], pos[n + l], bp.L[1], bp.hL[1]);
    float bz = min_image(pos[2 * n + j], pos[2 * n + l], bp.L[2], bp.hL[2]);
    float ra = sqrtf(ax * ax + ay * ay + az * az);
    float rb = sqrtf(bx * bx + by * by + bz * bz);
    float ira = 1.0f / ra, irb = 1.0f / rb;
    float ahx = ax * ira, ahy = ay * ira, ahz = az * ira;
    float bhx = bx * irb, bhy = by * irb, bhz = bz * irb;
    float c = ahx * bhx + ahy * bhy + ahz * bhz;
    c = fminf(1.0f, fmaxf(-1.0f, c));
    float theta = acosf(c);
    float dth = theta - tp.angle_t0[t];
    float dU = 2.0f * tp.angle_k[t] * dth;
    float s = sqrtf(fmaxf(1.0f - c * c, 1e-12f));
    float pre = dU / s;
    float fix = pre * (bhx - c * ahx) * ira, fiy = pre * (bhy - c * ahy) * ira,
          fiz = pre * (bhz - c * ahz) * ira;
    float flx = pre * (ahx - c * bhx) * irb, fly = pre * (ahy - c * bhy) * irb,
          flz = pre * (ahz - c * bhz) * irb;
    if (a == i) { fx += fix; fy += fiy; fz += fiz; }
    if (a == l) { fx += flx; fy += fly; fz += flz; }
    if (a == j) { fx -= fix + flx; fy -= fiy + fly; fz -= fiz + flz; }
    if (ENERGY && a == j) e_a += (double)(tp.angle_k[t] * dth * dth);
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

// Reciprocal-space force on an atom at p (charge p.w):
// F = -k_e q sum_k grad(theta(u - k)) phi(k) over its 4x4x4 stencil; the
// z planes t3 = t3_first, t3_first + t3_step, ... < 4 of the stencil only.
__device__ __forceinline__ void pme_gather_atom(float4 p, const float* __restrict__ phi,
                                                const PmeParams& pp, float& fx, float& fy,
                                                float& fz, int t3_first = 0, int t3_step = 1) {
  float xyz[3] = {p.x, p.y, p.z};
  int k0[3];
  float th[3][4], dth[3][4];
  for (int d = 0; d < 3; ++d) {
    float fr;
    grid_coord(xyz[d], pp.s_hi[d], pp.s_lo[d], pp.K[d], k0[d], fr);
    spline4(fr, th[d], dth[d]);
  }
  float gx = 0.f, gy = 0.f, gz = 0.f;
  for (int t3 = t3_first; t3 < 4; t3 += t3_step) {
    int z = k0[2] - t3;
    z += z < 0 ? pp.K[2] : 0;
    for (int t2 = 0; t2 < 4; ++t2) {
      int y = k0[1] - t2;
      y += y < 0 ? pp.K[1] : 0;
      const float* rowp = phi + ((size_t)z * pp.K[1] + y) * pp.K[0];
      float ayz = th[1][t2] * th[2][t3];
      float dyz = dth[1][t2] * th[2][t3];
      float ydz = th[1][t2] * dth[2][t3];
      for (int t1 = 0; t1 < 4; ++t1) {
        int x = k0[0] - t1;
        x += x < 0 ? pp.K[0] : 0;
        float v = rowp[x];
        gx += dth[0][t1] * ayz * v;
        gy += th[0][t1] * dyz * v;
        gz += th[0][t1] * ydz * v;
      }
    }
  }
  float c = -pp.coulomb_k * p.w;
  fx += c * gx * (pp.s_hi[0] + pp.s_lo[0]);
  fy += c * gy * (pp.s_hi[1] + pp.s_lo[1]);
  fz += c * gz * (pp.s_hi[2] + pp.s_lo[2]);
}

// Host helpers filling the parameter structs from a context.
BondedParams make_bonded_params(const Ctx& c);
Topology make_topology(const Ctx& c);
PmeParams make_pme_params(const Ctx& c);

}  // namespace mdx
