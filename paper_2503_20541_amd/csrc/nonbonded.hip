// Short-range forces (DIMOS Sec. II.A.1-2).
//
// k_pair: one wave per 4-atom i-cluster streams its list of 4x4 cluster
//   tiles four at a time: lane = (i slot, tile, j slot), i.e. the wave's four
//   16-lane rows each hold one i atom against 16 j atoms. Per pair: LJ
//   (Eqs. 4-5, type-pair table, optional Eq. 6 switch) + the minimum-image
//   real-space Ewald term (Eq. 10) for pairs whose mask bit is set and with
//   r2 < fl(r_c^2). A group of tiles with no such pair is skipped after the
//   distance test. The list holds both directions of every pair, so each
//   row only accumulates its own i force: a 16-lane row reduction at the end,
//   no atomics, bitwise reproducible. Energies accumulate per lane in FP64.
// k_bonded_excl: one thread per caller atom for the terms that involve it:
//   the FP64 erf exclusion correction and FP32 harmonic bonds/angles (Eqs. 1-2).
//   Each term's energy is booked once, by a designated member atom.
// k_reduce_rows: fixed-order FP64 reduction of per-block partial sums.
#include "mdx_internal.h"

namespace mdx {

// erfc(x) = exp(-x^2) R(x): R = t P(t), t = 1/(1 + 0.4 x), with P of degree 9
// fitted (weighted least squares iterated towards equal ripple) to the
// scaled complementary error function exp(x^2) erfc(x) on [0, 6]; relative
// error below 1e-9 in exact arithmetic, a few float32 ulps as evaluated.
// The caller multiplies by exp(-x^2), which it needs for the force anyway.
__device__ __forceinline__ float erfc_scaled(float x) {
  const float t = __builtin_amdgcn_rcpf(fmaf(0.4f, x, 1.0f));
  float p = -3.839134390e-02f;
  p = fmaf(p, t, 2.474407330e-01f);
  p = fmaf(p, t, -6.196206523e-01f);
  p = fmaf(p, t, 7.158111156e-01f);
  p = fmaf(p, t, -4.316577684e-01f);
  p = fmaf(p, t, 3.558386304e-01f);
  p = fmaf(p, t, 9.873089759e-02f);
  p = fmaf(p, t, 2.220756708e-01f);
  p = fmaf(p, t, 2.240124465e-01f);
  p = fmaf(p, t, 2.257602716e-01f);
  return p * t;
}

struct PairParams {
  float L[3], hL[3];
  float rc2;
  float alpha_hi, alpha_lo;   // Ewald alpha as a float pair
  float two_a_sqrtpi;         // 2 alpha / sqrt(pi)
  float coulomb_k;
  float r_s, r_c, inv_sw;     // switch r_s, r_c and 1/(r_c - r_s)
  int ntypes;
  double alpha_d;             // alpha for the FP64 energy terms
};

// Energies of a pair on measurement steps: the float32 squared distance (and
// the switch value) is widened and the pair energy is evaluated in FP64 with
// FP64 constants, so the only rounding left is the unbiased float32 rounding
// of each pair's distance; k_e is applied in the final FP64 reduction. (The
// real-space Coulomb sum cancels strongly, so a float32 erfc bias of 1e-7
// would show up at the 1e-6 level in the total.)
template <bool ENERGY, bool COUL, bool SWITCH>
__global__ void __launch_bounds__(256) k_pair(const float4* __restrict__ xs,
                                              const int* __restrict__ ts,
                                              const uint2* __restrict__ tiles,
                                              const int* __restrict__ tile_count,
                                              const int* __restrict__ meta, int cap,
                                              PairParams pp, const float4* __restrict__ lj_f,
                                              const double2* __restrict__ lj_d,
                                              const int* __restrict__ perm, int n,
                                              float* __restrict__ force,
                                              double* __restrict__ partials, int pstride) {
  __shared__ double red[16];
  const int w = threadIdx.x / kWave, lane = threadIdx.x & (kWave - 1);
  const int ic = blockIdx.x * 4 + w;
  const bool active = ic < meta[1];
  const int ia = lane >> 4, tt = (lane >> 2) & 3, jb = lane & 3;
  const int si = ic * kClusterSize + ia;
  const unsigned bitpos = (unsigned)(ia * kClusterSize + jb);
  float fx = 0.f, fy = 0.f, fz = 0.f;
  double e_lj = 0.0, e_c = 0.0;
  if (active) {
    const float4 pi = xs[si];
    const float lmx = pp.L[0] - pi.x, lmy = pp.L[1] - pi.y, lmz = pp.L[2] - pi.z;
    const int trow = ts[si] * pp.ntypes;
    const int cnt = tile_count[ic];
    const uint2* tl = tiles + (size_t)ic * cap;
    // lists are padded to groups of four; the prefetch of the next group is
    // clamped into the list's allocation and only used while g < cnt
    uint2 e_next = tl[tt];
    for (int g = 0; g < cnt; g += 4) {
      const uint2 e = e_next;
      e_next = tl[min(g + 4 + tt, cap - 1)];
      const bool on = (e.y >> bitpos) & 1u;
      const int sj = (int)e.x * kClusterSize + jb;
      const float4 pj = xs[sj];
      float dx = min_image_h(pi.x, lmx, pj.x, pp.L[0], pp.hL[0]);
      float dy = min_image_h(pi.y, lmy, pj.y, pp.L[1], pp.hL[1]);
      float dz = min_image_h(pi.z, lmz, pj.z, pp.L[2], pp.hL[2]);
      float r2 = dist2(dx, dy, dz);
      const bool in = on && r2 < pp.rc2;
      if (__ballot(in) == 0ull) continue;
      if (in) {
        const int tp = trow + ts[sj];
        float4 lj = lj_f[tp];             // c12, c6, 12 c12, 6 c6
        const float rinv = __builtin_amdgcn_rsqf(r2);   // r2 is never denormal here
        const float rinv2 = rinv * rinv;
        float r6 = rinv2 * rinv2 * rinv2;
        float f_over_r = r6 * (lj.z * r6 - lj.w) * rinv2;
        float S = 1.f;
        if (SWITCH) {
          float r = r2 * rinv;
          if (r > pp.r_s) {
            float x = (r - pp.r_s) * pp.inv_sw;
            float x2 = x * x, x3 = x2 * x;
            S = 1.0f + x3 * (-10.0f + x * (15.0f - 6.0f * x));
            float dS = x2 * (-30.0f + x * (60.0f - 30.0f * x)) * pp.inv_sw;
            float u_lj = r6 * (lj.x * r6 - lj.y);
            f_over_r = f_over_r * S - u_lj * dS * rinv;
          }
        }
        float ec = 0.f;
        if (COUL) {
          float r = r2 * rinv;
          float ar = fmaf(pp.alpha_hi, r, pp.alpha_lo * r);
          // exp(-x^2) as 2^(-x^2 log2 e) on the transcendental unit; the
          // energies on measurement steps are evaluated separately in FP64
          float ex = __builtin_amdgcn_exp2f(-ar * ar * 1.44269504088896341f);
          ec = erfc_scaled(ar) * ex;
          f_over_r += pp.coulomb_k * (pi.w * pj.w) * (ec * rinv + pp.two_a_sqrtpi * ex) * rinv2;
        }
        fx -= f_over_r * dx;
        fy -= f_over_r * dy;
        fz -= f_over_r * dz;
        if (ENERGY) {
          double2 c = lj_d[tp];
          double r2d = (double)r2;
          double r6d = 1.0 / (r2d * r2d * r2d);
          double u = r6d * (c.x * r6d - c.y);
          if (SWITCH) u *= (double)S;
          e_lj += u;
          if (COUL) {
            double rd = sqrt(r2d);
            e_c += (double)pi.w * (double)pj.w * erfc(pp.alpha_d * rd) / rd;
          }
        }
      }
    }
  }
  // sum the i force over the 16 lanes of the row
  for (int o = 8; o >= 1; o >>= 1) {
    fx += __shfl_xor(fx, o, kWave);
    fy += __shfl_xor(fy, o, kWave);
    fz += __shfl_xor(fz, o, kWave);
  }
  if (active && (lane & 15) == 0) {
    int a = perm[si];
    if (a >= 0) {
      force[a] = fx;
      force[n + a] = fy;
      force[2 * n + a] = fz;
    }
  }
  if (ENERGY) {
    // every pair was visited from both ends
    double s_lj = block_sum(0.5 * e_lj, red);
    double s_c = block_sum(0.5 * e_c, red);
    if (threadIdx.x == 0) {
      partials[kRowLJ * pstride + blockIdx.x] = s_lj;
      partials[kRowDir * pstride + blockIdx.x] = s_c;
    }
  }
}

struct BondedParams {
  float L[3], hL[3];
  double Ld[3];
  double alpha, two_a_sqrtpi, coulomb_k;
};

template <bool ENERGY, bool COUL>
__global__ void __launch_bounds__(256) k_bonded_excl(
    const float* __restrict__ pos, int n, BondedParams bp, const float* __restrict__ q,
    const int* __restrict__ ex_start, const int* __restrict__ ex_idx,
    const int* __restrict__ bonds, const float* __restrict__ bond_k,
    const float* __restrict__ bond_r0, const int* __restrict__ bt_start,
    const int* __restrict__ bt_idx, const int* __restrict__ angles,
    const float* __restrict__ angle_k, const float* __restrict__ angle_t0,
    const int* __restrict__ at_start, const int* __restrict__ at_idx, float* __restrict__ force,
    double* __restrict__ partials, int pstride) {
  __shared__ double red[16];
  int a = blockIdx.x * blockDim.x + threadIdx.x;
  double e_ex = 0.0, e_b = 0.0, e_a = 0.0;
  if (a < n) {
    float xa = pos[a], ya = pos[n + a], za = pos[2 * n + a];
    float fx = 0.f, fy = 0.f, fz = 0.f;
    if (COUL) {
      // -k_e q_a q_b erf(alpha r)/r over excluded partners, in FP64 with the
      // exact minimum-image displacement of the float32 coordinates.
      double gx = 0.0, gy = 0.0, gz = 0.0;
      double qa = (double)q[a];
      for (int k = ex_start[a]; k < ex_start[a + 1]; ++k) {
        int b = ex_idx[k];
        double d[3] = {(double)pos[b] - (double)xa, (double)pos[n + b] - (double)ya,
                       (double)pos[2 * n + b] - (double)za};
        for (int t = 0; t < 3; ++t) {
          if (d[t] > 0.5 * bp.Ld[t]) d[t] -= bp.Ld[t];
          else if (d[t] < -0.5 * bp.Ld[t]) d[t] += bp.Ld[t];
        }
        double r2 = d[0] * d[0] + d[1] * d[1] + d[2] * d[2];
        double r = sqrt(r2);
        double qq = bp.coulomb_k * qa * (double)q[b];
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
      }
      fx += (float)gx;
      fy += (float)gy;
      fz += (float)gz;
    }
    for (int k = bt_start[a]; k < bt_start[a + 1]; ++k) {
      int t = bt_idx[k];
      int i = bonds[2 * t], j = bonds[2 * t + 1];
      float dx = min_image(pos[i], pos[j], bp.L[0], bp.hL[0]);
      float dy = min_image(pos[n + i], pos[n + j], bp.L[1], bp.hL[1]);
      float dz = min_image(pos[2 * n + i], pos[2 * n + j], bp.L[2], bp.hL[2]);
      float r = sqrtf(dx * dx + dy * dy + dz * dz);
      float dr = r - bond_r0[t];
      float g = -2.0f * bond_k[t] * dr / r;   // force on j = g * d
      float sgn = (a == j) ? 1.0f : -1.0f;
      fx += sgn * g * dx;
      fy += sgn * g * dy;
      fz += sgn * g * dz;
      if (ENERGY && a == i) e_b += (double)(bond_k[t] * dr * dr);
    }
    for (int k = at_start[a]; k < at_start[a + 1]; ++k) {
      int t = at_idx[k];
      int i = angles[3 * t], j = angles[3 * t + 1], l = angles[3 * t + 2];
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
      float dth = theta - angle_t0[t];
      float dU = 2.0f * angle_k[t] * dth;
      float s = sqrtf(fmaxf(1.0f - c * c, 1e-12f));
      float pre = dU / s;
      float fix = pre * (bhx - c * ahx) * ira, fiy = pre * (bhy - c * ahy) * ira,
            fiz = pre * (bhz - c * ahz) * ira;
      float flx = pre * (ahx - c * bhx) * irb, fly = pre * (ahy - c * bhy) * irb,
            flz = pre * (ahz - c * bhz) * irb;
      if (a == i) { fx += fix; fy += fiy; fz += fiz; }
      if (a == l) { fx += flx; fy += fly; fz += flz; }
      if (a == j) { fx -= fix + flx; fy -= fiy + fly; fz -= fiz + flz; }
      if (ENERGY && a == j) e_a += (double)(angle_k[t] * dth * dth);
    }
    force[a] += fx;
    force[n + a] += fy;
    force[2 * n + a] += fz;
  }
  if (ENERGY) {
    double s1 = block_sum(e_ex, red);
    double s2 = block_sum(e_b, red);
    double s3 = block_sum(e_a, red);
    if (threadIdx.x == 0) {
      partials[kRowExcl * pstride + blockIdx.x] = s1;
      partials[kRowBond * pstride + blockIdx.x] = s2;
      partials[kRowAngle * pstride + blockIdx.x] = s3;
    }
  }
}

struct ReduceSpec {
  int nrows;
  int row[8];
  int nblk[8];
  int slot[8];
  double scale[8];
  int const_slot;      // -1: none
  double const_val;
  int zero_slot;       // -1: none
};

// One block per requested row: fixed-order sum of its partials.
__global__ void __launch_bounds__(256) k_reduce_rows(const double* __restrict__ partials,
                                                     int pstride, ReduceSpec spec,
                                                     double* __restrict__ out,
                                                     unsigned* __restrict__ flags) {
  __shared__ double red[16];
  int r = blockIdx.x;
  if (r < spec.nrows) {
    const double* p = partials + (size_t)spec.row[r] * pstride;
    double v = 0.0;
    for (int k = threadIdx.x; k < spec.nblk[r]; k += blockDim.x) v += p[k];
    double s = block_sum(v, red) * spec.scale[r];
    if (threadIdx.x == 0) {
      out[spec.slot[r]] = s;
      if (!isfinite(s)) atomicOr(flags, MDX_FLAG_NONFINITE);
    }
  } else if (threadIdx.x == 0) {
    if (spec.const_slot >= 0) out[spec.const_slot] = spec.const_val;
    if (spec.zero_slot >= 0) out[spec.zero_slot] = 0.0;
  }
}

hipError_t launch_nonbonded(Ctx& c, float* force, bool energy) {
  PairParams pp;
  for (int d = 0; d < 3; ++d) {
    pp.L[d] = c.cg.L[d];
    pp.hL[d] = c.cg.hL[d];
  }
  pp.rc2 = c.cg.rc2;
  pp.alpha_hi = (float)c.alpha;
  pp.alpha_lo = (float)(c.alpha - (double)pp.alpha_hi);
  pp.alpha_d = c.alpha;
  pp.ntypes = c.n_types;
  pp.two_a_sqrtpi = (float)(2.0 * c.alpha / sqrt(M_PI));
  pp.coulomb_k = (float)c.coulomb_k;
  pp.r_s = c.switch_r;
  pp.r_c = c.r_cut;
  pp.inv_sw = c.has_switch ? 1.0f / (c.r_cut - c.switch_r) : 0.f;
  const int nb = (c.max_clusters + 3) / 4;
  c.nb_blocks = nb;
#define MDX_PAIR(E, C, S)                                                                       \
  k_pair<E, C, S><<<nb, 256, 0, c.stream>>>(c.xs, c.ts, c.tiles, c.tile_count, c.meta, c.nl_cap, \
                                             pp, c.lj_f, c.lj_d, c.perm, c.n, force, c.partials, \
                                             c.max_blocks)
  bool C = c.has_coulomb, S = c.has_switch;
  if (energy) {
    if (C && S) MDX_PAIR(true, true, true);
    else if (C) MDX_PAIR(true, true, false);
    else if (S) MDX_PAIR(true, false, true);
    else MDX_PAIR(true, false, false);
  } else {
    if (C && S) MDX_PAIR(false, true, true);
    else if (C) MDX_PAIR(false, true, false);
    else if (S) MDX_PAIR(false, false, true);
    else MDX_PAIR(false, false, false);
  }
#undef MDX_PAIR
  return hipGetLastError();
}

hipError_t launch_bonded_excl(Ctx& c, const float* pos, float* force, bool energy) {
  BondedParams bp;
  for (int d = 0; d < 3; ++d) {
    bp.L[d] = c.cg.L[d];
    bp.hL[d] = c.cg.hL[d];
    bp.Ld[d] = (double)c.cg.L[d];
  }
  bp.alpha = c.alpha;
  bp.two_a_sqrtpi = 2.0 * c.alpha / sqrt(M_PI);
  bp.coulomb_k = c.coulomb_k;
  const int nb = (c.n + 255) / 256;
#define MDX_BX(E, C)                                                                        \
  k_bonded_excl<E, C><<<nb, 256, 0, c.stream>>>(                                           \
      pos, c.n, bp, c.q, c.ex_start, c.ex_idx, c.bonds, c.bond_k, c.bond_r0, c.bt_start,   \
      c.bt_idx, c.angles, c.angle_k, c.angle_t0, c.at_start, c.at_idx, force, c.partials, \
      c.max_blocks)
  bool C = c.has_coulomb;
  if (energy) {
    if (C) MDX_BX(true, true);
    else MDX_BX(true, false);
  } else {
    if (C) MDX_BX(false, true);
    else MDX_BX(false, false);
  }
#undef MDX_BX
  return hipGetLastError();
}

hipError_t launch_reduce_energy(Ctx& c, const int* rows, const int* nblk, int nrows, double* out,
                                int slot_base, double const_val, int const_slot, int zero_slot) {
  ReduceSpec spec{};
  spec.nrows = nrows;
  for (int r = 0; r < nrows; ++r) {
    spec.row[r] = rows[r];
    spec.nblk[r] = nblk[r];
    spec.scale[r] = rows[r] == kRowRec ? 0.5 * c.coulomb_k * c.pme_energy_scale
                    : (rows[r] == kRowDir ? c.coulomb_k : 1.0);
    int slot;
    switch (rows[r]) {
      case kRowLJ: slot = MDX_ENERGY_LJ; break;
      case kRowDir: slot = MDX_ENERGY_COUL_DIR; break;
      case kRowExcl: slot = MDX_ENERGY_COUL_EXCL; break;
      case kRowBond: slot = MDX_ENERGY_BOND; break;
      case kRowAngle: slot = MDX_ENERGY_ANGLE; break;
      case kRowRec: slot = MDX_ENERGY_COUL_REC; break;
      default: slot = MDX_ENERGY_KINETIC; break;
    }
    spec.slot[r] = slot - slot_base;
  }
  spec.const_slot = const_slot >= 0 ? const_slot - slot_base : -1;
  spec.const_val = const_val;
  spec.zero_slot = zero_slot >= 0 ? zero_slot - slot_base : -1;
  k_reduce_rows<<<nrows + 1, 256, 0, c.stream>>>(c.partials, c.max_blocks, spec, out, c.flags);
  return hipGetLastError();
}

}  // namespace mdx
