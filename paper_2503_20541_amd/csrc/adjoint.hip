// Reverse mode of a velocity-Verlet trajectory: gradients of a loss on the
// final state with respect to the initial positions and velocities, the LJ
// parameters per type, a charge direction and the time step (the paper's
// differentiable simulation, Sec. I and Sec. IV).
//
// With a(x) = c F(x) / m, J = da/dx and the adjoints p (of the half-step
// velocities) and q (of the positions), one reverse step over node n
// (positions x_n) is
//     p   <- p + dt q                               (p_n from p_{n+1}, q_{n+1})
//     dL/ddt += q . v'_n + w p . a_n                (v'_n: half-step velocity)
//     u    = c p / m
//     q   <- q + w dt dF(x_n)[u]                    (J^T p = dF[u], H symmetric)
//     dL/dtheta += w dt u . dF/dtheta (x_n)
// with w = 1/2 at the trajectory's first node and 1 elsewhere; it starts
// from p = 0, q = dL/dx_T and ends with q = dL/dx_0, p = dL/dv_0.
//
// dF[u] is the Hessian-vector product of the force field: per pair (force
// on j phi(r) d, d = x_j - x_i) it is phi delta + psi (d . delta) d with
// delta = u_j - u_i and psi = phi'(r) / r; the exclusion and bonded terms
// the same way (angles by forward-mode dual numbers); the reciprocal part
// is the gather of the potential with second spline derivatives plus the
// gather of the potential of the dipole grid sum_j q_j u_j . grad theta_j.
//
// Parameter derivatives are attributed per atom and summed per type in a
// fixed order: a pair's derivative with respect to eps_t (Lorentz-Berthelot,
// eps_ij = sqrt(eps_i eps_j)) splits into the part through atom i's type
// (d eps_ij / d eps_ti = sqrt(eps_tj / eps_ti) / 2) and through j's; the
// full list visits the pair from both ends, each end books its own part.
// A type with eps_t = 0 gets no eps derivative (it does not exist there).
#include "atom_terms.h"

namespace mdx {

// ---- small helpers ----------------------------------------------------------

// Forward-mode dual number (value, derivative along one direction).
struct Dual {
  float v, d;
};
__device__ __forceinline__ Dual operator+(Dual a, Dual b) { return {a.v + b.v, a.d + b.d}; }
__device__ __forceinline__ Dual operator-(Dual a, Dual b) { return {a.v - b.v, a.d - b.d}; }
__device__ __forceinline__ Dual operator*(Dual a, Dual b) {
  return {a.v * b.v, a.d * b.v + a.v * b.d};
}
__device__ __forceinline__ Dual operator*(float s, Dual a) { return {s * a.v, s * a.d}; }
__device__ __forceinline__ Dual operator/(Dual a, Dual b) {
  const float iv = 1.0f / b.v;
  return {a.v * iv, (a.d - a.v * iv * b.d) * iv};
}
__device__ __forceinline__ Dual dsqrt(Dual a) {
  const float s = sqrtf(a.v);
  return {s, a.d * 0.5f / s};
}

// Second derivatives of the cubic B-spline weights of spline4 with respect
// to u.
__device__ __forceinline__ void spline4_d2(float f, float d2[4]) {
  d2[0] = f;
  d2[1] = 1.0f - 3.0f * f;
  d2[2] = 3.0f * f - 2.0f;
  d2[3] = 1.0f - f;
}

// ---- kernels -----------------------------------------------------------------

// Opening of a reverse node, one thread per atom: p <- p + dt q, the dt
// gradient's dot products (FP64 block partials), the tangent u = c p / m,
// and (gmass non-null) the node's mass term -w dt p . a / m per atom
// (a = c F / m depends on m). open = 0: the trajectory's end node taken with
// half weight when the loss also depends on the final velocities (no p
// update and no drift term there).
__global__ void __launch_bounds__(256) k_adj_pre(int n, float dt, float w, int open,
                                                 const float* __restrict__ q,
                                                 float* __restrict__ p,
                                                 const float* __restrict__ v_n,
                                                 const float* __restrict__ f_n,
                                                 const float* __restrict__ acc_over_m,
                                                 const float* __restrict__ mass,
                                                 float* __restrict__ u,
                                                 double* __restrict__ partials,
                                                 double* __restrict__ gmass) {
  __shared__ double red[16];
  const int a = blockIdx.x * blockDim.x + threadIdx.x;
  double acc = 0.0;
  if (a < n) {
    const float am = acc_over_m[a];
    const float h = 0.5f * dt * am;
    double pa = 0.0;
    for (int d = 0; d < 3; ++d) {
      const size_t k = (size_t)d * n + a;
      const float qk = q[k];
      const float pk = open ? p[k] + dt * qk : p[k];
      const float vh = v_n[k] + h * f_n[k];   // the half-step velocity, as the step made it
      const double pak = (double)pk * (am * f_n[k]);
      acc += (open ? (double)qk * vh : 0.0) + (double)w * pak;
      pa += pak;
      p[k] = pk;
      u[k] = am * pk;
    }
    if (gmass) gmass[a] -= (double)w * dt * pa / (double)mass[a];
  }
  const double s = block_sum(acc, red);
  if (threadIdx.x == 0) partials[blockIdx.x] = s;
}

// Slot positions from pos (continued from the build position) and the r_g/2
// validity test, raising *gate for a rebuild.
__global__ void __launch_bounds__(256) k_adj_refresh(const float* __restrict__ pos,
                                                     const int* __restrict__ perm,
                                                     const float* __restrict__ q,
                                                     const float* __restrict__ x_build,
                                                     const int* __restrict__ meta, int n,
                                                     CellGrid cg, float half_skin2,
                                                     float4* __restrict__ xs, int* gate) {
  const int s = blockIdx.x * blockDim.x + threadIdx.x;
  if (s >= meta[0]) return;
  const int a = perm[s];
  if (a < 0) return;
  const float x = pos[a], y = pos[n + a], z = pos[2 * n + a];
  const float bx = x_build[a], by = x_build[n + a], bz = x_build[2 * n + a];
  const float dx = min_image(bx, x, cg.L[0], cg.hL[0]);
  const float dy = min_image(by, y, cg.L[1], cg.hL[1]);
  const float dz = min_image(bz, z, cg.L[2], cg.hL[2]);
  xs[s] = make_float4(bx + dx, by + dy, bz + dz, q[a]);
  if (dist2(dx, dy, dz) > half_skin2) atomicOr(gate, 1);
}

// Tangent by slot: (u_x, u_y, u_z, dq) of the slot's atom, zero for padding.
__global__ void __launch_bounds__(256) k_adj_slots(const int* __restrict__ perm,
                                                   const int* __restrict__ meta, int max_slots,
                                                   int n, const float* __restrict__ u,
                                                   const float* __restrict__ dq,
                                                   float4* __restrict__ us) {
  const int s = blockIdx.x * blockDim.x + threadIdx.x;
  if (s >= max_slots) return;
  const int a = s < meta[0] ? perm[s] : -1;
  us[s] = a >= 0 ? make_float4(u[a], u[n + a], u[2 * n + a], dq[a])
                 : make_float4(0.f, 0.f, 0.f, 0.f);
}

struct JvpPairParams {
  float L[3];
  float rc2;
  float alpha, exp_c, two_a_sqrtpi, coulomb_k, alpha2;
  float two_k_rf;
  double alpha_d, coulomb_kd, k_rf_d, c_rf_d;
  int ntypes;
};

// Pair kernel of the reverse step over the full tile list (every pair from
// both ends), lanes as in the force kernel (i slot, tile of the group of
// four, j slot). EPARAM = false: the Hessian-vector product along us.xyz by
// slot into dfs (stored), and the parameter derivatives u . dF/dtheta
// attributed to the i atom (FP64, per slot: eps of its type, sigma of its
// type, the charge direction). EPARAM = true: the derivatives of the pair
// energy dU/dtheta attributed the same way (FP64 from the float32 distance).
template <bool EPARAM, int COUL>
__global__ void __launch_bounds__(256) k_pair_jvp(
    const float4* __restrict__ xs, const int* __restrict__ ts, const float4* __restrict__ us,
    const uint2* __restrict__ tiles, const int* __restrict__ tile_count,
    const int* __restrict__ meta, int cap, JvpPairParams pp, const float4* __restrict__ lj_f,
    const float4* __restrict__ adj_f, const double4* __restrict__ adj_d,
    float* __restrict__ dfs, double* __restrict__ gslot, int stride) {
  extern __shared__ float4 tab[];   // [T*T] lj_f, then [T*T] adj_f (or adj_d as double4)
  __shared__ float4 img_am[64], img_cp[64];
  const int TT = pp.ntypes * pp.ntypes;
  float4* lj_s = tab;
  float4* af_s = tab + TT;
  double4* ad_s = reinterpret_cast<double4*>(tab + TT);
  for (int t = threadIdx.x; t < TT; t += blockDim.x) {
    lj_s[t] = lj_f[t];
    if (EPARAM) ad_s[t] = adj_d[t];
    else af_s[t] = adj_f[t];
  }
  if (threadIdx.x < 64) {
    float am[3], cp[3];
    for (int d = 0; d < 3; ++d) {
      const unsigned code = (threadIdx.x >> (2 * d)) & 3u;
      am[d] = code == 1u ? -pp.L[d] : 0.f;
      cp[d] = code == 2u ? pp.L[d] : 0.f;
    }
    img_am[threadIdx.x] = make_float4(am[0], am[1], am[2], 0.f);
    img_cp[threadIdx.x] = make_float4(cp[0], cp[1], cp[2], 0.f);
  }
  __syncthreads();
  const int w = threadIdx.x / kWave, lane = threadIdx.x & (kWave - 1);
  const int ic = blockIdx.x * 4 + w;
  const bool active = ic < meta[1];
  const int ia = lane >> 4, tt = (lane >> 2) & 3, jb = lane & 3;
  const int si = ic * kClusterSize + ia;
  const unsigned bitpos = (unsigned)(ia * kClusterSize + jb);
  float gx = 0.f, gy = 0.f, gz = 0.f;
  double ge = 0.0, gs = 0.0, gq = 0.0;
  if (active) {
    const float4 pi = xs[si];
    const float4 ui = us[si];
    const int trow = ts[si] * pp.ntypes;
    const int cnt = tile_count[ic];
    const uint2* tl = tiles + (size_t)ic * cap;
    for (int g = 0; g < cnt; g += 4) {
      const uint2 e = tl[min(g + tt, cap - 1)];
      const bool on = g + tt < cnt && ((e.y >> bitpos) & 1u);
      const unsigned sj = (g + tt < cnt ? e.x : 0u) * kClusterSize + (unsigned)jb;
      const float4 pj = xs[sj];
      const float4 am = img_am[(e.y >> 16) & 63u], cp = img_cp[(e.y >> 16) & 63u];
      const float dx = image_diff(pi.x, pj.x, am.x, cp.x);
      const float dy = image_diff(pi.y, pj.y, am.y, cp.y);
      const float dz = image_diff(pi.z, pj.z, am.z, cp.z);
      const float r2 = dist2(dx, dy, dz);
      if (!(on && r2 < pp.rc2)) continue;
      const int tp = trow + ts[sj];
      if (EPARAM) {
        const double4 c = ad_s[tp];
        const double r2d = (double)r2, r6d = 1.0 / (r2d * r2d * r2d);
        ge += (c.x * r6d - c.y) * r6d;
        gs += (c.z * r6d - c.w) * r6d;
        if (COUL != 0) {
          const double rd = sqrt(r2d);
          const double qq = pp.coulomb_kd * (double)ui.w * (double)pj.w;   // k dq_i q_j
          if (COUL == 1) gq += qq * erfc(pp.alpha_d * rd) / rd;
          else gq += qq * (1.0 / rd + pp.k_rf_d * r2d - pp.c_rf_d);
        }
        continue;
      }
      const float4 uj = us[sj];
      const float4 lj = lj_s[tp];        // c12, c6, 12 c12, 6 c6
      const float4 aj = af_s[tp];        // eps and sigma derivative factors
      const float rinv = __builtin_amdgcn_rsqf(r2);
      const float rinv2 = rinv * rinv;
      const float r6 = rinv2 * rinv2 * rinv2;
      const float r8 = r6 * rinv2;
      float phi = r8 * (lj.z * r6 - lj.w);                          // force on j / r
      float psi = r8 * rinv2 * (8.0f * lj.w - 14.0f * lj.z * r6);   // (d phi / dr) / r
      float phic = 0.f;                                               // Coulomb part per q_i q_j
      if (COUL == 1) {
        const float r = r2 * rinv;
        const float ex = __builtin_amdgcn_exp2f(pp.exp_c * r2);
        const float ec = erfcf(pp.alpha * r);
        const float kq = pp.coulomb_k;
        phic = kq * (ec * rinv + pp.two_a_sqrtpi * ex) * rinv2;
        const float psic = kq * rinv2 *
                           (-3.0f * ec * rinv * rinv2 -
                            pp.two_a_sqrtpi * ex * (3.0f * rinv2 + 2.0f * pp.alpha2));
        const float qq = pi.w * pj.w;
        phi += qq * phic;
        psi += qq * psic;
      } else if (COUL == 2) {
        const float kq = pp.coulomb_k;
        phic = kq * (rinv * rinv2 - pp.two_k_rf);
        const float qq = pi.w * pj.w;
        phi += qq * phic;
        psi += qq * kq * (-3.0f * rinv2 * rinv2 * rinv);
      }
      const float ddx = uj.x - ui.x, ddy = uj.y - ui.y, ddz = uj.z - ui.z;
      const float sd = dx * ddx + dy * ddy + dz * ddz;
      // force on i is minus the force on j
      gx -= phi * ddx + psi * sd * dx;
      gy -= phi * ddy + psi * sd * dy;
      gz -= phi * ddz + psi * sd * dz;
      ge += (double)(sd * r8 * (aj.x * r6 - aj.y));
      gs += (double)(sd * r8 * (aj.z * r6 - aj.w));
      if (COUL != 0) gq += (double)(sd * phic * ui.w * pj.w);
    }
  }
  // sum over the 16 lanes of the row (the row's i atom)
  for (int o = 8; o >= 1; o >>= 1) {
    gx += __shfl_xor(gx, o, kWave);
    gy += __shfl_xor(gy, o, kWave);
    gz += __shfl_xor(gz, o, kWave);
    ge += __shfl_xor(ge, o, kWave);
    gs += __shfl_xor(gs, o, kWave);
    gq += __shfl_xor(gq, o, kWave);
  }
  const int c3 = lane & 15;
  if (active) {
    if (!EPARAM && c3 < 3) dfs[(size_t)c3 * stride + si] = c3 == 0 ? gx : (c3 == 1 ? gy : gz);
    if (c3 == 0) {
      gslot[si] = ge;
      gslot[stride + si] = gs;
      gslot[2 * (size_t)stride + si] = gq;
    }
  }
}

struct JvpAtomArgs {
  const float* pos;       // [3][n] positions of the node (caller order)
  const float* u;         // [3][n] tangent
  const float* dq;        // [n] charge direction
  const int* inv_perm;
  const float4* xs;       // slot positions (PME gather)
  const float* dfs;       // [3][stride] pair Hessian-vector product by slot
  const double* gslot;    // [3][stride] pair parameter terms by slot
  const float* phi;       // potential of the node
  const float* dphi;      // potential of the dipole grid (not read with EPARAM)
  float* q;               // [3][n] position adjoint, q += wdt dF (not written with EPARAM)
  double* gatom;          // [3][n] parameter terms by atom
  int n, stride;
  float wdt;
};

// Per atom: the pair terms (by slot), the exclusion, bond and angle
// Hessian-vector products and the reciprocal part; q += wdt dF. EPARAM: the
// energy's parameter derivatives instead (exclusion, reciprocal).
template <bool EPARAM, bool COUL, bool PME>
__global__ void __launch_bounds__(256) k_jvp_finish(JvpAtomArgs g, BondedParams bp, Topology tp,
                                                    PmeParams pp) {
  const int a = blockIdx.x * blockDim.x + threadIdx.x;
  if (a >= g.n) return;
  const int n = g.n;
  const int s = g.inv_perm[a];
  const float* pos = g.pos;
  const float* u = g.u;
  float fx = 0.f, fy = 0.f, fz = 0.f;
  double ge = 0.0, gs = 0.0, gq = 0.0;
  if (s >= 0) {
    if (!EPARAM) {
      fx = g.dfs[s];
      fy = g.dfs[g.stride + s];
      fz = g.dfs[2 * (size_t)g.stride + s];
    }
    ge = g.gslot[s];
    gs = g.gslot[g.stride + s];
    gq = g.gslot[2 * (size_t)g.stride + s];
  }
  const float xa = pos[a], ya = pos[n + a], za = pos[2 * n + a];
  const float uxa = u[a], uya = u[n + a], uza = u[2 * n + a];
  const double qa = (double)tp.q[a], dqa = (double)g.dq[a];
  if (COUL) {
    // exclusion corrections -k q_a q_b erf(alpha r)/r, FP64: force on a is
    // s d (d = x_b - x_a, s = U'(r)/r); its derivative s delta + s' (d.delta) d
    double hx = 0.0, hy = 0.0, hz = 0.0;
    for (int k = tp.ex_start[a]; k < tp.ex_start[a + 1]; ++k) {
      const int b = tp.ex_idx[k];
      double d[3] = {(double)pos[b] - (double)xa, (double)pos[n + b] - (double)ya,
                     (double)pos[2 * n + b] - (double)za};
      for (int t = 0; t < 3; ++t) {
        if (d[t] > 0.5 * bp.Ld[t]) d[t] -= bp.Ld[t];
        else if (d[t] < -0.5 * bp.Ld[t]) d[t] += bp.Ld[t];
      }
      const double r2 = d[0] * d[0] + d[1] * d[1] + d[2] * d[2];
      const double r = sqrt(r2);
      const double ar = bp.alpha * r;
      const double erfv = erf(ar), ex = bp.two_a_sqrtpi * exp(-ar * ar);
      const double qb = (double)tp.q[b];
      // per unit k q_a q_b: U = -erf/r, U' = -(ex/r - erf/r^2),
      // U'' = -(2 erf/r^3 - ex (2 alpha^2 + 2/r^2))
      const double up = -(ex / r - erfv / r2);
      const double upp = -(2.0 * erfv / (r2 * r) - ex * (2.0 * bp.alpha * bp.alpha + 2.0 / r2));
      if (EPARAM) {
        gq += -bp.coulomb_k * dqa * qb * erfv / r;
        continue;
      }
      const double kqq = bp.coulomb_k * qa * qb;
      const double su = up / r, sp = (upp - up / r) / r2;   // per unit k q_a q_b
      const double dl[3] = {(double)u[b] - uxa, (double)u[n + b] - uya,
                            (double)u[2 * n + b] - uza};
      const double sd = d[0] * dl[0] + d[1] * dl[1] + d[2] * dl[2];
      hx += kqq * (su * dl[0] + sp * sd * d[0]);
      hy += kqq * (su * dl[1] + sp * sd * d[1]);
      hz += kqq * (su * dl[2] + sp * sd * d[2]);
      // u . dF/dt: pair total -(delta . d) ds/dt, a books the dq_a q_b part
      gq += -sd * bp.coulomb_k * su * dqa * qb;
    }
    fx += (float)hx;
    fy += (float)hy;
    fz += (float)hz;
  }
  if (!EPARAM) {
    // bonds U = k (r - r0)^2: force on j g d (d = x_j - x_i), g = -2k (r - r0)/r,
    // (dg/dr)/r = -2 k r0 / r^3
    for (int k = tp.bt_start[a]; k < tp.bt_start[a + 1]; ++k) {
      const int t = tp.bt_idx[k];
      const int i = tp.bonds[2 * t], j = tp.bonds[2 * t + 1];
      const float dx = min_image(pos[i], pos[j], bp.L[0], bp.hL[0]);
      const float dy = min_image(pos[n + i], pos[n + j], bp.L[1], bp.hL[1]);
      const float dz = min_image(pos[2 * n + i], pos[2 * n + j], bp.L[2], bp.hL[2]);
      const float r = sqrtf(dx * dx + dy * dy + dz * dz);
      const float kb = tp.bond_k[t], r0 = tp.bond_r0[t];
      const float gb = -2.0f * kb * (r - r0) / r;
      const float gp = -2.0f * kb * r0 / (r * r * r);
      const float ddx = u[j] - u[i], ddy = u[n + j] - u[n + i], ddz = u[2 * n + j] - u[2 * n + i];
      const float sd = dx * ddx + dy * ddy + dz * ddz;
      const float sgn = (a == j) ? 1.0f : -1.0f;
      fx += sgn * (gb * ddx + gp * sd * dx);
      fy += sgn * (gb * ddy + gp * sd * dy);
      fz += sgn * (gb * ddz + gp * sd * dz);
    }
    // angles k (theta - theta0)^2 with dual numbers along u
    for (int k = tp.at_start[a]; k < tp.at_start[a + 1]; ++k) {
      const int t = tp.at_idx[k];
      const int i = tp.angles[3 * t], j = tp.angles[3 * t + 1], l = tp.angles[3 * t + 2];
      Dual av[3], bv[3];
      for (int d = 0; d < 3; ++d) {
        const size_t o = (size_t)d * n;
        av[d] = {min_image(pos[o + j], pos[o + i], bp.L[d], bp.hL[d]), u[o + i] - u[o + j]};
        bv[d] = {min_image(pos[o + j], pos[o + l], bp.L[d], bp.hL[d]), u[o + l] - u[o + j]};
      }
      const Dual ra = dsqrt(av[0] * av[0] + av[1] * av[1] + av[2] * av[2]);
      const Dual rb = dsqrt(bv[0] * bv[0] + bv[1] * bv[1] + bv[2] * bv[2]);
      Dual ah[3], bh[3];
      for (int d = 0; d < 3; ++d) {
        ah[d] = av[d] / ra;
        bh[d] = bv[d] / rb;
      }
      Dual c = ah[0] * bh[0] + ah[1] * bh[1] + ah[2] * bh[2];
      if (c.v > 1.0f || c.v < -1.0f) c = {fminf(1.0f, fmaxf(-1.0f, c.v)), 0.0f};
      const float sv = sqrtf(fmaxf(1.0f - c.v * c.v, 1e-12f));
      const Dual theta = {acosf(c.v), -c.d / sv};
      const Dual s = dsqrt(Dual{fmaxf(1.0f - c.v * c.v, 1e-12f), -2.0f * c.v * c.d});
      const Dual pre = (2.0f * tp.angle_k[t]) * (theta - Dual{tp.angle_t0[t], 0.0f}) / s;
      float dFi[3], dFl[3];
      for (int d = 0; d < 3; ++d) {
        dFi[d] = (pre * (bh[d] - c * ah[d]) / ra).d;
        dFl[d] = (pre * (ah[d] - c * bh[d]) / rb).d;
      }
      if (a == i) { fx += dFi[0]; fy += dFi[1]; fz += dFi[2]; }
      if (a == l) { fx += dFl[0]; fy += dFl[1]; fz += dFl[2]; }
      if (a == j) {
        fx -= dFi[0] + dFl[0];
        fy -= dFi[1] + dFl[1];
        fz -= dFi[2] + dFl[2];
      }
    }
  }
  if (PME && s >= 0) {
    // F = -k q sum grad(theta) phi; its derivative along u:
    // -k q [sum (Hess(theta) u) phi + sum grad(theta) dphi]
    const float4 p = g.xs[s];
    const float xyz[3] = {p.x, p.y, p.z};
    int k0[3];
    float th[3][4], dth[3][4], d2[3][4], sc[3];
    for (int d = 0; d < 3; ++d) {
      float fr;
      grid_coord(xyz[d], pp.s_hi[d], pp.s_lo[d], pp.K[d], k0[d], fr);
      spline4(fr, th[d], dth[d]);
      spline4_d2(fr, d2[d]);
      sc[d] = pp.s_hi[d] + pp.s_lo[d];
    }
    const float ux = uxa * sc[0], uy = uya * sc[1], uz = uza * sc[2];
    float hx = 0.f, hy = 0.f, hz = 0.f;   // sum (Hess theta . u) phi, in grid units
    float ex = 0.f, ey = 0.f, ez = 0.f;   // sum grad(theta) dphi
    float gw = 0.f, wd = 0.f;             // u . sum grad(theta) phi and sum theta dphi
    float wphi = 0.f;                     // sum theta phi (EPARAM)
    for (int t3 = 0; t3 < 4; ++t3) {
      int z = k0[2] - t3;
      z += z < 0 ? pp.K[2] : 0;
      for (int t2 = 0; t2 < 4; ++t2) {
        int y = k0[1] - t2;
        y += y < 0 ? pp.K[1] : 0;
        const size_t row = ((size_t)z * pp.K[1] + y) * pp.K[0];
        for (int t1 = 0; t1 < 4; ++t1) {
          int x = k0[0] - t1;
          x += x < 0 ? pp.K[0] : 0;
          const float v = g.phi[row + x];
          const float W = th[0][t1] * th[1][t2] * th[2][t3];
          if (EPARAM) {
            wphi += W * v;
            continue;
          }
          const float Wx = dth[0][t1] * th[1][t2] * th[2][t3];
          const float Wy = th[0][t1] * dth[1][t2] * th[2][t3];
          const float Wz = th[0][t1] * th[1][t2] * dth[2][t3];
          const float Wxx = d2[0][t1] * th[1][t2] * th[2][t3];
          const float Wyy = th[0][t1] * d2[1][t2] * th[2][t3];
          const float Wzz = th[0][t1] * th[1][t2] * d2[2][t3];
          const float Wxy = dth[0][t1] * dth[1][t2] * th[2][t3];
          const float Wxz = dth[0][t1] * th[1][t2] * dth[2][t3];
          const float Wyz = th[0][t1] * dth[1][t2] * dth[2][t3];
          const float dv = g.dphi[row + x];
          hx += (Wxx * ux + Wxy * uy + Wxz * uz) * v;
          hy += (Wxy * ux + Wyy * uy + Wyz * uz) * v;
          hz += (Wxz * ux + Wyz * uy + Wzz * uz) * v;
          ex += Wx * dv;
          ey += Wy * dv;
          ez += Wz * dv;
          gw += (Wx * ux + Wy * uy + Wz * uz) * v;
          wd += W * dv;
        }
      }
    }
    if (EPARAM) {
      gq += (double)pp.coulomb_k * dqa * (double)wphi;
    } else {
      const float c = -pp.coulomb_k * p.w;
      fx += c * (hx + ex) * sc[0];
      fy += c * (hy + ey) * sc[1];
      fz += c * (hz + ez) * sc[2];
      gq += -(double)pp.coulomb_k * dqa * ((double)gw + (double)wd);
    }
  }
  if (!EPARAM) {
    g.q[a] += g.wdt * fx;
    g.q[n + a] += g.wdt * fy;
    g.q[2 * n + a] += g.wdt * fz;
  }
  g.gatom[a] = ge;
  g.gatom[n + a] = gs;
  g.gatom[2 * (size_t)n + a] = gq;
}

// q += gx - gU F, p += gv (each term optional): a loss term on an
// intermediate state joins the reverse pass there.
__global__ void __launch_bounds__(256) k_adj_inject(int n3, const float* __restrict__ gx,
                                                    const float* __restrict__ gv,
                                                    const double* __restrict__ gU,
                                                    const float* __restrict__ force,
                                                    float* __restrict__ q, float* __restrict__ p) {
  const int k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= n3) return;
  float dq = gx ? gx[k] : 0.f;
  if (gU) dq -= (float)*gU * force[k];
  q[k] += dq;
  if (gv) p[k] += gv[k];
}

// q = gx - gU F, p = gv (or 0): the start of the reverse pass.
__global__ void __launch_bounds__(256) k_adj_begin(int n3, const float* __restrict__ gx,
                                                   const float* __restrict__ gv,
                                                   const double* __restrict__ gU,
                                                   const float* __restrict__ force,
                                                   float* __restrict__ q, float* __restrict__ p) {
  const int k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= n3) return;
  const float gu = (float)*gU;
  q[k] = gx[k] - gu * force[k];
  p[k] = gv ? gv[k] : 0.f;
}

// grad[b] += scale (* *scale_dev) * sum, one block per entry: b < T the eps
// terms of type b, T <= b < 2T the sigma terms of type b - T, 2T the charge
// direction (plus q_const), 2T + 1 the dt partials (nblk of them, unscaled).
__global__ void __launch_bounds__(256) k_adj_reduce(const double* __restrict__ gatom,
                                                    const int* __restrict__ atype, int n, int T,
                                                    double scale,
                                                    const double* __restrict__ scale_dev,
                                                    double q_const,
                                                    const double* __restrict__ dt_part, int nblk,
                                                    double* __restrict__ grad) {
  __shared__ double red[16];
  const int b = blockIdx.x;
  double v = 0.0;
  if (b < 2 * T) {
    const int t = b < T ? b : b - T;
    const double* src = gatom + (size_t)(b < T ? 0 : 1) * n;
    for (int a = threadIdx.x; a < n; a += blockDim.x)
      if (atype[a] == t) v += src[a];
  } else if (b == 2 * T) {
    for (int a = threadIdx.x; a < n; a += blockDim.x) v += gatom[2 * (size_t)n + a];
  } else {
    for (int k = threadIdx.x; k < nblk; k += blockDim.x) v += dt_part[k];
  }
  const double sum = block_sum(v, red);
  if (threadIdx.x == 0) {
    if (b <= 2 * T) {
      const double sc = scale * (scale_dev ? *scale_dev : 1.0);
      grad[b] += sc * (sum + (b == 2 * T ? q_const : 0.0));
    } else {
      grad[b] += sum;
    }
  }
}

// out = pos + img L (unwrapped positions)
__global__ void __launch_bounds__(256) k_unwrap(int n, const float* __restrict__ pos,
                                                const int* __restrict__ img, float3 L,
                                                float* __restrict__ out) {
  const int k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= 3 * n) return;
  const int d = k / n;
  const float Ld = d == 0 ? L.x : (d == 1 ? L.y : L.z);
  out[k] = pos[k] + (float)img[k] * Ld;
}

// ---- launchers -------------------------------------------------------------------

namespace {
JvpPairParams make_jvp_params(const Ctx& c) {
  JvpPairParams pp;
  for (int d = 0; d < 3; ++d) pp.L[d] = c.cg.L[d];
  pp.rc2 = c.cg.rc2;
  pp.alpha = (float)c.alpha;
  pp.alpha2 = (float)(c.alpha * c.alpha);
  pp.exp_c = (float)(-c.alpha * c.alpha / M_LN2);
  pp.two_a_sqrtpi = (float)(2.0 * c.alpha / sqrt(M_PI));
  pp.coulomb_k = (float)c.coulomb_k;
  pp.two_k_rf = (float)(2.0 * c.k_rf);
  pp.alpha_d = c.alpha;
  pp.coulomb_kd = c.coulomb_k;
  pp.k_rf_d = c.k_rf;
  pp.c_rf_d = c.c_rf;
  pp.ntypes = c.n_types;
  return pp;
}
}  // namespace

hipError_t launch_adj_pre(Ctx& c, float dt, float w, bool open, const float* q, float* p,
                          const float* v_n, const float* f_n, double* gmass) {
  const int nb = (c.n + 255) / 256;
  k_adj_pre<<<nb, 256, 0, c.stream>>>(c.n, dt, w, open ? 1 : 0, q, p, v_n, f_n, c.hdt_scale,
                                      c.mass, c.adj.u, c.adj.dt_part, gmass);
  return hipGetLastError();
}

hipError_t launch_adj_slots(Ctx& c, const float* pos, bool refresh) {
  if (refresh) {
    hipError_t e = launch_fill_i32(c.adj.gate, 0, 1, c.stream);
    if (e != hipSuccess) return e;
    const float h = 0.5f * c.r_ghost;
    k_adj_refresh<<<(c.max_slots + 255) / 256, 256, 0, c.stream>>>(
        pos, c.perm, c.q, c.x_build, c.meta, c.n, c.cg, h * h, c.xs, c.adj.gate);
    e = launch_build_list(c, pos, c.adj.gate);
    if (e != hipSuccess) return e;
  }
  k_adj_slots<<<(c.max_slots + 255) / 256, 256, 0, c.stream>>>(c.perm, c.meta, c.max_slots, c.n,
                                                                c.adj.u, c.adj.dq, c.adj.us);
  return hipGetLastError();
}

hipError_t launch_pair_jvp(Ctx& c, bool eparam) {
  const JvpPairParams pp = make_jvp_params(c);
  const int TT = c.n_types * c.n_types;
  const size_t sh = (size_t)TT * sizeof(float4) + (size_t)TT * (eparam ? sizeof(double4)
                                                                        : sizeof(float4));
  const int nb = (c.max_clusters + 3) / 4;
  const int coul = c.has_coulomb ? 1 : (c.rf ? 2 : 0);
#define MDX_PJ(E, C)                                                                         \
  k_pair_jvp<E, C><<<nb, 256, sh, c.stream>>>(c.xs, c.ts, c.adj.us, c.tiles, c.tile_count,   \
                                              c.meta, c.nl_cap, pp, c.lj_f, c.adj.lj_f,      \
                                              c.adj.lj_d, c.adj.dfs, c.adj.gslot, c.max_slots)
  if (eparam) {
    if (coul == 1) MDX_PJ(true, 1);
    else if (coul == 2) MDX_PJ(true, 2);
    else MDX_PJ(true, 0);
  } else {
    if (coul == 1) MDX_PJ(false, 1);
    else if (coul == 2) MDX_PJ(false, 2);
    else MDX_PJ(false, 0);
  }
#undef MDX_PJ
  return hipGetLastError();
}

hipError_t launch_jvp_finish(Ctx& c, bool eparam, const float* pos, const float* phi,
                             const float* dphi, float* q, float wdt) {
  JvpAtomArgs g{pos,    c.adj.u,     c.adj.dq,   c.inv_perm, c.xs,  c.adj.dfs,
                c.adj.gslot, phi, dphi, q, c.adj.gatom, c.n, c.max_slots, wdt};
  const BondedParams bp = make_bonded_params(c);
  const Topology tp = make_topology(c);
  const PmeParams pp = c.has_pme ? make_pme_params(c) : PmeParams{};
  const int nb = (c.n + 255) / 256;
  const bool C = c.has_coulomb, P = c.has_pme;
#define MDX_JF(E, CC, PP) k_jvp_finish<E, CC, PP><<<nb, 256, 0, c.stream>>>(g, bp, tp, pp)
  if (eparam) {
    if (C && P) MDX_JF(true, true, true);
    else if (C) MDX_JF(true, true, false);
    else MDX_JF(true, false, false);
  } else {
    if (C && P) MDX_JF(false, true, true);
    else if (C) MDX_JF(false, true, false);
    else MDX_JF(false, false, false);
  }
#undef MDX_JF
  return hipGetLastError();
}

hipError_t launch_adj_begin(Ctx& c, const float* gx, const float* gv, const double* gU,
                            const float* force, float* q, float* p) {
  const int n3 = 3 * c.n;
  k_adj_begin<<<(n3 + 255) / 256, 256, 0, c.stream>>>(n3, gx, gv, gU, force, q, p);
  return hipGetLastError();
}

hipError_t launch_adj_inject(Ctx& c, const float* gx, const float* gv, const double* gU,
                             const float* force, float* q, float* p) {
  const int n3 = 3 * c.n;
  k_adj_inject<<<(n3 + 255) / 256, 256, 0, c.stream>>>(n3, gx, gv, gU, force, q, p);
  return hipGetLastError();
}

hipError_t launch_adj_reduce(Ctx& c, double scale, const double* scale_dev, double q_const,
                             int dt_blocks, double* grad) {
  const int T = c.n_types;
  k_adj_reduce<<<2 * T + 2, 256, 0, c.stream>>>(c.adj.gatom, c.atype, c.n, T, scale, scale_dev,
                                                q_const, c.adj.dt_part, dt_blocks, grad);
  return hipGetLastError();
}

hipError_t launch_unwrap(Ctx& c, const float* pos, float* out) {
  const float3 L = make_float3(c.box[0], c.box[1], c.box[2]);
  k_unwrap<<<(3 * c.n + 255) / 256, 256, 0, c.stream>>>(c.n, pos, c.img, L, out);
  return hipGetLastError();
}

}  // namespace mdx
