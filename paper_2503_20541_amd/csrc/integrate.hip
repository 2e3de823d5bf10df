// Velocity Verlet (DIMOS Sec. II.D.1): the half kick + drift of steps 1-2 and
// the closing half kick of step 5, with positions wrapped back into [0, L).
//
// k_begin_step / k_finish_step: the updates fused, per slot, with the
//   neighbour-list refresh and validity test (begin) and with the PME force
//   interpolation, the bonded and exclusion terms and the kinetic energy
//   (finish); mdx_integrate_step uses these.
#include "atom_terms.h"

namespace mdx {

// x wrapped into [0, L); wraps gets the box lengths subtracted (+1 / -1).
__device__ __forceinline__ float wrap_box(float x, float L, int& wraps) {
  wraps = 0;
  if (x >= L) {
    x -= L;
    wraps = 1;
  } else if (x < 0.f) {
    x += L;
    wraps = -1;
    if (x >= L) {   // a tiny negative x rounds onto L: it stays at 0
      x = 0.f;
      wraps = 0;
    }
  }
  return x;
}

// Opening half of a step (v += (dt/2) a, x += dt v wrapped) for atom a in
// slot s, with the slot position refreshed (as build position + minimum-image
// displacement), the r_g/2 validity test (raises gate_now) and the pruned
// list's validity test (raises pgate_now). Positions are read from pos_in
// and written to pos_out (the same array for the stand-alone kernel).
struct OpenStep {
  const float* pos_in;
  const float* lv_sig;   // Langevin: sqrt(kT accel / m) per atom (null: velocity Verlet)
  float lv_c1, lv_c2;
  unsigned long long lv_seed, lv_step;
  float* pos_out;
  const float* x_build;
  const float4* xp;
  const float* q;
  const float* acc_over_m;
  float4* xs;
  int* img;
  float* xc;
  float* vc;
  int* gate_now;
  int* gate_next;
  int* pgate_now;
  int* pgate_next;
  int force_rebuild;
  int n;
  CellGrid cg;
  float half_dt, dt, half_skin2, prune_move2;
};

// Thread 0 of the grid clears the flags of the step after (nothing else
// touches them in this kernel) and raises gate_now on a cadence rebuild.
__device__ __forceinline__ void open_step_flags(const OpenStep& o) {
  *o.gate_next = 0;
  *o.pgate_next = 0;
  if (o.force_rebuild) *o.gate_now = 1;
}

// Philox4x64-10 (Salmon, Moraes, Dror, Shaw, SC'11): ten rounds of two
// 64 x 64 -> 128-bit products with the Weyl-sequence key schedule.
__device__ __forceinline__ void philox4x64_10(unsigned long long c[4], unsigned long long k0,
                                              unsigned long long k1) {
  const unsigned long long M0 = 0xD2E7470EE14C6C93ull, M1 = 0xCA5A826395121157ull;
  const unsigned long long W0 = 0x9E3779B97F4A7C15ull, W1 = 0xBB67AE8584CAA73Bull;
  for (int r = 0; r < 10; ++r) {
    if (r) {
      k0 += W0;
      k1 += W1;
    }
    const unsigned long long hi0 = __umul64hi(M0, c[0]), lo0 = M0 * c[0];
    const unsigned long long hi1 = __umul64hi(M1, c[2]), lo1 = M1 * c[2];
    const unsigned long long n0 = hi1 ^ c[1] ^ k0, n2 = hi0 ^ c[3] ^ k1;
    c[0] = n0;
    c[1] = lo1;
    c[2] = n2;
    c[3] = lo0;
  }
}

// Three standard normals for atom a at a step: Box-Muller of the block's
// four uniforms (top 24 bits + 1) / 2^24 in (0, 1].
__device__ __forceinline__ void langevin_normals(unsigned long long seed, unsigned long long step,
                                                 int a, float z[3]) {
  unsigned long long c[4] = {(unsigned long long)a, step, 0ull, 0ull};
  philox4x64_10(c, seed, 0ull);
  float u[4];
  for (int k = 0; k < 4; ++k) u[k] = (float)((c[k] >> 40) + 1ull) * 5.9604644775390625e-8f;
  const float r1 = sqrtf(-2.0f * logf(u[0])), r2 = sqrtf(-2.0f * logf(u[2]));
  const float t1 = 6.28318530717958648f * u[1], t2 = 6.28318530717958648f * u[3];
  z[0] = r1 * cosf(t1);
  z[1] = r1 * sinf(t1);
  z[2] = r2 * cosf(t2);
}

// What the opening half reads of atom a (slot s) besides its force and
// velocity: position, build position, pruned-list position, charge, dt/2
// scale and the Langevin noise amplitude. Read ahead of the kick, these loads
// overlap the rest of the closing kernel's.
struct OpenIn {
  float x[3], b[3];
  float4 p0;
  float qa, acc, sig;
};

__device__ __forceinline__ void open_fetch(const OpenStep& o, int a, int s, OpenIn& in) {
  const unsigned un = o.n, ua = a;
  for (unsigned d = 0; d < 3; ++d) {
    in.x[d] = ld32(o.pos_in, d * un + ua);
    in.b[d] = ld32(o.x_build, d * un + ua);
  }
  in.p0 = ld32(o.xp, (unsigned)s);
  in.qa = ld32(o.q, ua);
  in.acc = ld32(o.acc_over_m, ua);
  in.sig = o.lv_sig ? ld32(o.lv_sig, ua) : 0.f;
}

// The rest of the opening half once the three new coordinates x of an atom
// in slot s are known (b: its build position, q0: its pruned-list position):
// slot refresh and the two validity tests.
__device__ __forceinline__ void open_tail_at(const OpenStep& o, int s, const float x[3],
                                             const float b[3], float qa, float4 q0) {
  const CellGrid& cg = o.cg;
  const float dx = min_image(b[0], x[0], cg.L[0], cg.hL[0]);
  const float dy = min_image(b[1], x[1], cg.L[1], cg.hL[1]);
  const float dz = min_image(b[2], x[2], cg.L[2], cg.hL[2]);
  // slot position continued from the build position (not wrapped between
  // builds), so the periodic image each list tile records stays valid
  o.xs[s] = make_float4(b[0] + dx, b[1] + dy, b[2] + dz, qa);
  if (dist2(dx, dy, dz) > o.half_skin2) atomicOr(o.gate_now, 1);
  // pruned list: displacement since it was made (same slot order)
  const float px = min_image(q0.x, x[0], cg.L[0], cg.hL[0]);
  const float py = min_image(q0.y, x[1], cg.L[1], cg.hL[1]);
  const float pz = min_image(q0.z, x[2], cg.L[2], cg.hL[2]);
  if (dist2(px, py, pz) > o.prune_move2) atomicOr(o.pgate_now, 1);
}

__device__ __forceinline__ void open_tail(const OpenStep& o, int a, int s, const float x[3]) {
  const int n = o.n;
  const float b[3] = {o.x_build[a], o.x_build[n + a], o.x_build[2 * n + a]};
  open_tail_at(o, s, x, b, o.q[a], o.xp[s]);
}

// Opening half for atom a in slot s from its force f and velocity v.
__device__ __forceinline__ void open_step_atom(const OpenStep& o, const OpenIn& in,
                                               const float f[3], const float v[3],
                                               float* __restrict__ vel, int a, int s) {
  const int n = o.n;
  const CellGrid& cg = o.cg;
  const float h = o.half_dt * in.acc;
  float x[3];
  if (o.lv_sig) {
    // Langevin, BAOAB: kick, half drift, Ornstein-Uhlenbeck step, half drift
    float z[3];
    langevin_normals(o.lv_seed, o.lv_step, a, z);
    const float sg = in.sig;
    const float hdt = 0.5f * o.dt;
    for (int d = 0; d < 3; ++d) {
      const size_t k = (size_t)d * n + a;
      int wraps;
      const float v1 = v[d] + h * f[d];
      const float xh = in.x[d] + hdt * v1;
      const float v2 = o.lv_c1 * v1 + o.lv_c2 * sg * z[d];
      vel[k] = v2;
      x[d] = wrap_box(xh + hdt * v2, cg.L[d], wraps);
      o.pos_out[k] = x[d];
      if (wraps) o.img[k] += wraps;
    }
  } else
  for (int d = 0; d < 3; ++d) {
    const size_t k = (size_t)d * n + a;
    int wraps;
    if (o.xc) {   // compensated sums (MDX_OPT_KAHAN_VV)
      float cv = o.vc[k], cx = o.xc[k];
      const float vv = kahan_add(v[d], h * f[d], cv);
      vel[k] = vv;
      x[d] = wrap_box(kahan_add(in.x[d], o.dt * vv, cx), cg.L[d], wraps);
      o.vc[k] = cv;
      o.xc[k] = cx;
    } else {
      const float vv = v[d] + h * f[d];
      vel[k] = vv;
      x[d] = wrap_box(in.x[d] + o.dt * vv, cg.L[d], wraps);
    }
    o.pos_out[k] = x[d];
    if (wraps) o.img[k] += wraps;
  }
  open_tail_at(o, s, x, in.b, in.qa, in.p0);
}

// Stand-alone opening half for every slot (the first step of a call).
__global__ void __launch_bounds__(256) k_begin_step(OpenStep o, const float* __restrict__ force,
                                                    float* __restrict__ vel,
                                                    const int* __restrict__ perm,
                                                    const int* __restrict__ meta) {
  const int s = blockIdx.x * blockDim.x + threadIdx.x;
  if (s == 0) open_step_flags(o);
  if (s >= meta[0]) return;
  const int a = perm[s];
  if (a < 0) return;
  OpenIn in;
  open_fetch(o, a, s, in);
  const int n = o.n;
  const float f[3] = {force[a], force[n + a], force[2 * n + a]};
  const float v[3] = {vel[a], vel[n + a], vel[2 * n + a]};
  open_step_atom(o, in, f, v, vel, a, s);
}

// Closing half of a step, two lanes per slot. Without SIDE, lane q of the
// pair takes z planes q and q + 2 of the PME stencil (with PME) and every
// second bonded / exclusion term of the atom; with a half list it also takes
// every second of the j partials naming its cluster. With SIDE (PME
// contexts of at least kSideStreamMinAtoms atoms) the reciprocal-space force
// and those terms were summed by slot into fside on the second stream
// (k_side_terms), and the kernel reads that sum. The pair of lanes sums its
// parts in a fixed order, and lane 0 adds the pair force the pair kernel
// stored in the slot array (clearing it), stores the total and applies
// v += (dt/2) a. FP64 energy partials (exclusion, bond, angle, kinetic) per
// block. With `open`, lane 0 then opens the next
// step for its atom (open_step_atom, from the velocity and force it has just
// computed): the same values as a separate opening kernel, one launch fewer
// per step. The bonded terms read the positions of other atoms from `pos`,
// so the new positions go to o.pos_out (another buffer).
//
// The kernel is bound by the latency of its dependent loads, so every load
// that does not need an earlier one's value is issued first: the slot's
// position and the atom's list bounds, lane 0's kick and opening inputs, then
// the PME planes and the first term of each kind (terms_fetch), and only
// then the arithmetic, in the same order as a plain evaluation.
constexpr int kFinishLanes = 2;
constexpr int kFinishPlanes = 4 / kFinishLanes;   // PME z planes per lane

template <bool ENERGY, bool COUL, bool PME, bool SIDE>
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(2))) k_finish_step(
    const float4* __restrict__ xs, const float* __restrict__ phi, PmeParams pp,
    const int* __restrict__ perm, const int* __restrict__ meta, const float* __restrict__ pos,
    int n, BondedParams bp, Topology tp, float* __restrict__ fslot, int fstride,
    float* __restrict__ force, float* __restrict__ vel,
    const float* __restrict__ acc_over_m, const float* __restrict__ mass, float half_dt,
    double inv_2acc, double* __restrict__ partials, int pstride, float* __restrict__ vc,
    OpenStep o, int open, JParts jp, const float* __restrict__ fside) {
  __shared__ double red[16];
  if (open && blockIdx.x == 0 && threadIdx.x == 0) open_step_flags(o);
  // neighbouring slots on one XCD (the same order as k_side_terms): the PME
  // potential they gather comes from one part of the grid
  const int lb = xcd_block((meta[0] * kFinishLanes + 255) / 256);
  const int gt = lb * blockDim.x + threadIdx.x;
  const int s = gt / kFinishLanes, q = gt & (kFinishLanes - 1);
  double e_ex = 0.0, e_b = 0.0, e_a = 0.0, ke = 0.0;
  const bool live = lb >= 0 && s < meta[0];
  const int a = live ? ld32(perm, (unsigned)s) : -1;
  float4 p;
  if (PME && !SIDE && live) p = ld32(xs, (unsigned)s);
  float fx = 0.f, fy = 0.f, fz = 0.f;
  float fs[3], sd[3], v[3], acc;
  OpenIn in;
  if (a >= 0) {
    AtomTerms t;
    if (!SIDE) terms_begin<COUL>(t, a, pos, n, tp, q);
    // lane 0's inputs, read by both lanes (one request per pair) so no
    // branch holds the loads back
    for (unsigned d = 0; d < 3; ++d) {
      fs[d] = ld32(fslot, d * fstride + s);
      if (SIDE) sd[d] = ld32(fside, d * fstride + s);
      v[d] = ld32(vel, d * n + a);
    }
    acc = ld32(acc_over_m, (unsigned)a);
    if (open) open_fetch(o, a, s, in);
    if (!SIDE) {
      PmeStencil st;
      float pv[kFinishPlanes][16];
      if (PME) {
        pme_stencil(p, pp, st);
        for (int k = 0; k < kFinishPlanes; ++k)
          pme_plane_load(st, phi, pp, q + k * kFinishLanes, pv[k]);
      }
      terms_fetch<COUL>(t, a, pos, n, tp);
      if (PME) {
        float gx = 0.f, gy = 0.f, gz = 0.f;
        for (int k = 0; k < kFinishPlanes; ++k) {
          const int t3 = q + k * kFinishLanes;
          pme_plane_add(st, pv[k], pick4(st.th[2], t3), pick4(st.dth[2], t3), gx, gy, gz);
        }
        pme_force_add(p, pp, gx, gy, gz, fx, fy, fz);
      }
      terms_apply<ENERGY, COUL, false>(t, a, pos, n, bp, tp, fx, fy, fz, e_ex, e_b, e_a,
                                       kFinishLanes, nullptr);
    }
    if (jp.jpart) add_jparts(jp, s, q, kFinishLanes, fx, fy, fz);
  }
  // sum over the slot's lanes (they share the slot, so a is uniform among them)
  for (int o = 1; o < kFinishLanes; o <<= 1) {
    fx += __shfl_xor(fx, o, kWave);
    fy += __shfl_xor(fy, o, kWave);
    fz += __shfl_xor(fz, o, kWave);
  }
  if (a >= 0 && q == 0) {
    fx += fs[0];
    fy += fs[1];
    fz += fs[2];
    if (SIDE) {
      fx += sd[0];
      fy += sd[1];
      fz += sd[2];
    }
    fslot[s] = 0.f;
    fslot[fstride + s] = 0.f;
    fslot[2 * fstride + s] = 0.f;
    force[a] = fx;
    force[n + a] = fy;
    force[2 * n + a] = fz;
    const float h = half_dt * acc;
    float v0, v1, v2;
    if (vc) {   // compensated sums (MDX_OPT_KAHAN_VV)
      float c0 = vc[a], c1 = vc[n + a], c2 = vc[2 * n + a];
      v0 = kahan_add(v[0], h * fx, c0);
      v1 = kahan_add(v[1], h * fy, c1);
      v2 = kahan_add(v[2], h * fz, c2);
      vc[a] = c0;
      vc[n + a] = c1;
      vc[2 * n + a] = c2;
    } else {
      v0 = v[0] + h * fx;
      v1 = v[1] + h * fy;
      v2 = v[2] + h * fz;
    }
    vel[a] = v0;
    vel[n + a] = v1;
    vel[2 * n + a] = v2;
    if (ENERGY)
      ke = (double)mass[a] * ((double)v0 * v0 + (double)v1 * v1 + (double)v2 * v2) * inv_2acc;
    if (open) {
      const float f3[3] = {fx, fy, fz}, v3[3] = {v0, v1, v2};
      open_step_atom(o, in, f3, v3, vel, a, s);
    }
  }
  if (ENERGY) {
    if (!SIDE) {   // (with SIDE the side kernel wrote these rows)
      double s1 = block_sum(e_ex, red);
      double s2 = block_sum(e_b, red);
      double s3 = block_sum(e_a, red);
      if (threadIdx.x == 0) {
        partials[kRowExcl * pstride + blockIdx.x] = s1;
        partials[kRowBond * pstride + blockIdx.x] = s2;
        partials[kRowAngle * pstride + blockIdx.x] = s3;
      }
    }
    double s4 = block_sum(ke, red);
    if (threadIdx.x == 0) partials[kRowKin * pstride + blockIdx.x] = s4;
  }
}

// The closing half's forces that do not need the pair kernel: the PME force
// interpolation and the bonded and exclusion terms, summed by slot into
// fside. Inside mdx_integrate_step they run on the second stream after the
// last FFT pass (the potential is complete there), beside the end of the
// pair kernel, and the closing kernel adds the sum. Lane q of the pair takes
// z planes q and q + 2 of the PME stencil and every second term; every load
// that does not need an earlier one's value is issued first. Same lanes,
// block order and grid as the closing kernel, so its energy rows (exclusion,
// bond, angle) line up with the closing kernel's kinetic row.
template <bool ENERGY>
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(2))) k_side_terms(
    const int* __restrict__ perm, const int* __restrict__ meta, const float* __restrict__ pos,
    int n, BondedParams bp, Topology tp, const float4* __restrict__ xs,
    const float* __restrict__ phi, PmeParams pp, float* __restrict__ fside, int fstride,
    double* __restrict__ partials, int pstride) {
  __shared__ double red[16];
  const int lb = xcd_block((meta[0] * kFinishLanes + 255) / 256);
  const int gt = lb * blockDim.x + threadIdx.x;
  const int s = gt / kFinishLanes, q = gt & (kFinishLanes - 1);
  const bool live = lb >= 0 && s < meta[0];
  const int a = live ? ld32(perm, (unsigned)s) : -1;
  float4 p;
  if (live) p = ld32(xs, (unsigned)s);
  double e_ex = 0.0, e_b = 0.0, e_a = 0.0;
  float fx = 0.f, fy = 0.f, fz = 0.f;
  if (a >= 0) {
    AtomTerms t;
    terms_begin<true>(t, a, pos, n, tp, q);
    PmeStencil st;
    float pv[kFinishPlanes][16];
    pme_stencil(p, pp, st);
    for (int k = 0; k < kFinishPlanes; ++k)
      pme_plane_load(st, phi, pp, q + k * kFinishLanes, pv[k]);
    terms_fetch<true>(t, a, pos, n, tp);
    {
      float gx = 0.f, gy = 0.f, gz = 0.f;
      for (int k = 0; k < kFinishPlanes; ++k) {
        const int t3 = q + k * kFinishLanes;
        pme_plane_add(st, pv[k], pick4(st.th[2], t3), pick4(st.dth[2], t3), gx, gy, gz);
      }
      pme_force_add(p, pp, gx, gy, gz, fx, fy, fz);
    }
    terms_apply<ENERGY, true, false>(t, a, pos, n, bp, tp, fx, fy, fz, e_ex, e_b, e_a,
                                     kFinishLanes, nullptr);
  }
  for (int o = 1; o < kFinishLanes; o <<= 1) {
    fx += __shfl_xor(fx, o, kWave);
    fy += __shfl_xor(fy, o, kWave);
    fz += __shfl_xor(fz, o, kWave);
  }
  if (a >= 0 && q == 0) {
    fside[s] = fx;
    fside[fstride + s] = fy;
    fside[2 * fstride + s] = fz;
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

namespace {
OpenStep make_open(const Ctx& c, const float* pos_in, float* pos_out, float dt,
                   const StepGates& g) {
  const float h = 0.5f * c.r_ghost;
  OpenStep o;
  o.pos_in = pos_in;
  o.pos_out = pos_out;
  o.x_build = c.x_build;
  o.xp = c.xp;
  o.q = c.q;
  o.acc_over_m = c.hdt_scale;
  o.xs = c.xs;
  o.img = c.img;
  o.xc = c.xc;
  o.vc = c.vc;
  o.gate_now = g.gate_now;
  o.gate_next = g.gate_next;
  o.pgate_now = g.pgate_now;
  o.pgate_next = g.pgate_next;
  o.force_rebuild = g.cadence ? 1 : 0;
  o.n = c.n;
  o.cg = c.cg;
  o.half_dt = 0.5f * dt;
  o.dt = dt;
  o.half_skin2 = h * h;
  o.prune_move2 = c.prune_move2;
  o.lv_sig = c.langevin ? c.lv_sig : nullptr;
  o.lv_c1 = (float)std::exp(-c.lv_gamma * (double)dt);
  o.lv_c2 = (float)std::sqrt(std::max(0.0, 1.0 - std::exp(-2.0 * c.lv_gamma * (double)dt)));
  o.lv_seed = c.lv_seed;
  o.lv_step = (unsigned long long)g.step;
  return o;
}
}  // namespace

// Rigid water (RATTLE): after the drift, each molecule's three distances
// (O-H1, O-H2, H1-H2) are restored by SHAKE iterations along the bond
// vectors of the previous positions x_old (minimum image), the velocities
// take the same correction over dt, and the atoms are wrapped, their slots
// refreshed and the validity tests redone; after the closing kick the
// velocities are projected onto the constraints (an exact 3x3 solve). One
// thread per molecule.
struct RigidArgs {
  const int* mols;     // [n_mol][3] caller atoms O, H1, H2
  int n_mol;
  float d[3];          // O-H1, O-H2, H1-H2
  const float* acc_over_m;
  int settle;          // closed form (every molecule's hydrogens weigh the same)
};

__device__ __forceinline__ double3 d3(float3 v) { return make_double3(v.x, v.y, v.z); }
__device__ __forceinline__ double3 operator+(double3 a, double3 b) {
  return make_double3(a.x + b.x, a.y + b.y, a.z + b.z);
}
__device__ __forceinline__ double3 operator-(double3 a, double3 b) {
  return make_double3(a.x - b.x, a.y - b.y, a.z - b.z);
}
__device__ __forceinline__ double3 operator*(double s, double3 a) {
  return make_double3(s * a.x, s * a.y, s * a.z);
}
__device__ __forceinline__ double dot3(double3 a, double3 b) {
  return a.x * b.x + a.y * b.y + a.z * b.z;
}
__device__ __forceinline__ double3 cross3(double3 a, double3 b) {
  return make_double3(a.y * b.z - a.z * b.y, a.z * b.x - a.x * b.z, a.x * b.y - a.y * b.x);
}
__device__ __forceinline__ double3 unit3(double3 a) { return rsqrt(dot3(a, a)) * a; }

// SETTLE: the closed-form solution of the three distance constraints (the
// fixed point SHAKE iterates to). Every displacement lies in the old plane,
// the centre of mass is kept, and the constraint moves carry no torque about
// the old plane's normal; in a frame with Z along that normal, the new Z
// coordinates fix the triangle's tilts (phi about X, psi about Y) and the
// torque condition alpha sin(theta) + beta cos(theta) = gamma its turn about
// Z. ob0, oc0: old H1 - O, H2 - O; ob1, oc1: the same after the drift;
// returns the displacements of O, H1, H2 from the drifted positions, false
// for a geometry with no solution. FP64 throughout (vectors of ~1 A).
__device__ bool settle_water(double3 ob0, double3 oc0, double3 ob1, double3 oc1, double mo,
                             double mh, double d_oh, double d_hh, double3 dl[3]) {
  const double M = mo + 2.0 * mh, rc = 0.5 * d_hh;
  const double h = sqrt(d_oh * d_oh - rc * rc), ra = 2.0 * mh * h / M, rb = h - ra;
  const double3 com0 = (mh / M) * (ob0 + oc0), com1 = (mh / M) * (ob1 + oc1);
  const double3 o0[3] = {-1.0 * com0, ob0 - com0, oc0 - com0};
  const double3 n1[3] = {-1.0 * com1, ob1 - com1, oc1 - com1};
  const double3 Z = unit3(cross3(ob0, oc0));
  const double3 X = unit3(cross3(n1[0], Z));
  const double3 Y = cross3(Z, X);
  double ox[3], oy[3], nx[3], ny[3], nz[3];
  for (int k = 0; k < 3; ++k) {
    ox[k] = dot3(o0[k], X);
    oy[k] = dot3(o0[k], Y);
    nx[k] = dot3(n1[k], X);
    ny[k] = dot3(n1[k], Y);
    nz[k] = dot3(n1[k], Z);
  }
  const double sphi = nz[0] / ra;
  if (!(fabs(sphi) < 1.0)) return false;
  const double cphi = sqrt(1.0 - sphi * sphi);
  const double spsi = (nz[1] - nz[2]) / (2.0 * rc * cphi);
  if (!(fabs(spsi) < 1.0)) return false;
  const double cpsi = sqrt(1.0 - spsi * spsi);
  const double tx[3] = {0.0, -rc * cpsi, rc * cpsi};
  const double ty[3] = {ra * cphi, -rb * cphi - rc * spsi * sphi, -rb * cphi + rc * spsi * sphi};
  const double tz[3] = {ra * sphi, -rb * sphi + rc * spsi * cphi, -rb * sphi - rc * spsi * cphi};
  const double w[3] = {mo, mh, mh};
  double al = 0.0, be = 0.0, ga = 0.0;
  for (int k = 0; k < 3; ++k) {
    al += w[k] * (ox[k] * tx[k] + oy[k] * ty[k]);
    be += w[k] * (ox[k] * ty[k] - oy[k] * tx[k]);
    ga += w[k] * (ox[k] * ny[k] - oy[k] * nx[k]);
  }
  const double ab = al * al + be * be, disc = ab - ga * ga;
  if (!(ab > 0.0) || !(disc >= 0.0)) return false;
  const double sth = (al * ga - be * sqrt(disc)) / ab;
  const double cth = sqrt(1.0 - sth * sth);
  const double3 rel[3] = {make_double3(0.0, 0.0, 0.0), ob1, oc1};   // drifted, from O
  for (int k = 0; k < 3; ++k) {
    const double x3 = tx[k] * cth - ty[k] * sth, y3 = tx[k] * sth + ty[k] * cth;
    dl[k] = com1 + (x3 * X + y3 * Y + tz[k] * Z) - rel[k];
  }
  return true;
}

__device__ __forceinline__ float3 mi3(float3 d, const CellGrid& cg) {
  return make_float3(min_image(0.f, d.x, cg.L[0], cg.hL[0]), min_image(0.f, d.y, cg.L[1], cg.hL[1]),
                     min_image(0.f, d.z, cg.L[2], cg.hL[2]));
}

// x_old: positions before the drift; y_in: after it; pos: where the
// constrained positions go (x_old and pos may be the same array: a thread
// reads and writes the coordinates of its own molecule only).
__global__ void __launch_bounds__(64) k_rigid_positions(RigidArgs r, OpenStep o,
                                                        const float* x_old,
                                                        const float* __restrict__ y_in,
                                                        float* pos,
                                                         float* __restrict__ vel,
                                                         const int* __restrict__ inv_perm,
                                                         unsigned* __restrict__ flags) {
  const int m = blockIdx.x * blockDim.x + threadIdx.x;
  if (m >= r.n_mol) return;
  // a molecule with an atom that a full column left out of the list was not
  // drifted: it is left as it is (the build latched MDX_FLAG_COLUMN_OVERFLOW)
  if (inv_perm[r.mols[3 * m]] < 0 || inv_perm[r.mols[3 * m + 1]] < 0 ||
      inv_perm[r.mols[3 * m + 2]] < 0)
    return;
  const int n = o.n;
  const CellGrid& cg = o.cg;
  int at[3];
  float3 y0[3], dl[3], ref[3], d0[3];
  float iw[3];
  for (int k = 0; k < 3; ++k) {
    at[k] = r.mols[3 * m + k];
    y0[k] = make_float3(y_in[at[k]], y_in[n + at[k]], y_in[2 * n + at[k]]);
    dl[k] = make_float3(0.f, 0.f, 0.f);
    iw[k] = r.acc_over_m[at[k]];   // accel / mass: only the ratios matter
  }
  // constraint c joins atoms (ca, cb): (0,1), (0,2), (1,2); directions from x_old
  const int ca[3] = {0, 0, 1}, cb[3] = {1, 2, 2};
  for (int c = 0; c < 3; ++c) {
    const int a = at[ca[c]], b = at[cb[c]];
    ref[c] = mi3(make_float3(x_old[a] - x_old[b], x_old[n + a] - x_old[n + b],
                             x_old[2 * n + a] - x_old[2 * n + b]), cg);
    d0[c] = mi3(make_float3(y0[ca[c]].x - y0[cb[c]].x, y0[ca[c]].y - y0[cb[c]].y,
                            y0[ca[c]].z - y0[cb[c]].z), cg);
  }
  if (r.settle) {
    // closed form, FP64 (ratios of the masses only: 1 / (accel / m))
    double3 dd[3];
    const bool ok = settle_water(-1.0 * d3(ref[0]), -1.0 * d3(ref[1]), -1.0 * d3(d0[0]),
                                 -1.0 * d3(d0[1]), 1.0 / (double)iw[0], 1.0 / (double)iw[1],
                                 (double)r.d[0], (double)r.d[2], dd);
    if (!ok) atomicOr(flags, MDX_FLAG_CONSTRAINT);
    for (int k = 0; k < 3; ++k)
      dl[k] = ok ? make_float3((float)dd[k].x, (float)dd[k].y, (float)dd[k].z)
                 : make_float3(0.f, 0.f, 0.f);
  } else {
  // The iteration moves the displacements dl (small numbers) rather than the
  // coordinates: the velocity correction dl/dt then carries no cancellation
  // between two coordinates of the size of the box.
  float worst = 0.f;
  for (int it = 0; it < 200; ++it) {
    worst = 0.f;
    for (int c = 0; c < 3; ++c) {
      const int a = ca[c], b = cb[c];
      const float3 d = make_float3(d0[c].x + (dl[a].x - dl[b].x), d0[c].y + (dl[a].y - dl[b].y),
                                   d0[c].z + (dl[a].z - dl[b].z));
      const float diff = d.x * d.x + d.y * d.y + d.z * d.z - r.d[c] * r.d[c];
      worst = fmaxf(worst, fabsf(diff) / (r.d[c] * r.d[c]));
      const float g = diff / (2.0f * (iw[a] + iw[b]) *
                              (d.x * ref[c].x + d.y * ref[c].y + d.z * ref[c].z));
      const float ga = g * iw[a], gb = g * iw[b];
      dl[a].x -= ga * ref[c].x;
      dl[a].y -= ga * ref[c].y;
      dl[a].z -= ga * ref[c].z;
      dl[b].x += gb * ref[c].x;
      dl[b].y += gb * ref[c].y;
      dl[b].z += gb * ref[c].z;
    }
    // 2e-6 in r^2 (1e-6 in length) stays well above the float32 rounding of
    // |d|^2 (a few 1e-7), so every molecule stops after a few sweeps
    if (worst < 2e-6f) break;
  }
  if (!(worst < 2e-6f)) atomicOr(flags, MDX_FLAG_CONSTRAINT);   // also for a NaN
  }
  for (int k = 0; k < 3; ++k) {
    const int a = at[k];
    const float inv_dt = 1.0f / o.dt;
    const float dx0[3] = {dl[k].x, dl[k].y, dl[k].z};
    float x[3] = {y0[k].x + dl[k].x, y0[k].y + dl[k].y, y0[k].z + dl[k].z};
    for (int d = 0; d < 3; ++d) {
      const size_t kk = (size_t)d * n + a;
      vel[kk] += dx0[d] * inv_dt;
      int wraps;
      x[d] = wrap_box(x[d], cg.L[d], wraps);
      pos[kk] = x[d];
      if (wraps) o.img[kk] += wraps;
    }
    const int s = inv_perm[a];
    open_tail(o, a, s, x);
  }
}

// ENERGY: the kinetic energy change of the projection, FP64, one partial per
// block (the closing kernel took the kinetic energy before it).
template <bool ENERGY>
__global__ void __launch_bounds__(64) k_rigid_velocities(RigidArgs r, CellGrid cg, int n,
                                                          const float* __restrict__ pos,
                                                          float* __restrict__ vel,
                                                          const float* __restrict__ mass,
                                                          double inv_2acc,
                                                          double* __restrict__ partials,
                                                          int pstride,
                                                          unsigned* __restrict__ flags) {
  __shared__ double red[16];
  const int m = blockIdx.x * blockDim.x + threadIdx.x;
  double dke = 0.0;
  if (m < r.n_mol) {
  int at[3];
  float3 v[3];
  float iw[3];
  for (int k = 0; k < 3; ++k) {
    at[k] = r.mols[3 * m + k];
    v[k] = make_float3(vel[at[k]], vel[n + at[k]], vel[2 * n + at[k]]);
    iw[k] = r.acc_over_m[at[k]];   // 1 / (mass / accel)
  }
  const int ca[3] = {0, 0, 1}, cb[3] = {1, 2, 2};
  float3 rc[3];
  for (int c = 0; c < 3; ++c) {
    const int a = at[ca[c]], b = at[cb[c]];
    rc[c] = mi3(make_float3(pos[a] - pos[b], pos[n + a] - pos[n + b], pos[2 * n + a] - pos[2 * n + b]),
                cg);
  }
  // A mu = rhs: r_c . (v_a - v_b) after v_i += sum_c' mu_c' s_c',i r_c' w_i^-1 vanishes
  double A[3][3], rhs[3];
  for (int c = 0; c < 3; ++c) {
    const int a = ca[c], b = cb[c];
    const float3 dv = make_float3(v[a].x - v[b].x, v[a].y - v[b].y, v[a].z - v[b].z);
    rhs[c] = -((double)rc[c].x * dv.x + (double)rc[c].y * dv.y + (double)rc[c].z * dv.z);
    for (int c2 = 0; c2 < 3; ++c2) {
      const int a2 = ca[c2], b2 = cb[c2];
      const double coef = (a2 == a ? iw[a] : 0.0) - (b2 == a ? iw[a] : 0.0) -
                          (a2 == b ? iw[b] : 0.0) + (b2 == b ? iw[b] : 0.0);
      A[c][c2] = ((double)rc[c].x * rc[c2].x + (double)rc[c].y * rc[c2].y +
                  (double)rc[c].z * rc[c2].z) * coef;
    }
  }
  // Cramer's rule (3x3)
  const double det = A[0][0] * (A[1][1] * A[2][2] - A[1][2] * A[2][1]) -
                     A[0][1] * (A[1][0] * A[2][2] - A[1][2] * A[2][0]) +
                     A[0][2] * (A[1][0] * A[2][1] - A[1][1] * A[2][0]);
  if (!(det != 0.0) || !isfinite(det)) atomicOr(flags, MDX_FLAG_CONSTRAINT);
  double mu[3];
  for (int c = 0; c < 3; ++c) {
    double B[3][3];
    for (int i = 0; i < 3; ++i)
      for (int j = 0; j < 3; ++j) B[i][j] = j == c ? rhs[i] : A[i][j];
    mu[c] = (B[0][0] * (B[1][1] * B[2][2] - B[1][2] * B[2][1]) -
             B[0][1] * (B[1][0] * B[2][2] - B[1][2] * B[2][0]) +
             B[0][2] * (B[1][0] * B[2][1] - B[1][1] * B[2][0])) / det;
  }
  for (int c = 0; c < 3; ++c) {
    const int a = ca[c], b = cb[c];
    v[a].x += (float)(mu[c] * rc[c].x * iw[a]);
    v[a].y += (float)(mu[c] * rc[c].y * iw[a]);
    v[a].z += (float)(mu[c] * rc[c].z * iw[a]);
    v[b].x -= (float)(mu[c] * rc[c].x * iw[b]);
    v[b].y -= (float)(mu[c] * rc[c].y * iw[b]);
    v[b].z -= (float)(mu[c] * rc[c].z * iw[b]);
  }
  for (int k = 0; k < 3; ++k) {
    const int a = at[k];
    if (ENERGY) {
      const double v0x = vel[a], v0y = vel[n + a], v0z = vel[2 * n + a];
      dke += (double)mass[a] *
             (((double)v[k].x * v[k].x + (double)v[k].y * v[k].y + (double)v[k].z * v[k].z) -
              (v0x * v0x + v0y * v0y + v0z * v0z)) * inv_2acc;
    }
    vel[a] = v[k].x;
    vel[n + a] = v[k].y;
    vel[2 * n + a] = v[k].z;
  }
  }
  if (ENERGY) {
    const double sb = block_sum(dke, red);
    if (threadIdx.x == 0) partials[kRowKinRigid * pstride + blockIdx.x] = sb;
  }
}

hipError_t launch_rigid_positions(Ctx& c, const float* x_old, const float* y_in, float* pos,
                                  float* vel, float dt, const StepGates& g) {
  RigidArgs r{c.rigid_mols, c.n_rigid, {c.rigid_d[0], c.rigid_d[1], c.rigid_d[2]}, c.hdt_scale,
              c.rigid_settle ? 1 : 0};
  // 64-lane groups: one molecule per lane, and enough groups to reach every CU
  k_rigid_positions<<<(c.n_rigid + 63) / 64, 64, 0, c.stream>>>(r, make_open(c, pos, pos, dt, g),
                                                                x_old, y_in, pos, vel, c.inv_perm,
                                                                c.flags);
  return hipGetLastError();
}

hipError_t launch_rigid_velocities(Ctx& c, const float* pos, float* vel, bool energy,
                                   int* blocks) {
  RigidArgs r{c.rigid_mols, c.n_rigid, {c.rigid_d[0], c.rigid_d[1], c.rigid_d[2]}, c.hdt_scale,
              c.rigid_settle ? 1 : 0};
  const int nb = (c.n_rigid + 63) / 64;
  if (blocks) *blocks = nb;
  if (energy && nb > c.max_blocks) return hipErrorInvalidValue;   // partial rows too short
  const double inv_2acc = 0.5 / c.accel;
  if (energy)
    k_rigid_velocities<true><<<nb, 64, 0, c.stream>>>(r, c.cg, c.n, pos, vel, c.mass, inv_2acc,
                                                       c.partials, c.max_blocks, c.flags);
  else
    k_rigid_velocities<false><<<nb, 64, 0, c.stream>>>(r, c.cg, c.n, pos, vel, c.mass, inv_2acc,
                                                        c.partials, c.max_blocks, c.flags);
  return hipGetLastError();
}

hipError_t launch_begin_step(Ctx& c, float* pos, float* vel, const float* force, float dt,
                             const StepGates& g, float* pos_out) {
  k_begin_step<<<(c.max_slots + 255) / 256, 256, 0, c.stream>>>(make_open(c, pos, pos_out ? pos_out : pos, dt, g),
                                                                 force, vel, c.perm, c.meta);
  return hipGetLastError();
}

hipError_t launch_side_terms(Ctx& c, const float* pos, bool energy, hipStream_t s,
                             hipEvent_t done) {
  if (!c.fside || !side_terms_used(c)) return hipErrorInvalidValue;
  const int nb = xcd_grid((c.max_slots * kFinishLanes + 255) / 256);
  BondedParams bp = make_bonded_params(c);
  Topology tp = make_topology(c);
  PmeParams pp = make_pme_params(c);
  const int* perm = c.perm;
  const int* meta = c.meta;
  const float4* xs = c.xs;
  const float* phi = c.grid_phi;
  int n = c.n, fstride = c.max_slots, pstride = c.max_blocks;
  float* fside = c.fside;
  double* partials = c.partials;
  const void* fn = energy ? reinterpret_cast<const void*>(k_side_terms<true>)
                          : reinterpret_cast<const void*>(k_side_terms<false>);
  void* args[] = {&perm, &meta, &pos, &n, &bp, &tp, &xs, &phi, &pp, &fside, &fstride, &partials,
                  &pstride};
  if (done && !c.capturing)
    return hipExtLaunchKernel(fn, dim3(nb), dim3(256), args, 0, s, nullptr, done, 0);
  hipError_t e = hipLaunchKernel(fn, dim3(nb), dim3(256), args, 0, s);
  if (e == hipSuccess && done) e = hipEventRecord(done, s);
  return e;
}

hipError_t launch_finish_step(Ctx& c, const float* pos, float* vel, float* force, float dt,
                              bool energy, const StepGates* next, float* pos_next) {
  if (next && (!pos_next || pos_next == pos)) return hipErrorInvalidValue;
  // PME contexts from kSideStreamMinAtoms atoms on: the reciprocal-space,
  // bonded and exclusion forces come from the side kernel of the same step
  const bool side = side_terms_used(c);
  if (side && (!c.fside || !c.has_coulomb)) return hipErrorInvalidValue;
  const StepGates none{c.gate, c.gate, c.gate, c.gate, false, 0};   // not used when !next
  const OpenStep o = make_open(c, pos, pos_next, dt, next ? *next : none);
  const int open = next ? 1 : 0;
  const int nb = xcd_grid((c.max_slots * kFinishLanes + 255) / 256);
  const BondedParams bp = make_bonded_params(c);
  const Topology tp = make_topology(c);
  const double inv_2acc = 0.5 / c.accel;
  c.finish_blocks = nb;
  const PmeParams pp = c.has_pme ? make_pme_params(c) : PmeParams{};
#define MDX_FIN(E, C, P, S)                                                                    \
  k_finish_step<E, C, P, S><<<nb, 256, 0, c.stream>>>(c.xs, c.grid_phi, pp, c.perm, c.meta, pos, \
                                                       c.n, bp, tp, c.fslot, c.max_slots, force, \
                                                       vel, c.hdt_scale, c.mass, 0.5f * dt,      \
                                                       inv_2acc, c.partials, c.max_blocks, c.vc, \
                                                       o, open, c.jparts(), c.fside)
  const bool C = c.has_coulomb, P = c.has_pme;
  if (energy) {
    if (side) MDX_FIN(true, true, true, true);
    else if (C && P) MDX_FIN(true, true, true, false);
    else if (C) MDX_FIN(true, true, false, false);
    else MDX_FIN(true, false, false, false);
  } else {
    if (side) MDX_FIN(false, true, true, true);
    else if (C && P) MDX_FIN(false, true, true, false);
    else if (C) MDX_FIN(false, true, false, false);
    else MDX_FIN(false, false, false, false);
  }
#undef MDX_FIN
  return hipGetLastError();
}

}  // namespace mdx
