// Short-range forces (DIMOS Sec. II.A.1-2).
//
// k_pair: one wave per 4-atom i-cluster streams its list of 4x4 cluster
//   tiles four at a time: lane = (i slot, tile, j slot), i.e. the wave's four
//   16-lane rows each hold one i atom against 16 j atoms. Per pair: LJ
//   (Eqs. 4-5, type-pair table, optional Eq. 6 switch) + the minimum-image
//   real-space Ewald term (Eq. 10) for pairs whose mask bit is set and with
//   r2 < fl(r_c^2). A group of tiles with no such pair is skipped after the
//   distance test. Full list (default): every pair is listed from both
//   ends, the wave stores its i forces and nothing else, so the result is
//   bitwise reproducible. Half list: every pair is listed once and its force
//   acts on both atoms: the i force accumulates per lane over the whole
//   list, the j forces of a group are summed over the four rows with lane
//   swaps and added to the slot force array with one float atomic per lane
//   (x, y, z of the 16 j atoms on rows 0-2). Energies accumulate per lane in
//   FP64 in both modes.
// k_bonded_excl: one thread per caller atom for the terms that involve it:
//   the FP64 erf exclusion correction and FP32 harmonic bonds/angles (Eqs. 1-2);
//   it also moves the atom's pair force out of the slot array (clearing it).
//   Each term's energy is booked once, by a designated member atom.
// k_reduce_rows: fixed-order FP64 reduction of per-block partial sums.
#include "atom_terms.h"

#include <hip/hip_ext.h>

#include <type_traits>

namespace mdx {

// erfc(x) = exp(-x^2) R(x): R = t P(t), t = 1/(1 + 0.42 x), with P of degree 7
// fitted (weighted least squares on the relative error, iterated towards
// equal ripple; fit_erfc.py beside this file) to the scaled complementary
// error function exp(x^2) erfc(x) on [0, 6]: relative error below 4e-8 in
// exact arithmetic, about 3.5e-7 as evaluated in float32 (the rounding of t
// dominates). Here x = alpha r and the caller passes r and c = 0.42 alpha.
// The caller multiplies by exp(-x^2), which it needs for the force anyway.
__device__ __forceinline__ float erfc_scaled(float r, float c) {
  const float t = __builtin_amdgcn_rcpf(fmaf(c, r, 1.0f));
  float p = 7.619556785e-02f;
  p = fmaf(p, t, -3.458804786e-01f);
  p = fmaf(p, t, 4.864609241e-01f);
  p = fmaf(p, t, -1.745370179e-01f);
  p = fmaf(p, t, 2.932607532e-01f);
  p = fmaf(p, t, 1.868254989e-01f);
  p = fmaf(p, t, 2.409472317e-01f);
  p = fmaf(p, t, 2.367275357e-01f);
  return p * t;
}

struct PairParams {
  float L[3], hL[3];
  float rc2;
  float alpha;                // Ewald alpha
  float alpha_t;              // 0.42 alpha: erfc's t = 1/(1 + alpha_t r)
  float exp_c;                // -alpha^2 log2(e): exp(-alpha^2 r^2) = 2^(exp_c r^2)
  float two_a_sqrtpi;         // 2 alpha / sqrt(pi)
  float coulomb_k;
  float r_s, r_c, inv_sw;     // switch r_s, r_c and 1/(r_c - r_s)
  int ntypes;
  double alpha_d;             // alpha for the FP64 energy terms
  double coulomb_kd;          // k_e and 2 alpha / sqrt(pi) for the FP64 virial
  double two_a_sqrtpi_d;
  float two_k_rf;             // reaction field (Eq. 8): 2 k_RF
  double k_rf_d, c_rf_d;      // k_RF, c_RF for the FP64 energy and virial
};

// Coulomb term of the pair kernel: none, real-space Ewald (Eq. 10) or the
// reaction field (Eq. 8).
constexpr int kCoulNone = 0, kCoulEwald = 1, kCoulRF = 2;

// Energies of a pair on measurement steps: the float32 squared distance (and
// the switch value) is widened and the pair energy is evaluated in FP64 with
// FP64 constants, so the only rounding left is the unbiased float32 rounding
// of each pair's distance; k_e is applied in the final FP64 reduction. (The
// real-space Coulomb sum cancels strongly, so a float32 erfc bias of 1e-7
// would show up at the 1e-6 level in the total.)
// Sum over the four 16-lane rows at this lane's position in its row
// (lanes l, l^16, l^32, l^48), returned on every lane in one fixed order.
__device__ __forceinline__ float sum_rows4(float x) {
  const unsigned u = __float_as_uint(x);
  const auto h = __builtin_amdgcn_permlane32_swap(u, u, false, false);
  const float s = __uint_as_float(h[0]) + __uint_as_float(h[1]);
  const unsigned us = __float_as_uint(s);
  const auto r = __builtin_amdgcn_permlane16_swap(us, us, false, false);
  return __uint_as_float(r[0]) + __uint_as_float(r[1]);
}

// The pair kernel stages the LJ type-pair table in LDS (at most
// kMaxLjTypes^2 type pairs, 16 KB; mdx_create rejects more types).

// Dynamic pruning (an optimisation of the Verlet list's use, Sec. II.A.2):
// the tiles with a pair within r_p = r_c + 0.4 r_g at the emitting step are
// kept in a second list, used while every atom stays within 0.19 r_g of its
// position at that step; a pair it drops was farther than r_p apart, so it
// cannot come within r_c (0.8 r_g of closing) before the list is refreshed.
struct PruneArgs {
  const int* gate_now;    // rebuild flag of this step (null: stand-alone call)
  const int* pgate_now;   // pruned list no longer valid (set by k_begin_step)
  uint2* ptiles;          // [max_clusters][cap]
  int* pcount;            // [max_clusters]
  float4* xp;             // [max_slots] positions at the emitting step
  float rp2;              // fl(r_p^2)
  // half list, stand-alone call: the in-step pruned-list flags of both step
  // parities, raised so that the next step walks the full list (this call
  // writes every tile's j partials for its own positions)
  int* invalidate;
};

// Half list (each pair once, Newton's third law): the wave of cluster ic
// stores its atoms' forces as with the full list, and the forces on each
// tile's j atoms, summed over the tile's four i atoms, go to jpart at the
// tile's position in the full list: [tile][component][j slot]. Every real
// tile of the list a step walks writes its entry, zero if no pair
// interacted; a tile the pruned list drops had no pair within r_p when it
// was dropped (that step walked the full list and wrote zeros for it), and
// has none within r_c while the pruned list is in use. The closing kernel
// adds, to each atom, the entries of the tiles whose j-cluster holds it, in
// the order of in_sorted: the tile search appends them to in_fill in any
// order, and on a build step (or a stand-alone call) the wave of each
// cluster sorts its own entries by full-list position. No float atomics:
// the forces do not depend on scheduling.
struct HalfArgs {
  float* jpart;          // [max_clusters * cap][3][4]
  int* ppos;             // [max_clusters][cap] pruned tile -> full-list position
  const int* in_count;   // [max_clusters]
  const int* in_fill;    // [max_clusters][cap]
  int* in_sorted;        // [max_clusters][cap]
};

// tiles whose keep flags a wave holds before writing them out (a power of two)
constexpr int kKeepTiles = 256;

template <bool ENERGY, int COUL, bool SWITCH, bool HALF, bool VIR = false>
__global__ void __launch_bounds__(256) k_pair(const float4* __restrict__ xs,
                                              const int* __restrict__ ts,
                                              const uint2* __restrict__ tiles,
                                              const int* __restrict__ tile_count,
                                              const int* __restrict__ meta, int cap,
                                              PairParams pp, const float4* __restrict__ lj_f,
                                              const double2* __restrict__ lj_d,
                                              float* __restrict__ fslot, int fstride,
                                              double* __restrict__ partials, int pstride,
                                              PruneArgs pr, HalfArgs ha) {
  __shared__ double red[16];
  // LJ type-pair table, ntypes^2 entries (dynamic: the concurrent PME
  // kernels keep the rest of the CU's LDS)
  extern __shared__ float4 lj_s[];
  // Reserve 80 VGPRs (the clobber marks v79 as used): at most 6 of the 8
  // wave slots per SIMD go to this kernel, and the PME FFT passes that run
  // concurrently on the second stream always find room on every CU. The
  // pair kernel is VALU-bound and loses little at 6 waves per SIMD.
  asm volatile("" ::: "v79");
  for (int t = threadIdx.x; t < pp.ntypes * pp.ntypes; t += blockDim.x) lj_s[t] = lj_f[t];
  // periodic image shifts by tile image code (2 bits per axis): x_j offset
  // am (-L for image 1) and cp (L for image 2), see image_diff
  __shared__ float4 img_am[64], img_cp[64];
  // per wave, on a walk that writes the pruned list: the keep flags of the
  // last kKeepTiles tiles, one byte per group of four
  __shared__ unsigned char keep_s[4][kKeepTiles / 4];
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
  // the wave index is the same on every lane: read it as such, so that the
  // cluster and its list rows are addressed from scalar registers
  const int w = __builtin_amdgcn_readfirstlane(threadIdx.x / kWave);
  const int lane = threadIdx.x & (kWave - 1);
  // neighbouring clusters on one XCD: their j clusters come from one region
  const int lb = xcd_block((meta[1] + 3) / 4);
  const int ic = lb * 4 + w;
  const bool active = lb >= 0 && ic < meta[1];
  if (HALF && pr.invalidate && blockIdx.x == 0 && threadIdx.x < 2) pr.invalidate[threadIdx.x] = 1;
  const int ia = lane >> 4, tt = (lane >> 2) & 3, jb = lane & 3;
  const int si = ic * kClusterSize + ia;
  const unsigned bitpos = (unsigned)(ia * kClusterSize + jb);
  float fx = 0.f, fy = 0.f, fz = 0.f;
  double e_lj = 0.0, e_c = 0.0;
  double wv[6] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0};   // virial (VIR)
  if (active) {
    const float4 pi = xs[si];
    const float qik = pp.coulomb_k * pi.w;   // k_e q_i, per lane
    const int trow = ts[si] * pp.ntypes;
    // List selection (the flags are the same for the whole grid): the full
    // list, emitting the pruned list and the prune positions, on a rebuild
    // step or when an atom has moved too far since the last emission; the
    // pruned list otherwise. Without flags (stand-alone force calls) the full
    // list, nothing emitted.
    const bool emit = __builtin_amdgcn_readfirstlane(
                          pr.gate_now && (*pr.gate_now != 0 || *pr.pgate_now != 0)) != 0;
    const bool pruned = pr.gate_now && !emit;
    const int cnt = pruned ? pr.pcount[ic] : tile_count[ic];
    const uint2* tl = (pruned ? pr.ptiles : tiles) + (size_t)ic * cap;
    uint2* const pl = pr.ptiles + (size_t)ic * cap;
    int pn = 0;
    // half list: full-list positions of the pruned tiles; this lane's j
    // partial (component ia of j slot jb) of the tile at full position f is
    // jpart[((ic * cap + f) * 3 + ia) * 4 + jb]
    int* const ppl = HALF ? ha.ppos + (size_t)ic * cap : nullptr;
    float* const jrow = HALF ? ha.jpart + (size_t)ic * cap * 12 + (ia < 3 ? ia : 0) * 4 + jb
                             : nullptr;
    // One group of four tiles (e: this lane's tile, sj / pj / tj: its j slot,
    // position and type; f: the tile's full-list position). EMIT (whether
    // this walk writes the pruned list) is a compile-time constant of each
    // of the two loops below.
    auto group = [&](auto emit_c, int g0, uint2 e, unsigned sj, float4 pj, int tj, int f) {
      constexpr bool EMIT = decltype(emit_c)::value;
      const bool on = (e.y >> bitpos) & 1u;
      // the tile's image: the same differences as the minimum-image rule
      // gives for its listed pairs, without the per-pair selects; when no
      // tile of the group wraps (the common case; the test is the same for
      // the whole wave) that is the plain difference
      const unsigned code = e.y >> 16;
      float dx, dy, dz;
      if (__builtin_amdgcn_ballot_w64(code != 0u) == 0ull) {
        dx = plain_diff(pi.x, pj.x);
        dy = plain_diff(pi.y, pj.y);
        dz = plain_diff(pi.z, pj.z);
      } else {
        const float4 am = img_am[code], cp = img_cp[code];
        dx = image_diff(pi.x, pj.x, am.x, cp.x);
        dy = image_diff(pi.y, pj.y, am.y, cp.y);
        dz = image_diff(pi.z, pj.z, am.z, cp.z);
      }
      float r2 = dist2(dx, dy, dz);
      const bool in = on && r2 < pp.rc2;
      if (EMIT) {
        // tile t of the group is kept if any of its pairs (lanes 16 a + 4 t
        // + b) is within r_p: four flags from one ballot (scalar work),
        // stored as the group's byte; the kept tiles are written out in list
        // order by compact()
        // (ballots of single compares, combined as masks; the folding is
        // integer work on the wave-uniform mask)
        unsigned long long m =
            __builtin_amdgcn_ballot_w64(on) & __builtin_amdgcn_ballot_w64(r2 < pr.rp2);
        m |= m >> 32;
        m |= m >> 16;                          // bit 4 t + b: any row
        unsigned x = (unsigned)m & 0xffffu;
        x |= x >> 2;
        x |= x >> 1;                           // bit 4 t: any pair of tile t
        const unsigned nib = (x & 1u) | ((x >> 3) & 2u) | ((x >> 6) & 4u) | ((x >> 9) & 8u);
        if (lane == 0) keep_s[w][(g0 >> 2) & (kKeepTiles / 4 - 1)] = (unsigned char)nib;
      }
      const unsigned long long hit = __builtin_amdgcn_ballot_w64(in);
      // half list: every real tile (mask != 0) writes its j partials
      const bool jw = HALF && ia < 3 && (e.y & 0xffffu) != 0u;
      if (hit == 0ull) {
        if (jw) jrow[(size_t)f * 12] = 0.f;
        return;
      }
      // Every lane evaluates the pair terms (the branch above is the same for
      // the whole wave, so no lane's registers need to be kept aside), and a
      // lane without a pair within r_c takes a zero factor: its operands may
      // be infinite or NaN (r2 = 0 on the diagonal), the select drops them.
      float gx, gy, gz;   // force on j (minus the force on i)
      {
        const int tp = trow + tj;
        const float4 lj = lj_s[tp];       // c12, c6, 12 c12, 6 c6
        // r2 of a pair within r_c is never denormal
        const float rinv = __builtin_amdgcn_rsqf(r2);
        const float rinv2 = rinv * rinv;
        const float r = r2 * rinv;
        float r6 = rinv2 * rinv2 * rinv2;
        // F/r is assembled as (F/r) r^2 and multiplied by 1/r^2 once
        float fr2 = r6 * (lj.z * r6 - lj.w);   // LJ
        float S = 1.f, dS = 0.f;
        if (SWITCH) {
          if (r > pp.r_s) {
            float x = (r - pp.r_s) * pp.inv_sw;
            float x2 = x * x, x3 = x2 * x;
            S = 1.0f + x3 * (-10.0f + x * (15.0f - 6.0f * x));
            dS = x2 * (-30.0f + x * (60.0f - 30.0f * x)) * pp.inv_sw;
            float u_lj = r6 * (lj.x * r6 - lj.y);
            fr2 = fr2 * S - u_lj * dS * r;
          }
        }
        const float qq = qik * pj.w;
        if (COUL == kCoulEwald) {
          // k q_i q_j exp(-alpha^2 r^2) (R(alpha r) / r + 2 alpha / sqrt(pi)),
          // with exp(-alpha^2 r^2) as 2^(exp_c r^2) on the transcendental
          // unit; the energies on measurement steps are evaluated separately
          // in FP64
          const float ex = __builtin_amdgcn_exp2f(pp.exp_c * r2);
          const float w = fmaf(erfc_scaled(r, pp.alpha_t), rinv, pp.two_a_sqrtpi);
          fr2 = fmaf(qq, ex * w, fr2);
        }
        if (COUL == kCoulRF) fr2 = fmaf(qq, fmaf(-pp.two_k_rf, r2, rinv), fr2);
        const float f_over_r = in ? fr2 * rinv2 : 0.f;
        gx = f_over_r * dx;
        gy = f_over_r * dy;
        gz = f_over_r * dz;
        fx -= gx;
        fy -= gy;
        fz -= gz;
        if (ENERGY && in) {
          double2 c = lj_d[tp];
          double r2d = (double)r2;
          double r6d = 1.0 / (r2d * r2d * r2d);
          double u = r6d * (c.x * r6d - c.y);
          if (SWITCH) u *= (double)S;
          e_lj += u;
          if (COUL == kCoulEwald) {
            double rd = sqrt(r2d);
            e_c += (double)pi.w * (double)pj.w * erfc(pp.alpha_d * rd) / rd;
          }
          if (COUL == kCoulRF) {
            double rd = sqrt(r2d);
            e_c += (double)pi.w * (double)pj.w * (1.0 / rd + pp.k_rf_d * r2d - pp.c_rf_d);
          }
          if (VIR) {
            // d (x) F_j with F_j = fr d, fr = -(dU/dr)/r in FP64 from the
            // widened float32 distance
            const double rd = sqrt(r2d);
            double fr = (12.0 * c.x * r6d - 6.0 * c.y) * r6d / r2d;
            if (SWITCH) fr = fr * (double)S - r6d * (c.x * r6d - c.y) * (double)dS / rd;
            if (COUL == kCoulEwald) {
              const double ar = pp.alpha_d * rd;
              fr += pp.coulomb_kd * (double)pi.w * (double)pj.w *
                    (erfc(ar) / rd + pp.two_a_sqrtpi_d * exp(-ar * ar)) / r2d;
            }
            if (COUL == kCoulRF)
              fr += pp.coulomb_kd * (double)pi.w * (double)pj.w *
                    (1.0 / (r2d * rd) - 2.0 * pp.k_rf_d);
            vir_add_dd(wv, fr, (double)dx, (double)dy, (double)dz);
          }
        }
      }
      if (HALF) {
        gx = sum_rows4(gx);
        gy = sum_rows4(gy);
        gz = sum_rows4(gz);
        if (jw) jrow[(size_t)f * 12] = ia == 0 ? gx : (ia == 1 ? gy : gz);
      }
    };
    // Software pipeline, two groups per iteration with fixed registers: while
    // group g is computed the j atoms of group g + 4 are in flight, and the
    // tiles of the groups after that. Lists are padded to groups of four
    // (padding tiles point at cluster 0); reads past the list are clamped
    // into its allocation and their cluster index is replaced by 0 before it
    // is used as an address. (Unsigned 32-bit indices let the loads use a
    // scalar base + 32-bit offset.)
    auto tile_at = [&](int g) {
      return *reinterpret_cast<const uint2*>(reinterpret_cast<const char*>(tl) +
                                             ((unsigned)min(g + tt, cap - 1) << 3));
    };
    // 32-bit byte offsets from the arrays' bases (the slot arrays are far
    // below 4 GB)
    auto pos_at = [&](unsigned s) {
      return *reinterpret_cast<const float4*>(reinterpret_cast<const char*>(xs) + (s << 4));
    };
    auto type_at = [&](unsigned s) {
      return *reinterpret_cast<const int*>(reinterpret_cast<const char*>(ts) + (s << 2));
    };
    // full-list position of this lane's tile of group g (half list)
    auto full_at = [&](int g) {
      if (!HALF) return 0;
      const int k = min(g + tt, cap - 1);
      return pruned ? ppl[k] : k;
    };
    // Writing the pruned list: the tiles [c0, c1) of the full list (c0 a
    // multiple of kKeepTiles) whose flags the walk has stored, appended in
    // list order, one wave instruction per 64 tiles.
    auto compact = [&](int c0, int c1) {
      __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
      __builtin_amdgcn_wave_barrier();
      __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
      for (int t0 = c0; t0 < c1; t0 += kWave) {
        const int t = t0 + lane;
        const bool k =
            t < c1 && ((keep_s[w][(t >> 2) & (kKeepTiles / 4 - 1)] >> (t & 3)) & 1u) != 0u;
        const unsigned long long km = __builtin_amdgcn_ballot_w64(k);
        if (k) {
          const int pos = pn + __popcll(km & ((1ull << lane) - 1ull));
          pl[pos] = tl[t];
          if (HALF) ppl[pos] = t;
        }
        pn += __popcll(km);
      }
      __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
      __builtin_amdgcn_wave_barrier();
      __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    };
    auto walk = [&](auto emit_c) {
      constexpr bool EMIT = decltype(emit_c)::value;
      // A walk that writes the pruned list takes the list in chunks of
      // kKeepTiles tiles and writes out each chunk's kept tiles after it:
      // the group loop itself then holds no other memory operations, and its
      // loads stay in flight across groups (with the writes inside the loop
      // every group waited for all of them).
      const int chunk = EMIT ? kKeepTiles : (cnt > 0 ? cnt : 1);
      for (int c0 = 0; c0 < cnt; c0 += chunk) {
        const int c1 = min(c0 + chunk, cnt);
        auto slot = [&](uint2 e, int g) {
          return (g < c1 ? e.x : 0u) * kClusterSize + (unsigned)jb;
        };
        uint2 eA = tile_at(c0), eB = tile_at(c0 + 4);
        uint2 eA2 = tile_at(c0 + 8), eB2 = tile_at(c0 + 12);
        int fA = full_at(c0), fB = full_at(c0 + 4);
        int fA2 = full_at(c0 + 8), fB2 = full_at(c0 + 12);
        unsigned sA = slot(eA, c0), sB = slot(eB, c0 + 4);
        float4 pA = pos_at(sA), pB = pos_at(sB);
        int tA = type_at(sA), tB = type_at(sB);
        for (int g = c0; g < c1; g += 8) {
          group(emit_c, g, eA, sA, pA, tA, fA);
          eA = eA2;
          fA = fA2;
          eA2 = tile_at(g + 16);
          fA2 = full_at(g + 16);
          sA = slot(eA, g + 8);
          pA = pos_at(sA);
          tA = type_at(sA);
          if (g + 4 < c1) group(emit_c, g + 4, eB, sB, pB, tB, fB);
          eB = eB2;
          fB = fB2;
          eB2 = tile_at(g + 20);
          fB2 = full_at(g + 20);
          sB = slot(eB, g + 12);
          pB = pos_at(sB);
          tB = type_at(sB);
        }
        if (EMIT) compact(c0, c1);
      }
    };
    if (emit) walk(std::true_type{});
    else walk(std::false_type{});
    if (emit) {
      // pad the pruned list to a whole group; record the prune positions
      const int padded = (pn + 3) & ~3;
      if (lane < padded - pn) pl[pn + lane] = make_uint2(0u, 0u);
      if (lane == 0) pr.pcount[ic] = padded;
      if ((lane & 15) == 0) pr.xp[si] = pi;
    }
    // half list, on a build step or a stand-alone call: this cluster's
    // incoming tiles in full-list order (rank of each distinct position)
    if (HALF && (!pr.gate_now || *pr.gate_now != 0)) {
      const int nin = min(ha.in_count[ic], cap);
      const int* src = ha.in_fill + (size_t)ic * cap;
      for (int k = lane; k < nin; k += kWave) {
        const int key = src[k];
        int rank = 0;
        for (int m = 0; m < nin; ++m) rank += src[m] < key ? 1 : 0;
        ha.in_sorted[(size_t)ic * cap + rank] = key;
      }
    }
  }
  // sum the i force over the 16 lanes of the row; lanes 0-2 of the row
  // store its x, y, z (the wave owns the slot)
  for (int o = 8; o >= 1; o >>= 1) {
    fx += __shfl_xor(fx, o, kWave);
    fy += __shfl_xor(fy, o, kWave);
    fz += __shfl_xor(fz, o, kWave);
  }
  const int c3 = lane & 15;
  if (active && c3 < 3) {
    const float v = c3 == 0 ? fx : (c3 == 1 ? fy : fz);
    fslot[(size_t)c3 * fstride + si] = v;
  }
  if (ENERGY) {
    // a full list visits every pair from both ends
    if (!HALF) {
      e_lj *= 0.5;
      e_c *= 0.5;
      for (int k = 0; k < 6; ++k) wv[k] *= 0.5;
    }
    double s_lj = block_sum(e_lj, red);
    double s_c = block_sum(e_c, red);
    if (threadIdx.x == 0) {
      partials[kRowLJ * pstride + blockIdx.x] = s_lj;
      partials[kRowDir * pstride + blockIdx.x] = s_c;
    }
    if (VIR) {
      for (int k = 0; k < 6; ++k) {
        const double sk = block_sum(wv[k], red);
        if (threadIdx.x == 0) partials[(kRowVir + k) * pstride + blockIdx.x] = sk;
      }
    }
  }
}

template <bool ENERGY, bool COUL, bool VIR>
__global__ void __launch_bounds__(256) k_bonded_excl(const float* __restrict__ pos, int n,
                                                     BondedParams bp, Topology tp,
                                                     const int* __restrict__ inv_perm,
                                                     float* __restrict__ fslot, int fstride,
                                                     float* __restrict__ force,
                                                     double* __restrict__ partials,
                                                     int pstride, JParts jp) {
  __shared__ double red[16];
  int a = blockIdx.x * blockDim.x + threadIdx.x;
  double e_ex = 0.0, e_b = 0.0, e_a = 0.0;
  double w[6] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
  if (a < n) {
    const int s = inv_perm[a];   // -1: an atom a full column left out of the list
    float fx = 0.f, fy = 0.f, fz = 0.f;
    if (s >= 0) {
      fx = fslot[s];
      fy = fslot[fstride + s];
      fz = fslot[2 * fstride + s];
      fslot[s] = 0.f;
      fslot[fstride + s] = 0.f;
      fslot[2 * fstride + s] = 0.f;
      if (jp.jpart) add_jparts(jp, s, 0, 1, fx, fy, fz);
    }
    bonded_excl_atom<ENERGY, COUL, VIR>(a, pos, n, bp, tp, fx, fy, fz, e_ex, e_b, e_a, 0, 1, w);
    force[a] = fx;
    force[n + a] = fy;
    force[2 * n + a] = fz;
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
  if (VIR) {
    for (int k = 0; k < 6; ++k) {
      const double sk = block_sum(w[k], red);
      if (threadIdx.x == 0) partials[(kRowVirB + k) * pstride + blockIdx.x] = sk;
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
  int kin_extra_blocks;   // > 0: the kinetic row also sums kRowKinRigid over these blocks
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
    if (spec.row[r] == kRowKin && spec.kin_extra_blocks > 0) {
      const double* pr = partials + (size_t)kRowKinRigid * pstride;
      for (int k = threadIdx.x; k < spec.kin_extra_blocks; k += blockDim.x) v += pr[k];
    }
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

hipError_t launch_nonbonded(Ctx& c, bool energy, const int* gate_now, const int* pgate_now,
                            bool virial, hipEvent_t t_start, hipEvent_t t_stop) {
  PairParams pp;
  for (int d = 0; d < 3; ++d) {
    pp.L[d] = c.cg.L[d];
    pp.hL[d] = c.cg.hL[d];
  }
  pp.rc2 = c.cg.rc2;
  pp.alpha = (float)c.alpha;
  pp.alpha_t = (float)(0.42 * c.alpha);
  pp.exp_c = (float)(-c.alpha * c.alpha / M_LN2);
  pp.alpha_d = c.alpha;
  pp.coulomb_kd = c.coulomb_k;
  pp.two_a_sqrtpi_d = 2.0 * c.alpha / sqrt(M_PI);
  pp.ntypes = c.n_types;
  pp.two_a_sqrtpi = (float)(2.0 * c.alpha / sqrt(M_PI));
  pp.coulomb_k = (float)c.coulomb_k;
  pp.r_s = c.switch_r;
  pp.r_c = c.r_cut;
  pp.inv_sw = c.has_switch ? 1.0f / (c.r_cut - c.switch_r) : 0.f;
  pp.two_k_rf = (float)(2.0 * c.k_rf);
  pp.k_rf_d = c.k_rf;
  pp.c_rf_d = c.c_rf;
  const int nb = xcd_grid((c.max_clusters + 3) / 4);
  c.nb_blocks = nb;
  const size_t lds = sizeof(float4) * (size_t)c.n_types * c.n_types;
  const PruneArgs pr{gate_now, pgate_now, c.ptiles, c.pcount, c.xp, c.prune_r2,
                     c.half_list && !gate_now ? c.gate + 2 : nullptr};
  const HalfArgs ha{c.jpart, c.ppos, c.in_count, c.in_fill, c.in_sorted};
  // the timing events (optional) are recorded by the dispatch itself: no
  // marker packets around the kernel
#define MDX_PAIR(E, C, S, H, V)                                                              \
  do {                                                                                        \
  if (t_start || t_stop)                                                                      \
    hipExtLaunchKernelGGL(k_pair<E, C, S, H, V>, dim3(nb), dim3(256), lds, c.stream, t_start, \
                          t_stop, 0u, static_cast<const float4*>(c.xs),                       \
                          static_cast<const int*>(c.ts), static_cast<const uint2*>(c.tiles),  \
                          static_cast<const int*>(c.tile_count),                              \
                          static_cast<const int*>(c.meta), c.nl_cap, pp,                      \
                          static_cast<const float4*>(c.lj_f),                                 \
                          static_cast<const double2*>(c.lj_d), c.fslot, c.max_slots,          \
                          c.partials, c.max_blocks, pr, ha);                                  \
  else                                                                                        \
    k_pair<E, C, S, H, V><<<nb, 256, lds, c.stream>>>(c.xs, c.ts, c.tiles, c.tile_count, c.meta, \
                                                      c.nl_cap, pp, c.lj_f, c.lj_d, c.fslot,  \
                                                      c.max_slots, c.partials, c.max_blocks, pr, \
                                                      ha);                                    \
  } while (0)
#define MDX_PAIR_H(E, C, S)             \
  if (c.half_list)                      \
    MDX_PAIR(E, C, S, true, false);     \
  else                                  \
    MDX_PAIR(E, C, S, false, false)
#define MDX_PAIR_V(C, S)                \
  if (c.half_list)                      \
    MDX_PAIR(true, C, S, true, true);   \
  else                                  \
    MDX_PAIR(true, C, S, false, true)
#define MDX_PAIR_VE(E, C, S) MDX_PAIR_V(C, S)
#define MDX_PAIR_S(M, E, C) \
  if (S) {                  \
    M(E, C, true);          \
  } else {                  \
    M(E, C, false);         \
  }
#define MDX_PAIR_C(M, E)                \
  if (C == kCoulEwald) {                \
    MDX_PAIR_S(M, E, kCoulEwald)        \
  } else if (C == kCoulRF) {            \
    MDX_PAIR_S(M, E, kCoulRF)           \
  } else {                              \
    MDX_PAIR_S(M, E, kCoulNone)         \
  }
  const int C = c.has_coulomb ? kCoulEwald : (c.rf ? kCoulRF : kCoulNone);
  const bool S = c.has_switch;
  if (virial) {
    MDX_PAIR_C(MDX_PAIR_VE, true)
  } else if (energy) {
    MDX_PAIR_C(MDX_PAIR_H, true)
  } else {
    MDX_PAIR_C(MDX_PAIR_H, false)
  }
#undef MDX_PAIR_C
#undef MDX_PAIR_S
#undef MDX_PAIR_VE
#undef MDX_PAIR_V
#undef MDX_PAIR_H
#undef MDX_PAIR
  return hipGetLastError();
}

BondedParams make_bonded_params(const Ctx& c) {
  BondedParams bp;
  for (int d = 0; d < 3; ++d) {
    bp.L[d] = c.cg.L[d];
    bp.hL[d] = c.cg.hL[d];
    bp.Ld[d] = (double)c.cg.L[d];
  }
  bp.alpha = c.alpha;
  bp.two_a_sqrtpi = 2.0 * c.alpha / sqrt(M_PI);
  bp.coulomb_k = c.coulomb_k;
  return bp;
}

Topology make_topology(const Ctx& c) {
  return Topology{c.q,      c.ex_start, c.ex_idx,  c.bonds,  c.bond_k,   c.bond_r0, c.bt_start,
                  c.bt_idx, c.angles,   c.angle_k, c.angle_t0, c.at_start, c.at_idx};
}

hipError_t launch_bonded_excl(Ctx& c, const float* pos, float* force, bool energy, bool virial) {
  const BondedParams bp = make_bonded_params(c);
  const Topology tp = make_topology(c);
  const int nb = (c.n + 255) / 256;
  hipStream_t s = c.stream;
  const bool C = c.has_coulomb;
#define MDX_BX(E, C, V)                                                                       \
  k_bonded_excl<E, C, V><<<nb, 256, 0, s>>>(pos, c.n, bp, tp, c.inv_perm, c.fslot, c.max_slots, \
                                            force, c.partials, c.max_blocks, c.jparts())
  if (virial) {
    if (C) MDX_BX(true, true, true);
    else MDX_BX(true, false, true);
  } else if (energy) {
    if (C) MDX_BX(true, true, false);
    else MDX_BX(true, false, false);
  } else {
    if (C) MDX_BX(false, true, false);
    else MDX_BX(false, false, false);
  }
#undef MDX_BX
  return hipGetLastError();
}

// One block per virial component: fixed-order sums over the sources' rows.
struct VirialSpec {
  int nsrc;
  int row0[2];
  int nblk[2];
  double scale[2];
};

__global__ void __launch_bounds__(256) k_reduce_virial(const double* __restrict__ partials,
                                                       int pstride, VirialSpec spec,
                                                       double* __restrict__ out,
                                                       unsigned* __restrict__ flags) {
  __shared__ double red[16];
  const int k = blockIdx.x;   // xx, yy, zz, xy, xz, yz
  double total = 0.0;
  for (int src = 0; src < spec.nsrc; ++src) {
    const double* p = partials + (size_t)(spec.row0[src] + k) * pstride;
    double v = 0.0;
    for (int b = threadIdx.x; b < spec.nblk[src]; b += blockDim.x) v += p[b];
    total += block_sum(v, red) * spec.scale[src];
  }
  if (threadIdx.x == 0) {
    const int ij[6][2] = {{0, 0}, {1, 1}, {2, 2}, {0, 1}, {0, 2}, {1, 2}};
    out[3 * ij[k][0] + ij[k][1]] = total;
    out[3 * ij[k][1] + ij[k][0]] = total;
    if (!isfinite(total)) atomicOr(flags, MDX_FLAG_NONFINITE);
  }
}

hipError_t launch_reduce_virial(Ctx& c, const int* row0, const int* nblk, const double* scale,
                                int nsrc, double* out) {
  if (nsrc < 1 || nsrc > 2) return hipErrorInvalidValue;
  VirialSpec spec{};
  spec.nsrc = nsrc;
  for (int s = 0; s < nsrc; ++s) {
    spec.row0[s] = row0[s];
    spec.nblk[s] = nblk[s];
    spec.scale[s] = scale[s];
  }
  k_reduce_virial<<<6, 256, 0, c.stream>>>(c.partials, c.max_blocks, spec, out, c.flags);
  return hipGetLastError();
}

hipError_t launch_reduce_energy(Ctx& c, const int* rows, const int* nblk, int nrows, double* out,
                                int slot_base, double const_val, int const_slot, int zero_slot,
                                int rigid_blocks) {
  ReduceSpec spec{};
  spec.kin_extra_blocks = rigid_blocks;
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
