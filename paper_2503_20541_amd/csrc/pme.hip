// Smooth particle-mesh Ewald (DIMOS Sec. II.A.2, PME paragraph).
//
//  k_pme_spread   one workgroup per grid brick; candidate atoms come from the
//                 column sort: columns within spline reach + r_g/2 of the
//                 brick, and in each the slots whose build z is in reach
//                 (ranges found by binary search once per list build).
//                 Grids of 11 or more points per axis: k_pme_spread_lines,
//                 every lane owns one z-line of the brick in registers and
//                 the wave walks the atoms whose stencil meets the brick
//                 (no atomics). Smaller grids and the dipole grid of the
//                 adjoint: each lane takes one atom and adds its stencil
//                 values inside the brick into its wave's own LDS copy of
//                 the brick. Either way the copies are summed in a fixed
//                 order (no global atomics).
//  k_fft_rows_*   x-direction real<->half-complex transforms, P rows per block
//  k_fft_cols     y (forward / inverse) and z (forward, influence multiply
//                 with the FP64 energy partial, inverse) pencils
//  k_pme_gather   one thread per atom: F = -k_e q sum grad(theta) phi
//
// The 1D transforms are radix-2/3/4/5/7 Stockham FFTs in LDS with a twiddle
// table exp(-2 pi i k/N) computed on the host in double precision.
#include "atom_terms.h"

#include <hip/hip_ext.h>

namespace mdx {

struct FftPlan {
  int N;
  int nst;
  int radix[16];
};

constexpr int kSpreadThreads = 256;
constexpr int kSpreadWaves = kSpreadThreads / kWave;
// B_z planes of B_x * B_y + 2 points (padded, see below)
constexpr int kMaxBrick = kBrickZ * (kBrickXY * kBrickXY + 2);
constexpr int kMaxCandCells = 512;
constexpr int kCandList = 2048;      // candidate slots a brick lists in LDS

// The LDS brick copies store point (lx, ly, lz) at lx + B_x ly + (B_x B_y + 2) lz
// (the padding spreads the planes over the banks).
__device__ __forceinline__ int brick_index(int lx, int ly, int lz, const PmeParams& pp) {
  return (lz * pp.B[1] + ly) * pp.B[0] + 2 * lz + lx;
}

// Candidate f of a brick: slot index from the LDS list, or (for bricks with
// more candidates than the list holds) by binary search over the segment
// offsets.
__device__ __forceinline__ int spread_candidate(int f, int total, int ncand,
                                                const int* cand_list, const int* cand_start,
                                                const int* cand_off) {
  if (total <= kCandList) return cand_list[f];
  int lo = 0, hi = ncand - 1;             // last segment with cand_off <= f
  while (lo < hi) {
    int mid = (lo + hi + 1) >> 1;
    if (cand_off[mid] <= f) lo = mid; else hi = mid - 1;
  }
  return cand_start[lo] + (f - cand_off[lo]);
}

// One workgroup per brick. Each lane takes one candidate atom, computes its
// B-spline weights in registers and adds its (up to) 64 stencil values that
// fall inside the brick into its wave's private LDS copy of the brick; the
// copies are summed in a fixed order. No global atomics, and the result does
// not depend on scheduling.
//
// DIPOLE: the tangent of the charge grid along per-slot displacements u
// (us[slot].xyz): each atom adds q u . grad(theta) instead of q theta, the
// grid the Hessian-vector product of the reciprocal force convolves.
template <bool DIPOLE>
__global__ void __launch_bounds__(kSpreadThreads) k_pme_spread(
    const float4* __restrict__ xs, const int4* __restrict__ brick_zr,
    const int* __restrict__ brick_cols, PmeParams pp, CellGrid cg,
    float* __restrict__ grid_q, const float4* __restrict__ us) {
  __shared__ float lgrid[kSpreadWaves][kMaxBrick];
  __shared__ int cand_start[kMaxCandCells];
  __shared__ int cand_off[kMaxCandCells + 1];
  __shared__ int cand_list[kCandList];

  const int brick = blockIdx.x;
  const int bx = brick % pp.nb[0], by = (brick / pp.nb[0]) % pp.nb[1],
            bz = brick / (pp.nb[0] * pp.nb[1]);
  const int g0x = bx * pp.B[0], g0y = by * pp.B[1], g0z = bz * pp.B[2];
  const int bex = min(pp.B[0], pp.K[0] - g0x), bey = min(pp.B[1], pp.K[1] - g0y),
            bez = min(pp.B[2], pp.K[2] - g0z);
  // candidate columns (first, count along x and y); the slot ranges inside
  // each column that reach this brick layer come from the list build
  const int* bcx = brick_cols + 2 * bx;
  const int* bcy = brick_cols + 2 * pp.nb[0] + 2 * by;
  const int ncx = bcx[1], ncy = bcy[1];
  const int ncol = ncx * ncy;
  const int ncand = 2 * ncol;    // up to two z segments per column (periodic wrap)
  const int w = threadIdx.x / kWave, lane = threadIdx.x & (kWave - 1);

  for (int t = threadIdx.x; t < kSpreadWaves * kMaxBrick; t += blockDim.x)
    (&lgrid[0][0])[t] = 0.f;
  const int4* zr = brick_zr + (size_t)bz * cg.ncell;
  for (int t = threadIdx.x; t < ncol; t += blockDim.x) {
    int cx = (bcx[0] + t % ncx) % cg.n[0], cy = (bcy[0] + t / ncx) % cg.n[1];
    const int4 r = zr[cy * cg.n[0] + cx];
    cand_start[2 * t] = r.x;
    cand_off[2 * t + 1] = r.y;
    cand_start[2 * t + 1] = r.z;
    cand_off[2 * t + 2] = r.w;
  }
  __syncthreads();
  if (w == 0) {   // inclusive scan of the segment sizes by the first wave
    int carry = 0;
    for (int base = 0; base < ncand; base += kWave) {
      const int i = base + lane;
      int v = i < ncand ? cand_off[i + 1] : 0;
      for (int o = 1; o < kWave; o <<= 1) {
        const int u = __shfl_up(v, o, kWave);
        if (lane >= o) v += u;
      }
      if (i < ncand) cand_off[i + 1] = carry + v;
      carry += __shfl(v, kWave - 1, kWave);
    }
    if (lane == 0) cand_off[0] = 0;
  }
  __syncthreads();
  const int total = cand_off[ncand];
  if (total <= kCandList) {
    for (int t = threadIdx.x; t < ncand; t += blockDim.x) {
      const int b = cand_off[t], e = cand_off[t + 1], s0 = cand_start[t];
      for (int k = b; k < e; ++k) cand_list[k] = s0 + (k - b);
    }
    __syncthreads();
  }
  float* my_grid = lgrid[w];
  const int plane = pp.B[0] * pp.B[1] + 2;

  for (int ch = w; ch * kWave < total; ch += kSpreadWaves) {
    const int f = ch * kWave + lane;
    if (f >= total) continue;
    const int sl = spread_candidate(f, total, ncand, cand_list, cand_start, cand_off);
    const float4 p = xs[sl];
    int kx, ky, kz;
    float fx, fy, fz;
    grid_coord(p.x, pp.s_hi[0], pp.s_lo[0], pp.K[0], kx, fx);
    grid_coord(p.y, pp.s_hi[1], pp.s_lo[1], pp.K[1], ky, fy);
    grid_coord(p.z, pp.s_hi[2], pp.s_lo[2], pp.K[2], kz, fz);
    // stencil point t sits at k0 - t; its brick-local offset is k0 - g0 - t
    int dx = kx - g0x, dy = ky - g0y, dz = kz - g0z;
    if (dx < 0) dx += pp.K[0];
    if (dy < 0) dy += pp.K[1];
    if (dz < 0) dz += pp.K[2];
    float tx[4], ty[4], tz[4], dtx[4], dty[4], dtz[4];
    spline4(fx, tx, dtx);
    spline4(fy, ty, dty);
    spline4(fz, tz, dtz);
    // dipole mode: q u_d (K_d / L_d) scales the derivative factor along d
    float ux = 0.f, uy = 0.f, uz = 0.f;
    if (DIPOLE) {
      const float4 u = us[sl];
      ux = p.w * u.x * (pp.s_hi[0] + pp.s_lo[0]);
      uy = p.w * u.y * (pp.s_hi[1] + pp.s_lo[1]);
      uz = p.w * u.z * (pp.s_hi[2] + pp.s_lo[2]);
    }
#pragma unroll
    for (int t1 = 0; t1 < 4; ++t1) {
      int lx = dx - t1;
      if (lx < 0) lx += pp.K[0];
      if (lx >= bex) continue;
      const float wx = p.w * tx[t1];
#pragma unroll
      for (int t2 = 0; t2 < 4; ++t2) {
        int ly = dy - t2;
        if (ly < 0) ly += pp.K[1];
        if (ly >= bey) continue;
        const float wxy = wx * ty[t2];
        // dipole: (ux dtx ty + uy tx dty) tz + uz tx ty dtz
        const float a = DIPOLE ? ux * dtx[t1] * ty[t2] + uy * tx[t1] * dty[t2] : 0.f;
        const float b = DIPOLE ? uz * tx[t1] * ty[t2] : 0.f;
        float* row = my_grid + ly * pp.B[0] + lx;
#pragma unroll
        for (int t3 = 0; t3 < 4; ++t3) {
          int lz = dz - t3;
          if (lz < 0) lz += pp.K[2];
          if (lz < bez)
            atomicAdd(row + lz * plane, DIPOLE ? a * tz[t3] + b * dtz[t3] : wxy * tz[t3]);
        }
      }
    }
  }
  __syncthreads();
  const int nloc = bex * bey * bez;
  for (int t = threadIdx.x; t < nloc; t += blockDim.x) {
    int lx = t % bex, ly = (t / bex) % bey, lz = t / (bex * bey);
    int li = brick_index(lx, ly, lz, pp);
    float s = lgrid[0][li];
    for (int c = 1; c < kSpreadWaves; ++c) s += lgrid[c][li];
    grid_q[((size_t)(g0z + lz) * pp.K[1] + (g0y + ly)) * pp.K[0] + g0x + lx] = s;
  }
}

// The spread and the FFT passes share the chip with the pair kernel (they run
// on a second stream): their waves take a raised issue priority so the short
// chain of reciprocal-space kernels is not starved by the long-running pair
// waves on the same SIMDs.
__device__ __forceinline__ void fft_priority() { __builtin_amdgcn_s_setprio(2); }

// grid_coord's k0 and f, with the reduction into [0, K) done in float from
// the kernel parameters (K and 1/K) instead of an integer remainder: the
// remainder's multiplier would sit in a vector register for the kernel's
// whole run. kf is an integer below 2^24 in magnitude, so kf - K q is exact
// and the two corrections absorb an off-by-one quotient.
__device__ __forceinline__ int grid_coord_f(float x, float s_hi, float s_lo, float Kf, float invK,
                                            float& f) {
  float kf = floorf(x * s_hi);
  f = fmaf(x, s_hi, -kf) + x * s_lo;
  if (f < 0.f) { f += 1.0f; kf -= 1.0f; }
  if (f >= 1.0f) { f -= 1.0f; kf += 1.0f; }
  if (f < 0.f) f = 0.f;
  kf = fmaf(-Kf, floorf(kf * invK), kf);
  if (kf >= Kf) kf -= Kf;
  if (kf < 0.f) kf += Kf;
  return (int)kf;
}

// Owner-computes spreading for grids of at least B + 3 points along every
// axis (then B = 8 and no stencil point wraps back into the brick it left).
// Lane (lx, ly) of every wave owns the brick's z-line at (lx, ly) and holds
// its 8 points in registers; the waves take the candidates in chunks of 64
// (one per lane: grid coordinates and weights q t_x, t_y, t_z into the wave's
// LDS table), then walk the chunk's atoms whose stencil meets the brick one at
// a time: every lane adds that atom's weights on its own line (at most 16 of
// the 64 lines, 4 points each). The four waves' bricks are summed in wave
// order at the end. No atomics; every point's sum runs in a fixed order
// (chunk, lane, wave), so the grid does not depend on scheduling.
//
// Written to fit in 32 VGPRs (each weight row is computed and stored before
// the next): the pair kernel running beside it on the first stream leaves 32
// of a SIMD's 512 registers per lane free, and a larger wave would wait for
// the pair waves to retire.
__global__ void __launch_bounds__(kSpreadThreads) k_pme_spread_lines(
    const float4* __restrict__ xs, const int4* __restrict__ brick_zr,
    const int* __restrict__ brick_cols, PmeParams pp, CellGrid cg,
    float* __restrict__ grid_q) {
  constexpr int B = 8;
  fft_priority();
  // 20 KB of LDS in all, so that LDS leaves room for 8 waves per SIMD and
  // the register allocation stays at what the code uses (the compiler sizes
  // it to the occupancy the LDS allows). Per candidate: q t_x[0..3],
  // t_y[0..3], and the weights of the brick's 8 z planes (t_z[dz - lz] where
  // the stencil covers lz, else 0); after its chunks each wave keeps its
  // brick lines ([lz][ly B + lx]) in its own part of the table. Stored
  // component-major ([wave][k][lane]): a row write is then one 16-byte
  // store per lane at consecutive addresses (no bank conflicts).
  __shared__ float4 wts[kSpreadWaves][4][kWave];
  // the candidate slot ranges (two per column, periodic wrap) and the
  // inclusive prefix sums of their sizes
  __shared__ int seg_start[kMaxCandCells];
  __shared__ int seg_end[kMaxCandCells];

  const int brick = blockIdx.x;
  const int bx = brick % pp.nb[0], by = (brick / pp.nb[0]) % pp.nb[1],
            bz = brick / (pp.nb[0] * pp.nb[1]);
  const int g0x = bx * B, g0y = by * B, g0z = bz * B;
  const int bex = min(B, pp.K[0] - g0x), bey = min(B, pp.K[1] - g0y), bez = min(B, pp.K[2] - g0z);
  const int* bcx = brick_cols + 2 * bx;
  const int* bcy = brick_cols + 2 * pp.nb[0] + 2 * by;
  const int ncx = bcx[1], ncy = bcy[1];
  const int ncol = ncx * ncy;
  const int ncand = 2 * ncol;
  const int w = threadIdx.x / kWave, lane = threadIdx.x & (kWave - 1);
  const int4* zr = brick_zr + (size_t)bz * cg.ncell;
  for (int t = threadIdx.x; t < ncol; t += blockDim.x) {
    int cx = (bcx[0] + t % ncx) % cg.n[0], cy = (bcy[0] + t / ncx) % cg.n[1];
    const int4 r = zr[cy * cg.n[0] + cx];
    seg_start[2 * t] = r.x;
    seg_end[2 * t] = r.y;
    seg_start[2 * t + 1] = r.z;
    seg_end[2 * t + 1] = r.w;
  }
  __syncthreads();
  if (w == 0) {
    int carry = 0;
    for (int base = 0; base < ncand; base += kWave) {
      const int i = base + lane;
      int v = i < ncand ? seg_end[i] : 0;
      for (int o = 1; o < kWave; o <<= 1) {
        const int u = __shfl_up(v, o, kWave);
        if (lane >= o) v += u;
      }
      if (i < ncand) seg_end[i] = carry + v;
      carry += __shfl(v, kWave - 1, kWave);
    }
  }
  __syncthreads();
  const int total = ncand > 0 ? seg_end[ncand - 1] : 0;
  // candidate f: the first segment whose end passes f (never an empty one)
  auto candidate = [&](int f) {
    int lo = 0, hi = ncand - 1;
    while (lo < hi) {
      const int mid = (lo + hi) >> 1;
      if (seg_end[mid] > f) hi = mid; else lo = mid + 1;
    }
    return seg_start[lo] + f - (lo > 0 ? seg_end[lo - 1] : 0);
  };

  const int lx = lane & (B - 1), ly = lane / B;
  float acc[B] = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
  for (int ch = w; ch * kWave < total; ch += kSpreadWaves) {
    const int f = ch * kWave + lane;
    unsigned packed = 0u;
    bool meets = false;
    if (f < total) {
      const int sl = candidate(f);
      const float4 p = xs[sl];
      auto row = [&](int k) -> float4& { return wts[w][k][lane]; };
      float t[4], dt[4];
      // stencil point t sits at brick-local offset d - t (d = k0 - g0 mod K)
      int k;
      float fr;
      k = grid_coord_f(p.x, pp.s_hi[0], pp.s_lo[0], pp.Kf[0], pp.invK[0], fr);
      int dx = k - g0x;
      if (dx < 0) dx += pp.K[0];
      spline4(fr, t, dt);
      row(0) = make_float4(p.w * t[0], p.w * t[1], p.w * t[2], p.w * t[3]);
      __builtin_amdgcn_sched_barrier(0);
      k = grid_coord_f(p.y, pp.s_hi[1], pp.s_lo[1], pp.Kf[1], pp.invK[1], fr);
      int dy = k - g0y;
      if (dy < 0) dy += pp.K[1];
      spline4(fr, t, dt);
      row(1) = make_float4(t[0], t[1], t[2], t[3]);
      packed = (unsigned)dx | (unsigned)dy << 8;
      const bool meets_xy = dx < bex + 3 && dy < bey + 3;
      __builtin_amdgcn_sched_barrier(0);
      k = grid_coord_f(p.z, pp.s_hi[2], pp.s_lo[2], pp.Kf[2], pp.invK[2], fr);
      int dz = k - g0z;
      if (dz < 0) dz += pp.K[2];
      spline4(fr, t, dt);
      // weight of plane lz: t_z[dz - lz] where 0 <= dz - lz <= 3
      auto zw = [&](int lz) {
        const int t3 = dz - lz;
        const float lo = (t3 & 1) ? t[1] : t[0], hi = (t3 & 1) ? t[3] : t[2];
        const float v = (t3 & 2) ? hi : lo;
        return (unsigned)t3 < 4u ? v : 0.f;
      };
#pragma unroll
      for (int lz = 0; lz < B; ++lz) {
        reinterpret_cast<float*>(&row(2 + lz / 4))[lz % 4] = zw(lz);
        __builtin_amdgcn_sched_barrier(0);
      }
      meets = meets_xy && dz < bez + 3;
    }
    unsigned long long m = __ballot(meets);
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    while (m) {
      const int a = __builtin_ctzll(m);
      m &= m - 1ull;
      const unsigned pa = __builtin_amdgcn_readlane(packed, a);
      const int t1 = (int)(pa & 255u) - lx, t2 = (int)((pa >> 8) & 255u) - ly;
      const float wxv = reinterpret_cast<const float*>(&wts[w][0][a])[t1 & 3];
      const float wyv = reinterpret_cast<const float*>(&wts[w][1][a])[t2 & 3];
      const float4 z0 = wts[w][2][a], z1 = wts[w][3][a];
      const float wv = ((unsigned)t1 < 4u && (unsigned)t2 < 4u) ? wxv * wyv : 0.f;
      acc[0] += wv * z0.x;
      acc[1] += wv * z0.y;
      acc[2] += wv * z0.z;
      acc[3] += wv * z0.w;
      acc[4] += wv * z1.x;
      acc[5] += wv * z1.y;
      acc[6] += wv * z1.z;
      acc[7] += wv * z1.w;
    }
    // the next chunk rewrites the table
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
  }
  float* const mine = reinterpret_cast<float*>(&wts[w][0][0]);
#pragma unroll
  for (int z = 0; z < B; ++z) mine[z * kWave + lane] = acc[z];
  __syncthreads();
  auto line = [&](int c, int z, int col) {
    return reinterpret_cast<const float*>(&wts[c][0][0])[z * kWave + col];
  };
  for (int t = threadIdx.x; t < B * kWave; t += blockDim.x) {
    const int z = t / kWave, col = t % kWave, x = col % B, y = col / B;
    if (x < bex && y < bey && z < bez) {
      const float s = ((line(0, z, col) + line(1, z, col)) + line(2, z, col)) + line(3, z, col);
      grid_q[((size_t)(g0z + z) * pp.K[1] + (g0y + y)) * pp.K[0] + g0x + x] = s;
    }
  }
}

// The line kernel covers grids with at least 11 points along every axis.
__host__ __forceinline__ bool spread_by_lines(const PmeParams& pp) {
  return pp.K[0] >= 11 && pp.K[1] >= 11 && pp.K[2] >= 11;
}


// ---------------------------------------------------------------------------
// LDS FFT: Stockham autosort, radix 4/2/3/5 (7 by table), twiddles from a
// host-built table exp(-2 pi i m/N). Lengths with a compiled plan (kFftSizes)
// run a fully unrolled stage sequence with constant strides; other lengths
// use the same stages with run-time strides.
// ---------------------------------------------------------------------------
struct Radices {
  int n;
  int r[16];
};

__host__ __device__ constexpr Radices factor_radices(int N) {
  Radices f{};
  int m = N;
  while (m % 10 == 0 && f.n < 16) { f.r[f.n++] = 10; m /= 10; }
  while (m % 4 == 0 && f.n < 16) { f.r[f.n++] = 4; m /= 4; }
  while (m % 2 == 0 && f.n < 16) { f.r[f.n++] = 2; m /= 2; }
  while (m % 3 == 0 && f.n < 16) { f.r[f.n++] = 3; m /= 3; }
  while (m % 5 == 0 && f.n < 16) { f.r[f.n++] = 5; m /= 5; }
  while (m % 7 == 0 && f.n < 16) { f.r[f.n++] = 7; m /= 7; }
  if (m != 1) f.n = -1;
  return f;
}

__device__ __forceinline__ float2 cmul(float2 a, float2 b) {
  return make_float2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}

// exp(SIGN * 2 pi i m / N) from the forward table exp(-2 pi i m / N).
template <int SIGN>
__device__ __forceinline__ float2 twid(const float2* tw, int m) {
  float2 t = tw[m];
  if (SIGN > 0) t.y = -t.y;
  return t;
}

// SIGN * i * z
template <int SIGN>
__device__ __forceinline__ float2 mul_si(float2 z) {
  return SIGN > 0 ? make_float2(-z.y, z.x) : make_float2(z.y, -z.x);
}

// In-register DFT of length R with kernel exp(SIGN 2 pi i r k / R).
template <int R, int SIGN>
__device__ __forceinline__ void dft_fixed(float2* v, const float2* tw, int N) {
  if constexpr (R == 2) {
    float2 a = v[0], b = v[1];
    v[0] = make_float2(a.x + b.x, a.y + b.y);
    v[1] = make_float2(a.x - b.x, a.y - b.y);
  } else if constexpr (R == 4) {
    float2 a = v[0], b = v[1], c = v[2], d = v[3];
    float2 s0 = make_float2(a.x + c.x, a.y + c.y), s1 = make_float2(a.x - c.x, a.y - c.y);
    float2 s2 = make_float2(b.x + d.x, b.y + d.y), s3 = make_float2(b.x - d.x, b.y - d.y);
    float2 is3 = mul_si<SIGN>(s3);
    v[0] = make_float2(s0.x + s2.x, s0.y + s2.y);
    v[2] = make_float2(s0.x - s2.x, s0.y - s2.y);
    v[1] = make_float2(s1.x + is3.x, s1.y + is3.y);
    v[3] = make_float2(s1.x - is3.x, s1.y - is3.y);
  } else if constexpr (R == 3) {
    // y1,2 = v0 - (v1+v2)/2 +- SIGN i sin(2pi/3) (v1 - v2)
    const float s3 = 0.86602540378443865f;
    float2 t1 = make_float2(v[1].x + v[2].x, v[1].y + v[2].y);
    float2 t2 = make_float2(s3 * (v[1].x - v[2].x), s3 * (v[1].y - v[2].y));
    float2 a = make_float2(v[0].x - 0.5f * t1.x, v[0].y - 0.5f * t1.y);
    float2 b = mul_si<SIGN>(t2);
    v[0] = make_float2(v[0].x + t1.x, v[0].y + t1.y);
    v[1] = make_float2(a.x + b.x, a.y + b.y);
    v[2] = make_float2(a.x - b.x, a.y - b.y);
  } else if constexpr (R == 5) {
    // cos/sin of 2pi/5 and 4pi/5; pairs (1,4) and (2,3) combine into
    // a1,2 (cosine parts) and b1,2 (sine parts)
    const float c1 = 0.30901699437494742f, c2 = -0.80901699437494742f;
    const float s1 = 0.95105651629515357f, s2 = 0.58778525229247313f;
    float2 t1 = make_float2(v[1].x + v[4].x, v[1].y + v[4].y);
    float2 t2 = make_float2(v[2].x + v[3].x, v[2].y + v[3].y);
    float2 t3 = make_float2(v[1].x - v[4].x, v[1].y - v[4].y);
    float2 t4 = make_float2(v[2].x - v[3].x, v[2].y - v[3].y);
    float2 a1 = make_float2(v[0].x + c1 * t1.x + c2 * t2.x, v[0].y + c1 * t1.y + c2 * t2.y);
    float2 a2 = make_float2(v[0].x + c2 * t1.x + c1 * t2.x, v[0].y + c2 * t1.y + c1 * t2.y);
    float2 b1 = mul_si<SIGN>(make_float2(s1 * t3.x + s2 * t4.x, s1 * t3.y + s2 * t4.y));
    float2 b2 = mul_si<SIGN>(make_float2(s2 * t3.x - s1 * t4.x, s2 * t3.y - s1 * t4.y));
    v[0] = make_float2(v[0].x + t1.x + t2.x, v[0].y + t1.y + t2.y);
    v[1] = make_float2(a1.x + b1.x, a1.y + b1.y);
    v[4] = make_float2(a1.x - b1.x, a1.y - b1.y);
    v[2] = make_float2(a2.x + b2.x, a2.y + b2.y);
    v[3] = make_float2(a2.x - b2.x, a2.y - b2.y);
  } else if constexpr (R == 10) {
    // prime-factor (Good-Thomas) split 10 = 2 x 5, no twiddles: with input
    // x[(5 a + 2 b) mod 10] and output X[(5 c + 6 d) mod 10], X is the
    // 2-point DFT over a of the 5-point DFTs over b
    float2 e[5], o[5];
#pragma unroll
    for (int b = 0; b < 5; ++b) {
      e[b] = v[(2 * b) % 10];
      o[b] = v[(5 + 2 * b) % 10];
    }
    dft_fixed<5, SIGN>(e, tw, N);
    dft_fixed<5, SIGN>(o, tw, N);
#pragma unroll
    for (int d = 0; d < 5; ++d) {
      v[(6 * d) % 10] = make_float2(e[d].x + o[d].x, e[d].y + o[d].y);
      v[(5 + 6 * d) % 10] = make_float2(e[d].x - o[d].x, e[d].y - o[d].y);
    }
  } else {
    float2 in[R];
    for (int r = 0; r < R; ++r) in[r] = v[r];
    const int step = N / R;
    for (int k = 0; k < R; ++k) {
      float2 acc = in[0];
      for (int r = 1; r < R; ++r) {
        float2 p = cmul(in[r], twid<SIGN>(tw, ((r * k) % R) * step));
        acc.x += p.x;
        acc.y += p.y;
      }
      v[k] = acc;
    }
  }
}

// One Stockham stage on P pencils stored with stride SP: radix R, NS points
// already combined. All threads of the block take part.
template <int R, int SIGN>
__device__ __forceinline__ void fft_stage(const float2* __restrict__ a, float2* __restrict__ b,
                                          int N, int SP, int NS, int P, const float2* tw) {
  const int NR = N / R;
  const int ts = N / (NS * R);
  for (int idx = threadIdx.x; idx < P * NR; idx += blockDim.x) {
    const int p = idx / NR, j = idx - p * NR;
    const int k = j % NS;
    const float2* in = a + p * SP;
    float2* out = b + p * SP;
    float2 v[R];
    v[0] = in[j];
#pragma unroll
    for (int r = 1; r < R; ++r) v[r] = cmul(in[j + r * NR], twid<SIGN>(tw, k * r * ts));
    dft_fixed<R, SIGN>(v, tw, N);
    const int base = (j / NS) * NS * R + k;
#pragma unroll
    for (int r = 0; r < R; ++r) out[base + r * NS] = v[r];
  }
  __syncthreads();
}

// Compiled plan: stage S of length N (constant strides, unrolled sequence).
template <int N, int SIGN, int S, int NS>
__device__ __forceinline__ float2* fft_ct(float2* a, float2* b, int SP, int P, const float2* tw) {
  constexpr Radices f = factor_radices(N);
  if constexpr (S >= f.n) {
    return a;
  } else {
    constexpr int R = f.r[S];
    fft_stage<R, SIGN>(a, b, N, SP, NS, P, tw);
    return fft_ct<N, SIGN, S + 1, NS * R>(b, a, SP, P, tw);
  }
}

// Run-time plan for lengths without a compiled one.
template <int SIGN>
__device__ float2* fft_rt(float2* a, float2* b, int SP, int P, const FftPlan& pl,
                          const float2* tw) {
  int NS = 1;
  for (int s = 0; s < pl.nst; ++s) {
    const int R = pl.radix[s];
    switch (R) {
      case 4: fft_stage<4, SIGN>(a, b, pl.N, SP, NS, P, tw); break;
      case 2: fft_stage<2, SIGN>(a, b, pl.N, SP, NS, P, tw); break;
      case 3: fft_stage<3, SIGN>(a, b, pl.N, SP, NS, P, tw); break;
      case 5: fft_stage<5, SIGN>(a, b, pl.N, SP, NS, P, tw); break;
      case 10: fft_stage<10, SIGN>(a, b, pl.N, SP, NS, P, tw); break;
      default: fft_stage<7, SIGN>(a, b, pl.N, SP, NS, P, tw); break;
    }
    float2* t = a;
    a = b;
    b = t;
    NS *= R;
  }
  return a;
}

template <int N, int SIGN>
__device__ __forceinline__ float2* fft_any(float2* a, float2* b, int SP, int P, const FftPlan& pl,
                                           const float2* tw) {
  if constexpr (N > 0) {
    return fft_ct<N, SIGN, 0, 1>(a, b, SP, P, tw);
  } else {
    return fft_rt<SIGN>(a, b, SP, P, pl, tw);
  }
}

// x-direction forward: real rows [Kz*Ky][Kx] -> half spectrum [Kz*Ky][Kxh].
// Two real rows per complex transform: pencil q holds rows a = r0 + 2q (real
// part) and b = a + 1 (imaginary part) of the block's 2P rows; with Z the
// transform, X_a(k) = (Z(k) + conj Z(L-k)) / 2 and X_b(k) = (Z(k) -
// conj Z(L-k)) / (2i).
template <int N>
__global__ void __launch_bounds__(256) k_fft_rows_r2c(const float* __restrict__ in,
                                                      float2* __restrict__ out, int nrows,
                                                      int P, int Kxh, FftPlan pl,
                                                      const float2* __restrict__ twg) {
  fft_priority();
  extern __shared__ float2 sm[];
  const int L = N > 0 ? N : pl.N;
  float2* tw = sm;
  float2* a = sm + L;
  float2* b = a + P * L;
  for (int t = threadIdx.x; t < L; t += blockDim.x) tw[t] = twg[t];
  const int r0 = blockIdx.x * 2 * P;
  for (int idx = threadIdx.x; idx < P * L; idx += blockDim.x) {
    const int q = idx / L, x = idx - q * L;
    const int ra = r0 + 2 * q, rb = ra + 1;
    a[idx] = make_float2(ra < nrows ? in[(size_t)ra * L + x] : 0.f,
                         rb < nrows ? in[(size_t)rb * L + x] : 0.f);
  }
  __syncthreads();
  float2* res = fft_any<N, -1>(a, b, L, P, pl, tw);
  for (int idx = threadIdx.x; idx < P * Kxh; idx += blockDim.x) {
    const int q = idx / Kxh, k = idx - q * Kxh;
    const float2 zk = res[q * L + k], zm = res[q * L + (k == 0 ? 0 : L - k)];
    const int ra = r0 + 2 * q, rb = ra + 1;
    if (ra < nrows)
      out[(size_t)ra * Kxh + k] = make_float2(0.5f * (zk.x + zm.x), 0.5f * (zk.y - zm.y));
    if (rb < nrows)
      out[(size_t)rb * Kxh + k] = make_float2(0.5f * (zk.y + zm.y), 0.5f * (zm.x - zk.x));
  }
}

// x-direction inverse: half spectrum -> real rows (Hermitian completion).
// Two rows per complex transform: pencil q holds Z = X_a + i X_b over the
// full spectrum, each X completed by X(L-k) = conj X(k); the imaginary parts
// of X(0) and X(L/2), which are zero for a real row, are set to zero, so the
// real and imaginary parts of the inverse are the two rows.
template <int N>
__global__ void __launch_bounds__(256) k_fft_rows_c2r(const float2* __restrict__ in,
                                                      float* __restrict__ out, int nrows,
                                                      int P, int Kxh, FftPlan pl,
                                                      const float2* __restrict__ twg) {
  fft_priority();
  extern __shared__ float2 sm[];
  const int L = N > 0 ? N : pl.N;
  float2* tw = sm;
  float2* a = sm + L;
  float2* b = a + P * L;
  for (int t = threadIdx.x; t < L; t += blockDim.x) tw[t] = twg[t];
  const int r0 = blockIdx.x * 2 * P;
  for (int idx = threadIdx.x; idx < P * L; idx += blockDim.x) {
    const int q = idx / L, k = idx - q * L;
    const int ra = r0 + 2 * q, rb = ra + 1;
    const bool hi = k >= Kxh;
    const int kk = hi ? L - k : k;
    const bool self_conj = k == 0 || 2 * k == L;
    float2 xa = make_float2(0.f, 0.f), xb = make_float2(0.f, 0.f);
    if (ra < nrows) xa = in[(size_t)ra * Kxh + kk];
    if (rb < nrows) xb = in[(size_t)rb * Kxh + kk];
    if (hi) {
      xa.y = -xa.y;
      xb.y = -xb.y;
    }
    if (self_conj) {
      xa.y = 0.f;
      xb.y = 0.f;
    }
    a[idx] = make_float2(xa.x - xb.y, xa.y + xb.x);
  }
  __syncthreads();
  float2* res = fft_any<N, +1>(a, b, L, P, pl, tw);
  for (int idx = threadIdx.x; idx < P * L; idx += blockDim.x) {
    const int q = idx / L, x = idx - q * L;
    const int ra = r0 + 2 * q, rb = ra + 1;
    const float2 z = res[idx];
    if (ra < nrows) out[(size_t)ra * L + x] = z.x;
    if (rb < nrows) out[(size_t)rb * L + x] = z.y;
  }
}

// Column pencils of the half spectrum, P consecutive kx per block, stored in
// LDS with an odd stride (L + 1) so the transposing load is conflict-free.
// MODE 0: y forward, 1: y inverse, 2: z forward, influence multiply + energy
// partial, z inverse.
template <int N, int MODE>
__global__ void __launch_bounds__(256) k_fft_cols(float2* __restrict__ grid, PmeParams pp,
                                                  int P, FftPlan pl,
                                                  const float2* __restrict__ twg,
                                                  const double* __restrict__ bmx,
                                                  const double* __restrict__ bmy,
                                                  const double* __restrict__ bmz,
                                                  const double* __restrict__ mx,
                                                  const double* __restrict__ my,
                                                  const double* __restrict__ mz,
                                                  const double* __restrict__ gtab,
                                                  double* __restrict__ partials, int pstride) {
  fft_priority();
  extern __shared__ float2 sm[];
  __shared__ double red[16];
  const int L = N > 0 ? N : pl.N;
  const int SP = L + 1;
  float2* tw = sm;
  float2* a = sm + L;
  float2* b = a + P * SP;
  for (int t = threadIdx.x; t < L; t += blockDim.x) tw[t] = twg[t];
  const int Kxh = pp.Kxh;
  const int ntile = (Kxh + P - 1) / P;
  const int outer = blockIdx.x / ntile;       // z for the y pass, ky for the z pass
  const int kx0 = (blockIdx.x - outer * ntile) * P;
  size_t base, stride;
  if (MODE >= 2) {
    base = (size_t)outer * Kxh;
    stride = (size_t)pp.K[1] * Kxh;
  } else {
    base = (size_t)outer * pp.K[1] * Kxh;
    stride = Kxh;
  }
  // element i P + p of the tile (i along the pencil, p the pencil): each
  // thread steps (i, p) by the block size, without a division per element
  const int di = (int)blockDim.x / P, dp = (int)blockDim.x - di * P;
  const int i0 = (int)threadIdx.x / P, p0 = (int)threadIdx.x - i0 * P;
  for (int i = i0, p = p0; i < L;) {
    const int kx = kx0 + p;
    a[p * SP + i] = kx < Kxh ? grid[base + (size_t)i * stride + kx] : make_float2(0.f, 0.f);
    i += di;
    p += dp;
    if (p >= P) {
      p -= P;
      ++i;
    }
  }
  __syncthreads();
  float2* res;
  if (MODE == 1) {
    res = fft_any<N, +1>(a, b, SP, P, pl, tw);
  } else {
    res = fft_any<N, -1>(a, b, SP, P, pl, tw);
  }
  if (MODE >= 2) {
    // influence function G = B(m) C(m) on the half spectrum. G is formed in
    // FP64 (its float32 value scales Q^; the FP64 value, without the
    // constant 1/(pi V) applied in the reduction, weights |Q^|^2 for E_rec).
    // MODE 3 also sums the virial: each E(m) times
    // delta_ab - 2 (1 + pi^2 m^2 / alpha^2) m_a m_b / m^2.
    double e = 0.0;
    double w[6] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
    const int ky = outer;
    for (int idx = threadIdx.x; idx < P * L; idx += blockDim.x) {
      int p = idx / L, kz = idx - p * L;
      int kx = kx0 + p;
      float2 v = res[p * SP + kz];
      float g = 0.f;
      if (kx < Kxh) {
        // G from the context's table (the virial pass needs m^2 and forms it
        // here); zero at m = 0
        double msq = 0.0, gd = 0.0;
        if (MODE == 3) {
          msq = mx[kx] * mx[kx] + my[ky] * my[ky] + mz[kz] * mz[kz];
          if (msq > 0.0) gd = bmx[kx] * bmy[ky] * bmz[kz] * exp(-pp.exp_fac * msq) / msq;
        } else {
          gd = gtab[((size_t)ky * Kxh + kx) * L + kz];
        }
        if (gd != 0.0) {
          int wgt = (kx == 0 || (2 * kx == pp.K[0])) ? 1 : 2;
          const double ew = (double)wgt * gd * ((double)v.x * v.x + (double)v.y * v.y);
          e += ew;
          if (MODE == 3) {
            const double fac = 2.0 * (1.0 + pp.exp_fac * msq) / msq;
            const double m0 = mx[kx], m1 = my[ky], m2 = mz[kz];
            w[0] += ew * (1.0 - fac * m0 * m0);
            w[1] += ew * (1.0 - fac * m1 * m1);
            w[2] += ew * (1.0 - fac * m2 * m2);
            w[3] -= ew * fac * m0 * m1;
            w[4] -= ew * fac * m0 * m2;
            w[5] -= ew * fac * m1 * m2;
          }
          g = (float)(gd * pp.inv_piV);
        }
      }
      res[p * SP + kz] = make_float2(v.x * g, v.y * g);
    }
    double s = block_sum(e, red);
    if (threadIdx.x == 0) partials[kRowRec * pstride + blockIdx.x] = s;
    if (MODE == 3) {
      for (int k = 0; k < 6; ++k) {
        const double sk = block_sum(w[k], red);
        if (threadIdx.x == 0) partials[(kRowVir + k) * pstride + blockIdx.x] = sk;
      }
    }
    __syncthreads();
    float2* other = (res == a) ? b : a;
    res = fft_any<N, +1>(res, other, SP, P, pl, tw);
  }
  for (int i = i0, p = p0; i < L;) {
    const int kx = kx0 + p;
    if (kx < Kxh) grid[base + (size_t)i * stride + kx] = res[p * SP + i];
    i += di;
    p += dp;
    if (p >= P) {
      p -= P;
      ++i;
    }
  }
}

// One thread per slot (padding slots return): F = -k_e q grad(theta) . phi.
__global__ void __launch_bounds__(256) k_pme_gather(const float4* __restrict__ xs,
                                                    const int* __restrict__ perm,
                                                    const int* __restrict__ meta,
                                                    const float* __restrict__ phi, int n,
                                                    PmeParams pp, float* __restrict__ force) {
  int s = blockIdx.x * blockDim.x + threadIdx.x;
  if (s >= meta[0]) return;
  const int a = perm[s];
  if (a < 0) return;
  float fx = 0.f, fy = 0.f, fz = 0.f;
  pme_gather_atom(xs[s], phi, pp, fx, fy, fz);
  force[a] += fx;
  force[n + a] += fy;
  force[2 * n + a] += fz;
}

// ---------------------------------------------------------------------------
static FftPlan make_plan(int N) {
  FftPlan p{};
  Radices f = factor_radices(N);
  p.N = N;
  p.nst = f.n;
  for (int s = 0; s < 16; ++s) p.radix[s] = f.r[s];
  return p;
}

bool pme_size_supported(int K) { return K >= 4 && K <= 1024 && make_plan(K).nst > 0; }

// Pencils (consecutive kx) per block of the column passes: the count in
// [12, 24] that leaves the fewest padding columns in the last tile of the
// Kxh columns (17 for Kxh = 51: three full tiles), the larger on a tie.
int pme_col_pencils(int kxh) {
  int best = 16, waste = 1 << 30;
  for (int pc = 12; pc <= 24; ++pc) {
    const int w = (kxh + pc - 1) / pc * pc - kxh;
    if (w <= waste) {
      best = pc;
      waste = w;
    }
  }
  return best;
}

static int pencils_for(int N) {
  int P = 2048 / N;
  if (P > 32) P = 32;
  if (P < 1) P = 1;
  return P;
}

// Lengths with a compiled FFT plan; others take the run-time plan.
#define MDX_FFT_SIZES(X) X(32) X(48) X(64) X(96) X(100) X(128)

template <int N>
static void launch_rows_r2c(int blocks, size_t sh, hipStream_t s, const float* in, float2* out,
                            int rows, int P, int Kxh, const FftPlan& pl, const float2* tw) {
  k_fft_rows_r2c<N><<<blocks, 256, sh, s>>>(in, out, rows, P, Kxh, pl, tw);
}
// The last pass may record `done` as part of its own dispatch (no separate
// marker on the stream).
template <int N>
static void launch_rows_c2r(int blocks, size_t sh, hipStream_t s, const float2* in, float* out,
                            int rows, int P, int Kxh, const FftPlan& pl, const float2* tw,
                            hipEvent_t done) {
  if (!done) {
    k_fft_rows_c2r<N><<<blocks, 256, sh, s>>>(in, out, rows, P, Kxh, pl, tw);
    return;
  }
  FftPlan plan = pl;
  void* args[] = {&in, &out, &rows, &P, &Kxh, &plan, &tw};
  (void)hipExtLaunchKernel(reinterpret_cast<const void*>(k_fft_rows_c2r<N>), dim3(blocks),
                           dim3(256), args, sh, s, nullptr, done, 0);
}
template <int N, int MODE>
static void launch_cols(int blocks, size_t sh, hipStream_t s, Ctx& c, const PmeParams& pp, int P,
                        const FftPlan& pl, const float2* tw) {
  k_fft_cols<N, MODE><<<blocks, 256, sh, s>>>(c.grid_c, pp, P, pl, tw, c.bmod[0], c.bmod[1],
                                               c.bmod[2], c.mrec[0], c.mrec[1], c.mrec[2],
                                               c.pme_g, c.partials, c.max_blocks);
}

static void rows_r2c(int N, int blocks, size_t sh, hipStream_t s, const float* in, float2* out,
                     int rows, int P, int Kxh, const FftPlan& pl, const float2* tw) {
  switch (N) {
#define X(n) case n: launch_rows_r2c<n>(blocks, sh, s, in, out, rows, P, Kxh, pl, tw); return;
    MDX_FFT_SIZES(X)
#undef X
    default: launch_rows_r2c<0>(blocks, sh, s, in, out, rows, P, Kxh, pl, tw);
  }
}
static void rows_c2r(int N, int blocks, size_t sh, hipStream_t s, const float2* in, float* out,
                     int rows, int P, int Kxh, const FftPlan& pl, const float2* tw,
                     hipEvent_t done) {
  switch (N) {
#define X(n) case n: launch_rows_c2r<n>(blocks, sh, s, in, out, rows, P, Kxh, pl, tw, done); return;
    MDX_FFT_SIZES(X)
#undef X
    default: launch_rows_c2r<0>(blocks, sh, s, in, out, rows, P, Kxh, pl, tw, done);
  }
}
template <int MODE>
static void cols(int N, int blocks, size_t sh, hipStream_t s, Ctx& c, const PmeParams& pp, int P,
                 const FftPlan& pl, const float2* tw) {
  switch (N) {
#define X(n) case n: launch_cols<n, MODE>(blocks, sh, s, c, pp, P, pl, tw); return;
    MDX_FFT_SIZES(X)
#undef X
    default: launch_cols<0, MODE>(blocks, sh, s, c, pp, P, pl, tw);
  }
}

PmeParams make_pme_params(const Ctx& c) {
  const PmeGrid& g = c.pg;
  PmeParams pp;
  for (int d = 0; d < 3; ++d) {
    pp.K[d] = g.K[d];
    pp.B[d] = g.B[d];
    pp.nb[d] = g.nb[d];
    pp.s_hi[d] = g.scale_hi[d];
    pp.s_lo[d] = g.scale_lo[d];
    pp.Kf[d] = (float)g.K[d];
    pp.invK[d] = 1.0f / (float)g.K[d];
  }
  pp.Kxh = g.Kxh;
  pp.coulomb_k = (float)c.coulomb_k;
  pp.exp_fac = M_PI * M_PI / (c.alpha * c.alpha);
  pp.inv_piV = c.pme_energy_scale;
  return pp;
}

// Charge spreading onto grid_q on stream s; `done` (if given) is recorded by
// the kernel's own dispatch when it completes.
hipError_t launch_pme_spread(Ctx& c, hipStream_t s, hipEvent_t done) {
  static_assert(kBrickXY == 8 && kBrickZ == 8, "the line kernel holds 8-point bricks");
  const PmeParams pp = make_pme_params(c);
  const bool lines = spread_by_lines(pp);
  if (!done) {
    if (lines)
      k_pme_spread_lines<<<c.pg.nbrick, kSpreadThreads, 0, s>>>(c.xs, c.brick_zr, c.brick_cols, pp,
                                                                c.cg, c.grid_q);
    else
      k_pme_spread<false><<<c.pg.nbrick, kSpreadThreads, 0, s>>>(c.xs, c.brick_zr, c.brick_cols,
                                                                 pp, c.cg, c.grid_q, nullptr);
    return hipGetLastError();
  }
  const float4* xs = c.xs;
  const int4* zr = c.brick_zr;
  const int* bc = c.brick_cols;
  CellGrid cg = c.cg;
  float* q = c.grid_q;
  PmeParams p = pp;
  const float4* us = nullptr;
  if (lines) {
    void* args[] = {&xs, &zr, &bc, &p, &cg, &q};
    return hipExtLaunchKernel(reinterpret_cast<const void*>(k_pme_spread_lines),
                              dim3(c.pg.nbrick), dim3(kSpreadThreads), args, 0, s, nullptr, done, 0);
  }
  void* args[] = {&xs, &zr, &bc, &p, &cg, &q, &us};
  return hipExtLaunchKernel(reinterpret_cast<const void*>(k_pme_spread<false>),
                            dim3(c.pg.nbrick), dim3(kSpreadThreads), args, 0, s, nullptr, done, 0);
}

hipError_t launch_pme_spread_dipole(Ctx& c, const float4* us) {
  const PmeParams pp = make_pme_params(c);
  k_pme_spread<true><<<c.pg.nbrick, kSpreadThreads, 0, c.stream>>>(c.xs, c.brick_zr, c.brick_cols,
                                                                   pp, c.cg, c.grid_q, us);
  return hipGetLastError();
}

// The five FFT passes (forward transform, influence multiply with the energy
// partials, inverse) on stream s: grid_q -> potential in grid_phi; `done`
// (if given) is recorded by the last pass's dispatch.
hipError_t launch_pme_fft(Ctx& c, hipStream_t s, hipEvent_t done, bool virial) {
  const PmeGrid& g = c.pg;
  const PmeParams pp = make_pme_params(c);
  FftPlan px = make_plan(g.K[0]), py = make_plan(g.K[1]), pz = make_plan(g.K[2]);
  const int rows = g.K[1] * g.K[2];
  // row passes: P pencils of two rows each per block
  const int P = std::max(1, pencils_for(g.K[0]) / 2);
  const size_t sh = (size_t)(g.K[0] + 2 * P * g.K[0]) * sizeof(float2);
  const int rblocks = (rows + 2 * P - 1) / (2 * P);
  rows_r2c(g.K[0], rblocks, sh, s, c.grid_q, c.grid_c, rows, P, g.Kxh, px, c.tw[0]);
  const int Pc = pme_col_pencils(g.Kxh);
  const int ntile = (g.Kxh + Pc - 1) / Pc;
  const size_t shy = (size_t)(g.K[1] + 2 * Pc * (g.K[1] + 1)) * sizeof(float2);
  const size_t shz = (size_t)(g.K[2] + 2 * Pc * (g.K[2] + 1)) * sizeof(float2);
  cols<0>(g.K[1], g.K[2] * ntile, shy, s, c, pp, Pc, py, c.tw[1]);
  if (virial) cols<3>(g.K[2], g.K[1] * ntile, shz, s, c, pp, Pc, pz, c.tw[2]);
  else cols<2>(g.K[2], g.K[1] * ntile, shz, s, c, pp, Pc, pz, c.tw[2]);
  c.pme_blocks = g.K[1] * ntile;
  cols<1>(g.K[1], g.K[2] * ntile, shy, s, c, pp, Pc, py, c.tw[1]);
  rows_c2r(g.K[0], rblocks, sh, s, c.grid_c, c.grid_phi, rows, P, g.Kxh, px, c.tw[0], done);
  return hipGetLastError();
}

hipError_t launch_pme(Ctx& c, float* force, bool energy, bool virial) {
  (void)energy;   // the z pass always writes its energy partials
  hipError_t e = launch_pme_spread(c, c.stream, nullptr);
  if (e == hipSuccess) e = launch_pme_fft(c, c.stream, nullptr, virial);
  if (e != hipSuccess) return e;
  const PmeParams pp = make_pme_params(c);
  k_pme_gather<<<(c.max_slots + 255) / 256, 256, 0, c.stream>>>(c.xs, c.perm, c.meta, c.grid_phi,
                                                                c.n, pp, force);
  return hipGetLastError();
}

}  // namespace mdx
