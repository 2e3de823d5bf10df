// Cluster-pair Verlet list (DIMOS Sec. II.A.2, "Neighborlists").
//
// The list holds every non-excluded pair closer than r_nl = r_c + r_g. It is
// stored as tiles of 4-atom clusters: atoms are binned into x-y columns
// (edge ~ the cube holding four atoms), sorted by z inside each column (ties
// by atom index) and cut into consecutive clusters of four slots (the last
// cluster of a column is padded with empty slots). For every i-cluster the
// list keeps the j-clusters whose bounding boxes come closer than r_nl, each
// with a 16-bit mask whose bit 4*a + b says that slot pair (a, b) passes the
// float32 inclusion predicate of mdx.h and is not excluded. By default every
// pair is held from both ends (full list). With a half list every unordered
// pair is held once (Newton's third law: the force kernel applies each pair
// force to both atoms): a pair of distinct clusters is listed by one of the
// two, chosen by index parity, and a cluster's own tile keeps the slot pairs
// a < b; the tile search also lists every tile under its j-cluster
// (in_count / in_fill), from which the force kernel's j-side sums are
// gathered. The set bits are exactly the pair list, so the exported list is
// the definition's, while the force kernel streams whole 4x4 tiles.
//
// Build phases (gated: with a gate they do nothing unless it is raised):
//   bin (column of every atom, appended to that column's fixed-capacity
//   list) -> scan (atom and padded-slot offsets per column) -> column sort
//   (rank by z, write slot data), then the column's cluster boxes and PME
//   spreading ranges -> tile search (one wave per i-cluster). By default
//   these are three kernels (the last block to finish binning runs the
//   scan);
//   k_build_all runs them all in one cooperative launch with grid-wide
//   barriers between phases (optional: cooperative launches use a separate
//   hardware queue, and the resident grid is smaller than the per-phase
//   grids).
#include "mdx_internal.h"

#include <hip/hip_cooperative_groups.h>

#include <algorithm>

namespace mdx {

__global__ void k_fill_i32(int* __restrict__ p, int v, int count) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < count) p[i] = v;
}

hipError_t launch_fill_i32(int* p, int v, int count, hipStream_t s) {
  if (count <= 0) return hipSuccess;
  k_fill_i32<<<(count + 255) / 256, 256, 0, s>>>(p, v, count);
  return hipGetLastError();
}

__device__ __forceinline__ int bin_coord(float x, float inv_w, int n) {
  int c = (int)(x * inv_w);          // x >= 0: truncation is floor
  c = c < 0 ? 0 : c;
  return c >= n ? n - 1 : c;
}

__device__ __forceinline__ bool gated_off(const int* gate) { return gate && *gate == 0; }

// For the PME spreading: per (brick layer along z, column) the slots of the
// column whose build z lies in the layer's reach [lo, hi) - one segment, or
// two when the reach wraps around the periodic box.
struct ZRangeArgs {
  const float* zb;
  const int* slot_start;
  const int* col_start;   // atom offsets: the column's atom count is the difference
  const float* layer_z;   // [layers][2] lo, hi
  int layers;
  int ncol;
  float Lz;
  int4* out;              // [layers][ncol] (first, count) of both segments
};

__device__ void column_zrange(int e, const ZRangeArgs& z) {
  const int layer = e / z.ncol, col = e - layer * z.ncol;
  const float zlo = z.layer_z[2 * layer], zhi = z.layer_z[2 * layer + 1];
  const int sb = z.slot_start[col], se = sb + (z.col_start[col + 1] - z.col_start[col]);
  float a0 = zlo, b0 = zhi, a1 = 0.f, b1 = 0.f;
  if (zlo < 0.f) {
    a0 = 0.f; b0 = zhi; a1 = zlo + z.Lz; b1 = z.Lz;
  } else if (zhi > z.Lz) {
    a0 = zlo; b0 = z.Lz; a1 = 0.f; b1 = zhi - z.Lz;
  }
  const int s0 = lower_bound_f(z.zb, sb, se, a0), e0 = lower_bound_f(z.zb, sb, se, b0);
  int s1 = sb, e1 = sb;
  if (b1 > a1) {
    s1 = lower_bound_f(z.zb, sb, se, a1);
    e1 = lower_bound_f(z.zb, sb, se, b1);
  }
  z.out[e] = make_int4(s0, max(0, e0 - s0), s1, max(0, e1 - s1));
}

// Everything the build phases read and write.
struct BuildArgs {
  const int* gate;
  const float* pos;
  int n;
  CellGrid cg;
  int* col_of;
  int* col_count;
  float* x_build;
  unsigned* flags;
  int* col_start;
  int* slot_start;
  int* meta;
  int* nl_needed;
  int* col_atoms;   // [ncol][col_cap]
  int col_cap;
  const float* q;
  const int* atype;
  int* perm;
  int* inv_perm;
  float4* xs;
  int* ts;
  float* zb;
  float4* box_lo;
  float4* box_hi;
  float4* col_xy;
  ZRangeArgs zr;
  const int* ex_start;
  const int* ex_idx;
  int cap;
  int half;
  int2* zbin;
  uint2* tiles;
  int* tile_count;
  int max_clusters;
  // half list: tiles listed per j-cluster (cleared by the binning, appended
  // by the tile search in any order)
  int* in_count;   // [max_clusters]
  int* in_fill;    // [max_clusters][cap]: i-cluster * cap + full-list position
};

// Binning order. Every atom is binned once per build, in the slot order of
// the previous build when that build placed every atom (meta[4], set by the
// scan: the clamped column counts add up to n), else in atom order. In slot
// order the lanes of a wave fall into one or two columns, and each run of
// lanes with the same column takes its places in that column's list with a
// single atomic; in atom order the runs are short and this is one atomic
// per atom, as before. Which order was used does not change the list: the
// column sort ranks each column's atoms by (build z, atom index).
__device__ __forceinline__ bool bin_by_slot(const BuildArgs& a) { return a.meta[4] != 0; }
__device__ __forceinline__ int bin_count(const BuildArgs& a, bool by_slot) {
  return by_slot ? a.meta[0] : a.n;
}
__device__ __forceinline__ int bin_atom_at(const BuildArgs& a, bool by_slot, int j) {
  if (j >= bin_count(a, by_slot)) return -1;
  return by_slot ? a.perm[j] : j;
}

// Column of atom i (-1: none for this lane), atoms per column (the atom goes
// to the next free place of its column's fixed-capacity list), build-position
// snapshot. Called by every lane of the wave (the runs are found with
// cross-lane operations).
__device__ void bin_atom(const BuildArgs& a, int i) {
  const bool active = i >= 0;
  int c = -1;
  if (active) {
    const int n = a.n;
    float x = a.pos[i], y = a.pos[n + i], z = a.pos[2 * n + i];
    bool inside = x >= 0.f && x < a.cg.L[0] && y >= 0.f && y < a.cg.L[1] && z >= 0.f &&
                  z < a.cg.L[2];
    if (!inside) atomicOr(a.flags, MDX_FLAG_OUT_OF_BOX);
    int cx = bin_coord(x, a.cg.inv_w[0], a.cg.n[0]);
    int cy = bin_coord(y, a.cg.inv_w[1], a.cg.n[1]);
    c = cy * a.cg.n[0] + cx;
    a.col_of[i] = c;
    a.x_build[i] = x;
    a.x_build[n + i] = y;
    a.x_build[2 * n + i] = z;
  }
  // runs of consecutive active lanes with the same column: the first lane of
  // a run adds the run's length, the others take the following places
  const int lane = threadIdx.x & (kWave - 1);
  const int prev = __shfl_up(c, 1, kWave);
  const bool head = active && (lane == 0 || prev != c);
  const unsigned long long heads = __ballot(head);
  const unsigned long long stops = __ballot(head || !active);
  const unsigned long long below = lane == kWave - 1 ? ~0ull : (2ull << lane) - 1ull;
  const int leader = active ? kWave - 1 - __clzll(heads & below) : lane;
  int base = 0;
  if (head) {
    const unsigned long long after = lane == kWave - 1 ? 0ull : stops >> (lane + 1);
    const int len = after ? __ffsll((long long)after) : kWave - lane;
    base = atomicAdd(&a.col_count[c], len);
  }
  base = __shfl(base, leader, kWave);
  if (active) {
    const int k = base + (lane - leader);
    if (k < a.col_cap) {
      a.col_atoms[(size_t)c * a.col_cap + k] = i;
    } else {
      // left out of this list: no slot (the column sort writes the slots of
      // the atoms it places only)
      a.inv_perm[i] = -1;
      atomicOr(a.flags, MDX_FLAG_COLUMN_OVERFLOW);
    }
  }
}

// Exclusive scans of the column counts (atoms) and of the counts rounded up
// to whole clusters (slots), by one block; a wave-level shuffle scan
// combines per-thread chunk sums. meta[0] = slots, meta[1] = clusters,
// meta[2] counts the builds. The counts are cleared once read (ready for the
// next build's binning; they start at zero) and so is nl_needed.
__device__ void scan_columns(const BuildArgs& a) {
  __shared__ int wave_tot[2][16];
  const int ncol = a.cg.ncell;
  int* count = a.col_count;
  int t = threadIdx.x;
  int chunk = (ncol + blockDim.x - 1) / blockDim.x;
  int b = t * chunk, e = min(b + chunk, ncol);
  int s = 0, sp = 0;
  // the counts were formed by other blocks' atomics: read them at device scope
  for (int i = b; i < e; ++i) {
    const int ci = min(__hip_atomic_load(&count[i], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT),
                       a.col_cap);
    s += ci;
    sp += (ci + kClusterSize - 1) / kClusterSize * kClusterSize;
  }
  int lane = t & (kWave - 1), w = t / kWave;
  int v = s, vp = sp;
  for (int o = 1; o < kWave; o <<= 1) {
    int u = __shfl_up(v, o, kWave);
    int up = __shfl_up(vp, o, kWave);
    if (lane >= o) {
      v += u;
      vp += up;
    }
  }
  if (lane == kWave - 1) {
    wave_tot[0][w] = v;
    wave_tot[1][w] = vp;
  }
  __syncthreads();
  if (t == 0) {
    int acc = 0, accp = 0;
    for (int i = 0; i < (int)(blockDim.x / kWave); ++i) {
      int tmp = wave_tot[0][i], tmpp = wave_tot[1][i];
      wave_tot[0][i] = acc;
      wave_tot[1][i] = accp;
      acc += tmp;
      accp += tmpp;
    }
    a.col_start[ncol] = acc;
    a.slot_start[ncol] = accp;
    a.meta[0] = accp;
    a.meta[1] = accp / kClusterSize;
    a.meta[2] += 1;
    // every atom placed: the next build may bin in this build's slot order
    a.meta[4] = acc == a.n ? 1 : 0;
    *a.nl_needed = 0;
  }
  __syncthreads();
  int run = wave_tot[0][w] + v - s;
  int runp = wave_tot[1][w] + vp - sp;
  for (int i = b; i < e; ++i) {
    const int ci = min(__hip_atomic_load(&count[i], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT),
                       a.col_cap);
    a.col_start[i] = run;
    a.slot_start[i] = runp;
    run += ci;
    runp += (ci + kClusterSize - 1) / kClusterSize * kClusterSize;
    count[i] = 0;
  }
}

// One block per column: rank its atoms by (build z, atom index) - an order
// that does not depend on the binning's atomic order - and write the slot
// data; padding slots of the column's last cluster are emptied. Columns of
// up to kColStage atoms are ranked from LDS (st), larger ones from global
// memory.
constexpr int kColThreads = 128;
constexpr int kColStage = 1024;

// Sort key of a build z: a NaN coordinate (a diverged trajectory, flagged
// out of box by the binning) ranks as +inf, so that (key, atom index) stays
// a strict total order and each slot of the column is written exactly once.
__device__ __forceinline__ float z_key(float z) { return z == z ? z : __builtin_inff(); }

__device__ void sort_column(const BuildArgs& a, int c, float2* st) {
  const int n = a.n;
  const int b = a.col_start[c], e = a.col_start[c + 1];
  const int cnt = e - b;
  const int sb = a.slot_start[c], se = a.slot_start[c + 1];
  const bool staged = cnt <= kColStage;
  __syncthreads();   // st may still be read for the previous column
  if (staged) {
    for (int p = threadIdx.x; p < cnt; p += blockDim.x) {
      const int v = a.col_atoms[(size_t)c * a.col_cap + p];
      st[p] = make_float2(z_key(a.pos[2 * n + v]), __int_as_float(v));
    }
    __syncthreads();
  }
  for (int p = threadIdx.x; p < cnt; p += blockDim.x) {
    int v, rank = 0;
    float zv;
    if (staged) {
      const float2 me = st[p];
      zv = me.x;
      v = __float_as_int(me.y);
      for (int k = 0; k < cnt; ++k) {
        const float2 o = st[k];
        const int u = __float_as_int(o.y);
        rank += (o.x < zv || (o.x == zv && u < v)) ? 1 : 0;
      }
    } else {
      v = a.col_atoms[(size_t)c * a.col_cap + p];
      zv = z_key(a.pos[2 * n + v]);
      for (int k = 0; k < cnt; ++k) {
        const int u = a.col_atoms[(size_t)c * a.col_cap + k];
        const float zu = z_key(a.pos[2 * n + u]);
        rank += (zu < zv || (zu == zv && u < v)) ? 1 : 0;
      }
    }
    const int s = sb + rank;
    a.perm[s] = v;
    a.inv_perm[v] = s;
    a.xs[s] = make_float4(a.pos[v], a.pos[n + v], a.pos[2 * n + v], a.q[v]);
    a.ts[s] = a.atype[v];
    a.zb[s] = zv;
  }
  for (int s = sb + cnt + threadIdx.x; s < se; s += blockDim.x) {
    a.perm[s] = -1;
    a.xs[s] = make_float4(0.f, 0.f, 0.f, 0.f);
    a.ts[s] = 0;
    a.zb[s] = 3.0e38f;
  }
}

__device__ void cluster_box(const BuildArgs& a, int c);
__device__ __forceinline__ int first_ge(const float4* __restrict__ b, int lo, int hi, float x);
__device__ __forceinline__ int first_gt(const float4* __restrict__ b, int lo, int hi, float x);

// Column c's sort, then (reading back what this block just wrote, ordered by
// the block barrier) the bounding boxes of its clusters and its slot ranges
// for every PME brick layer.
__device__ void sort_column_boxes(const BuildArgs& a, int c, float2* st) {
  sort_column(a, c, st);
  __syncthreads();
  const int c0 = a.slot_start[c] / kClusterSize, c1 = a.slot_start[c + 1] / kClusterSize;
  for (int k = c0 + (int)threadIdx.x; k < c1; k += blockDim.x) cluster_box(a, k);
  for (int l = threadIdx.x; l < a.zr.layers; l += blockDim.x) column_zrange(l * a.zr.ncol + c, a.zr);
  __syncthreads();
  // x-y extent of the column's atoms (empty column: an inverted box), for
  // the tile search's column reach test
  if (threadIdx.x < kWave) {
    float xl = 3e38f, xh = -3e38f, yl = 3e38f, yh = -3e38f;
    for (int k = c0 + (int)threadIdx.x; k < c1; k += kWave) {
      const float4 lo = a.box_lo[k], hi = a.box_hi[k];
      if (lo.w > 0.f) {
        xl = fminf(xl, lo.x); xh = fmaxf(xh, hi.x);
        yl = fminf(yl, lo.y); yh = fmaxf(yh, hi.y);
      }
    }
    for (int o = 1; o < kWave; o <<= 1) {
      xl = fminf(xl, __shfl_xor(xl, o, kWave));
      xh = fmaxf(xh, __shfl_xor(xh, o, kWave));
      yl = fminf(yl, __shfl_xor(yl, o, kWave));
      yh = fmaxf(yh, __shfl_xor(yh, o, kWave));
    }
    if (threadIdx.x == 0) a.col_xy[c] = make_float4(xl, xh, yl, yh);
  }
  // lookup table of the column's z-sorted clusters: for bin edge z_b = b L/nzb
  // the first cluster whose max z >= z_b and the first whose min z > z_b
  const int nzb = a.cg.nzb;
  int2* zt = a.zbin + (size_t)c * (nzb + 1);
  for (int b = threadIdx.x; b <= nzb; b += blockDim.x) {
    const float zb = (float)b / a.cg.inv_zb;
    const int f = first_ge(a.box_hi, c0, c1, zb);
    zt[b] = make_int2(f, first_gt(a.box_lo, f, c1, zb));
  }
}

// Bounding box of cluster c's real atoms at the build positions.
__device__ void cluster_box(const BuildArgs& a, int c) {
  if (c >= a.meta[1]) return;
  float lx = 3e38f, ly = 3e38f, lz = 3e38f, hx = -3e38f, hy = -3e38f, hz = -3e38f;
  int nvalid = 0;
  for (int k = 0; k < kClusterSize; ++k) {
    int s = c * kClusterSize + k;
    if (a.perm[s] < 0) continue;
    float4 p = a.xs[s];
    lx = fminf(lx, p.x); ly = fminf(ly, p.y); lz = fminf(lz, p.z);
    hx = fmaxf(hx, p.x); hy = fmaxf(hy, p.y); hz = fmaxf(hz, p.z);
    ++nvalid;
  }
  a.box_lo[c] = make_float4(lx, ly, lz, (float)nvalid);
  a.box_hi[c] = make_float4(hx, hy, hz, 0.f);
}

// Each unordered pair of distinct clusters is listed once, from the cluster
// that index parity designates: for ic < jc the lower index owns the pair
// when ic + jc is even, the higher one when it is odd, so every cluster owns
// about half of its partners on either side of its own index. A cluster's
// pairs with itself are kept in its own tile (slot pairs a < b).
// With a full list (half == 0) every cluster keeps all of its partners.
__device__ __forceinline__ bool owns_pair(int ic, int jc, int half) {
  return !half || jc == ic || ((ic < jc) != (((ic + jc) & 1) != 0));
}

// Periodic gap between two intervals along one axis (0 if they overlap).
__device__ __forceinline__ float axis_gap(float alo, float ahi, float blo, float bhi, float L) {
  float ca = 0.5f * (alo + ahi), cb = 0.5f * (blo + bhi);
  float d = fabsf(cb - ca);
  d = fminf(d, L - d);
  return fmaxf(0.f, d - 0.5f * (ahi - alo) - 0.5f * (bhi - blo));
}

// The image (image_code values) every pair of points of two boxes takes
// along one axis under min_image_h's rule, or 3 when pairs differ. Rounded
// subtraction is monotonic in each operand, so the differences of the box
// extremes bound every pair's.
__device__ __forceinline__ unsigned box_image(float ilo, float ihi, float jlo, float jhi,
                                              float hL) {
#pragma clang fp contract(off)
  const float smin = jlo - ihi, smax = jhi - ilo;
  if (smin > hL) return 1u;
  if (smax < -hL) return 2u;
  return (smax <= hL && smin >= -hL) ? 0u : 3u;
}

// bbox-passing j-clusters one i-cluster may have; an entry holds
// 4 * j-cluster + (its real atoms - 1), never negative, and its image byte
// the 6-bit image code all its pairs share, or kMixedImage
constexpr int kSearchCand = 1024;
constexpr int kSearchSegs = 64;     // (column, z segment) units handled per chunk
constexpr unsigned char kMixedImage = 0xff;

// Per-wave scratch of the tile search.
struct SearchLds {
  int cand[kSearchCand];
  unsigned char img[kSearchCand];
  int seg_first[kSearchSegs];        // per unit: first cluster,
  int seg_pre[kSearchSegs + 1];      // clusters before it
};

// Offsets of image_diff by image code (2 bits per axis), per block.
__device__ void fill_image_tables(float4* am, float4* cp, const CellGrid& cg) {
  for (int t = threadIdx.x; t < 64; t += blockDim.x) {
    float m[3], p[3];
    for (int d = 0; d < 3; ++d) {
      const unsigned code = ((unsigned)t >> (2 * d)) & 3u;
      m[d] = code == 1u ? -cg.L[d] : 0.f;
      p[d] = code == 2u ? cg.L[d] : 0.f;
    }
    am[t] = make_float4(m[0], m[1], m[2], 0.f);
    cp[t] = make_float4(p[0], p[1], p[2], 0.f);
  }
}

// First cluster in [lo, hi) whose value v(k) >= x (v nondecreasing).
__device__ __forceinline__ int first_ge(const float4* __restrict__ b, int lo, int hi, float x) {
  while (lo < hi) {
    int mid = (lo + hi) >> 1;
    if (b[mid].z < x) lo = mid + 1; else hi = mid;
  }
  return lo;
}
// First cluster in [lo, hi) whose value v(k) > x.
__device__ __forceinline__ int first_gt(const float4* __restrict__ b, int lo, int hi, float x) {
  while (lo < hi) {
    int mid = (lo + hi) >> 1;
    if (b[mid].z <= x) lo = mid + 1; else hi = mid;
  }
  return lo;
}

// One wave per i-cluster ic: (1) enumerate the j-clusters of the columns whose
// atoms come within reach of its box in x-y - inside a column only the
// z-sorted clusters that overlap the z reach left by that x-y distance (one
// or two periodic segments, table lookups) - and keep those the i-cluster
// owns (owns_pair) whose boxes come closer than r_nl (+ margin), with the
// periodic image all their pairs take if there is one; (2) test the 16 slot
// pairs of four candidate tiles at once (one lane per pair) with the exact
// predicate and the exclusions; tiles with a non-empty mask are appended to
// the i-cluster's list in enumeration order.
__device__ void search_cluster(const BuildArgs& a, int ic, SearchLds& sl, const float4* img_am,
                               const float4* img_cp) {
  int* const mycand = sl.cand;
  unsigned char* const myimg = sl.img;
  int* const seg_first = sl.seg_first;
  int* const seg_pre = sl.seg_pre;
  const int lane = threadIdx.x & (kWave - 1);
  const int nclu = a.meta[1];
  if (ic >= nclu) return;
  const float4 ilo = a.box_lo[ic], ihi = a.box_hi[ic];
  int ncand = 0;
  bool overflow = false;
  if (ilo.w > 0.f) {
    const float reach = a.cg.r_search;
    // column ranges (periodic) that can hold a box within reach
    int cx0 = (int)floorf((ilo.x - reach) * a.cg.inv_w[0]);
    int cx1 = (int)floorf((ihi.x + reach) * a.cg.inv_w[0]);
    int cy0 = (int)floorf((ilo.y - reach) * a.cg.inv_w[1]);
    int cy1 = (int)floorf((ihi.y + reach) * a.cg.inv_w[1]);
    int nx = min(cx1 - cx0 + 1, a.cg.n[0]);
    int ny = min(cy1 - cy0 + 1, a.cg.n[1]);
    if (nx == a.cg.n[0]) cx0 = 0;
    if (ny == a.cg.n[1]) cy0 = 0;
    const int ncols = nx * ny;
    const float reach2 = reach * reach;
    // z reach as up to two segments inside [0, L): one unit per column if
    // the full reach neither wraps nor spans the column, else two (per
    // column the reach shrinks with its x-y distance, and a unit may be empty)
    const float Lz = a.cg.L[2];
    const float margin = 1e-3f * reach;
    const int nseg =
        (ilo.z - reach - margin >= 0.f && ihi.z + reach + margin < Lz &&
         (ihi.z + reach + margin) - (ilo.z - reach - margin) < Lz) ? 1 : 2;
    const int nunits = ncols * nseg;
    for (int u0 = 0; u0 < nunits; u0 += kSearchSegs) {
      const int nu = min(kSearchSegs, nunits - u0);
      int cnt = 0, first = 0;
      if (lane < nu) {
        int u = u0 + lane;
        int t = u / nseg, sg = u - t * nseg;
        int x = cx0 + t % nx, y = cy0 + t / nx;
        x %= a.cg.n[0]; x += x < 0 ? a.cg.n[0] : 0;
        y %= a.cg.n[1]; y += y < 0 ? a.cg.n[1] : 0;
        int col = y * a.cg.n[0] + x;
        // the column's x-y gap to the i-box bounds the z reach it needs
        const float4 cxy = a.col_xy[col];
        float gap2 = 3e38f;
        if (cxy.x <= cxy.y) {
          const float gx = axis_gap(ilo.x, ihi.x, cxy.x, cxy.y, a.cg.L[0]);
          const float gy = axis_gap(ilo.y, ihi.y, cxy.z, cxy.w, a.cg.L[1]);
          gap2 = gx * gx + gy * gy;
        }
        if (gap2 < reach2) {
          const float zr = sqrtf(reach2 - gap2) + margin;
          const float za = ilo.z - zr, zb_ = ihi.z + zr;
          float sa[2], sz[2];
          bool two = true;
          if (zb_ - za >= Lz) {
            sa[0] = -1.f; sz[0] = 2.f * Lz; two = false;
          } else if (za < 0.f) {
            sa[0] = 0.f; sz[0] = zb_; sa[1] = za + Lz; sz[1] = 2.f * Lz;
          } else if (zb_ >= Lz) {
            sa[0] = za; sz[0] = 2.f * Lz; sa[1] = -1.f; sz[1] = zb_ - Lz;
          } else {
            sa[0] = za; sz[0] = zb_; two = false;
          }
          // clusters overlapping [sa, sz] (max z >= sa and min z <= sz),
          // from the column's lookup table one bin wider on each side: a
          // superset, the box test below removes the extra clusters
          const int2* zt = a.zbin + (size_t)col * (a.cg.nzb + 1);
          auto lower = [&](float z) {
            return min(max((int)floorf(z * a.cg.inv_zb) - 1, 0), a.cg.nzb);
          };
          auto upper = [&](float z) {
            return min(max((int)ceilf(z * a.cg.inv_zb) + 1, 0), a.cg.nzb);
          };
          if (sg == 0 || two) {
            int f = zt[lower(sa[sg])].x;
            int l = zt[upper(sz[sg])].y;
            if (sg == 1) {
              // the two segments sit at opposite ends of the column; a
              // cluster reaching into both is taken once, by segment 0
              const int f0 = zt[lower(sa[0])].x, l0 = zt[upper(sz[0])].y;
              if (sa[1] > sa[0]) f = max(f, l0);
              else l = min(l, f0);
            }
            first = f;
            cnt = max(0, l - f);
          }
        }
      }
      int v = cnt;
      for (int o = 1; o < kWave; o <<= 1) {
        int uu = __shfl_up(v, o, kWave);
        if (lane >= o) v += uu;
      }
      if (lane < nu) {
        seg_first[lane] = first;
        seg_pre[lane + 1] = v;
      }
      if (lane == 0) seg_pre[0] = 0;
      __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
      __builtin_amdgcn_wave_barrier();
      __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
      const int total = __shfl(v, nu - 1, kWave);
      // cluster f of the units, from a binary search over them
      auto cluster_of = [&](int f) {
        int lo = 0, hi = nu - 1;
        while (lo < hi) {
          int mid = (lo + hi + 1) >> 1;
          if (seg_pre[mid] <= f) lo = mid; else hi = mid - 1;
        }
        return seg_first[lo] + (f - seg_pre[lo]);
      };
      // the boxes of the next 64 clusters are loaded while the current ones
      // are tested
      int jcn = lane < total ? cluster_of(lane) : 0;
      float4 lon = lane < total ? a.box_lo[jcn] : make_float4(0.f, 0.f, 0.f, 0.f);
      float4 hin = lane < total ? a.box_hi[jcn] : make_float4(0.f, 0.f, 0.f, 0.f);
      for (int f0 = 0; f0 < total; f0 += kWave) {
        const int jc = jcn;
        const float4 jlo = lon, jhi = hin;
        const int fn = f0 + kWave + lane;
        if (fn < total) {
          jcn = cluster_of(fn);
          lon = a.box_lo[jcn];
          hin = a.box_hi[jcn];
        }
        bool pass = false;
        int nvj = 0;
        unsigned cimg = 0;
        if (f0 + lane < total) {
          nvj = (int)jlo.w;
          if (jlo.w > 0.f && owns_pair(ic, jc, a.half)) {
            float gx = axis_gap(ilo.x, ihi.x, jlo.x, jhi.x, a.cg.L[0]);
            float gy = axis_gap(ilo.y, ihi.y, jlo.y, jhi.y, a.cg.L[1]);
            float gz = axis_gap(ilo.z, ihi.z, jlo.z, jhi.z, a.cg.L[2]);
            pass = gx * gx + gy * gy + gz * gz < reach2;
            const unsigned bx = box_image(ilo.x, ihi.x, jlo.x, jhi.x, a.cg.hL[0]);
            const unsigned by = box_image(ilo.y, ihi.y, jlo.y, jhi.y, a.cg.hL[1]);
            const unsigned bz = box_image(ilo.z, ihi.z, jlo.z, jhi.z, a.cg.hL[2]);
            cimg = (bx == 3u || by == 3u || bz == 3u) ? kMixedImage : (bx | by << 2 | bz << 4);
          }
        }
        unsigned long long m = __ballot(pass);
        int before = __popcll(m & ((1ull << lane) - 1ull));
        if (pass) {
          int slot = ncand + before;
          if (slot < kSearchCand) {
            mycand[slot] = jc * kClusterSize + (nvj - 1);
            myimg[slot] = (unsigned char)cimg;
          }
        }
        ncand += __popcll(m);
      }
      __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
      __builtin_amdgcn_wave_barrier();
      __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    }
    if (ncand > kSearchCand) {
      overflow = true;
      ncand = kSearchCand;
    }
  }
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");

  // (2) masks: lane = (tile t of 4, i slot a, j slot b). Padding slots are
  // the last slots of a cluster (a slot is real iff its index in the cluster
  // is below the cluster's real-atom count). The i atom's excluded partners
  // are held as slot indices in registers (the list walk is the fallback
  // for atoms with more than four exclusions).
  const int t = lane >> 4, ia = (lane >> 2) & 3, b = lane & 3;
  const int si = ic * kClusterSize + ia;
  const bool ivalid = ia < (int)ilo.w;
  const float4 pi = a.xs[si];
  const float lmx = a.cg.L[0] - pi.x, lmy = a.cg.L[1] - pi.y, lmz = a.cg.L[2] - pi.z;
  int ex0 = -1, ex1 = -1, ex2 = -1, ex3 = -1;
  int eb = 0, ee = 0;
  if (ivalid) {
    const int ai = a.perm[si];
    eb = a.ex_start[ai];
    ee = a.ex_start[ai + 1];
    const int ne = ee - eb;
    if (ne > 0) ex0 = a.inv_perm[a.ex_idx[eb]];
    if (ne > 1) ex1 = a.inv_perm[a.ex_idx[eb + 1]];
    if (ne > 2) ex2 = a.inv_perm[a.ex_idx[eb + 2]];
    if (ne > 3) ex3 = a.inv_perm[a.ex_idx[eb + 3]];
  }
  const bool ex_more = ee - eb > 4;
  int count = 0;
  // Appends the tiles of the pairs in tk (bit 4a + b of tile t's mask is
  // lane 16t + 4a + b) with image code limg, in tile order.
  auto emit = [&](int jc, unsigned long long tk, unsigned limg) {
    const unsigned mask = (unsigned)((tk >> (16 * t)) & 0xffffull);
    const unsigned long long nonempty = __ballot(b == 0 && ia == 0 && mask != 0);
    const int before = __popcll(nonempty & ((1ull << lane) - 1ull));
    if (ia == 0 && b == 0 && mask != 0) {
      const int k = count + before;
      if (k < a.cap) {
        a.tiles[(size_t)ic * a.cap + k] = make_uint2((unsigned)jc, mask | limg << 16);
        if (a.in_count) {
          // the tile's j partials (jpart at ic * cap + k) belong to jc
          const int r = atomicAdd(&a.in_count[jc], 1);
          if (r < a.cap) {
            a.in_fill[(size_t)jc * a.cap + r] = ic * a.cap + k;
          } else {
            atomicOr(a.flags, MDX_FLAG_NL_OVERFLOW);
            atomicMax(a.nl_needed, r + 1);
          }
        }
      }
    }
    count += __popcll(nonempty);
  };
  // One group of four candidate tiles: c = this lane's candidate entry (-1
  // past the end), cimg its image byte, pj its j slot's position.
  auto group = [&](int c, unsigned cimg, float4 pj) {
    const int jc = c >= 0 ? c / kClusterSize : -1;
    const int nv = c >= 0 ? c % kClusterSize + 1 : 0;
    // every candidate of the group with one image for all its pairs: the
    // differences from the image table (rounded as min_image_h rounds them)
    const bool shared = __ballot(c >= 0 && cimg == kMixedImage) == 0ull;
    const int sj = jc * kClusterSize + b;
    // the cluster's own tile: slot pairs a < b (half list) or a != b
    const bool cand =
        (jc >= 0) & ivalid & (b < nv) & ((jc != ic) | (b > ia) | (!a.half & (b < ia)));
    if (shared) {
      // Without branches: every lane forms its pair's difference and the
      // predicate (candidate, within r_nl, not excluded) decides its bit;
      // only atoms with more than four exclusions walk their list.
      float dx, dy, dz;
      if (__ballot(cimg != 0u) == 0ull) {   // no candidate of the group wraps
        dx = plain_diff(pi.x, pj.x);
        dy = plain_diff(pi.y, pj.y);
        dz = plain_diff(pi.z, pj.z);
      } else {
        const float4 am = img_am[cimg], cp = img_cp[cimg];
        dx = image_diff(pi.x, pj.x, am.x, cp.x);
        dy = image_diff(pi.y, pj.y, am.y, cp.y);
        dz = image_diff(pi.z, pj.z, am.z, cp.z);
      }
      const bool within = cand & (dist2(dx, dy, dz) < a.cg.rnl2);
      bool excluded = (sj == ex0) | (sj == ex1) | (sj == ex2) | (sj == ex3);
      const bool walk = within & ex_more & !excluded;
      if (__ballot(walk) != 0ull && walk) {
        const int aj = a.perm[sj];
        for (int k = eb + 4; k < ee; ++k) excluded |= (a.ex_idx[k] == aj);
      }
      emit(jc, __ballot(within & !excluded), cimg);
      return;
    }
    unsigned bit = 0, img = 0;
    if (cand) {
      const float dx = min_image_h(pi.x, lmx, pj.x, a.cg.L[0], a.cg.hL[0]);
      const float dy = min_image_h(pi.y, lmy, pj.y, a.cg.L[1], a.cg.hL[1]);
      const float dz = min_image_h(pi.z, lmz, pj.z, a.cg.L[2], a.cg.hL[2]);
      if (dist2(dx, dy, dz) < a.cg.rnl2) {
        bool excluded = sj == ex0 || sj == ex1 || sj == ex2 || sj == ex3;
        if (ex_more && !excluded) {
          const int aj = a.perm[sj];
          for (int k = eb + 4; k < ee; ++k) excluded |= (a.ex_idx[k] == aj);
        }
        bit = excluded ? 0u : 1u;
        img = image_code(pi.x, pj.x, a.cg.hL[0]) | image_code(pi.y, pj.y, a.cg.hL[1]) << 2 |
              image_code(pi.z, pj.z, a.cg.hL[2]) << 4;
      }
    }
    unsigned long long rem = __ballot(bit != 0);
    // One tile entry per periodic image among a tile's pairs (several only
    // in a box small next to the clusters and the list radius): in each
    // round, the pairs sharing the image of the tile's first remaining pair.
    while (rem) {
      const unsigned tm = (unsigned)((rem >> (16 * t)) & 0xffffull);
      const int lead = 16 * t + (tm ? __ffs(tm) - 1 : 0);
      const unsigned limg = (unsigned)__shfl((int)img, lead, kWave);
      const unsigned long long tk = __ballot(((rem >> lane) & 1ull) && img == limg);
      emit(jc, tk, limg);
      rem &= ~tk;
    }
  };
  // two groups per iteration with fixed registers: the j positions of the
  // next group of each half are in flight while a group is tested
  auto cand_at = [&](int g) { return (g + t < ncand) ? mycand[g + t] : -1; };
  auto img_at = [&](int g) { return (g + t < ncand) ? (unsigned)myimg[g + t] : 0u; };
  // unconditional loads (slot b of cluster 0 past the end, ignored there):
  // a load under a branch makes the compiler wait for every load in flight
  // before the group, including the prefetched one (2 % of the search)
  auto pos_of = [&](int c) { return a.xs[(c >= 0 ? (c & ~(kClusterSize - 1)) : 0) + b]; };
  int cA = cand_at(0), cB = cand_at(4);
  unsigned iA = img_at(0), iB = img_at(4);
  float4 pA = pos_of(cA), pB = pos_of(cB);
  for (int g = 0; g < ncand; g += 8) {
    group(cA, iA, pA);
    cA = cand_at(g + 8);
    iA = img_at(g + 8);
    pA = pos_of(cA);
    if (g + 4 < ncand) group(cB, iB, pB);
    cB = cand_at(g + 12);
    iB = img_at(g + 12);
    pB = pos_of(cB);
  }
  // pad the list to whole groups of four tiles with empty tiles (mask 0)
  const int kept = count < a.cap ? count : a.cap;
  const int padded = min((kept + 3) & ~3, a.cap);
  if (lane < padded - kept) a.tiles[(size_t)ic * a.cap + kept + lane] = make_uint2(0u, 0u);
  if (lane == 0) {
    a.tile_count[ic] = padded;
    // only a cluster whose tiles fill more than two thirds of the capacity
    // reports its count (one device-scope atomic per wave on one address
    // would serialize): an explicit build then grows the list ahead of the
    // rebuilds inside mdx_integrate_step, which cannot grow it
    if (count > a.cap - a.cap / 3) atomicMax(a.nl_needed, count);
    if (count > a.cap) atomicOr(a.flags, MDX_FLAG_NL_OVERFLOW);
    if (overflow) atomicOr(a.flags, MDX_FLAG_CELL_OVERFLOW);
  }
}

// ---- one kernel per phase ---------------------------------------------------
// Binning; the last block to finish (counted in meta[3]) runs the scan.
// Half list: no tile is listed under any j-cluster before the tile search.
__device__ __forceinline__ void clear_in_counts(const BuildArgs& a, int tid, int nthreads) {
  if (!a.in_count) return;
  for (int c = tid; c < a.max_clusters; c += nthreads) a.in_count[c] = 0;
}

__global__ void __launch_bounds__(256) k_bin_scan(BuildArgs a) {
  if (gated_off(a.gate)) return;
  __shared__ int last;
  clear_in_counts(a, blockIdx.x * blockDim.x + threadIdx.x, gridDim.x * blockDim.x);
  const bool by_slot = bin_by_slot(a);
  bin_atom(a, bin_atom_at(a, by_slot, blockIdx.x * blockDim.x + threadIdx.x));
  // The counts are atomics whose results every lane has received before the
  // barrier; one device-scope release per block (not a cache write-back per
  // wave) orders them before the block is counted, and the last block's
  // acquire before the scan reads them.
  __syncthreads();
  if (threadIdx.x == 0)
    last = __hip_atomic_fetch_add(&a.meta[3], 1, __ATOMIC_ACQ_REL, __HIP_MEMORY_SCOPE_AGENT) ==
           (int)gridDim.x - 1;
  __syncthreads();
  if (!last) return;
  scan_columns(a);
  if (threadIdx.x == 0) a.meta[3] = 0;
}

__global__ void __launch_bounds__(kColThreads) k_col_sort(BuildArgs a) {
  if (gated_off(a.gate)) return;
  __shared__ float2 st[kColStage];   // (build z, atom index bits)
  sort_column_boxes(a, blockIdx.x, st);
}

__global__ void __launch_bounds__(256) k_tile_search(BuildArgs a) {
  if (gated_off(a.gate)) return;
  __shared__ SearchLds sl[4];
  __shared__ float4 img_am[64], img_cp[64];
  fill_image_tables(img_am, img_cp, a.cg);
  __syncthreads();
  const int w = threadIdx.x / kWave;
  // neighbouring i-clusters on one XCD: their candidates come from one region
  const int lb = xcd_block((a.meta[1] + 3) / 4);
  if (lb < 0) return;
  search_cluster(a, lb * 4 + w, sl[w], img_am, img_cp);
}

// ---- all phases in one cooperative launch ------------------------------------
// Every block runs every phase (grid-stride loops) with grid-wide barriers in
// between; the gate test comes first and is the same for all blocks, so
// either every block reaches every barrier or none does.
constexpr int kBuildThreads = 256;

__global__ void __launch_bounds__(kBuildThreads) k_build_all(BuildArgs a) {
  if (gated_off(a.gate)) return;
  cooperative_groups::grid_group grid = cooperative_groups::this_grid();
  __shared__ float2 st[kColStage];
  __shared__ SearchLds sl[4];
  __shared__ float4 img_am[64], img_cp[64];
  fill_image_tables(img_am, img_cp, a.cg);
  __syncthreads();
  const int nthreads = gridDim.x * blockDim.x;
  const int tid = blockIdx.x * blockDim.x + threadIdx.x;
  // bounds rounded to whole blocks: the atom loops stay uniform per wave
  const bool by_slot = bin_by_slot(a);
  const int nround = (bin_count(a, by_slot) + blockDim.x - 1) / blockDim.x * blockDim.x;
  clear_in_counts(a, tid, nthreads);
  // every block has read meta before the barrier after the binning, and the
  // scan (block 0) writes it after that barrier
  for (int j = tid; j < nround; j += nthreads) bin_atom(a, bin_atom_at(a, by_slot, j));
  grid.sync();
  if (blockIdx.x == 0) scan_columns(a);
  grid.sync();
  for (int c = blockIdx.x; c < a.cg.ncell; c += gridDim.x) sort_column_boxes(a, c, st);
  grid.sync();
  const int w = threadIdx.x / kWave;
  for (int ic = blockIdx.x * 4 + w; ic < a.max_clusters; ic += gridDim.x * 4)
    search_cluster(a, ic, sl[w], img_am, img_cp);
}

int build_coop_blocks(int max_clusters, int n, int ncol) {
  int dev = 0, coop = 0, ncu = 0, per_cu = 0;
  if (hipGetDevice(&dev) != hipSuccess) return 0;
  if (hipDeviceGetAttribute(&coop, hipDeviceAttributeCooperativeLaunch, dev) != hipSuccess ||
      !coop)
    return 0;
  if (hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess)
    return 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k_build_all, kBuildThreads, 0) !=
          hipSuccess ||
      per_cu <= 0)
    return 0;
  const int useful = std::max({(n + kBuildThreads - 1) / kBuildThreads, ncol,
                               (max_clusters + 3) / 4, 1});
  return std::min(per_cu * ncu, useful);
}

// Copy the current positions into the slot array and test the list's
// validity: an atom that moved more than r_g/2 since the build invalidates
// the list (Sec. II.A.2) and latches NL_STALE.
__global__ void k_refresh(const float* __restrict__ pos, const int* __restrict__ perm,
                          const float* __restrict__ q, const float* __restrict__ x_build,
                          const int* __restrict__ meta, int n, CellGrid cg, float half_skin2,
                          float4* __restrict__ xs, unsigned* __restrict__ flags) {
  int s = blockIdx.x * blockDim.x + threadIdx.x;
  if (s >= meta[0]) return;
  int a = perm[s];
  if (a < 0) return;
  float x = pos[a], y = pos[n + a], z = pos[2 * n + a];
  bool inside = x >= 0.f && x < cg.L[0] && y >= 0.f && y < cg.L[1] && z >= 0.f && z < cg.L[2];
  const float bx = x_build[a], by = x_build[n + a], bz = x_build[2 * n + a];
  float dx = min_image(bx, x, cg.L[0], cg.hL[0]);
  float dy = min_image(by, y, cg.L[1], cg.hL[1]);
  float dz = min_image(bz, z, cg.L[2], cg.hL[2]);
  // continued from the build position, as the list's tile images require
  xs[s] = make_float4(bx + dx, by + dy, bz + dz, q[a]);
  unsigned f = 0;
  if (dist2(dx, dy, dz) > half_skin2) f |= MDX_FLAG_NL_STALE;
  if (!inside) f |= MDX_FLAG_OUT_OF_BOX;
  if (f) atomicOr(flags, f);
}

hipError_t launch_build_list(Ctx& c, const float* pos, const int* gate, hipEvent_t done) {
  hipStream_t s = c.stream;
  const int n = c.n;
  const int ncol = c.cg.ncell;
  BuildArgs a{gate, pos, n, c.cg, c.cell_of, c.cell_count, c.x_build, c.flags,
              c.cell_start, c.slot_start, c.meta, c.nl_needed,
              c.col_atoms, c.col_cap, c.q, c.atype, c.perm, c.inv_perm, c.xs, c.ts, c.zb,
              c.box_lo, c.box_hi, c.col_xy,
              ZRangeArgs{c.zb, c.slot_start, c.cell_start, c.brick_z,
                         c.has_pme ? c.pg.nb[2] : 0, ncol, c.cg.L[2], c.brick_zr},
              c.ex_start, c.ex_idx, c.nl_cap, c.half_list ? 1 : 0, c.zbin, c.tiles,
              c.tile_count, c.max_clusters, c.in_count, c.in_fill};
  if (c.coop_blocks > 0) {
    void* args[] = {&a};
    hipError_t e = hipLaunchCooperativeKernel(reinterpret_cast<const void*>(k_build_all),
                                              dim3(c.coop_blocks), dim3(kBuildThreads), args, 0, s);
    if (e == hipSuccess && done) e = hipEventRecord(done, s);
    return e;
  }
  // binning in slot order visits up to max_slots entries
  const int nb = (std::max(n, c.max_slots) + 255) / 256;
  k_bin_scan<<<nb, 256, 0, s>>>(a);
  k_col_sort<<<ncol, kColThreads, 0, s>>>(a);
  // `done` is recorded by the tile search's own dispatch (the slot positions
  // and the PME brick ranges were complete after the column sort; work
  // forked from here starts together with the force kernel)
  const int sb = xcd_grid((c.max_clusters + 3) / 4);
  if (done && !c.capturing) {
    void* args[] = {&a};
    return hipExtLaunchKernel(reinterpret_cast<const void*>(k_tile_search), dim3(sb), dim3(256),
                              args, 0, s, nullptr, done, 0);
  }
  k_tile_search<<<sb, 256, 0, s>>>(a);
  // under graph capture the event becomes a dependency edge after the search
  if (done) return hipEventRecord(done, s);
  return hipGetLastError();
}

hipError_t launch_refresh_sorted(Ctx& c, const float* pos) {
  float h = 0.5f * c.r_ghost;
  k_refresh<<<(c.max_slots + 255) / 256, 256, 0, c.stream>>>(pos, c.perm, c.q, c.x_build, c.meta,
                                                             c.n, c.cg, h * h, c.xs, c.flags);
  return hipGetLastError();
}

}  // namespace mdx
