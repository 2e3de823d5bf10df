// Cell-list Verlet neighbour list (DIMOS Sec. II.A.2, "Neighborlists").
//
// Build = bin atoms into cells of edge >= r_nl / m -> counting sort by cell
// (histogram, one-block scan, scatter, per-cell rank sort by caller index so
// the order is a pure function of (cell, atom index)) -> per-atom search of
// the (2m+1)^3 stencil with the float32 predicate of mdx.h. The list is a
// full (both directions) ELL array nl[k * npad + i] of sorted slot indices,
// so the k-th entries of 64 consecutive atoms are one coalesced 256-byte row.
#include "mdx_internal.h"

namespace mdx {

__global__ void k_fill_i32(int* __restrict__ p, int v, int count) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < count) p[i] = v;
}

__global__ void k_copy_f32(float* __restrict__ d, const float* __restrict__ s, int count) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < count) d[i] = s[i];
}

hipError_t launch_fill_i32(int* p, int v, int count, hipStream_t s) {
  if (count <= 0) return hipSuccess;
  k_fill_i32<<<(count + 255) / 256, 256, 0, s>>>(p, v, count);
  return hipGetLastError();
}

hipError_t launch_copy_f32(float* dst, const float* src, int count, hipStream_t s) {
  if (count <= 0) return hipSuccess;
  k_copy_f32<<<(count + 255) / 256, 256, 0, s>>>(dst, src, count);
  return hipGetLastError();
}

__device__ __forceinline__ int bin_coord(float x, float inv_w, int n) {
  int c = (int)(x * inv_w);          // x >= 0: truncation is floor
  c = c < 0 ? 0 : c;
  return c >= n ? n - 1 : c;
}

__device__ __forceinline__ bool gated_off(const int* gate) { return gate && *gate == 0; }

__global__ void k_prepare(const int* __restrict__ gate, int* __restrict__ cell_count, int ncell,
                          int* __restrict__ nl_needed) {
  if (gated_off(gate)) return;
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < ncell) cell_count[i] = 0;
  if (i == 0) *nl_needed = 0;
}

// Bin every caller atom, count atoms per cell, snapshot the build positions.
__global__ void k_bin(const int* __restrict__ gate, const float* __restrict__ pos, int n,
                      CellGrid cg, int* __restrict__ cell_of, int* __restrict__ cell_count,
                      float* __restrict__ x_build, unsigned* __restrict__ flags) {
  if (gated_off(gate)) return;
  int a = blockIdx.x * blockDim.x + threadIdx.x;
  if (a >= n) return;
  float x = pos[a], y = pos[n + a], z = pos[2 * n + a];
  bool inside = x >= 0.f && x < cg.L[0] && y >= 0.f && y < cg.L[1] && z >= 0.f && z < cg.L[2];
  if (!inside) atomicOr(flags, MDX_FLAG_OUT_OF_BOX);
  int cx = bin_coord(x, cg.inv_w[0], cg.n[0]);
  int cy = bin_coord(y, cg.inv_w[1], cg.n[1]);
  int cz = bin_coord(z, cg.inv_w[2], cg.n[2]);
  int c = (cz * cg.n[1] + cy) * cg.n[0] + cx;
  cell_of[a] = c;
  atomicAdd(&cell_count[c], 1);
  x_build[a] = x;
  x_build[n + a] = y;
  x_build[2 * n + a] = z;
}

// Exclusive scan of the cell counts in one 1024-thread block: each thread
// sums a contiguous chunk, a wave-level shuffle scan combines the chunk sums.
__global__ void __launch_bounds__(1024) k_scan(const int* __restrict__ gate,
                                               const int* __restrict__ count, int ncell,
                                               int* __restrict__ start, int* __restrict__ cursor) {
  if (gated_off(gate)) return;
  __shared__ int wave_tot[16];
  int t = threadIdx.x;
  int chunk = (ncell + blockDim.x - 1) / blockDim.x;
  int b = t * chunk, e = min(b + chunk, ncell);
  int s = 0;
  for (int i = b; i < e; ++i) s += count[i];
  // inclusive scan of s across the wave
  int lane = t & (kWave - 1), w = t / kWave;
  int v = s;
  for (int o = 1; o < kWave; o <<= 1) {
    int u = __shfl_up(v, o, kWave);
    if (lane >= o) v += u;
  }
  if (lane == kWave - 1) wave_tot[w] = v;
  __syncthreads();
  if (t == 0) {
    int acc = 0;
    for (int i = 0; i < (int)(blockDim.x / kWave); ++i) {
      int tmp = wave_tot[i];
      wave_tot[i] = acc;
      acc += tmp;
    }
  }
  __syncthreads();
  int run = wave_tot[w] + v - s;   // exclusive prefix of this thread's chunk
  for (int i = b; i < e; ++i) {
    start[i] = run;
    cursor[i] = run;
    run += count[i];
  }
  if (e == ncell && b < e) start[ncell] = run;
  if (ncell == 0 && t == 0) start[0] = 0;
}

__global__ void k_scatter(const int* __restrict__ gate, const int* __restrict__ cell_of, int n,
                          int* __restrict__ cursor, int* __restrict__ perm_unsorted) {
  if (gated_off(gate)) return;
  int a = blockIdx.x * blockDim.x + threadIdx.x;
  if (a >= n) return;
  int slot = atomicAdd(&cursor[cell_of[a]], 1);
  perm_unsorted[slot] = a;
}

// One wave per cell: rank every atom of the cell by caller index (stable
// order independent of the scatter's atomic order), then write the sorted
// slot data.
__global__ void k_cell_sort(const int* __restrict__ gate, const int* __restrict__ cell_start,
                            int ncell, const int* __restrict__ perm_unsorted,
                            const float* __restrict__ pos, int n, const float* __restrict__ q,
                            const int* __restrict__ atype, int* __restrict__ perm,
                            int* __restrict__ inv_perm, int* __restrict__ cell_sorted,
                            float4* __restrict__ xs, int* __restrict__ ts) {
  if (gated_off(gate)) return;
  int c = blockIdx.x * (blockDim.x / kWave) + threadIdx.x / kWave;
  int lane = threadIdx.x & (kWave - 1);
  if (c >= ncell) return;
  int b = cell_start[c], e = cell_start[c + 1];
  int cnt = e - b;
  for (int p = lane; p < cnt; p += kWave) {
    int v = perm_unsorted[b + p];
    int rank = 0;
    for (int k = 0; k < cnt; ++k) rank += perm_unsorted[b + k] < v ? 1 : 0;
    int s = b + rank;
    perm[s] = v;
    inv_perm[v] = s;
    cell_sorted[s] = c;
    xs[s] = make_float4(pos[v], pos[n + v], pos[2 * n + v], q[v]);
    ts[s] = atype[v];
  }
}

// Stencil search: one thread per sorted atom i.
__global__ void __launch_bounds__(256) k_nl_search(
    const int* __restrict__ gate, const float4* __restrict__ xs, const int* __restrict__ cell_sorted,
    const int* __restrict__ cell_start, const int* __restrict__ perm,
    const int* __restrict__ ex_start, const int* __restrict__ ex_idx, int n, int npad, int cap,
    CellGrid cg, int* __restrict__ nl, int* __restrict__ nl_count, int* __restrict__ nl_needed,
    unsigned* __restrict__ flags) {
  if (gated_off(gate)) return;
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  float4 pi = xs[i];
  int ci = cell_sorted[i];
  int cx = ci % cg.n[0], cy = (ci / cg.n[0]) % cg.n[1], cz = ci / (cg.n[0] * cg.n[1]);
  int a = perm[i];
  int eb = ex_start[a], ee = ex_start[a + 1];
  int cnt = 0;
  for (int oz = 0; oz < cg.nofs[2]; ++oz) {
    int z = cz + cg.ofs[2][oz];
    z += z < 0 ? cg.n[2] : 0;
    z -= z >= cg.n[2] ? cg.n[2] : 0;
    for (int oy = 0; oy < cg.nofs[1]; ++oy) {
      int y = cy + cg.ofs[1][oy];
      y += y < 0 ? cg.n[1] : 0;
      y -= y >= cg.n[1] ? cg.n[1] : 0;
      int row = (z * cg.n[1] + y) * cg.n[0];
      for (int ox = 0; ox < cg.nofs[0]; ++ox) {
        int x = cx + cg.ofs[0][ox];
        x += x < 0 ? cg.n[0] : 0;
        x -= x >= cg.n[0] ? cg.n[0] : 0;
        int c = row + x;
        int jb = cell_start[c], je = cell_start[c + 1];
        for (int j = jb; j < je; ++j) {
          if (j == i) continue;
          float4 pj = xs[j];
          float dx = min_image(pi.x, pj.x, cg.L[0], cg.hL[0]);
          float dy = min_image(pi.y, pj.y, cg.L[1], cg.hL[1]);
          float dz = min_image(pi.z, pj.z, cg.L[2], cg.hL[2]);
          float r2 = dist2(dx, dy, dz);
          if (r2 < cg.rnl2) {
            bool excluded = false;
            if (ee > eb) {
              int bj = perm[j];
              for (int k = eb; k < ee; ++k) excluded |= (ex_idx[k] == bj);
            }
            if (!excluded) {
              if (cnt < cap) nl[(size_t)cnt * npad + i] = j;
              ++cnt;
            }
          }
        }
      }
    }
  }
  nl_count[i] = cnt < cap ? cnt : cap;
  if (cnt > cap) {
    atomicOr(flags, MDX_FLAG_NL_OVERFLOW);
  }
  atomicMax(nl_needed, cnt);
}

// Copy the current positions into the sorted float4 array and test the
// list's validity: an atom that moved more than r_g/2 since the build
// invalidates the list (Sec. II.A.2). Without a gate this latches
// NL_STALE; with one it requests a rebuild before the forces are taken.
__global__ void k_refresh(const float* __restrict__ pos, const int* __restrict__ perm,
                          const float* __restrict__ q, const float* __restrict__ x_build, int n,
                          CellGrid cg, float half_skin2, float4* __restrict__ xs,
                          unsigned* __restrict__ flags, int* __restrict__ gate,
                          int force_rebuild) {
  int s = blockIdx.x * blockDim.x + threadIdx.x;
  if (gate && force_rebuild && s == 0) *gate = 1;
  if (s >= n) return;
  int a = perm[s];
  float x = pos[a], y = pos[n + a], z = pos[2 * n + a];
  xs[s] = make_float4(x, y, z, q[a]);
  bool inside = x >= 0.f && x < cg.L[0] && y >= 0.f && y < cg.L[1] && z >= 0.f && z < cg.L[2];
  float dx = min_image(x_build[a], x, cg.L[0], cg.hL[0]);
  float dy = min_image(x_build[n + a], y, cg.L[1], cg.hL[1]);
  float dz = min_image(x_build[2 * n + a], z, cg.L[2], cg.hL[2]);
  bool stale = dist2(dx, dy, dz) > half_skin2;
  unsigned f = 0;
  if (stale) {
    if (gate) atomicOr(gate, 1);
    else f |= MDX_FLAG_NL_STALE;
  }
  if (!inside) f |= MDX_FLAG_OUT_OF_BOX;
  if (f) atomicOr(flags, f);
}

hipError_t launch_build_list(Ctx& c, const float* pos, const int* gate) {
  hipStream_t s = c.stream;
  const int n = c.n;
  const int nb = (n + 255) / 256;
  const int ncell = c.cg.ncell;
  k_prepare<<<(ncell + 255) / 256, 256, 0, s>>>(gate, c.cell_count, ncell, c.nl_needed);
  k_bin<<<nb, 256, 0, s>>>(gate, pos, n, c.cg, c.cell_of, c.cell_count, c.x_build, c.flags);
  k_scan<<<1, 1024, 0, s>>>(gate, c.cell_count, ncell, c.cell_start, c.cell_cursor);
  k_scatter<<<nb, 256, 0, s>>>(gate, c.cell_of, n, c.cell_cursor, c.perm_unsorted);
  k_cell_sort<<<(ncell + 3) / 4, 256, 0, s>>>(gate, c.cell_start, ncell, c.perm_unsorted, pos, n,
                                              c.q, c.atype, c.perm, c.inv_perm, c.cell_sorted,
                                              c.xs, c.ts);
  k_nl_search<<<nb, 256, 0, s>>>(gate, c.xs, c.cell_sorted, c.cell_start, c.perm, c.ex_start,
                                 c.ex_idx, n, c.npad, c.nl_cap, c.cg, c.nl, c.nl_count,
                                 c.nl_needed, c.flags);
  return hipGetLastError();
}

hipError_t launch_refresh_sorted(Ctx& c, const float* pos, int* gate, bool force_rebuild) {
  const int n = c.n;
  float h = 0.5f * c.r_ghost;
  k_refresh<<<(n + 255) / 256, 256, 0, c.stream>>>(pos, c.perm, c.q, c.x_build, n, c.cg, h * h,
                                                   c.xs, c.flags, gate, force_rebuild ? 1 : 0);
  return hipGetLastError();
}

}  // namespace mdx
