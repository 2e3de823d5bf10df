// Host runtime and C ABI (mdx.h): descriptor validation, one-time device
// allocation, the cell/PME geometry, and the call sequences of each entry
// point. Everything computed per step runs in the kernels of nl.hip,
// nonbonded.hip, pme.hip and integrate.hip.
#include <algorithm>
#include <cmath>
#include <complex>
#include <cstdio>
#include <cstring>
#include <new>
#include <set>
#include <utility>
#include <vector>

#include "mdx_internal.h"

struct mdx_ctx {
  mdx::Ctx c;
  std::vector<void*> allocs;
  // event pairs per timing group, reused across recordings
  unsigned timing = 0;   // bit g: record group g
  std::vector<std::pair<hipEvent_t, hipEvent_t>> ev[3];
  size_t used[3] = {0, 0, 0};
  // second stream for the PME potential inside mdx_integrate_step, forked
  // from and joined back into the context's stream every step
  hipStream_t aux = nullptr;
  hipEvent_t ev_fork = nullptr, ev_join = nullptr;
  // graph replay of integrate_step chunks (mdx_set_graph): the chunk length,
  // the stream captures are recorded on, the instantiated graph and what it
  // was captured for
  int graph_chunk = 0;
  hipStream_t cap = nullptr;
  hipGraph_t graph = nullptr;
  hipGraphExec_t gexec = nullptr;
  struct GraphKey {
    const float* pos = nullptr;
    const float* vel = nullptr;
    const float* force = nullptr;
    float dt = 0.f;
    uint64_t version = 0;
    int steps_since_build = -2;
  } gkey;
  int64_t graph_launches = 0;
};

namespace {

using mdx::Ctx;

#define MDX_TRY(expr)                               \
  do {                                              \
    hipError_t _e = (expr);                         \
    if (_e != hipSuccess) return MDX_E_HIP;         \
  } while (0)

template <typename T>
int dev_alloc(mdx_ctx* x, T** p, size_t count) {
  *p = nullptr;
  if (count == 0) count = 1;
  void* q = nullptr;
  hipError_t e = hipMalloc(&q, count * sizeof(T));
  if (e != hipSuccess) {
    (void)hipGetLastError();
    return MDX_E_OUT_OF_MEMORY;
  }
  x->allocs.push_back(q);
  *p = static_cast<T*>(q);
  return MDX_OK;
}

template <typename T>
int dev_upload(mdx_ctx* x, T** p, const std::vector<T>& h) {
  int rc = dev_alloc(x, p, h.size());
  if (rc != MDX_OK) return rc;
  if (!h.empty() && hipMemcpy(*p, h.data(), h.size() * sizeof(T), hipMemcpyHostToDevice) != hipSuccess)
    return MDX_E_HIP;
  return MDX_OK;
}

void dev_free(mdx_ctx* x, void* p) {
  if (!p) return;
  auto it = std::find(x->allocs.begin(), x->allocs.end(), p);
  if (it != x->allocs.end()) x->allocs.erase(it);
  (void)hipFree(p);
}

// v with zeros appended up to m entries. The closing kernel reads entry 0 of
// each topology array (and members 0..2 of term 0) whether or not an atom
// has terms of that kind, so these arrays are never empty.
template <typename T>
std::vector<T> padded(std::vector<T> v, size_t m) {
  if (v.size() < m) v.resize(m, T(0));
  return v;
}

// CSR of per-atom item lists from (atom, item) pairs.
void build_csr(int n, const std::vector<std::pair<int, int>>& items, std::vector<int>& start,
               std::vector<int>& idx) {
  start.assign(n + 1, 0);
  for (auto& p : items) start[p.first + 1]++;
  for (int i = 0; i < n; ++i) start[i + 1] += start[i];
  idx.assign(items.size(), 0);
  std::vector<int> cur(start.begin(), start.end() - 1);
  for (auto& p : items) idx[cur[p.first]++] = p.second;
  for (int i = 0; i < n; ++i) std::sort(idx.begin() + start[i], idx.begin() + start[i + 1]);
}

// Cubic B-spline value at the integers 1, 2, 3 (uniform basis).
double m4_at(int k) { return k == 2 ? 2.0 / 3.0 : (k == 1 || k == 3 ? 1.0 / 6.0 : 0.0); }

// Tiles per i-cluster: clusters whose boxes lie within r_list of a box of
// edge ~a, with headroom.
int default_capacity(int n, const float box[3], float r_list, double a, int max_clusters,
                     bool full_list) {
  double V = (double)box[0] * box[1] * box[2];
  double rho = n / V;
  double r = (double)r_list + a;
  // clusters whose boxes reach within r_list; a half list holds each pair
  // once. The build regrows a list whose largest per-cluster count passes two
  // thirds of the capacity, and the largest count runs above this mean, so
  // the capacity starts at 2.25 times it.
  double expect = (full_list ? 1.0 : 0.5) * rho * 4.0 / 3.0 * M_PI * r * r * r /
                  mdx::kClusterSize;
  int cap = (int)std::ceil(2.25 * expect + 16.0);
  cap = (cap + 15) / 16 * 16;
  // in a box small next to r_list a j-cluster can take one tile per periodic
  // image its pairs use, so the bound is a few times the cluster count
  return std::max(16, std::min(cap, (4 * max_clusters + 15) / 16 * 16));
}

// LJ type-pair tables from the current per-type sigma and epsilon (Eqs. 4-5,
// FP64 mixing): the force kernel's (c12, c6, 12 c12, 6 c6) in float32 and
// (c12, c6) in FP64, and the reverse pass's parameter-derivative factors
// (per ordered type pair, for the i end: a = sqrt(eps_tj / eps_ti) / 2,
// 0 when eps_ti = 0):
//   force: (48 a s^12, 24 a s^6, 288 eps s^11, 72 eps s^5)
//   energy: (4 a s^12, 4 a s^6, 24 eps s^11, 12 eps s^5)
// uploaded into the context's tables (allocated on the first call).
int upload_lj_tables(mdx_ctx* x) {
  Ctx& c = x->c;
  const int T = c.n_types;
  std::vector<float4> ljf((size_t)T * T), adf((size_t)T * T);
  std::vector<double2> ljd((size_t)T * T);
  std::vector<double4> add((size_t)T * T);
  for (int a = 0; a < T; ++a)
    for (int b = 0; b < T; ++b) {
      const double ea = c.eps_h[a], eb = c.eps_h[b];
      double sig = 0.5 * ((double)c.sig_h[a] + (double)c.sig_h[b]);
      double eps = std::sqrt(std::max(0.0, ea * eb));
      double s6 = sig * sig * sig * sig * sig * sig;
      double c6 = 4.0 * eps * s6, c12 = 4.0 * eps * s6 * s6;
      const size_t k = (size_t)a * T + b;
      ljf[k] = make_float4((float)c12, (float)c6, (float)(12.0 * c12), (float)(6.0 * c6));
      ljd[k] = make_double2(c12, c6);
      const double at = ea > 0.0 ? 0.5 * std::sqrt(std::max(0.0, eb) / ea) : 0.0;
      const double s5 = s6 / sig, s11 = s6 * s5, s12 = s6 * s6;
      adf[k] = make_float4((float)(48.0 * at * s12), (float)(24.0 * at * s6),
                           (float)(288.0 * eps * s11), (float)(72.0 * eps * s5));
      add[k] = make_double4(4.0 * at * s12, 4.0 * at * s6, 24.0 * eps * s11, 12.0 * eps * s5);
    }
  int rc;
  if (!c.lj_f) {
    if ((rc = dev_alloc(x, &c.lj_f, ljf.size())) != MDX_OK) return rc;
    if ((rc = dev_alloc(x, &c.lj_d, ljd.size())) != MDX_OK) return rc;
    if ((rc = dev_alloc(x, &c.adj.lj_f, adf.size())) != MDX_OK) return rc;
    if ((rc = dev_alloc(x, &c.adj.lj_d, add.size())) != MDX_OK) return rc;
  }
  MDX_TRY(hipMemcpy(c.lj_f, ljf.data(), sizeof(float4) * ljf.size(), hipMemcpyHostToDevice));
  MDX_TRY(hipMemcpy(c.lj_d, ljd.data(), sizeof(double2) * ljd.size(), hipMemcpyHostToDevice));
  MDX_TRY(hipMemcpy(c.adj.lj_f, adf.data(), sizeof(float4) * adf.size(), hipMemcpyHostToDevice));
  MDX_TRY(hipMemcpy(c.adj.lj_d, add.data(), sizeof(double4) * add.size(), hipMemcpyHostToDevice));
  return MDX_OK;
}

// Eq. 12 times k_e plus the neutralising term, from the current charges.
double self_energy(const Ctx& c) {
  if (!c.has_coulomb) return 0.0;
  double q2 = 0.0, qsum = 0.0;
  for (float q : c.q_h) {
    q2 += (double)q * q;
    qsum += q;
  }
  const double V = (double)c.box[0] * c.box[1] * c.box[2];
  return -c.coulomb_k * c.alpha / std::sqrt(M_PI) * q2 -
         c.coulomb_k * M_PI * qsum * qsum / (2.0 * V * c.alpha * c.alpha);
}

int alloc_list(mdx_ctx* x, int cap) {
  Ctx& c = x->c;
  cap = std::max(4, (cap + 3) / 4 * 4);   // lists are padded to groups of four tiles
  dev_free(x, c.tiles);
  dev_free(x, c.ptiles);
  dev_free(x, c.jpart);
  dev_free(x, c.ppos);
  dev_free(x, c.in_fill);
  dev_free(x, c.in_sorted);
  c.tiles = nullptr;
  c.ptiles = nullptr;
  c.jpart = nullptr;
  c.ppos = nullptr;
  c.in_fill = nullptr;
  c.in_sorted = nullptr;
  c.version++;   // a graph captured before holds the old addresses
  const size_t nt = (size_t)cap * c.max_clusters;
  int rc = dev_alloc(x, &c.tiles, nt);
  if (rc != MDX_OK) return rc;
  if ((rc = dev_alloc(x, &c.ptiles, nt)) != MDX_OK) return rc;
  if (c.half_list) {
    if ((rc = dev_alloc(x, &c.jpart, 12 * nt)) != MDX_OK) return rc;
    if ((rc = dev_alloc(x, &c.ppos, nt)) != MDX_OK) return rc;
    if ((rc = dev_alloc(x, &c.in_fill, nt)) != MDX_OK) return rc;
    if ((rc = dev_alloc(x, &c.in_sorted, nt)) != MDX_OK) return rc;
    if (!c.in_count) {
      if ((rc = dev_alloc(x, &c.in_count, (size_t)c.max_clusters)) != MDX_OK) return rc;
    }
    // no list yet: nothing listed as anyone's j-cluster
    MDX_TRY(hipMemset(c.in_count, 0, sizeof(int) * c.max_clusters));
    MDX_TRY(hipMemset(c.jpart, 0, sizeof(float) * 12 * nt));
  }
  c.nl_cap = cap;
  return MDX_OK;
}

int setup_pme(mdx_ctx* x, const mdx_system_desc* d) {
  Ctx& c = x->c;
  mdx::PmeGrid& g = c.pg;
  for (int k = 0; k < 3; ++k) {
    g.K[k] = d->pme_grid[k];
    g.B[k] = std::min(k < 2 ? mdx::kBrickXY : mdx::kBrickZ, g.K[k]);
    g.nb[k] = (g.K[k] + g.B[k] - 1) / g.B[k];
    double s = (double)g.K[k] / (double)c.box[k];
    g.scale_hi[k] = (float)s;
    g.scale_lo[k] = (float)(s - (double)g.scale_hi[k]);
  }
  g.Kxh = g.K[0] / 2 + 1;
  g.nbrick = g.nb[0] * g.nb[1] * g.nb[2];
  g.disp_max = (float)(0.5 * (double)c.r_ghost * 1.001 + 1e-3);

  // Per brick index: the columns (along x and y) and the build-z range that can
  // hold an atom whose spline support reaches the brick, allowing r_g/2 of
  // motion since the build.
  std::vector<int> bc;
  std::vector<float> bz;
  int maxc[2] = {0, 0};
  for (int k = 0; k < 3; ++k) {
    double L = c.box[k], h = L / g.K[k];
    for (int b = 0; b < g.nb[k]; ++b) {
      int g0 = b * g.B[k];
      int beff = std::min(g.B[k], g.K[k] - g0);
      double lo = g0 * h - g.disp_max;
      double hi = (g0 + beff + 3) * h + g.disp_max;
      if (k < 2) {
        double w = L / c.cg.n[k];
        long first = (long)std::floor(lo / w);
        long last = (long)std::floor(hi / w);
        long count = last - first + 1;
        if (count >= c.cg.n[k]) {
          first = 0;
          count = c.cg.n[k];
        }
        first = ((first % c.cg.n[k]) + c.cg.n[k]) % c.cg.n[k];
        bc.push_back((int)first);
        bc.push_back((int)count);
        maxc[k] = std::max(maxc[k], (int)count);
      } else {
        if (hi - lo >= L) {
          lo = 0.0;
          hi = L;
        }
        bz.push_back((float)lo);
        bz.push_back((float)hi);
      }
    }
  }
  if ((long)maxc[0] * maxc[1] > 256) return MDX_E_UNSUPPORTED;
  int rc = dev_upload(x, &c.brick_cols, bc);
  if (rc != MDX_OK) return rc;
  if ((rc = dev_upload(x, &c.brick_z, bz)) != MDX_OK) return rc;
  if ((rc = dev_alloc(x, &c.brick_zr, (size_t)g.nb[2] * c.cg.ncell)) != MDX_OK) return rc;

  std::vector<double> bmh[3], mrh[3];
  for (int k = 0; k < 3; ++k) {
    const int K = g.K[k];
    std::vector<float2> tw(K);
    for (int m = 0; m < K; ++m) {
      double a = -2.0 * M_PI * m / K;
      tw[m] = make_float2((float)std::cos(a), (float)std::sin(a));
    }
    std::vector<double> bm(K), mr(K);
    for (int m = 0; m < K; ++m) {
      std::complex<double> s(0.0, 0.0);
      for (int t = 0; t <= 2; ++t)
        s += m4_at(t + 1) * std::exp(std::complex<double>(0.0, 2.0 * M_PI * m * t / K));
      bm[m] = 1.0 / std::norm(s);
      int mp = (m <= K / 2) ? m : m - K;
      mr[m] = (double)mp / (double)c.box[k];
    }
    if ((rc = dev_upload(x, &c.tw[k], tw)) != MDX_OK) return rc;
    if ((rc = dev_upload(x, &c.bmod[k], bm)) != MDX_OK) return rc;
    if ((rc = dev_upload(x, &c.mrec[k], mr)) != MDX_OK) return rc;
    bmh[k] = bm;
    mrh[k] = mr;
  }
  {
    // the influence function on the half spectrum, in the z pass's order
    // [ky][kx][kz]: G(m) = B(m) exp(-pi^2 m^2 / alpha^2) / m^2 (smooth PME,
    // Sec. II.A.2)
    const double exp_fac = M_PI * M_PI / (c.alpha * c.alpha);
    std::vector<double> gt((size_t)g.K[1] * g.Kxh * g.K[2], 0.0);
    for (int ky = 0; ky < g.K[1]; ++ky)
      for (int kx = 0; kx < g.Kxh; ++kx)
        for (int kz = 0; kz < g.K[2]; ++kz) {
          const double msq =
              mrh[0][kx] * mrh[0][kx] + mrh[1][ky] * mrh[1][ky] + mrh[2][kz] * mrh[2][kz];
          if (msq > 0.0)
            gt[((size_t)ky * g.Kxh + kx) * g.K[2] + kz] =
                bmh[0][kx] * bmh[1][ky] * bmh[2][kz] * std::exp(-exp_fac * msq) / msq;
        }
    if ((rc = dev_upload(x, &c.pme_g, gt)) != MDX_OK) return rc;
  }
  c.pme_energy_scale = 1.0 / (M_PI * (double)c.box[0] * c.box[1] * c.box[2]);
  size_t ng = (size_t)g.K[0] * g.K[1] * g.K[2];
  if ((rc = dev_alloc(x, &c.grid_q, ng)) != MDX_OK) return rc;
  if ((rc = dev_alloc(x, &c.grid_phi, ng)) != MDX_OK) return rc;
  if ((rc = dev_alloc(x, &c.grid_c, (size_t)g.Kxh * g.K[1] * g.K[2])) != MDX_OK) return rc;
  return MDX_OK;
}

int create_impl(mdx_ctx* x, const mdx_system_desc* d) {
  Ctx& c = x->c;
  const int n = d->n_atoms;
  if (d->n_types > mdx::kMaxLjTypes || n > mdx::kMaxAtoms) return MDX_E_UNSUPPORTED;
  if (n <= 0 || !d->charge || !d->mass || !d->atom_type || d->n_types <= 0 || !d->type_sigma ||
      !d->type_epsilon)
    return MDX_E_INVALID;
  for (int k = 0; k < 3; ++k)
    if (!(d->box[k] > 0.f) || !std::isfinite(d->box[k])) return MDX_E_INVALID;
  if (!(d->r_cut > 0.f) || !(d->r_ghost >= 0.f)) return MDX_E_INVALID;
  if ((d->n_exclusions > 0 && !d->exclusions) || d->n_exclusions < 0) return MDX_E_INVALID;
  if ((d->n_bonds > 0 && (!d->bonds || !d->bond_k || !d->bond_r0)) || d->n_bonds < 0)
    return MDX_E_INVALID;
  if ((d->n_angles > 0 && (!d->angles || !d->angle_k || !d->angle_theta0)) || d->n_angles < 0)
    return MDX_E_INVALID;
  for (int i = 0; i < n; ++i) {
    if (d->atom_type[i] < 0 || d->atom_type[i] >= d->n_types) return MDX_E_INVALID;
    if (!(d->mass[i] > 0.f)) return MDX_E_INVALID;
  }
  if (d->options & ~(MDX_OPT_HALF_LIST | MDX_OPT_COOPERATIVE_BUILD | MDX_OPT_KAHAN_VV))
    return MDX_E_INVALID;
  const int cdiv = d->cell_divisions == 0 ? 2 : d->cell_divisions;
  if (cdiv < 1 || cdiv > 4) return MDX_E_INVALID;
  if (d->switch_r > 0.f && !(d->switch_r < d->r_cut)) return MDX_E_INVALID;

  c.n = n;
  for (int k = 0; k < 3; ++k) c.box[k] = d->box[k];
  c.r_cut = d->r_cut;
  c.r_ghost = d->r_ghost;
  c.r_list = d->r_cut + d->r_ghost;   // float32 sum
  c.switch_r = d->switch_r;
  c.has_switch = d->switch_r > 0.f;
  c.coulomb_k = d->coulomb_k;
  c.accel = d->accel > 0 ? d->accel : 1.0;
  c.boltzmann = d->boltzmann;
  c.cell_div = cdiv;
  c.half_list = (d->options & MDX_OPT_HALF_LIST) != 0;
  c.rebuild_every = d->rebuild_every > 0 ? d->rebuild_every : 10;
  for (int k = 0; k < 3; ++k)
    if ((double)c.r_list > 0.5 * (double)c.box[k]) return MDX_E_BOX_TOO_SMALL;

  // Ewald splitting parameter: explicit, or Eq. 13 from the tolerance.
  if (d->ewald_alpha > 0.0) c.alpha = d->ewald_alpha;
  else if (d->ewald_delta > 0.0) {
    if (d->ewald_delta >= 0.5) return MDX_E_INVALID;
    c.alpha = std::sqrt(-std::log(2.0 * d->ewald_delta)) / (double)d->r_cut;
  } else c.alpha = 0.0;
  bool any_q = false;
  for (int i = 0; i < n; ++i) any_q |= d->charge[i] != 0.f;
  c.has_coulomb = c.alpha > 0.0 && d->coulomb_k != 0.0 && any_q;
  const bool want_pme = d->pme_grid[0] > 0 || d->pme_grid[1] > 0 || d->pme_grid[2] > 0;
  // reaction field (Eq. 8, with eps_s in both constants): no Ewald parts
  if (!(d->rf_epsilon >= 0.0)) return MDX_E_INVALID;
  if (d->rf_epsilon > 0.0) {
    if (d->ewald_alpha > 0.0 || d->ewald_delta > 0.0 || want_pme) return MDX_E_INVALID;
    const double rc = (double)d->r_cut, es = d->rf_epsilon;
    if (std::isinf(es)) {
      c.k_rf = 1.0 / (2.0 * rc * rc * rc);
      c.c_rf = 3.0 / (2.0 * rc);
    } else {
      c.k_rf = (es - 1.0) / ((2.0 * es + 1.0) * rc * rc * rc);
      c.c_rf = 3.0 * es / ((2.0 * es + 1.0) * rc);
    }
    c.rf = d->coulomb_k != 0.0 && any_q;
  }
  if (want_pme) {
    if (d->pme_order != 4 && d->pme_order != 0) return MDX_E_UNSUPPORTED;
    for (int k = 0; k < 3; ++k)
      if (!mdx::pme_size_supported(d->pme_grid[k])) return MDX_E_UNSUPPORTED;
    if (!(c.alpha > 0.0)) return MDX_E_INVALID;
  }
  c.has_pme = want_pme && c.has_coulomb;

  // ---- column grid and predicate constants ----
  // Columns of edge ~ the cube that holds one cluster of atoms (scaled by
  // 2/cell_divisions); the list does not depend on this choice.
  mdx::CellGrid& g = c.cg;
  const double rho = n / ((double)c.box[0] * c.box[1] * c.box[2]);
  const double a_clu = std::cbrt(mdx::kClusterSize / rho);
  const double wcol = a_clu * 2.0 / cdiv;
  g.ncell = 1;
  for (int k = 0; k < 3; ++k) {
    int nk = k < 2 ? (int)std::floor((double)c.box[k] / wcol) : 1;
    nk = std::max(1, std::min(nk, 4096));
    g.n[k] = nk;
    g.ncell *= nk;
    g.L[k] = c.box[k];
    g.hL[k] = c.box[k] * 0.5f;
    g.inv_w[k] = (float)nk / c.box[k];
  }
  g.rnl2 = c.r_list * c.r_list;
  g.rc2 = c.r_cut * c.r_cut;
  g.r_search = c.r_list * 1.001f + 1e-4f;
  // z bins of about half a cluster's height for the tile search's lookups
  g.nzb = std::max(1, std::min(1024, (int)std::ceil((double)c.box[2] / (0.5 * a_clu))));
  g.inv_zb = (float)g.nzb / c.box[2];
  c.max_slots = n + (mdx::kClusterSize - 1) * g.ncell;
  c.max_slots = (c.max_slots + mdx::kClusterSize - 1) / mdx::kClusterSize * mdx::kClusterSize;
  c.max_clusters = c.max_slots / mdx::kClusterSize;
  c.coop_blocks = (d->options & MDX_OPT_COOPERATIVE_BUILD)
                      ? mdx::build_coop_blocks(c.max_clusters, n, g.ncell)
                      : 0;

  // ---- per-atom parameters and the LJ type-pair table (Eqs. 4-5) ----
  std::vector<float> q(n), am(n), ms(n);
  std::vector<int> ty(n);
  for (int i = 0; i < n; ++i) {
    q[i] = c.has_coulomb || c.rf ? d->charge[i] : 0.f;
    ty[i] = d->atom_type[i];
    am[i] = (float)(c.accel / (double)d->mass[i]);
    ms[i] = d->mass[i];
  }
  const int T = d->n_types;
  c.n_types = T;
  c.sig_h.assign(d->type_sigma, d->type_sigma + T);
  c.eps_h.assign(d->type_epsilon, d->type_epsilon + T);
  c.q_h = q;
  c.e_self = self_energy(c);
  int rc;
  if ((rc = upload_lj_tables(x)) != MDX_OK) return rc;
  if ((rc = dev_upload(x, &c.q, q)) != MDX_OK) return rc;
  if ((rc = dev_upload(x, &c.atype, ty)) != MDX_OK) return rc;
  if ((rc = dev_upload(x, &c.hdt_scale, am)) != MDX_OK) return rc;
  if ((rc = dev_upload(x, &c.mass, ms)) != MDX_OK) return rc;
  c.mass_h = ms;

  // ---- topology ----
  std::set<std::pair<int, int>> ex;
  for (int e = 0; e < d->n_exclusions; ++e) {
    int a = d->exclusions[2 * e], b = d->exclusions[2 * e + 1];
    if (a < 0 || b < 0 || a >= n || b >= n || a == b) return MDX_E_INVALID;
    ex.insert({std::min(a, b), std::max(a, b)});
  }
  std::vector<std::pair<int, int>> items;
  for (auto& p : ex) {
    items.push_back({p.first, p.second});
    items.push_back({p.second, p.first});
  }
  std::vector<int> st, ix;
  build_csr(n, items, st, ix);
  c.n_excl = (int)ex.size();
  if ((rc = dev_upload(x, &c.ex_start, st)) != MDX_OK) return rc;
  if ((rc = dev_upload(x, &c.ex_idx, padded(ix, 1))) != MDX_OK) return rc;

  std::vector<int> bidx(2 * d->n_bonds);
  std::vector<float> bk(d->n_bonds), br(d->n_bonds);
  items.clear();
  for (int b = 0; b < d->n_bonds; ++b) {
    int i = d->bonds[2 * b], j = d->bonds[2 * b + 1];
    if (i < 0 || j < 0 || i >= n || j >= n || i == j) return MDX_E_INVALID;
    bidx[2 * b] = i;
    bidx[2 * b + 1] = j;
    bk[b] = d->bond_k[b];
    br[b] = d->bond_r0[b];
    items.push_back({i, b});
    items.push_back({j, b});
  }
  build_csr(n, items, st, ix);
  c.n_bonds = d->n_bonds;
  if ((rc = dev_upload(x, &c.bonds, padded(bidx, 2))) != MDX_OK) return rc;
  if ((rc = dev_upload(x, &c.bond_k, padded(bk, 1))) != MDX_OK) return rc;
  if ((rc = dev_upload(x, &c.bond_r0, padded(br, 1))) != MDX_OK) return rc;
  if ((rc = dev_upload(x, &c.bt_start, st)) != MDX_OK) return rc;
  if ((rc = dev_upload(x, &c.bt_idx, padded(ix, 1))) != MDX_OK) return rc;

  std::vector<int> aidx(3 * d->n_angles);
  std::vector<float> ak(d->n_angles), at(d->n_angles);
  items.clear();
  for (int a = 0; a < d->n_angles; ++a) {
    int i = d->angles[3 * a], j = d->angles[3 * a + 1], l = d->angles[3 * a + 2];
    if (i < 0 || j < 0 || l < 0 || i >= n || j >= n || l >= n || i == j || j == l || i == l)
      return MDX_E_INVALID;
    aidx[3 * a] = i;
    aidx[3 * a + 1] = j;
    aidx[3 * a + 2] = l;
    ak[a] = d->angle_k[a];
    at[a] = d->angle_theta0[a];
    items.push_back({i, a});
    items.push_back({j, a});
    items.push_back({l, a});
  }
  build_csr(n, items, st, ix);
  c.n_angles = d->n_angles;
  if ((rc = dev_upload(x, &c.angles, padded(aidx, 3))) != MDX_OK) return rc;
  if ((rc = dev_upload(x, &c.angle_k, padded(ak, 1))) != MDX_OK) return rc;
  if ((rc = dev_upload(x, &c.angle_t0, padded(at, 1))) != MDX_OK) return rc;
  if ((rc = dev_upload(x, &c.at_start, st)) != MDX_OK) return rc;
  if ((rc = dev_upload(x, &c.at_idx, padded(ix, 1))) != MDX_OK) return rc;

  // ---- column sort, cluster slots and tile list storage ----
  const int ncol = g.ncell;
  if ((rc = dev_alloc(x, &c.cell_of, n)) != MDX_OK) return rc;
  if ((rc = dev_alloc(x, &c.cell_count, ncol)) != MDX_OK) return rc;
  MDX_TRY(hipMemset(c.cell_count, 0, sizeof(int) * ncol));
  if ((rc = dev_alloc(x, &c.cell_start, ncol + 1)) != MDX_OK) return rc;
  if ((rc = dev_alloc(x, &c.slot_start, ncol + 1)) != MDX_OK) return rc;
  // meta: slots, clusters, builds, binning blocks done, slot-order binning
  // allowed (meta[4]); padded to 8
  if ((rc = dev_alloc(x, &c.meta, 8)) != MDX_OK) return rc;
  MDX_TRY(hipMemset(c.meta, 0, 8 * sizeof(int)));
  // atoms binned per column: twice the mean with headroom (a column that
  // overflows latches MDX_FLAG_COLUMN_OVERFLOW; mdx_build_neighbors grows it)
  c.col_cap = std::min(n, std::max(64, 2 * ((n + ncol - 1) / ncol) + 32));
  if ((rc = dev_alloc(x, &c.col_atoms, (size_t)ncol * c.col_cap)) != MDX_OK) return rc;
  if ((rc = dev_alloc(x, &c.perm, c.max_slots)) != MDX_OK) return rc;
  MDX_TRY(hipMemset(c.perm, 0xff, sizeof(int) * c.max_slots));   // every slot empty (-1)
  if ((rc = dev_alloc(x, &c.inv_perm, n)) != MDX_OK) return rc;
  // an atom a column could not hold keeps its previous slot: a valid index
  MDX_TRY(hipMemset(c.inv_perm, 0, sizeof(int) * n));
  if ((rc = dev_alloc(x, &c.xs, c.max_slots)) != MDX_OK) return rc;
  if ((rc = dev_alloc(x, &c.zbin, (size_t)ncol * (g.nzb + 1))) != MDX_OK) return rc;
  if ((rc = dev_alloc(x, &c.fslot, (size_t)3 * c.max_slots)) != MDX_OK) return rc;
  MDX_TRY(hipMemset(c.fslot, 0, sizeof(float) * 3 * c.max_slots));
  if (mdx::side_terms_used(c) && (rc = dev_alloc(x, &c.fside, (size_t)3 * c.max_slots)) != MDX_OK)
    return rc;
  if ((rc = dev_alloc(x, &c.ts, c.max_slots)) != MDX_OK) return rc;
  if ((rc = dev_alloc(x, &c.zb, c.max_slots)) != MDX_OK) return rc;
  if ((rc = dev_alloc(x, &c.box_lo, c.max_clusters)) != MDX_OK) return rc;
  if ((rc = dev_alloc(x, &c.box_hi, c.max_clusters)) != MDX_OK) return rc;
  if ((rc = dev_alloc(x, &c.col_xy, ncol)) != MDX_OK) return rc;
  if ((rc = dev_alloc(x, &c.img, (size_t)3 * n)) != MDX_OK) return rc;
  if ((rc = dev_alloc(x, &c.pos_alt, (size_t)3 * n)) != MDX_OK) return rc;
  MDX_TRY(hipMemset(c.pos_alt, 0, sizeof(float) * 3 * (size_t)n));
  MDX_TRY(hipMemset(c.img, 0, sizeof(int) * 3 * (size_t)n));
  if (d->options & MDX_OPT_KAHAN_VV) {
    if ((rc = dev_alloc(x, &c.xc, (size_t)3 * n)) != MDX_OK) return rc;
    if ((rc = dev_alloc(x, &c.vc, (size_t)3 * n)) != MDX_OK) return rc;
    MDX_TRY(hipMemset(c.xc, 0, sizeof(float) * 3 * (size_t)n));
    MDX_TRY(hipMemset(c.vc, 0, sizeof(float) * 3 * (size_t)n));
  }
  if ((rc = dev_alloc(x, &c.x_build, (size_t)3 * n)) != MDX_OK) return rc;
  if ((rc = dev_alloc(x, &c.tile_count, c.max_clusters)) != MDX_OK) return rc;
  if ((rc = dev_alloc(x, &c.nl_needed, 1)) != MDX_OK) return rc;
  if ((rc = dev_alloc(x, &c.flags, 1)) != MDX_OK) return rc;
  MDX_TRY(hipMemset(c.flags, 0, sizeof(unsigned)));
  if ((rc = dev_alloc(x, &c.gate, 4)) != MDX_OK) return rc;
  {
    const int g0[4] = {0, 0, 1, 1};   // no pruned list yet
    MDX_TRY(hipMemcpy(c.gate, g0, sizeof(g0), hipMemcpyHostToDevice));
  }
  if ((rc = dev_alloc(x, &c.pcount, c.max_clusters)) != MDX_OK) return rc;
  MDX_TRY(hipMemset(c.pcount, 0, sizeof(int) * c.max_clusters));
  if ((rc = dev_alloc(x, &c.xp, c.max_slots)) != MDX_OK) return rc;
  MDX_TRY(hipMemset(c.xp, 0, sizeof(float4) * c.max_slots));
  {
    const float rp = c.r_cut + 0.4f * c.r_ghost;
    const float mv = 0.19f * c.r_ghost;
    c.prune_r2 = rp * rp;
    c.prune_move2 = mv * mv;
  }
  int cap = d->nl_capacity > 0 ? d->nl_capacity
                               : default_capacity(n, c.box, c.r_list, a_clu, c.max_clusters,
                                                   !c.half_list);
  if ((rc = alloc_list(x, cap)) != MDX_OK) return rc;

  if (c.has_pme) {
    if ((rc = setup_pme(x, d)) != MDX_OK) return rc;
  }
  // ---- reductions ----
  // partial rows hold one entry per block of the widest energy kernel
  int mb = std::max({(n + 255) / 256, mdx::xcd_grid((c.max_clusters + 3) / 4),
                     mdx::xcd_grid((c.max_slots * 4 + 255) / 256)});
  if (c.has_pme) {
    const int pc = mdx::pme_col_pencils(c.pg.Kxh);
    int ntile = (c.pg.Kxh + pc - 1) / pc;
    mb = std::max(mb, c.pg.K[1] * ntile);
  }
  c.max_blocks = mb;
  if ((rc = dev_alloc(x, &c.partials, (size_t)mdx::kRowCount * mb)) != MDX_OK) return rc;
  MDX_TRY(hipMemset(c.partials, 0, sizeof(double) * mdx::kRowCount * mb));
  if ((rc = dev_alloc(x, &c.energy_scratch, MDX_N_ENERGY)) != MDX_OK) return rc;
  MDX_TRY(hipDeviceSynchronize());
  return MDX_OK;
}

int check_ctx(mdx_ctx* x) { return x ? MDX_OK : MDX_E_INVALID; }

constexpr size_t kMaxTimed = 8192;

// Event pairs of the timed groups. timing_slot hands out the next pair of
// `group` (*slot = nullptr unless the group is recorded) for a caller that
// has a dispatch record them; timing_begin also records the first event on
// `stream` (close the interval with timing_end); timed() brackets the
// launches made by `fn`.
hipError_t timing_slot(mdx_ctx* x, int group, std::pair<hipEvent_t, hipEvent_t>** slot) {
  *slot = nullptr;
  if (!((x->timing >> group) & 1u) || x->used[group] >= kMaxTimed) return hipSuccess;
  auto& v = x->ev[group];
  if (x->used[group] == v.size()) {
    hipEvent_t a, b;
    hipError_t e = hipEventCreate(&a);
    if (e != hipSuccess) return e;
    if ((e = hipEventCreate(&b)) != hipSuccess) return e;
    v.push_back({a, b});
  }
  *slot = &v[x->used[group]++];
  return hipSuccess;
}

hipError_t timing_begin(mdx_ctx* x, int group, hipStream_t stream,
                        std::pair<hipEvent_t, hipEvent_t>** slot) {
  hipError_t e = timing_slot(x, group, slot);
  if (e != hipSuccess || !*slot) return e;
  return hipEventRecord((*slot)->first, stream);
}

hipError_t timing_end(std::pair<hipEvent_t, hipEvent_t>* slot, hipStream_t stream) {
  return slot ? hipEventRecord(slot->second, stream) : hipSuccess;
}

template <typename F>
hipError_t timed(mdx_ctx* x, int group, hipStream_t stream, F&& fn) {
  std::pair<hipEvent_t, hipEvent_t>* slot;
  hipError_t e = timing_begin(x, group, stream, &slot);
  if (e != hipSuccess) return e;
  if ((e = fn()) != hipSuccess) return e;
  return timing_end(slot, stream);
}

}  // namespace

extern "C" {

const char* mdx_error_string(int code) {
  switch (code) {
    case MDX_OK: return "ok";
    case MDX_E_INVALID: return "invalid argument";
    case MDX_E_BOX_TOO_SMALL: return "box too small: r_cut + r_ghost exceeds half a box edge";
    case MDX_E_HIP: return "HIP runtime error";
    case MDX_E_CAPACITY: return "caller buffer too small";
    case MDX_E_NO_LIST: return "no neighbour list: call mdx_build_neighbors first";
    case MDX_E_NO_PME: return "PME not configured for this context";
    case MDX_E_OUT_OF_MEMORY: return "device allocation failed";
    case MDX_E_UNSUPPORTED: return "unsupported option";
    default: return "unknown error";
  }
}

int mdx_create(mdx_ctx** out, const mdx_system_desc* d, void* hip_stream) {
  if (!out) return MDX_E_INVALID;
  *out = nullptr;
  if (!d) return MDX_E_INVALID;
  mdx_ctx* x = new (std::nothrow) mdx_ctx();
  if (!x) return MDX_E_OUT_OF_MEMORY;
  if (hipGetDevice(&x->c.device) != hipSuccess) {
    delete x;
    return MDX_E_HIP;
  }
  x->c.stream = static_cast<hipStream_t>(hip_stream);
  // these events only order the two streams on this device: no timestamps,
  // and a device-scope release (not a system-scope one, which writes the
  // caches back for the host) when they are recorded
  const unsigned ev_flags = hipEventDisableTiming | hipEventReleaseToDevice;
  if (hipStreamCreateWithFlags(&x->aux, hipStreamNonBlocking) != hipSuccess ||
      hipEventCreateWithFlags(&x->ev_fork, ev_flags) != hipSuccess ||
      hipEventCreateWithFlags(&x->ev_join, ev_flags) != hipSuccess) {
    mdx_destroy(x);
    return MDX_E_HIP;
  }
  int rc = create_impl(x, d);
  if (rc != MDX_OK) {
    mdx_destroy(x);
    return rc;
  }
  // the device address of the fixed scratch array of
  // mdx_compute_ewald_direct_noalloc (once per device)
  if (mdx::ewald_scratch_setup(x->c.device) != hipSuccess) {
    mdx_destroy(x);
    return MDX_E_HIP;
  }
  *out = x;
  return MDX_OK;
}

int mdx_destroy(mdx_ctx* x) {
  if (!x) return MDX_OK;
  (void)hipStreamSynchronize(x->c.stream);
  if (x->aux) {
    (void)hipStreamSynchronize(x->aux);
    (void)hipStreamDestroy(x->aux);
  }
  if (x->ev_fork) (void)hipEventDestroy(x->ev_fork);
  if (x->ev_join) (void)hipEventDestroy(x->ev_join);
  if (x->gexec) (void)hipGraphExecDestroy(x->gexec);
  if (x->graph) (void)hipGraphDestroy(x->graph);
  if (x->cap) (void)hipStreamDestroy(x->cap);
  for (auto& v : x->ev)
    for (auto& p : v) {
      (void)hipEventDestroy(p.first);
      (void)hipEventDestroy(p.second);
    }
  for (void* p : x->allocs) (void)hipFree(p);
  delete x;
  return MDX_OK;
}

int mdx_set_stream(mdx_ctx* x, void* hip_stream) {
  if (check_ctx(x)) return MDX_E_INVALID;
  x->c.stream = static_cast<hipStream_t>(hip_stream);
  return MDX_OK;
}

int mdx_build_neighbors(mdx_ctx* x, const float* pos) {
  if (check_ctx(x) || !pos) return MDX_E_INVALID;
  Ctx& c = x->c;
  // a new list (new slot order) invalidates the pruned list
  MDX_TRY(mdx::launch_fill_i32(c.gate + 2, 1, 2, c.stream));
  // a new state: the Kahan compensation starts again from zero (all-zero
  // bits are 0.0f)
  if (c.xc) {
    MDX_TRY(mdx::launch_fill_i32(reinterpret_cast<int*>(c.xc), 0, 3 * c.n, c.stream));
    MDX_TRY(mdx::launch_fill_i32(reinterpret_cast<int*>(c.vc), 0, 3 * c.n, c.stream));
  }
  // A column list grows by doubling up to n atoms (where it cannot
  // overflow), the tile list to 1.5 times the largest count the build
  // reported when that count overflows or fills more than two thirds of the
  // capacity (headroom for the rebuilds inside mdx_integrate_step, which
  // cannot grow it), so this ends after a few attempts.
  for (int attempt = 0; attempt < 40; ++attempt) {
    MDX_TRY(timed(x, MDX_TIMING_BUILD, c.stream, [&] { return mdx::launch_build_list(c, pos); }));
    int needed = 0;
    MDX_TRY(hipMemcpyAsync(&needed, c.nl_needed, sizeof(int), hipMemcpyDeviceToHost, c.stream));
    MDX_TRY(hipStreamSynchronize(c.stream));
    c.steps_since_build = 0;
    unsigned fl = 0;
    MDX_TRY(hipMemcpy(&fl, c.flags, sizeof(unsigned), hipMemcpyDeviceToHost));
    if (fl & MDX_FLAG_CELL_OVERFLOW) return MDX_E_UNSUPPORTED;
    if (fl & MDX_FLAG_COLUMN_OVERFLOW) {
      c.version++;
      dev_free(x, c.col_atoms);
      c.col_atoms = nullptr;
      c.col_cap = std::min(c.n, 2 * c.col_cap);
      int rc = dev_alloc(x, &c.col_atoms, (size_t)c.cg.ncell * c.col_cap);
      if (rc != MDX_OK) return rc;
      // the tile count of an incomplete list says nothing: build again first
    } else if (needed <= c.nl_cap - c.nl_cap / 3) {
      return MDX_OK;
    } else {
      int rc = alloc_list(x, (needed + needed / 2 + 16 + 15) / 16 * 16);
      if (rc != MDX_OK) return rc;
    }
    // clear the overflow bits this build latched, and build again
    fl &= ~(MDX_FLAG_NL_OVERFLOW | MDX_FLAG_COLUMN_OVERFLOW);
    MDX_TRY(hipMemcpy(c.flags, &fl, sizeof(unsigned), hipMemcpyHostToDevice));
  }
  return MDX_E_HIP;
}

}  // extern "C"

namespace {

// Host copy of the last built list: slot permutation, tiles per cluster and
// the tiles themselves (synchronising).
struct HostList {
  int nslot = 0, nclu = 0, builds = 0;
  std::vector<int> perm, cnt;
  std::vector<uint2> tl;
};

int read_list(Ctx& c, HostList& h) {
  MDX_TRY(hipStreamSynchronize(c.stream));
  int meta[3];
  MDX_TRY(hipMemcpy(meta, c.meta, sizeof(meta), hipMemcpyDeviceToHost));
  h.nslot = meta[0];
  h.nclu = meta[1];
  h.builds = meta[2];
  h.perm.assign(h.nslot, 0);
  h.cnt.assign(h.nclu, 0);
  h.tl.assign((size_t)h.nclu * c.nl_cap, uint2{0u, 0u});
  if (h.nslot > 0) {
    MDX_TRY(hipMemcpy(h.perm.data(), c.perm, sizeof(int) * h.nslot, hipMemcpyDeviceToHost));
    MDX_TRY(hipMemcpy(h.cnt.data(), c.tile_count, sizeof(int) * h.nclu, hipMemcpyDeviceToHost));
    MDX_TRY(hipMemcpy(h.tl.data(), c.tiles, sizeof(uint2) * h.tl.size(), hipMemcpyDeviceToHost));
  }
  return MDX_OK;
}

}  // namespace

extern "C" {

int mdx_get_neighbor_pairs(mdx_ctx* x, int32_t* pairs_host, int64_t cap, int64_t* n_out) {
  if (check_ctx(x) || !n_out || cap < 0 || (cap > 0 && !pairs_host)) return MDX_E_INVALID;
  Ctx& c = x->c;
  if (c.steps_since_build < 0) return MDX_E_NO_LIST;
  HostList h;
  if (int rc = read_list(c, h)) return rc;
  const int nclu = h.nclu;
  const std::vector<int>& perm = h.perm;
  const std::vector<int>& cnt = h.cnt;
  const std::vector<uint2>& tl = h.tl;
  std::vector<std::pair<int, int>> pairs;
  for (int ic = 0; ic < nclu; ++ic)
    for (int k = 0; k < cnt[ic]; ++k) {
      const uint2 e = tl[(size_t)ic * c.nl_cap + k];
      for (int bit = 0; bit < 16; ++bit) {
        if (!((e.y >> bit) & 1u)) continue;
        int a = perm[ic * mdx::kClusterSize + bit / 4];
        int b = perm[(int)e.x * mdx::kClusterSize + bit % 4];
        // a full list holds both directions; a half list each pair once
        if (c.half_list || a < b) pairs.push_back({std::min(a, b), std::max(a, b)});
      }
    }
  std::sort(pairs.begin(), pairs.end());
  *n_out = (int64_t)pairs.size();
  if ((int64_t)pairs.size() > cap) return MDX_E_CAPACITY;
  for (size_t p = 0; p < pairs.size(); ++p) {
    pairs_host[2 * p] = pairs[p].first;
    pairs_host[2 * p + 1] = pairs[p].second;
  }
  return MDX_OK;
}

int mdx_compute_nonbonded(mdx_ctx* x, const float* pos, float* force, double* energy,
                          double* virial) {
  if (check_ctx(x) || !pos || !force) return MDX_E_INVALID;
  Ctx& c = x->c;
  if (c.steps_since_build < 0) return MDX_E_NO_LIST;
  const bool v = virial != nullptr;
  const bool e = energy != nullptr || v;
  MDX_TRY(mdx::launch_refresh_sorted(c, pos));
  MDX_TRY(timed(x, MDX_TIMING_PAIR, c.stream,
                [&] { return mdx::launch_nonbonded(c, e, nullptr, nullptr, v); }));
  MDX_TRY(mdx::launch_bonded_excl(c, pos, force, e, v));
  if (v) {
    const int row0[2] = {mdx::kRowVir, mdx::kRowVirB};
    const int nblk[2] = {c.nb_blocks, (c.n + 255) / 256};
    const double scale[2] = {1.0, 1.0};
    MDX_TRY(mdx::launch_reduce_virial(c, row0, nblk, scale, 2, virial));
  }
  if (energy) {
    const int nb = (c.n + 255) / 256;
    int rows[5] = {mdx::kRowLJ, mdx::kRowDir, mdx::kRowExcl, mdx::kRowBond, mdx::kRowAngle};
    int nblk[5] = {c.nb_blocks, c.nb_blocks, nb, nb, nb};
    MDX_TRY(mdx::launch_reduce_energy(c, rows, nblk, 5, energy, 0, c.e_self,
                                      MDX_ENERGY_COUL_SELF));
  }
  return MDX_OK;
}

int mdx_compute_pme(mdx_ctx* x, const float* pos, float* force, double* energy, double* virial) {
  if (check_ctx(x) || !pos || !force) return MDX_E_INVALID;
  Ctx& c = x->c;
  if (!c.has_pme) return MDX_E_NO_PME;
  if (c.steps_since_build < 0) return MDX_E_NO_LIST;
  MDX_TRY(mdx::launch_refresh_sorted(c, pos));
  MDX_TRY(timed(x, MDX_TIMING_PME, c.stream, [&] {
    return mdx::launch_pme(c, force, energy != nullptr, virial != nullptr);
  }));
  if (virial) {
    const int row0[1] = {mdx::kRowVir};
    const int nblk[1] = {c.pme_blocks};
    const double scale[1] = {0.5 * c.coulomb_k * c.pme_energy_scale};
    MDX_TRY(mdx::launch_reduce_virial(c, row0, nblk, scale, 1, virial));
  }
  if (energy) {
    int rows[1] = {mdx::kRowRec};
    int nblk[1] = {c.pme_blocks};
    MDX_TRY(mdx::launch_reduce_energy(c, rows, nblk, 1, energy, MDX_ENERGY_COUL_REC, 0.0, -1));
  }
  return MDX_OK;
}

}  // extern "C"

namespace {

// The steps of mdx_integrate_step as launches on the context's stream (and
// its second stream); under graph capture the same sequence is recorded.
int integrate_eager(mdx_ctx* x, float* pos, float* vel, float* force, int32_t n_steps,
                    float dt, double* energies) {
  Ctx& c = x->c;
  if (c.steps_since_build < 0) {
    MDX_TRY(mdx::launch_build_list(c, pos));
    c.steps_since_build = 0;
  }
  const bool e = energies != nullptr;
  // The list is rebuilt on the cadence, and in between whenever an atom has
  // moved more than r_g/2 since the last build: the opening half of a step
  // raises the step's gate, the build kernels run only if it is raised. Two
  // gates alternate with the step parity, so the kernel that clears the next
  // step's gate never touches the one being raised.
  auto gates_of = [&](int64_t step) {
    mdx::StepGates g;
    g.gate_now = c.gate + (step & 1);
    g.gate_next = c.gate + ((step + 1) & 1);
    g.pgate_now = g.gate_now + 2;
    g.pgate_next = g.gate_next + 2;
    g.cadence = ++c.steps_since_build >= c.rebuild_every;
    if (g.cadence) c.steps_since_build = 0;
    g.step = (long long)step;
    return g;
  };
  // The first step opens with its own kernel; every later one is opened by
  // the closing kernel of the step before, which reads the positions from
  // one buffer and writes the new ones to the other (the caller's array and
  // pos_alt, alternating); the last positions are copied back if needed.
  float* pos_cur = pos;
  float* pos_other = c.pos_alt;
  // Rigid water: every step opens with its own kernel, followed by the
  // position constraints, and closes with the velocity projection. When every
  // atom belongs to a rigid molecule the drift writes pos_alt and the
  // constraint kernel writes every position back to pos; otherwise pos_alt
  // keeps a copy of the positions before the drift, which happens in place.
  const bool rigid = c.n_rigid > 0;
  const bool rigid_all = 3 * (size_t)c.n_rigid == (size_t)c.n;   // molecules are disjoint
  auto open_rigid = [&](const mdx::StepGates& gs) -> hipError_t {
    if (rigid_all) {
      hipError_t err = mdx::launch_begin_step(c, pos, vel, force, dt, gs, c.pos_alt);
      if (err == hipSuccess) err = mdx::launch_rigid_positions(c, pos, c.pos_alt, pos, vel, dt, gs);
      return err;
    }
    hipError_t err = hipMemcpyAsync(c.pos_alt, pos, sizeof(float) * 3 * (size_t)c.n,
                                    hipMemcpyDeviceToDevice, c.stream);
    if (err == hipSuccess) err = mdx::launch_begin_step(c, pos, vel, force, dt, gs);
    if (err == hipSuccess) err = mdx::launch_rigid_positions(c, c.pos_alt, pos, pos, vel, dt, gs);
    return err;
  };
  int rigid_blocks = 0;   // blocks of the velocity projection's kinetic partials
  mdx::StepGates g = gates_of(c.steps_taken);
  if (rigid) MDX_TRY(open_rigid(g));
  else MDX_TRY(mdx::launch_begin_step(c, pos_cur, vel, force, dt, g));
  for (int s = 0; s < n_steps; ++s) {
    int* gate_now = g.gate_now;
    int* pgate_now = g.pgate_now;
    MDX_TRY(timed(x, MDX_TIMING_BUILD, c.stream, [&] {
      return mdx::launch_build_list(c, pos_cur, gate_now, c.has_pme ? x->ev_fork : nullptr);
    }));
    // The reciprocal-space potential only needs this step's slot positions
    // and the PME brick slot ranges: the spread and the FFT passes run on the
    // second stream, from the end of the list build on, concurrently with
    // the pair kernel. The PME force interpolation and the bonded and
    // exclusion terms do not need the pair forces either: they follow on the
    // second stream (side terms), beside the end of the pair kernel. The
    // closing kernel (pair-force add, kick, opening half) waits for them.
    // The fork and join events are recorded by the tile search's and the
    // side kernel's own dispatches (no marker packets between kernels).
    // (Below kSideStreamMinAtoms the second stream is the longer one already,
    // and the closing kernel evaluates those terms.)
    if (c.has_pme) {
      const bool side = mdx::side_terms_used(c);
      MDX_TRY(hipStreamWaitEvent(x->aux, x->ev_fork, 0));
      std::pair<hipEvent_t, hipEvent_t>* tslot;
      MDX_TRY(timing_begin(x, MDX_TIMING_PME, x->aux, &tslot));
      MDX_TRY(mdx::launch_pme_spread(c, x->aux, nullptr));
      // the join event is recorded by the last kernel's dispatch, or (timing
      // of the FFT passes, graph capture) explicitly after it
      const bool by_dispatch = !tslot && !c.capturing;
      MDX_TRY(mdx::launch_pme_fft(c, x->aux, by_dispatch && !side ? x->ev_join : nullptr));
      MDX_TRY(timing_end(tslot, x->aux));
      if (side) MDX_TRY(mdx::launch_side_terms(c, pos_cur, e, x->aux, x->ev_join));
      else if (!by_dispatch) MDX_TRY(hipEventRecord(x->ev_join, x->aux));
    }
    {
      // timed by events that the pair kernel's dispatch records (marker
      // packets between kernels would lengthen the step)
      std::pair<hipEvent_t, hipEvent_t>* ps;
      MDX_TRY(timing_slot(x, MDX_TIMING_PAIR, &ps));
      MDX_TRY(mdx::launch_nonbonded(c, e, gate_now, pgate_now, false,
                                    ps ? ps->first : nullptr, ps ? ps->second : nullptr));
    }
    if (c.has_pme) MDX_TRY(hipStreamWaitEvent(c.stream, x->ev_join, 0));
    if (rigid) {
      MDX_TRY(mdx::launch_finish_step(c, pos_cur, vel, force, dt, e));
      MDX_TRY(mdx::launch_rigid_velocities(c, pos_cur, vel, e, &rigid_blocks));
      if (s + 1 < n_steps) {
        g = gates_of(c.steps_taken + 1);
        MDX_TRY(open_rigid(g));
      }
    } else if (s + 1 < n_steps) {
      const mdx::StepGates next = gates_of(c.steps_taken + 1);
      MDX_TRY(mdx::launch_finish_step(c, pos_cur, vel, force, dt, e, &next, pos_other));
      std::swap(pos_cur, pos_other);
      g = next;
    } else {
      MDX_TRY(mdx::launch_finish_step(c, pos_cur, vel, force, dt, e));
    }
    if (e) {
      int rows[7] = {mdx::kRowLJ,    mdx::kRowDir, mdx::kRowExcl, mdx::kRowBond,
                     mdx::kRowAngle, mdx::kRowKin, mdx::kRowRec};
      int nblk[7] = {c.nb_blocks,      c.nb_blocks,      c.finish_blocks, c.finish_blocks,
                     c.finish_blocks,  c.finish_blocks,  c.pme_blocks};
      const int nrows = c.has_pme ? 7 : 6;
      double* out = energies + (size_t)s * MDX_N_ENERGY;
      MDX_TRY(mdx::launch_reduce_energy(c, rows, nblk, nrows, out, 0, c.e_self,
                                        MDX_ENERGY_COUL_SELF,
                                        c.has_pme ? -1 : MDX_ENERGY_COUL_REC,
                                        rigid ? rigid_blocks : 0));
    }
    c.steps_taken++;
  }
  if (pos_cur != pos)
    MDX_TRY(hipMemcpyAsync(pos, pos_cur, sizeof(float) * 3 * (size_t)c.n,
                           hipMemcpyDeviceToDevice, c.stream));
  return MDX_OK;
}

// A chunk of `chunk` steps replays as one graph when nothing it recorded has
// changed: the same buffers and dt, no reallocation or configuration change,
// the same rebuild phase, no energies, timing or Langevin (whose noise is
// keyed by the step index the launches carry).
bool graph_eligible(const mdx_ctx* x, int32_t n_steps, double* energies) {
  const Ctx& c = x->c;
  return x->graph_chunk > 0 && n_steps % x->graph_chunk == 0 && !energies && x->timing == 0 &&
         !c.langevin && c.steps_since_build >= 0;
}

bool graph_matches(const mdx_ctx* x, const float* pos, const float* vel, const float* force,
                   float dt) {
  const mdx_ctx::GraphKey& k = x->gkey;
  return x->gexec && k.pos == pos && k.vel == vel && k.force == force && k.dt == dt &&
         k.version == x->c.version && k.steps_since_build == x->c.steps_since_build;
}

// Records one chunk on the capture stream (launches are recorded, nothing
// runs; the host counters advance as for an eager chunk) and instantiates it.
int capture_chunk(mdx_ctx* x, float* pos, float* vel, float* force, float dt) {
  Ctx& c = x->c;
  if (!x->cap) MDX_TRY(hipStreamCreateWithFlags(&x->cap, hipStreamNonBlocking));
  if (x->gexec) (void)hipGraphExecDestroy(x->gexec);
  if (x->graph) (void)hipGraphDestroy(x->graph);
  x->gexec = nullptr;
  x->graph = nullptr;
  mdx_ctx::GraphKey key{pos, vel, force, dt, c.version, c.steps_since_build};
  hipStream_t user = c.stream;
  c.stream = x->cap;
  c.capturing = true;
  hipError_t e = hipStreamBeginCapture(x->cap, hipStreamCaptureModeRelaxed);
  int rc = e == hipSuccess ? integrate_eager(x, pos, vel, force, x->graph_chunk, dt, nullptr)
                           : MDX_E_HIP;
  hipGraph_t g = nullptr;
  const hipError_t e2 = hipStreamEndCapture(x->cap, &g);
  c.stream = user;
  c.capturing = false;
  if (rc != MDX_OK || e2 != hipSuccess || !g) {
    if (g) (void)hipGraphDestroy(g);
    (void)hipGetLastError();
    return rc != MDX_OK ? rc : MDX_E_HIP;
  }
  x->graph = g;
  MDX_TRY(hipGraphInstantiate(&x->gexec, g, nullptr, nullptr, 0));
  // the rebuild phase repeats every chunk (chunk is a multiple of the cadence)
  x->gkey = key;
  return MDX_OK;
}

}  // namespace

extern "C" {

int mdx_integrate_step(mdx_ctx* x, float* pos, float* vel, float* force, int32_t n_steps,
                       float dt, double* energies) {
  if (check_ctx(x) || !pos || !vel || !force || n_steps < 1 || !(dt > 0.f)) return MDX_E_INVALID;
  Ctx& c = x->c;
  if (c.steps_since_build < 0) {
    MDX_TRY(mdx::launch_build_list(c, pos));
    c.steps_since_build = 0;
  }
  if (!graph_eligible(x, n_steps, energies)) return integrate_eager(x, pos, vel, force, n_steps,
                                                                     dt, energies);
  for (int done = 0; done < n_steps; done += x->graph_chunk) {
    if (!graph_matches(x, pos, vel, force, dt)) {
      // the capture advances the host counters by one chunk without running
      // it; the launch below runs it
      if (int rc = capture_chunk(x, pos, vel, force, dt)) return rc;
    } else {
      c.steps_taken += x->graph_chunk;
    }
    MDX_TRY(hipGraphLaunch(x->gexec, c.stream));
    x->graph_launches++;
  }
  return MDX_OK;
}

}  // extern "C"

struct mdx_batch {
  std::vector<mdx_ctx*> ctx;
  int chunk = 0;
  std::vector<hipStream_t> streams;   // per replica: the stream its graph launches go to
  hipEvent_t ev_start = nullptr;      // the caller's stream reached the batch call
  std::vector<hipEvent_t> ev_end;     // per replica: its launches are done
};

namespace {

// Mean time per step of `steps` steps of a fresh context for desc (after
// `steps` untimed ones), from events on `stream`.
int time_config(const mdx_system_desc* d, const float* pos, const float* vel, float dt,
                int steps, hipStream_t stream, double* ms) {
  mdx_ctx* x = nullptr;
  int rc = mdx_create(&x, d, stream);
  if (rc != MDX_OK) return rc;
  const size_t b3 = sizeof(float) * 3 * (size_t)d->n_atoms;
  float *p = nullptr, *v = nullptr, *f = nullptr;
  hipEvent_t e0 = nullptr, e1 = nullptr;
  auto done = [&](int code) {
    if (p) (void)hipFree(p);
    if (v) (void)hipFree(v);
    if (f) (void)hipFree(f);
    if (e0) (void)hipEventDestroy(e0);
    if (e1) (void)hipEventDestroy(e1);
    mdx_destroy(x);
    return code;
  };
  if (hipMalloc(&p, b3) != hipSuccess || hipMalloc(&v, b3) != hipSuccess ||
      hipMalloc(&f, b3) != hipSuccess || hipEventCreate(&e0) != hipSuccess ||
      hipEventCreate(&e1) != hipSuccess)
    return done(MDX_E_OUT_OF_MEMORY);
  if (hipMemcpyAsync(p, pos, b3, hipMemcpyDeviceToDevice, stream) != hipSuccess ||
      hipMemcpyAsync(v, vel, b3, hipMemcpyDeviceToDevice, stream) != hipSuccess ||
      hipMemsetAsync(f, 0, b3, stream) != hipSuccess)
    return done(MDX_E_HIP);
  if ((rc = mdx_build_neighbors(x, p)) != MDX_OK) return done(rc);
  if ((rc = mdx_compute_nonbonded(x, p, f, nullptr, nullptr)) != MDX_OK) return done(rc);
  if (x->c.has_pme && (rc = mdx_compute_pme(x, p, f, nullptr, nullptr)) != MDX_OK)
    return done(rc);
  if ((rc = mdx_integrate_step(x, p, v, f, steps, dt, nullptr)) != MDX_OK) return done(rc);
  if (hipEventRecord(e0, stream) != hipSuccess) return done(MDX_E_HIP);
  if ((rc = mdx_integrate_step(x, p, v, f, steps, dt, nullptr)) != MDX_OK) return done(rc);
  if (hipEventRecord(e1, stream) != hipSuccess || hipEventSynchronize(e1) != hipSuccess)
    return done(MDX_E_HIP);
  float t = 0.f;
  if (hipEventElapsedTime(&t, e0, e1) != hipSuccess) return done(MDX_E_HIP);
  *ms = (double)t / steps;
  return done(MDX_OK);
}

}  // namespace

extern "C" {

int mdx_batch_create(mdx_batch** out, mdx_ctx* const* ctxs, int32_t n_rep, int32_t chunk) {
  if (!out) return MDX_E_INVALID;
  *out = nullptr;
  if (!ctxs || n_rep < 1 || chunk < 0) return MDX_E_INVALID;
  for (int r = 0; r < n_rep; ++r) {
    if (!ctxs[r]) return MDX_E_INVALID;
    if (chunk > 0 && chunk % ctxs[r]->c.rebuild_every != 0) return MDX_E_INVALID;
    for (int q = 0; q < r; ++q)
      if (ctxs[q] == ctxs[r]) return MDX_E_INVALID;   // each context once
  }
  mdx_batch* b = new (std::nothrow) mdx_batch();
  if (!b) return MDX_E_OUT_OF_MEMORY;
  b->ctx.assign(ctxs, ctxs + n_rep);
  b->chunk = chunk;
  b->ev_end.assign(n_rep, nullptr);
  b->streams.assign(n_rep, nullptr);
  const unsigned fl = hipEventDisableTiming;
  bool ok = hipEventCreateWithFlags(&b->ev_start, fl) == hipSuccess;
  for (int r = 0; r < n_rep && ok; ++r)
    ok = hipEventCreateWithFlags(&b->ev_end[r], fl) == hipSuccess &&
         hipStreamCreateWithFlags(&b->streams[r], hipStreamNonBlocking) == hipSuccess;
  if (!ok) {
    mdx_batch_destroy(b);
    return MDX_E_HIP;
  }
  // with a chunk, every member replays its steps in graphs of that length
  for (int r = 0; r < n_rep && chunk > 0; ++r)
    if (mdx_set_graph(ctxs[r], chunk) != MDX_OK) {
      mdx_batch_destroy(b);
      return MDX_E_INVALID;
    }
  *out = b;
  return MDX_OK;
}

int mdx_batch_destroy(mdx_batch* b) {
  if (!b) return MDX_OK;
  for (hipStream_t st : b->streams)
    if (st) {
      (void)hipStreamSynchronize(st);
      (void)hipStreamDestroy(st);
    }
  for (hipEvent_t e : b->ev_end)
    if (e) (void)hipEventDestroy(e);
  if (b->ev_start) (void)hipEventDestroy(b->ev_start);
  delete b;
  return MDX_OK;
}

int mdx_batch_integrate(mdx_batch* b, float* const* pos, float* const* vel, float* const* force,
                        int32_t n_steps, const float* dt, void* hip_stream) {
  if (!b || !pos || !vel || !force || !dt || n_steps < 1 ||
      (b->chunk > 0 && n_steps % b->chunk != 0))
    return MDX_E_INVALID;
  hipStream_t stream = static_cast<hipStream_t>(hip_stream);
  const size_t n = b->ctx.size();
  for (size_t r = 0; r < n; ++r) {
    mdx_ctx* x = b->ctx[r];
    if (!pos[r] || !vel[r] || !force[r] || !(dt[r] > 0.f)) return MDX_E_INVALID;
    if (b->chunk > 0 && (x->c.langevin || x->timing)) return MDX_E_UNSUPPORTED;
    if (x->c.steps_since_build < 0) return MDX_E_NO_LIST;
  }
  // every replica on its own stream, ordered after the caller's stream and
  // joined back into it; each replica's chunks are its own graph launches
  MDX_TRY(hipEventRecord(b->ev_start, stream));
  for (size_t r = 0; r < n; ++r) {
    mdx_ctx* x = b->ctx[r];
    hipStream_t user = x->c.stream;
    x->c.stream = b->streams[r];
    int rc = hipStreamWaitEvent(b->streams[r], b->ev_start, 0) == hipSuccess ? MDX_OK : MDX_E_HIP;
    if (rc == MDX_OK) rc = mdx_integrate_step(x, pos[r], vel[r], force[r], n_steps, dt[r], nullptr);
    if (rc == MDX_OK && (hipEventRecord(b->ev_end[r], b->streams[r]) != hipSuccess ||
                         hipStreamWaitEvent(stream, b->ev_end[r], 0) != hipSuccess))
      rc = MDX_E_HIP;
    x->c.stream = user;
    if (rc != MDX_OK) return rc;
  }
  return MDX_OK;
}

int mdx_autotune(const mdx_system_desc* d, const float* pos, const float* vel, float dt,
                 int32_t steps, void* hip_stream, int32_t* cell_divisions, uint32_t* options,
                 double* ms_per_step) {
  if (!d || !pos || !vel || !(dt > 0.f) || steps < 1 || !cell_divisions || !options)
    return MDX_E_INVALID;
  hipStream_t stream = static_cast<hipStream_t>(hip_stream);
  double best = 0.0;
  int best_m = 0;
  uint32_t best_o = 0;
  for (int coop = 0; coop < 2; ++coop)
    for (int m = 1; m <= 4; ++m) {
      mdx_system_desc t = *d;
      t.cell_divisions = m;
      t.options = (d->options & ~(uint32_t)MDX_OPT_COOPERATIVE_BUILD) |
                  (coop ? (uint32_t)MDX_OPT_COOPERATIVE_BUILD : 0u);
      double ms = 0.0;
      int rc = time_config(&t, pos, vel, dt, steps, stream, &ms);
      if (rc != MDX_OK) return rc;
      if (ms_per_step) ms_per_step[coop * 4 + m - 1] = ms;
      if (best_m == 0 || ms < best) {
        best = ms;
        best_m = m;
        best_o = t.options;
      }
    }
  *cell_divisions = best_m;
  *options = best_o;
  return MDX_OK;
}

int mdx_set_graph(mdx_ctx* x, int32_t chunk) {
  if (check_ctx(x) || chunk < 0) return MDX_E_INVALID;
  Ctx& c = x->c;
  if (chunk > 0 && chunk % c.rebuild_every != 0) return MDX_E_INVALID;
  x->graph_chunk = chunk;
  if (x->gexec) (void)hipGraphExecDestroy(x->gexec);
  if (x->graph) (void)hipGraphDestroy(x->graph);
  x->gexec = nullptr;
  x->graph = nullptr;
  return MDX_OK;
}

int mdx_get_status(mdx_ctx* x, uint32_t* flags) {
  if (check_ctx(x) || !flags) return MDX_E_INVALID;
  Ctx& c = x->c;
  unsigned f = 0;
  MDX_TRY(hipMemcpyAsync(&f, c.flags, sizeof(unsigned), hipMemcpyDeviceToHost, c.stream));
  MDX_TRY(hipStreamSynchronize(c.stream));
  MDX_TRY(hipMemsetAsync(c.flags, 0, sizeof(unsigned), c.stream));
  MDX_TRY(hipStreamSynchronize(c.stream));
  *flags = f;
  return MDX_OK;
}

int mdx_compute_ewald_direct(mdx_ctx* x, const float* pos, float* force, double* energy,
                             int32_t n_max) {
  if (check_ctx(x) || !pos || !force || n_max < 1 || n_max > 64) return MDX_E_INVALID;
  Ctx& c = x->c;
  if (!c.has_coulomb) return MDX_E_INVALID;
  if (n_max > c.ew_nmax) {
    const size_t w = 2 * (size_t)n_max + 1, K = (w * w * w - 1) / 2;
    dev_free(x, c.ew_tab);
    dev_free(x, c.ew_S);
    dev_free(x, c.ew_eterm);
    c.ew_tab = nullptr;
    c.ew_S = nullptr;
    c.ew_eterm = nullptr;
    c.ew_nmax = 0;
    int rc;
    if ((rc = dev_alloc(x, &c.ew_tab, 3 * w * (size_t)c.n)) != MDX_OK) return rc;
    if ((rc = dev_alloc(x, &c.ew_S, K)) != MDX_OK) return rc;
    if ((rc = dev_alloc(x, &c.ew_eterm, K)) != MDX_OK) return rc;
    c.ew_nmax = n_max;
  }
  MDX_TRY(mdx::launch_ewald_direct(c, pos, force, energy, n_max, c.ew_tab, c.ew_S, c.ew_eterm));
  return MDX_OK;
}

int mdx_compute_ewald_direct_noalloc(mdx_ctx* x, const float* pos, float* force,
                                     double* energy, int32_t n_max) {
  if (check_ctx(x) || !pos || !force || n_max < 1 || n_max > 64) return MDX_E_INVALID;
  Ctx& c = x->c;
  if (!c.has_coulomb) return MDX_E_INVALID;
  if (mdx::ewald_scratch_bytes(c.n, n_max) > mdx::kEwScratchBytes) return MDX_E_CAPACITY;
  MDX_TRY(mdx::launch_ewald_direct_static(c, pos, force, energy, n_max));
  return MDX_OK;
}

int mdx_ewald_direct_noalloc_bytes(int32_t n_atoms, int32_t n_max, int64_t* bytes,
                                   int64_t* limit) {
  if (n_atoms < 1 || n_max < 1 || n_max > 64 || !bytes) return MDX_E_INVALID;
  *bytes = (int64_t)mdx::ewald_scratch_bytes(n_atoms, n_max);
  if (limit) *limit = (int64_t)mdx::kEwScratchBytes;
  return MDX_OK;
}

int mdx_set_rigid_water(mdx_ctx* x, const int32_t* mols, int32_t n_mol, double d_oh,
                        double d_hh) {
  if (check_ctx(x) || n_mol < 0 || (n_mol > 0 && (!mols || !(d_oh > 0.0) || !(d_hh > 0.0))))
    return MDX_E_INVALID;
  Ctx& c = x->c;
  if (n_mol > 0 && (c.xc || c.langevin)) return MDX_E_UNSUPPORTED;
  std::vector<int> seen(c.n, 0);
  for (int64_t i = 0; i < 3 * (int64_t)n_mol; ++i) {
    const int a = mols[i];
    if (a < 0 || a >= c.n || seen[a]++) return MDX_E_INVALID;   // in range, each atom once
  }
  if (n_mol > c.n_rigid) {
    dev_free(x, c.rigid_mols);
    c.rigid_mols = nullptr;
    int rc = dev_alloc(x, &c.rigid_mols, (size_t)3 * n_mol);
    if (rc != MDX_OK) return rc;
  }
  if (n_mol > 0)
    MDX_TRY(hipMemcpy(c.rigid_mols, mols, sizeof(int) * 3 * (size_t)n_mol,
                      hipMemcpyHostToDevice));
  c.version++;
  c.n_rigid = n_mol;
  c.rigid_d[0] = c.rigid_d[1] = (float)d_oh;
  c.rigid_d[2] = (float)d_hh;
  // the closed form (SETTLE) when every molecule's hydrogens weigh the same
  // and the triangle exists, SHAKE iterations otherwise
  c.rigid_settle = d_hh < 2.0 * d_oh;
  for (int64_t k = 0; k < n_mol && c.rigid_settle; ++k)
    c.rigid_settle = c.mass_h[mols[3 * k + 1]] == c.mass_h[mols[3 * k + 2]];
  return MDX_OK;
}

int mdx_set_langevin(mdx_ctx* x, double kT, double gamma, uint64_t seed) {
  if (check_ctx(x) || !(kT >= 0.0) || !(gamma >= 0.0) || !std::isfinite(kT) ||
      !std::isfinite(gamma))
    return MDX_E_INVALID;
  Ctx& c = x->c;
  if (c.xc && gamma > 0.0) return MDX_E_UNSUPPORTED;
  if (c.n_rigid > 0 && gamma > 0.0) return MDX_E_UNSUPPORTED;
  c.version++;
  c.langevin = gamma > 0.0;
  c.lv_kT = kT;
  c.lv_gamma = gamma;
  c.lv_seed = seed;
  if (!c.langevin) return MDX_OK;
  std::vector<float> sig(c.n);
  for (int i = 0; i < c.n; ++i) sig[i] = (float)std::sqrt(kT * c.accel / (double)c.mass_h[i]);
  if (!c.lv_sig) {
    int rc = dev_alloc(x, &c.lv_sig, (size_t)c.n);
    if (rc != MDX_OK) return rc;
  }
  MDX_TRY(hipMemcpy(c.lv_sig, sig.data(), sizeof(float) * c.n, hipMemcpyHostToDevice));
  return MDX_OK;
}

int mdx_get_images(mdx_ctx* x, int32_t* img) {
  if (check_ctx(x) || !img) return MDX_E_INVALID;
  Ctx& c = x->c;
  MDX_TRY(hipMemcpyAsync(img, c.img, sizeof(int32_t) * 3 * (size_t)c.n,
                         hipMemcpyDeviceToDevice, c.stream));
  return MDX_OK;
}

}  // extern "C"

namespace {

// Layout of a saved state: a header, then the device arrays that a later step
// reads, each starting at a multiple of 256 bytes.
constexpr uint64_t kStateMagic = 0x3154535844584d44ull;   // "DMXDXST1"
constexpr int64_t kStateVersion = 2;

struct StateHeader {
  uint64_t magic;
  int64_t version;
  int64_t total;                  // bytes, header included
  // geometry that must match the loading context
  int64_t n, max_slots, max_clusters, ncol, nzb, brick_layers;
  int64_t kahan, half_list, has_pme;
  // capacities (the loading context adopts them)
  int64_t nl_cap, col_cap;
  // host counters
  int64_t steps_since_build, steps_taken;
};

struct Segment {
  void* p;
  size_t bytes;
};

size_t align256(size_t b) { return (b + 255) / 256 * 256; }

// The arrays, in state order, of a context with the given capacities.
std::vector<Segment> state_segments(const Ctx& c) {
  const size_t n = (size_t)c.n, ns = (size_t)c.max_slots, nc = (size_t)c.max_clusters;
  const size_t ncol = (size_t)c.cg.ncell;
  std::vector<Segment> s = {
      {c.img, sizeof(int) * 3 * n},          {c.x_build, sizeof(float) * 3 * n},
      {c.gate, sizeof(int) * 4},             {c.meta, sizeof(int) * 4},
      {c.perm, sizeof(int) * ns},            {c.inv_perm, sizeof(int) * n},
      {c.cell_of, sizeof(int) * n},          {c.cell_count, sizeof(int) * ncol},
      {c.cell_start, sizeof(int) * (ncol + 1)}, {c.slot_start, sizeof(int) * (ncol + 1)},
      {c.zbin, sizeof(int2) * ncol * (c.cg.nzb + 1)},
      {c.xs, sizeof(float4) * ns},           {c.ts, sizeof(int) * ns},
      {c.zb, sizeof(float) * ns},            {c.box_lo, sizeof(float4) * nc},
      {c.box_hi, sizeof(float4) * nc},       {c.col_xy, sizeof(float4) * ncol},
      {c.tiles, sizeof(uint2) * nc * c.nl_cap}, {c.tile_count, sizeof(int) * nc},
      {c.nl_needed, sizeof(int)},            {c.ptiles, sizeof(uint2) * nc * c.nl_cap},
      {c.pcount, sizeof(int) * nc},          {c.xp, sizeof(float4) * ns},
  };
  if (c.xc) {
    s.push_back({c.xc, sizeof(float) * 3 * n});
    s.push_back({c.vc, sizeof(float) * 3 * n});
  }
  if (c.has_pme) s.push_back({c.brick_zr, sizeof(int4) * (size_t)c.pg.nb[2] * ncol});
  if (c.half_list) {
    // the tiles' j partials (a pruned step keeps the dropped tiles' zeros)
    // and the incoming lists
    const size_t nt = nc * (size_t)c.nl_cap;
    s.push_back({c.jpart, sizeof(float) * 12 * nt});
    s.push_back({c.ppos, sizeof(int) * nt});
    s.push_back({c.in_count, sizeof(int) * nc});
    s.push_back({c.in_fill, sizeof(int) * nt});
    s.push_back({c.in_sorted, sizeof(int) * nt});
  }
  return s;
}

StateHeader state_header(const Ctx& c) {
  StateHeader h{};
  h.magic = kStateMagic;
  h.version = kStateVersion;
  h.n = c.n;
  h.max_slots = c.max_slots;
  h.max_clusters = c.max_clusters;
  h.ncol = c.cg.ncell;
  h.nzb = c.cg.nzb;
  h.brick_layers = c.has_pme ? c.pg.nb[2] : 0;
  h.kahan = c.xc != nullptr;
  h.half_list = c.half_list;
  h.has_pme = c.has_pme;
  h.nl_cap = c.nl_cap;
  h.col_cap = c.col_cap;
  h.steps_since_build = c.steps_since_build;
  h.steps_taken = c.steps_taken;
  size_t total = align256(sizeof(StateHeader));
  for (const Segment& sg : state_segments(c)) total += align256(sg.bytes);
  h.total = (int64_t)total;
  return h;
}

}  // namespace

extern "C" {

int mdx_state_size(mdx_ctx* x, int64_t* bytes) {
  if (check_ctx(x) || !bytes) return MDX_E_INVALID;
  *bytes = state_header(x->c).total;
  return MDX_OK;
}

int mdx_save_state(mdx_ctx* x, void* state, int64_t capacity) {
  if (check_ctx(x) || !state || capacity < 0 || (reinterpret_cast<uintptr_t>(state) & 7u))
    return MDX_E_INVALID;
  Ctx& c = x->c;
  const StateHeader h = state_header(c);
  if (capacity < h.total) return MDX_E_CAPACITY;
  char* dst = static_cast<char*>(state);
  MDX_TRY(hipMemcpyAsync(dst, &h, sizeof(h), hipMemcpyHostToDevice, c.stream));
  size_t off = align256(sizeof(StateHeader));
  for (const Segment& sg : state_segments(c)) {
    MDX_TRY(hipMemcpyAsync(dst + off, sg.p, sg.bytes, hipMemcpyDeviceToDevice, c.stream));
    off += align256(sg.bytes);
  }
  MDX_TRY(hipStreamSynchronize(c.stream));   // the header is read from the host stack
  return MDX_OK;
}

int mdx_load_state(mdx_ctx* x, const void* state, int64_t size) {
  if (check_ctx(x) || !state || size < (int64_t)sizeof(StateHeader) ||
      (reinterpret_cast<uintptr_t>(state) & 7u))
    return MDX_E_INVALID;
  Ctx& c = x->c;
  StateHeader h;
  MDX_TRY(hipStreamSynchronize(c.stream));
  MDX_TRY(hipMemcpy(&h, state, sizeof(h), hipMemcpyDeviceToHost));
  const StateHeader mine = state_header(c);
  if (h.magic != kStateMagic || h.version != kStateVersion || h.n != mine.n ||
      h.max_slots != mine.max_slots || h.max_clusters != mine.max_clusters ||
      h.ncol != mine.ncol || h.nzb != mine.nzb || h.brick_layers != mine.brick_layers ||
      h.kahan != mine.kahan || h.half_list != mine.half_list || h.has_pme != mine.has_pme ||
      h.nl_cap < 4 || h.col_cap < 1 || h.col_cap > c.n || h.total > size ||
      h.steps_since_build < -1 || h.steps_taken < 0)
    return MDX_E_INVALID;
  // adopt the saved capacities, so the arrays have the saved sizes
  if (h.nl_cap != c.nl_cap) {
    int rc = alloc_list(x, (int)h.nl_cap);
    if (rc != MDX_OK) return rc;
    if (c.nl_cap != h.nl_cap) return MDX_E_INVALID;   // not a capacity alloc_list makes
  }
  c.version++;
  if (h.col_cap != c.col_cap) {
    dev_free(x, c.col_atoms);
    c.col_atoms = nullptr;
    c.col_cap = (int)h.col_cap;
    int rc = dev_alloc(x, &c.col_atoms, (size_t)c.cg.ncell * c.col_cap);
    if (rc != MDX_OK) return rc;
  }
  if (state_header(c).total != h.total) return MDX_E_INVALID;
  const char* src = static_cast<const char*>(state);
  size_t off = align256(sizeof(StateHeader));
  for (const Segment& sg : state_segments(c)) {
    MDX_TRY(hipMemcpyAsync(sg.p, src + off, sg.bytes, hipMemcpyDeviceToDevice, c.stream));
    off += align256(sg.bytes);
  }
  // the next build bins in atom order (the slot-order hint, meta[4], is not
  // part of the state; the list does not depend on the binning order)
  MDX_TRY(mdx::launch_fill_i32(c.meta + 4, 0, 1, c.stream));
  MDX_TRY(hipStreamSynchronize(c.stream));
  c.steps_since_build = (int)h.steps_since_build;
  c.steps_taken = h.steps_taken;
  return MDX_OK;
}

int mdx_set_parameters(mdx_ctx* x, const float* type_sigma, const float* type_epsilon,
                       const float* charge) {
  if (check_ctx(x)) return MDX_E_INVALID;
  Ctx& c = x->c;
  const int T = c.n_types;
  for (int t = 0; type_sigma && t < T; ++t)
    if (!(type_sigma[t] > 0.f) || !std::isfinite(type_sigma[t])) return MDX_E_INVALID;
  for (int t = 0; type_epsilon && t < T; ++t)
    if (!(type_epsilon[t] >= 0.f) || !std::isfinite(type_epsilon[t])) return MDX_E_INVALID;
  for (int i = 0; charge && i < c.n; ++i) {
    if (!std::isfinite(charge[i])) return MDX_E_INVALID;
    // electrostatics were configured (or not) at mdx_create
    if (!c.has_coulomb && !c.rf && charge[i] != 0.f) return MDX_E_UNSUPPORTED;
  }
  MDX_TRY(hipStreamSynchronize(c.stream));   // kernels in flight read the tables
  if (type_sigma) c.sig_h.assign(type_sigma, type_sigma + T);
  if (type_epsilon) c.eps_h.assign(type_epsilon, type_epsilon + T);
  if (type_sigma || type_epsilon) {
    int rc = upload_lj_tables(x);
    if (rc != MDX_OK) return rc;
  }
  if (charge) {
    c.q_h.assign(charge, charge + c.n);
    MDX_TRY(hipMemcpy(c.q, c.q_h.data(), sizeof(float) * c.n, hipMemcpyHostToDevice));
    c.e_self = self_energy(c);
  }
  return MDX_OK;
}

}  // extern "C"

namespace {

int ensure_adjoint(mdx_ctx* x) {
  Ctx& c = x->c;
  mdx::AdjScratch& a = c.adj;
  if (a.ready) return MDX_OK;
  const size_t n3 = 3 * (size_t)c.n, ns = (size_t)c.max_slots;
  int rc;
  if ((rc = dev_alloc(x, &a.u, n3)) != MDX_OK) return rc;
  if ((rc = dev_alloc(x, &a.us, ns)) != MDX_OK) return rc;
  if ((rc = dev_alloc(x, &a.dfs, 3 * ns)) != MDX_OK) return rc;
  if ((rc = dev_alloc(x, &a.gslot, 3 * ns)) != MDX_OK) return rc;
  if ((rc = dev_alloc(x, &a.gatom, n3)) != MDX_OK) return rc;
  if ((rc = dev_alloc(x, &a.dq, (size_t)c.n)) != MDX_OK) return rc;
  if ((rc = dev_alloc(x, &a.dt_part, (size_t)(c.n + 255) / 256)) != MDX_OK) return rc;
  if ((rc = dev_alloc(x, &a.gate, 1)) != MDX_OK) return rc;
  if ((rc = dev_alloc(x, &a.pos, n3)) != MDX_OK) return rc;
  if ((rc = dev_alloc(x, &a.vel, n3)) != MDX_OK) return rc;
  if ((rc = dev_alloc(x, &a.force, n3)) != MDX_OK) return rc;
  if (c.has_pme) {
    const size_t K3 = (size_t)c.pg.K[0] * c.pg.K[1] * c.pg.K[2];
    if ((rc = dev_alloc(x, &a.phi2, K3)) != MDX_OK) return rc;
  }
  MDX_TRY(hipMemset(a.dq, 0, sizeof(float) * c.n));
  a.dq_h.assign(c.n, 0.f);
  a.ready = true;
  return MDX_OK;
}

int ensure_records(mdx_ctx* x, int steps) {
  Ctx& c = x->c;
  mdx::AdjScratch& a = c.adj;
  if (steps <= a.rec_steps) return MDX_OK;
  dev_free(x, a.rec_x);
  dev_free(x, a.rec_v);
  dev_free(x, a.rec_f);
  dev_free(x, a.rec_phi);
  a.rec_x = a.rec_v = a.rec_f = a.rec_phi = nullptr;
  a.rec_steps = 0;
  const size_t m = (size_t)(steps + 1) * 3 * c.n;
  int rc;
  if ((rc = dev_alloc(x, &a.rec_x, m)) != MDX_OK) return rc;
  if ((rc = dev_alloc(x, &a.rec_v, m)) != MDX_OK) return rc;
  if ((rc = dev_alloc(x, &a.rec_f, m)) != MDX_OK) return rc;
  if (c.has_pme) {
    const size_t K3 = (size_t)c.pg.K[0] * c.pg.K[1] * c.pg.K[2];
    if ((rc = dev_alloc(x, &a.rec_phi, (size_t)(steps + 1) * K3)) != MDX_OK) return rc;
  }
  a.rec_steps = steps;
  return MDX_OK;
}

// The reverse pass covers plain velocity Verlet with the full list and the
// unswitched pair potentials.
int adjoint_supported(const Ctx& c) {
  if (c.half_list || c.langevin || c.n_rigid > 0 || c.has_switch) return MDX_E_UNSUPPORTED;
  return MDX_OK;
}

// d E_self / dt for charges q + t dq (Eq. 12 and the neutralising term).
double self_energy_charge_derivative(const Ctx& c) {
  if (!c.has_coulomb) return 0.0;
  double qdq = 0.0, qs = 0.0, dqs = 0.0;
  for (int i = 0; i < c.n; ++i) {
    qdq += (double)c.q_h[i] * c.adj.dq_h[i];
    qs += c.q_h[i];
    dqs += c.adj.dq_h[i];
  }
  const double V = (double)c.box[0] * c.box[1] * c.box[2];
  return -2.0 * c.coulomb_k * c.alpha / std::sqrt(M_PI) * qdq -
         c.coulomb_k * M_PI * qs * dqs / (V * c.alpha * c.alpha);
}

// The potential of the dipole grid of the tangent by slot into adj.phi2.
hipError_t dipole_potential(Ctx& c) {
  hipError_t e = mdx::launch_pme_spread_dipole(c, c.adj.us);
  if (e != hipSuccess) return e;
  std::swap(c.grid_phi, c.adj.phi2);
  e = mdx::launch_pme_fft(c, c.stream, nullptr);
  std::swap(c.grid_phi, c.adj.phi2);
  return e;
}

}  // namespace

extern "C" {

int mdx_set_charge_direction(mdx_ctx* x, const float* dq) {
  if (check_ctx(x) || !dq) return MDX_E_INVALID;
  Ctx& c = x->c;
  for (int i = 0; i < c.n; ++i)
    if (!std::isfinite(dq[i])) return MDX_E_INVALID;
  if (int rc = ensure_adjoint(x)) return rc;
  MDX_TRY(hipStreamSynchronize(c.stream));
  c.adj.dq_h.assign(dq, dq + c.n);
  MDX_TRY(hipMemcpy(c.adj.dq, dq, sizeof(float) * c.n, hipMemcpyHostToDevice));
  return MDX_OK;
}

int mdx_reset_images(mdx_ctx* x) {
  if (check_ctx(x)) return MDX_E_INVALID;
  MDX_TRY(mdx::launch_fill_i32(x->c.img, 0, 3 * x->c.n, x->c.stream));
  return MDX_OK;
}

int mdx_get_unwrapped(mdx_ctx* x, const float* pos, float* out) {
  if (check_ctx(x) || !pos || !out) return MDX_E_INVALID;
  MDX_TRY(mdx::launch_unwrap(x->c, pos, out));
  return MDX_OK;
}

int mdx_set_masses(mdx_ctx* x, const float* mass) {
  if (check_ctx(x) || !mass) return MDX_E_INVALID;
  Ctx& c = x->c;
  for (int i = 0; i < c.n; ++i)
    if (!(mass[i] > 0.f) || !std::isfinite(mass[i])) return MDX_E_INVALID;
  MDX_TRY(hipStreamSynchronize(c.stream));   // kernels in flight read the arrays
  c.mass_h.assign(mass, mass + c.n);
  std::vector<float> am(c.n);
  for (int i = 0; i < c.n; ++i) am[i] = (float)(c.accel / (double)mass[i]);
  MDX_TRY(hipMemcpy(c.mass, mass, sizeof(float) * c.n, hipMemcpyHostToDevice));
  MDX_TRY(hipMemcpy(c.hdt_scale, am.data(), sizeof(float) * c.n, hipMemcpyHostToDevice));
  if (c.langevin) {
    std::vector<float> sig(c.n);
    for (int i = 0; i < c.n; ++i) sig[i] = (float)std::sqrt(c.lv_kT * c.accel / (double)mass[i]);
    MDX_TRY(hipMemcpy(c.lv_sig, sig.data(), sizeof(float) * c.n, hipMemcpyHostToDevice));
  }
  if (c.n_rigid > 0) {
    // the closed form needs equal hydrogen masses in every molecule
    std::vector<int> mols(3 * (size_t)c.n_rigid);
    MDX_TRY(hipMemcpy(mols.data(), c.rigid_mols, sizeof(int) * mols.size(),
                      hipMemcpyDeviceToHost));
    bool settle = c.rigid_d[2] < 2.0f * c.rigid_d[0];
    for (int k = 0; k < c.n_rigid && settle; ++k)
      settle = c.mass_h[mols[3 * k + 1]] == c.mass_h[mols[3 * k + 2]];
    if (settle != c.rigid_settle) c.version++;
    c.rigid_settle = settle;
  }
  return MDX_OK;
}

int mdx_adjoint_begin(mdx_ctx* x, const float* pos, const float* force, const float* gx,
                      const float* gv, const double* gU, float* q, float* p, double* grad) {
  if (check_ctx(x) || !pos || !force || !gx || !gU || !q || !p || !grad) return MDX_E_INVALID;
  Ctx& c = x->c;
  if (int rc = adjoint_supported(c)) return rc;
  if (int rc = ensure_adjoint(x)) return rc;
  const int T = c.n_types;
  MDX_TRY(mdx::launch_fill_i32(reinterpret_cast<int*>(grad), 0, 2 * (2 * T + 2), c.stream));
  // the energy's parameter derivatives at pos, scaled by dL/dU
  MDX_TRY(mdx::launch_build_list(c, pos));
  c.steps_since_build = 0;
  MDX_TRY(mdx::launch_fill_i32(reinterpret_cast<int*>(c.adj.u), 0, 3 * c.n, c.stream));
  MDX_TRY(mdx::launch_adj_slots(c, pos, false));
  if (c.has_pme) {
    MDX_TRY(mdx::launch_pme_spread(c, c.stream, nullptr));
    MDX_TRY(mdx::launch_pme_fft(c, c.stream, nullptr));
  }
  MDX_TRY(mdx::launch_pair_jvp(c, true));
  MDX_TRY(mdx::launch_jvp_finish(c, true, pos, c.grid_phi, nullptr, nullptr, 0.f));
  MDX_TRY(mdx::launch_adj_reduce(c, 1.0, gU, self_energy_charge_derivative(c), 0, grad));
  MDX_TRY(mdx::launch_adj_begin(c, gx, gv, gU, force, q, p));
  return MDX_OK;
}

int mdx_adjoint_inject(mdx_ctx* x, const float* force, const float* gx, const float* gv,
                       const double* gU, float* q, float* p) {
  if (check_ctx(x) || !q || !p || (gU && !force)) return MDX_E_INVALID;
  MDX_TRY(mdx::launch_adj_inject(x->c, gx, gv, gU, force, q, p));
  return MDX_OK;
}

int mdx_adjoint_segment(mdx_ctx* x, const float* x0, const float* v0, const float* f0,
                        int32_t n_steps, float dt, int32_t flags, float* q, float* p,
                        double* grad, double* grad_mass) {
  if (check_ctx(x) || !x0 || !v0 || !f0 || !q || !p || !grad || n_steps < 1 || !(dt > 0.f) ||
      (flags & ~(MDX_ADJ_FIRST | MDX_ADJ_LAST)))
    return MDX_E_INVALID;
  const bool first = flags & MDX_ADJ_FIRST;
  Ctx& c = x->c;
  if (c.steps_since_build < 0) return MDX_E_NO_LIST;
  if (int rc = adjoint_supported(c)) return rc;
  if (int rc = ensure_adjoint(x)) return rc;
  if (int rc = ensure_records(x, n_steps)) return rc;
  mdx::AdjScratch& a = c.adj;
  const size_t n3 = 3 * (size_t)c.n;
  const size_t K3 = c.has_pme ? (size_t)c.pg.K[0] * c.pg.K[1] * c.pg.K[2] : 0;
  const size_t b3 = sizeof(float) * n3;
  auto copy = [&](void* dst, const void* src, size_t bytes) {
    return hipMemcpyAsync(dst, src, bytes, hipMemcpyDeviceToDevice, c.stream);
  };
  // the segment again, from its saved start, recording every state
  MDX_TRY(copy(a.pos, x0, b3));
  MDX_TRY(copy(a.vel, v0, b3));
  MDX_TRY(copy(a.force, f0, b3));
  MDX_TRY(copy(a.rec_x, x0, b3));
  MDX_TRY(copy(a.rec_v, v0, b3));
  MDX_TRY(copy(a.rec_f, f0, b3));
  if (c.has_pme) {
    MDX_TRY(mdx::launch_refresh_sorted(c, x0));
    MDX_TRY(mdx::launch_pme_spread(c, c.stream, nullptr));
    MDX_TRY(mdx::launch_pme_fft(c, c.stream, nullptr));
    MDX_TRY(copy(a.rec_phi, c.grid_phi, sizeof(float) * K3));
  }
  for (int k = 0; k < n_steps; ++k) {
    if (int rc = mdx_integrate_step(x, a.pos, a.vel, a.force, 1, dt, nullptr)) return rc;
    MDX_TRY(copy(a.rec_x + (k + 1) * n3, a.pos, b3));
    MDX_TRY(copy(a.rec_v + (k + 1) * n3, a.vel, b3));
    MDX_TRY(copy(a.rec_f + (k + 1) * n3, a.force, b3));
    if (c.has_pme) MDX_TRY(copy(a.rec_phi + (k + 1) * K3, c.grid_phi, sizeof(float) * K3));
  }
  // reverse over the segment's nodes; with MDX_ADJ_LAST first its end node
  // with half weight (the loss's velocity adjoint in p reaches the positions)
  const int nblk = (c.n + 255) / 256;
  for (int k = (flags & MDX_ADJ_LAST) ? n_steps : n_steps - 1; k >= 0; --k) {
    const bool end = k == n_steps;
    const float w = ((first && k == 0) || end) ? 0.5f : 1.0f;
    const float* xk = a.rec_x + k * n3;
    MDX_TRY(mdx::launch_adj_pre(c, dt, w, !end, q, p, a.rec_v + k * n3, a.rec_f + k * n3,
                                grad_mass));
    MDX_TRY(mdx::launch_adj_slots(c, xk, true));
    MDX_TRY(mdx::launch_pair_jvp(c, false));
    if (c.has_pme) MDX_TRY(dipole_potential(c));
    MDX_TRY(mdx::launch_jvp_finish(c, false, xk, c.has_pme ? a.rec_phi + k * K3 : nullptr,
                                   a.phi2, q, w * dt));
    MDX_TRY(mdx::launch_adj_reduce(c, (double)w * dt, nullptr, 0.0, nblk, grad));
  }
  return MDX_OK;
}

int mdx_get_info(mdx_ctx* x, mdx_info* info) {
  if (check_ctx(x) || !info) return MDX_E_INVALID;
  Ctx& c = x->c;
  std::memset(info, 0, sizeof(*info));
  info->n_atoms = c.n;
  for (int k = 0; k < 3; ++k) {
    info->cell_dims[k] = c.cg.n[k];
    info->pme_grid[k] = c.has_pme ? c.pg.K[k] : 0;
    info->pme_brick[k] = c.has_pme ? c.pg.B[k] : 0;
  }
  info->cell_divisions = c.cell_div;
  info->nl_capacity = c.nl_cap;
  info->alpha = c.alpha;
  info->r_list = (double)c.r_list;
  info->n_list_entries = -1;
  info->steps_taken = c.steps_taken;
  info->n_builds = 0;
  info->n_list_tiles = -1;
  if (c.steps_since_build >= 0) {
    HostList h;
    if (int rc = read_list(c, h)) return rc;
    int64_t entries = 0, tiles = 0;
    for (int ic = 0; ic < h.nclu; ++ic) {
      tiles += h.cnt[ic];
      for (int k = 0; k < h.cnt[ic]; ++k)
        entries += __builtin_popcount(h.tl[(size_t)ic * c.nl_cap + k].y & 0xffffu);
    }
    info->n_list_entries = entries;
    info->n_list_tiles = tiles;
    info->n_builds = h.builds;
  }
  return MDX_OK;
}

int mdx_set_timing(mdx_ctx* x, int groups) {
  if (check_ctx(x) || groups < 0 || groups > 7) return MDX_E_INVALID;
  x->timing = (unsigned)groups;
  for (int g = 0; g < 3; ++g)
    if ((x->timing >> g) & 1u) x->used[g] = 0;
  return MDX_OK;
}

int mdx_get_timing(mdx_ctx* x, int group, double* mean_ms, int64_t* launches) {
  if (check_ctx(x) || group < 0 || group > 2 || !mean_ms || !launches) return MDX_E_INVALID;
  MDX_TRY(hipStreamSynchronize(x->c.stream));
  double tot = 0.0;
  for (size_t k = 0; k < x->used[group]; ++k) {
    float ms = 0.f;
    MDX_TRY(hipEventElapsedTime(&ms, x->ev[group][k].first, x->ev[group][k].second));
    tot += ms;
  }
  *launches = (int64_t)x->used[group];
  *mean_ms = x->used[group] ? tot / (double)x->used[group] : 0.0;
  return MDX_OK;
}

}  // extern "C"
