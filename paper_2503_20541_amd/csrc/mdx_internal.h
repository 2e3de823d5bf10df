// Internal declarations shared by the translation units of libmdx.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <vector>

#include "mdx.h"

namespace mdx {

constexpr int kWave = 64;
constexpr int kClusterSize = 4;   // atoms per cluster (slots per tile side)

// Workgroups go to the chip's eight XCDs in turn (block b to XCD b mod 8),
// and each XCD has its own L2. A kernel whose consecutive blocks work on
// neighbouring atoms numbers its blocks with xcd_block(nwork), nwork being
// the blocks that hold work at this launch (the grid is sized for the
// largest count): XCD x takes the contiguous logical blocks
// [x p, (x+1) p), p = ceil(nwork / 8), so its L2 holds the data of one region
// of the box instead of the whole box, and the work stays even over the
// XCDs. Blocks left over return -1 (no work). The grid is a multiple of
// eight blocks (xcd_grid) and at least nwork.
constexpr int kXcds = 8;
inline int xcd_grid(int nb) { return (nb + kXcds - 1) / kXcds * kXcds; }
__device__ __forceinline__ int xcd_block(int nwork) {
  const int per = (nwork + kXcds - 1) / kXcds;
  const int i = (int)(blockIdx.x / kXcds);
  return i < per ? (int)(blockIdx.x % kXcds) * per + i : -1;
}
// Atoms per context: kernels address per-atom arrays ([3][n] floats at most)
// and the slot arrays by 32-bit byte offsets (ld32).
constexpr int kMaxAtoms = 100000000;
// Atoms from which mdx_integrate_step evaluates the PME force gather and the
// bonded and exclusion terms in a side kernel on the second stream, beside
// the pair kernel; in smaller systems the second stream is the longer one
// already, and the closing kernel evaluates them.
constexpr int kSideStreamMinAtoms = 40000;
constexpr int kMaxLjTypes = 32;   // LJ atom types (the pair kernel keeps the type-pair table in LDS)
// PME spreading bricks: kBrickXY x kBrickXY x kBrickZ grid points (smaller
// along a dimension with fewer grid points)
constexpr int kBrickXY = 8;
constexpr int kBrickZ = 8;

// Indices into the FP64 partial-sum rows written by force kernels.
// kRowVir + k and kRowVirB + k: virial component k (xx, yy, zz, xy, xz, yz) of
// the pair kernel (or of the PME z pass) and of the bonded/exclusion kernel.
enum PartialRow {
  kRowLJ = 0, kRowDir, kRowExcl, kRowBond, kRowAngle, kRowRec, kRowKin,
  kRowKinRigid,   // rigid water: kinetic energy change of the velocity projection
  kRowVir, kRowVirB = kRowVir + 6, kRowCount = kRowVirB + 6
};

// Adds s * d (x) d (symmetric: xx, yy, zz, xy, xz, yz) to w.
__device__ __forceinline__ void vir_add_dd(double* w, double s, double dx, double dy, double dz) {
  w[0] += s * dx * dx;
  w[1] += s * dy * dy;
  w[2] += s * dz * dz;
  w[3] += s * dx * dy;
  w[4] += s * dx * dz;
  w[5] += s * dy * dz;
}

// Half list: the forces that the tiles naming slot s's cluster as their
// j-cluster put on s (the tiles' j partials), entries first, first + step, ...
// of the cluster's incoming list, in list order. jpart null: full list.
struct JParts {
  const float* jpart;       // [tile][3][4]
  const int* in_count;      // [max_clusters]
  const int* in_sorted;     // [max_clusters][cap]
  int cap;
};

__device__ __forceinline__ void add_jparts(const JParts& jp, int s, int first, int step, float& fx,
                                           float& fy, float& fz) {
  const int c = s / kClusterSize, jb = s - c * kClusterSize;
  const int nin = min(jp.in_count[c], jp.cap);
  const int* lst = jp.in_sorted + (size_t)c * jp.cap;
  for (int k = first; k < nin; k += step) {
    const float* t = jp.jpart + (size_t)lst[k] * 12 + jb;
    fx += t[0];
    fy += t[4];
    fz += t[8];
  }
}

// Geometry of the x-y column grid and the float32 predicate constants.
struct CellGrid {
  int n[3];          // columns along x and y (n[2] = 1)
  int ncell;         // columns
  float inv_w[3];    // n_d / L_d (float32, used only for binning)
  float L[3];
  float hL[3];
  float rnl2;        // fl(r_nl * r_nl)
  float rc2;         // fl(r_c * r_c)
  float r_search;    // cluster-box distance below which a tile is tested
  int nzb;           // z bins of the per-column cluster lookup tables
  float inv_zb;      // nzb / L_z
};

struct PmeGrid {
  int K[3];
  int Kxh;           // K_x / 2 + 1
  int B[3];          // brick edge (grid points)
  int nb[3];         // bricks per dimension
  int nbrick;
  float scale_hi[3]; // K_d / L_d as a float32 pair (hi + lo)
  float scale_lo[3];
  float disp_max;    // r_g / 2 plus margin: how far an atom may sit outside its cell
};

// Scratch of the reverse (adjoint) pass, allocated by its first call.
struct AdjScratch {
  bool ready = false;
  float* u = nullptr;          // [3][n] tangent c p / m of the node
  float4* us = nullptr;        // [max_slots] (u, charge direction) by slot
  float* dfs = nullptr;        // [3][max_slots] pair Hessian-vector product by slot
  double* gslot = nullptr;     // [3][max_slots] pair parameter terms by slot
  double* gatom = nullptr;     // [3][n] parameter terms by atom
  float* dq = nullptr;         // [n] charge direction (mdx_set_charge_direction)
  float* phi2 = nullptr;       // [K^3] potential of the dipole grid
  double* dt_part = nullptr;   // [blocks] dt-gradient partials of a node
  int* gate = nullptr;         // [1] rebuild request of a node
  float4* lj_f = nullptr;      // [T*T] parameter-derivative factors (e1, e2, g1, g2)
  double4* lj_d = nullptr;     // [T*T] energy parameter-derivative factors
  // one segment's forward states: positions, velocities, forces, potential
  int rec_steps = 0;
  float* rec_x = nullptr;      // [rec_steps + 1][3][n]
  float* rec_v = nullptr;
  float* rec_f = nullptr;
  float* rec_phi = nullptr;    // [rec_steps + 1][K^3]
  float* pos = nullptr;        // [3][n] the segment's running state
  float* vel = nullptr;
  float* force = nullptr;
  std::vector<float> dq_h;     // host copy of the charge direction
};

struct Ctx {
  int device = 0;
  hipStream_t stream = nullptr;
  // the launches are being captured into a graph: no events recorded by a
  // kernel's own dispatch (explicit records instead)
  bool capturing = false;
  // bumped by every change that a captured graph would not see (buffers
  // reallocated, rigid water, Langevin, a new list build phase)
  uint64_t version = 0;
  int n = 0;              // atoms
  int npad = 0;           // n rounded up to a wave multiple (ELL stride)
  float box[3];
  float r_cut, r_ghost, r_list, switch_r;
  double alpha = 0.0;
  double coulomb_k = 0.0, accel = 1.0, boltzmann = 1.0;
  double e_self = 0.0;    // Eq. 12 + neutralising term (host FP64, fixed charges)
  bool has_coulomb = false, has_pme = false, has_switch = false;   // has_coulomb: Ewald
  bool rf = false;             // reaction-field Coulomb (Eq. 8) instead of Ewald
  double k_rf = 0.0, c_rf = 0.0;
  bool half_list = false;      // each pair once (MDX_OPT_HALF_LIST), j forces through jpart
  int coop_blocks = 0;         // grid of the single-launch list build (0: one kernel per phase)
  int n_types = 0, n_excl = 0, n_bonds = 0, n_angles = 0;
  int cell_div = 2;
  int nl_cap = 0;               // tiles per i-cluster
  int rebuild_every = 10;
  int steps_since_build = -1;   // -1: no list
  int64_t steps_taken = 0;
  CellGrid cg{};
  PmeGrid pg{};

  // ---- per-atom parameters (caller order) ----
  float* q = nullptr;          // charge
  int* atype = nullptr;        // LJ type
  float4* lj_f = nullptr;      // [T*T] (c12, c6, 12 c12, 6 c6), c_n = 4 eps sigma^n, FP32
  double2* lj_d = nullptr;     // [T*T] (c12, c6) in FP64 for energies
  float* hdt_scale = nullptr;  // accel / m_i  (times dt/2 at use)
  float* pos_alt = nullptr;    // [3][n] second position buffer of mdx_integrate_step
  // Langevin (BAOAB) opening half, mdx_set_langevin
  bool langevin = false;
  double lv_kT = 0.0, lv_gamma = 0.0;
  unsigned long long lv_seed = 0;
  float* lv_sig = nullptr;     // [n] sqrt(kT accel / m_i)
  std::vector<float> mass_h;   // [n] masses (host copy)
  // current parameters (host copies; mdx_set_parameters replaces them)
  std::vector<float> sig_h, eps_h;   // [n_types]
  std::vector<float> q_h;            // [n] charges as used (0 without electrostatics)
  AdjScratch adj;
  // rigid water (mdx_set_rigid_water)
  int n_rigid = 0;
  int* rigid_mols = nullptr;   // [n_rigid][3] caller atoms O, H1, H2
  float rigid_d[3] = {0.f, 0.f, 0.f};
  bool rigid_settle = false;   // closed form: both hydrogens of every molecule weigh the same
  // direct reciprocal Ewald sum (mdx_compute_ewald_direct): scratch for the
  // largest n_max asked for so far
  int ew_nmax = 0;
  double2* ew_tab = nullptr;   // [3][2 n_max + 1][n] phase factors
  double2* ew_S = nullptr;     // [K] structure factors of the half-space vectors
  double* ew_eterm = nullptr;  // [K] their energy terms
  float* mass = nullptr;
  // exclusions per atom (CSR, caller order, both directions)
  int* ex_start = nullptr;
  int* ex_idx = nullptr;
  // bonded terms and per-atom term lists (CSR)
  int* bonds = nullptr;  float* bond_k = nullptr;  float* bond_r0 = nullptr;
  int* angles = nullptr; float* angle_k = nullptr; float* angle_t0 = nullptr;
  int* bt_start = nullptr; int* bt_idx = nullptr;   // bond ids per atom
  int* at_start = nullptr; int* at_idx = nullptr;   // angle ids per atom

  // ---- column sort / cluster slots ----
  int max_slots = 0;           // n + (kClusterSize - 1) * columns, a bound on the slots
  int max_clusters = 0;
  int* cell_of = nullptr;      // [n] column of each caller atom at build
  int* cell_count = nullptr;   // [ncol] atoms per column
  int* cell_start = nullptr;   // [ncol + 1] first atom (unpadded) of each column
  int* slot_start = nullptr;   // [ncol + 1] first slot of each column (padded to clusters)
  int* meta = nullptr;         // [8] slots, clusters of the last build; builds so far;
                               // blocks done binning (the last one scans, then clears it);
                               // 1 if the last build placed every atom (the next one
                               // may bin in its slot order)
  int* col_atoms = nullptr;    // [ncol][col_cap] atoms binned into each column (unordered)
  int col_cap = 0;
  int* perm = nullptr;         // [max_slots] slot -> caller atom, -1 for padding
  int* inv_perm = nullptr;     // [n] caller atom -> slot
  int2* zbin = nullptr;        // [columns][nzb + 1] first cluster with max z >= bin z, first
                               // cluster with min z > bin z (per build)
  float4* xs = nullptr;        // [max_slots] (x, y, z, q) at the current positions
  float* fslot = nullptr;      // [3][max_slots] pair forces by slot; all zero between
                               // a force evaluation's consumer and the next pair kernel
  float* fside = nullptr;      // [3][max_slots] bonded + exclusion forces by slot, from
                               // the second stream (PME contexts; mdx_integrate_step)
  int* ts = nullptr;           // [max_slots] LJ type
  float* zb = nullptr;         // [max_slots] z at the last build (sorted within a column)
  float4* box_lo = nullptr;    // [max_clusters] cluster box (w = real atoms)
  float4* box_hi = nullptr;
  float4* col_xy = nullptr;     // [ncell] x min, x max, y min, y max of a column's atoms
  int* img = nullptr;           // [3][n] periodic image counters (atom order)
  float* xc = nullptr;          // [3][n] Kahan compensation of x and v (MDX_OPT_KAHAN_VV)
  float* vc = nullptr;
  float* x_build = nullptr;    // [3][n] positions at the last build (caller order)
  // [max_clusters][nl_cap] tiles: x = j-cluster, y = 16-bit pair mask (bit
  // 4 a + b: i slot a, j slot b) | periodic image of the j-cluster << 16
  // (2 bits per axis, image_code values; one image for all pairs of a tile)
  uint2* tiles = nullptr;
  int* tile_count = nullptr;   // [max_clusters]
  int* nl_needed = nullptr;    // [1] max tiles one cluster needed in the last build, if
                               // above nl_cap (0 otherwise)
  unsigned* flags = nullptr;   // [1] latched MDX_FLAG_*
  int* gate = nullptr;         // [4] rebuild requests inside mdx_integrate_step (step parity),
                               // then pruned-list invalid flags (step parity)
  uint2* ptiles = nullptr;     // [max_clusters][nl_cap] pruned tile list
  int* pcount = nullptr;       // [max_clusters]
  float4* xp = nullptr;        // [max_slots] slot positions when the pruned list was made
  // Half list: the j-atom forces of each tile (summed over its 4 i atoms) go
  // to jpart at the tile's full-list position [max_clusters * nl_cap][3][4]
  // (component, j slot); ppos gives a pruned tile's full-list position. The
  // tiles whose j-cluster is c are listed, by full-list position, at
  // in_sorted[c * nl_cap ...] (in_count[c] of them; the tile search appends
  // them to in_fill in any order, the pair kernel sorts them), and the
  // closing kernel sums them in that order.
  float* jpart = nullptr;
  int* ppos = nullptr;         // [max_clusters][nl_cap]
  int* in_count = nullptr;     // [max_clusters]
  int* in_fill = nullptr;      // [max_clusters][nl_cap]
  int* in_sorted = nullptr;    // [max_clusters][nl_cap]
  JParts jparts() const { return JParts{jpart, in_count, in_sorted, nl_cap}; }
  float prune_r2 = 0.f;        // fl(r_p^2), r_p = r_c + 0.4 r_g
  float prune_move2 = 0.f;     // (0.19 r_g)^2: displacement that invalidates the pruned list

  // ---- PME ----
  float* grid_q = nullptr;     // [Kz][Ky][Kx] real
  float2* grid_c = nullptr;    // [Kz][Ky][Kxh] complex
  float* grid_phi = nullptr;   // [Kz][Ky][Kx]
  float2* tw[3] = {nullptr, nullptr, nullptr};  // twiddles exp(-2 pi i k/K_d)
  double* bmod[3] = {nullptr, nullptr, nullptr}; // |b_d(m)|^2
  double* mrec[3] = {nullptr, nullptr, nullptr}; // m'_d / L_d
  double* pme_g = nullptr;     // [Ky][Kxh][Kz] influence function B(m) exp(-pi^2 m^2 / alpha^2)
                               // / m^2 (0 at m = 0), without 1/(pi V); box and alpha are fixed
  double pme_energy_scale = 0.0;                 // 1 / (pi V)
  int* brick_cols = nullptr;   // per brick index along x, y: first column, count
  float* brick_z = nullptr;    // per brick index along z: z range [lo, hi) of atoms that reach it
  int4* brick_zr = nullptr;    // [brick layers along z][columns] (first slot, count) of the two
                               // periodic segments of the column inside that z range (per build)

  // ---- reductions ----
  double* partials = nullptr;  // [kRowCount][max_blocks]
  int max_blocks = 0;
  double* energy_scratch = nullptr;   // [MDX_N_ENERGY]
  float* force_scratch = nullptr;     // [3][n] forces inside integrate_step
  int nb_blocks = 0;                  // blocks used by the last nonbonded launch
  int pme_blocks = 0;
  int finish_blocks = 0;              // blocks of the fused closing kernel
};

// ---- launchers (each returns hipError_t of the launch) ----
hipError_t launch_fill_i32(int* p, int v, int count, hipStream_t s);
// gate == nullptr: unconditional build; otherwise every build kernel returns
// at once unless *gate != 0. `done` (if given) is recorded by the column
// sort's dispatch: the slot positions and the PME brick slot ranges are then
// in place (before the tile search), for work on another stream that needs
// only those.
hipError_t launch_build_list(Ctx& c, const float* pos, const int* gate = nullptr,
                             hipEvent_t done = nullptr);
// Copies pos into the slot array (as build position + minimum-image
// displacement, like the integrator) and tests the r_g/2 validity rule; a
// violation latches MDX_FLAG_NL_STALE.
hipError_t launch_refresh_sorted(Ctx& c, const float* pos);
// Blocks of the cooperative list build that are co-resident on the current
// device (0 if cooperative launches are not available).
int build_coop_blocks(int max_clusters, int n, int ncol);
// gate_now / pgate_now: the step's rebuild and prune flags inside
// mdx_integrate_step (null for stand-alone calls: full list, no pruning).
// virial: also the FP64 virial partial rows (kRowVir), implies energy.
// t_start / t_stop (optional): events recorded by the kernel's dispatch.
hipError_t launch_nonbonded(Ctx& c, bool energy, const int* gate_now = nullptr,
                            const int* pgate_now = nullptr, bool virial = false,
                            hipEvent_t t_start = nullptr, hipEvent_t t_stop = nullptr);
// virial: also the partial rows kRowVirB, implies energy.
hipError_t launch_bonded_excl(Ctx& c, const float* pos, float* force, bool energy,
                              bool virial = false);
// out[9] (row-major, symmetric) = sum over the sources s of scale[s] times the
// partial rows row0[s] + k (k = xx, yy, zz, xy, xz, yz) over nblk[s] blocks.
hipError_t launch_reduce_virial(Ctx& c, const int* row0, const int* nblk, const double* scale,
                                int nsrc, double* out);
// Sums the FP64 partial rows into out[slot - slot_base] (slots MDX_ENERGY_*);
// const_slot >= 0 also stores const_val there, zero_slot >= 0 stores 0.
// rigid_blocks > 0: the kinetic row also takes the kRowKinRigid partials of
// that many blocks.
hipError_t launch_reduce_energy(Ctx& c, const int* rows, const int* nblk, int nrows, double* out,
                                int slot_base, double const_val, int const_slot,
                                int zero_slot = -1, int rigid_blocks = 0);
bool pme_size_supported(int K);
// virial: also the reciprocal-space virial partial rows (kRowVir).
hipError_t launch_pme(Ctx& c, float* force, bool energy, bool virial = false);
// Fused per-slot step kernels used by mdx_integrate_step.
// The flags of one step: its rebuild and prune gates, the next step's (which
// the opening kernel clears), and whether the rebuild cadence falls on it.
struct StepGates {
  int* gate_now;
  int* gate_next;
  int* pgate_now;
  int* pgate_next;
  bool cadence;
  long long step;   // the step's index among all the context's steps (Langevin noise)
};
// Opening half of a step: positions read from pos and written to pos_out
// (in place when pos_out is null).
hipError_t launch_begin_step(Ctx& c, float* pos, float* vel, const float* force, float dt,
                             const StepGates& g, float* pos_out = nullptr);
// Closing half of a step at positions pos. With `next`, the same kernel then
// opens the following step (gates *next) from the closing kick's velocities
// and forces, reading pos and writing the new positions to pos_next (another
// buffer: the bonded terms of other atoms still read pos).
// Whether the closing half's PME, bonded and exclusion forces come from the
// side kernel (PME contexts of at least kSideStreamMinAtoms atoms).
inline bool side_terms_used(const Ctx& c) { return c.has_pme && c.n >= kSideStreamMinAtoms; }
// When side_terms_used, the PME, bonded and exclusion forces are not
// evaluated here: their sum by slot is read from c.fside (launch_side_terms
// of the same step, which must precede it).
hipError_t launch_finish_step(Ctx& c, const float* pos, float* vel, float* force, float dt,
                              bool energy, const StepGates* next = nullptr,
                              float* pos_next = nullptr);
// side_terms_used contexts: the closing half's PME force interpolation and bonded and
// exclusion terms at positions pos (slot positions c.xs), summed by slot into
// c.fside (and their energy rows of the closing kernel's partials) on stream
// s, after the FFT passes; `done` (if given) is recorded by the kernel's own
// dispatch.
hipError_t launch_side_terms(Ctx& c, const float* pos, bool energy, hipStream_t s,
                             hipEvent_t done);
// Rigid water: SHAKE after the drift (x_old: positions before it) with the
// velocity correction, wrap, slot refresh and validity tests (x_old: positions
// before the drift, y_in: after it, pos: output, which may be x_old or y_in);
// RATTLE velocity projection after the closing kick.
hipError_t launch_rigid_positions(Ctx& c, const float* x_old, const float* y_in, float* pos,
                                  float* vel, float dt, const StepGates& g);
// energy: also the kinetic energy change of the projection (kRowKinRigid
// partials, one per 64 molecules; returns the block count in *blocks).
hipError_t launch_rigid_velocities(Ctx& c, const float* pos, float* vel, bool energy = false,
                                   int* blocks = nullptr);
// Spread + FFT passes only (the potential grid), for the fused closing kernel.
// `done` (may be null) is recorded by the last kernel's own dispatch.
hipError_t launch_pme_spread(Ctx& c, hipStream_t s, hipEvent_t done);
// Pencils per block of the FFT column passes for a half spectrum of kxh
// columns (the z pass writes one energy partial per block).
int pme_col_pencils(int kxh);
// The tangent of the charge grid along per-slot displacements us[slot].xyz
// (sum of q u . grad theta) into grid_q, on the context's stream.
hipError_t launch_pme_spread_dipole(Ctx& c, const float4* us);
// virial: the z pass also writes the reciprocal-space virial rows (kRowVir).
hipError_t launch_pme_fft(Ctx& c, hipStream_t s, hipEvent_t done, bool virial = false);
// Direct reciprocal Ewald sum over |n_d| <= nmax into force (accumulated);
// energy (dev double[1], may be null) overwritten. Scratch sized for nmax.
hipError_t launch_ewald_direct(Ctx& c, const float* pos, float* force, double* energy, int nmax,
                               double2* tab, double2* S, double* eterm);
// The same sum with its scratch (phase tables, structure factors, energy
// terms) in the library's fixed per-device array of kEwScratchBytes, so the
// call allocates nothing. ewald_scratch_setup(device), with that device
// current, takes the array's device address once (mdx_create calls it).
// hipErrorInvalidValue when the scratch of (n, nmax) exceeds the array.
constexpr size_t kEwScratchBytes = 32u << 20;
hipError_t ewald_scratch_setup(int device);
size_t ewald_scratch_bytes(int n, int nmax, size_t* off_S = nullptr, size_t* off_e = nullptr);
hipError_t launch_ewald_direct_static(Ctx& c, const float* pos, float* force, double* energy,
                                      int nmax);

// Reverse pass (adjoint.hip). A node: launch_adj_pre (p <- p + dt q, dt
// partials, tangent u), launch_adj_slots (slot refresh and gated rebuild at
// pos when `refresh`, tangent by slot), launch_pair_jvp, the dipole spread
// and FFT passes, launch_jvp_finish (q += wdt dF, parameter terms by atom),
// launch_adj_reduce. eparam: the energy's parameter derivatives instead.
hipError_t launch_adj_pre(Ctx& c, float dt, float w, bool open, const float* q, float* p,
                          const float* v_n, const float* f_n, double* gmass);
hipError_t launch_adj_slots(Ctx& c, const float* pos, bool refresh);
hipError_t launch_pair_jvp(Ctx& c, bool eparam);
hipError_t launch_jvp_finish(Ctx& c, bool eparam, const float* pos, const float* phi,
                             const float* dphi, float* q, float wdt);
hipError_t launch_adj_begin(Ctx& c, const float* gx, const float* gv, const double* gU,
                            const float* force, float* q, float* p);
hipError_t launch_adj_inject(Ctx& c, const float* gx, const float* gv, const double* gU,
                             const float* force, float* q, float* p);
hipError_t launch_adj_reduce(Ctx& c, double scale, const double* scale_dev, double q_const,
                             int dt_blocks, double* grad);
hipError_t launch_unwrap(Ctx& c, const float* pos, float* out);

// Device helpers shared by kernels -------------------------------------------

// Accurate float32 minimum-image displacement x_j - x_i (see mdx.h); the
// operations are not contracted so the result is the specified expression.
// First index in [lo, hi) with a[index] >= v (a nondecreasing).
__device__ __forceinline__ int lower_bound_f(const float* __restrict__ a, int lo, int hi, float v) {
  while (lo < hi) {
    int mid = (lo + hi) >> 1;
    if (a[mid] < v) lo = mid + 1; else hi = mid;
  }
  return lo;
}

__device__ __forceinline__ float min_image(float xi, float xj, float L, float hL) {
#pragma clang fp contract(off)
  float s = xj - xi;
  float up = (xj - L) - xi;
  float dn = xj + (L - xi);
  float d = s > hL ? up : s;
  return s < -hL ? dn : d;
}

// The same expression with L - x_i supplied by the caller (hoisted out of a
// loop over j); every operand is computed, so it compiles to selects.
__device__ __forceinline__ float min_image_h(float xi, float Lmxi, float xj, float L, float hL) {
#pragma clang fp contract(off)
  float s = xj - xi;
  float up = (xj - L) - xi;
  float dn = xj + Lmxi;
  float d = s > hL ? up : s;
  return s < -hL ? dn : d;
}

// The image min_image_h takes for x_j: 0 (x_j itself), 1 (x_j - L) or
// 2 (x_j + L).
__device__ __forceinline__ unsigned image_code(float xi, float xj, float hL) {
#pragma clang fp contract(off)
  const float s = xj - xi;
  return s > hL ? 1u : (s < -hL ? 2u : 0u);
}

// x_j - x_i at a given image, rounded exactly as min_image_h rounds it: am is
// -L for image 1 and 0 otherwise, cp is L for image 2 and 0 otherwise.
__device__ __forceinline__ float image_diff(float xi, float xj, float am, float cp) {
#pragma clang fp contract(off)
  return (xj + am) + (cp - xi);
}

// image_diff at image 0 (am = cp = 0): (x_j + 0) + (0 - x_i) is x_j - x_i
// rounded once, the same value in one operation.
__device__ __forceinline__ float plain_diff(float xi, float xj) { return xj - xi; }

// Kahan-compensated s + y: c carries the rounding error of the previous sum
// into this one and receives this one's.
__device__ __forceinline__ float kahan_add(float s, float y, float& c) {
#pragma clang fp contract(off)
  const float yc = y - c;
  const float t = s + yc;
  c = (t - s) - yc;
  return t;
}

// Element i of a device array, addressed as the array's (wave-uniform) base
// plus a 32-bit byte offset: the load then takes a scalar base and one 32-bit
// lane offset instead of 64-bit per-lane address arithmetic. The arrays read
// this way stay below 4 GB (kMaxAtoms).
template <typename T>
__device__ __forceinline__ T ld32(const T* __restrict__ base, unsigned i) {
  return *reinterpret_cast<const T*>(reinterpret_cast<const char*>(base) +
                                     i * (unsigned)sizeof(T));
}

__device__ __forceinline__ float dist2(float dx, float dy, float dz) {
#pragma clang fp contract(off)
  float a = dx * dx;
  float b = dy * dy;
  float c = dz * dz;
  return (a + b) + c;
}

// Wave-level sum of a double (all 64 lanes participate).
__device__ __forceinline__ double wave_sum(double v) {
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, kWave);
  return v;
}

// Block-level deterministic FP64 sum (blockDim.x multiple of 64, <= 1024).
__device__ __forceinline__ double block_sum(double v, double* lds) {
  v = wave_sum(v);
  int lane = threadIdx.x & (kWave - 1), w = threadIdx.x / kWave;
  if (lane == 0) lds[w] = v;
  __syncthreads();
  double r = 0.0;
  if (threadIdx.x == 0) {
    int nw = blockDim.x / kWave;
    for (int i = 0; i < nw; ++i) r += lds[i];
  }
  __syncthreads();
  return r;
}

}  // namespace mdx
