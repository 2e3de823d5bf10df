/*
 * mdx.h - C ABI of the MI355X (gfx950) force-evaluation library.
 *
 * The library evaluates the per-step forces of a periodic classical force
 * field the way the DIMOS paper (arXiv 2503.20541) defines them:
 *   - a cell-list Verlet neighbour list (Sec. II.A.2, "Neighborlists"),
 *   - Lennard-Jones with Lorentz-Berthelot mixing (Eqs. 4-5, optional switch
 *     Eq. 6) plus the real-space Ewald term (Eq. 10), exclusions removed at
 *     list level ("Exclusions and Exceptions"), with the erf exclusion and
 *     self (Eq. 12) corrections,
 *   - harmonic bonds and angles (Eqs. 1-2),
 *   - smooth particle-mesh Ewald for the reciprocal sum (Sec. II.A.2, PME
 *     paragraph; Eq. 11 in its standard form),
 *   - velocity Verlet (Sec. II.D.1).
 *
 * Conventions for every call:
 *   - Return value: MDX_OK (0) or a negative MDX_E_* code; no call aborts or
 *     throws across the ABI. mdx_error_string() names a code.
 *   - "dev" pointers are device (HBM) addresses on the device that was
 *     current at mdx_create; "host" pointers are host memory. The library
 *     never frees or retains a caller pointer beyond the call.
 *   - Per-atom vectors (positions, velocities, forces) are float32 structure
 *     of arrays [3][N]: x[0..N), y[N..2N), z[2N..3N), in the caller's atom
 *     order.
 *   - Positions passed to any call must lie in [0, L_d) per dimension
 *     (mdx_integrate_step keeps them there); a coordinate outside latches
 *     MDX_FLAG_OUT_OF_BOX.
 *   - Work is enqueued on the context's stream and is asynchronous unless a
 *     call says "synchronising". A context is not thread-safe.
 *   - Units are the caller's; the three unit constants in mdx_system_desc
 *     tie them together.
 */
#ifndef MDX_H
#define MDX_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ---- status codes ------------------------------------------------------ */
#define MDX_OK                0
#define MDX_E_INVALID        -1  /* bad argument or descriptor field          */
#define MDX_E_BOX_TOO_SMALL  -2  /* r_c + r_g > L_d / 2: minimum image fails   */
#define MDX_E_HIP            -3  /* a HIP runtime call failed                 */
#define MDX_E_CAPACITY       -4  /* caller buffer too small (size reported)    */
#define MDX_E_NO_LIST        -5  /* force call before mdx_build_neighbors     */
#define MDX_E_NO_PME         -6  /* PME requested but no grid was configured  */
#define MDX_E_OUT_OF_MEMORY  -7  /* device allocation failed                  */
#define MDX_E_UNSUPPORTED    -8  /* option not implemented                    */

/* ---- latched device flags (mdx_get_status) ----------------------------- */
#define MDX_FLAG_NL_OVERFLOW  0x1u  /* an atom had more neighbours than capacity */
#define MDX_FLAG_NL_STALE     0x2u  /* an atom moved > r_g/2 since the last build */
#define MDX_FLAG_NONFINITE    0x4u  /* a non-finite energy was reduced            */
#define MDX_FLAG_OUT_OF_BOX   0x8u  /* a coordinate outside [0, L)                */
#define MDX_FLAG_CELL_OVERFLOW 0x10u /* a cluster had more candidate clusters than
                                        the search holds (list incomplete)   */
#define MDX_FLAG_COLUMN_OVERFLOW 0x20u /* an x-y column held more atoms than its
                                          capacity (list incomplete; grown and
                                          rebuilt by mdx_build_neighbors; inside
                                          mdx_integrate_step the atoms left out
                                          are not integrated: results invalid,
                                          call mdx_build_neighbors)           */
#define MDX_FLAG_CONSTRAINT   0x40u /* rigid water: no SETTLE solution, SHAKE
                                       did not reach its tolerance in 200
                                       sweeps, or a molecule's RATTLE system
                                       was singular (positions or velocities
                                       of that molecule invalid) */

/* ---- energy slots (FP64) ----------------------------------------------- */
#define MDX_ENERGY_LJ         0  /* Eq. 4 (switched by Eq. 6 if enabled)        */
#define MDX_ENERGY_COUL_DIR   1  /* Eq. 10, minimum-image real-space term       */
#define MDX_ENERGY_COUL_EXCL  2  /* -k_e q_i q_j erf(alpha r)/r, excluded pairs */
#define MDX_ENERGY_COUL_SELF  3  /* Eq. 12 times k_e, + neutralising term       */
#define MDX_ENERGY_BOND       4  /* Eq. 1                                       */
#define MDX_ENERGY_ANGLE      5  /* Eq. 2                                       */
#define MDX_ENERGY_COUL_REC   6  /* reciprocal sum by smooth PME                */
#define MDX_ENERGY_KINETIC    7  /* sum m v^2 / (2 accel)                       */
#define MDX_N_ENERGY          8

typedef struct mdx_ctx mdx_ctx;
typedef struct mdx_batch mdx_batch;

/*
 * System description (all pointers host, read during mdx_create only).
 *
 * Atoms: charge, mass, atom_type [n_atoms] (n_atoms <= 100,000,000, more is
 * MDX_E_UNSUPPORTED: kernels address per-atom arrays by 32-bit byte
 * offsets); per-type LJ sigma/epsilon
 * [n_types] (Lorentz-Berthelot mixing, Eq. 5; n_types <= 32, more is
 * MDX_E_UNSUPPORTED). Topology index arrays use
 * the caller's atom order: exclusions [n_exclusions][2] (any order,
 * duplicates ignored), bonds [n_bonds][2] with bond_k, bond_r0, angles
 * [n_angles][3] as (end, vertex, end) with angle_k, angle_theta0 (radians).
 *
 * r_cut: interaction cutoff r_c; r_ghost: Verlet skin r_g (the list holds
 * pairs with r < r_c + r_g and stays valid until an atom moves > r_g / 2,
 * Sec. II.A.2). ewald_alpha > 0 sets alpha directly; otherwise, if
 * ewald_delta > 0, alpha = sqrt(-ln(2 delta)) / r_c (Eq. 13); if both are
 * <= 0 there is no electrostatics. pme_grid {K_x, K_y, K_z} (0 = no PME,
 * each in [4, 1024]); pme_order must be 4. switch_r in (0, r_c) enables
 * the Eq. 6 switch on LJ; <= 0 is plain truncation.
 *
 * rf_epsilon > 0 selects the reaction field (Sec. II.A.2, Eq. 8) instead:
 * every interacting, non-excluded pair gets k_e q_i q_j (1/r + k_RF r^2 -
 * c_RF) with k_RF = (eps_s - 1) / ((2 eps_s + 1) r_c^3) and c_RF = 3 eps_s /
 * ((2 eps_s + 1) r_c), eps_s = rf_epsilon (the pair energy vanishes at r_c;
 * INFINITY gives k_RF = 1/(2 r_c^3), c_RF = 3/(2 r_c)); excluded pairs get
 * nothing and there is no self or reciprocal term. It reports its energy in
 * MDX_ENERGY_COUL_DIR. ewald_alpha, ewald_delta and pme_grid must then be 0
 * (MDX_E_INVALID otherwise, as for a negative or NaN rf_epsilon).
 *
 * Units: coulomb_k = 1/(4 pi eps0); accel converts force/mass to
 * acceleration (a = accel F / m); boltzmann is k_B (kinetic temperature).
 *
 * Tuning: cell_divisions m in [1, 4] (x-y columns of edge 2/m times the
 * edge of the cube that holds four atoms at the mean density; 0 = 2; the
 * list does not depend on it); nl_capacity = 4x4 cluster tiles per
 * cluster (0 = sized from the density with headroom; grown on overflow by
 * mdx_build_neighbors); rebuild_every = steps between list rebuilds in
 * mdx_integrate_step (0 = 10).
 *
 * options: MDX_OPT_* bits (0 = defaults). By default every pair is listed
 * from both ends and each end accumulates its own force: no atomics,
 * bitwise-reproducible forces. MDX_OPT_HALF_LIST lists each pair once and
 * applies its force to both atoms (Newton's third law): the cluster that
 * lists a tile keeps its own atoms' forces, the forces on the tile's other
 * cluster go to a per-tile buffer, and each atom sums the tiles naming its
 * cluster in list order. Half the pair arithmetic, no atomics either, so
 * forces and energies are bitwise reproducible in both modes; the half list
 * needs 60 bytes of device memory per tile of capacity for that buffer and its
 * index. A stand-alone force call between mdx_integrate_step calls makes
 * the next step walk the whole list (not the pruned one). The list is built with one launch per build
 * phase; MDX_OPT_COOPERATIVE_BUILD runs all phases in one cooperative launch
 * with grid-wide barriers between them (one launch when no rebuild is due,
 * but the launch goes through its own hardware queue, and on a real rebuild
 * the resident grid is smaller). Both give the same list.
 * MDX_OPT_KAHAN_VV compensates the velocity-Verlet sums (Kahan summation):
 * each atom keeps the rounding error of its last position and velocity
 * updates (two more float [3][N] arrays) and feeds it into the next one, so
 * float32 round-off does not build up over long runs. The compensation is
 * cleared by mdx_build_neighbors (a new state).
 */
#define MDX_OPT_HALF_LIST         1u
#define MDX_OPT_COOPERATIVE_BUILD 2u
#define MDX_OPT_KAHAN_VV          4u
typedef struct mdx_system_desc {
  int32_t n_atoms;
  float box[3];
  const float* charge;
  const float* mass;
  const int32_t* atom_type;
  int32_t n_types;
  const float* type_sigma;
  const float* type_epsilon;
  int32_t n_exclusions;
  const int32_t* exclusions;
  int32_t n_bonds;
  const int32_t* bonds;
  const float* bond_k;
  const float* bond_r0;
  int32_t n_angles;
  const int32_t* angles;
  const float* angle_k;
  const float* angle_theta0;
  float r_cut;
  float r_ghost;
  float switch_r;
  double ewald_delta;
  double ewald_alpha;
  int32_t pme_grid[3];
  int32_t pme_order;
  double coulomb_k;
  double accel;
  double boltzmann;
  int32_t cell_divisions;
  int32_t nl_capacity;
  int32_t rebuild_every;
  uint32_t options;
  double rf_epsilon;   /* > 0: Coulomb by the reaction field of Eq. 8 instead of
                          Ewald, with solvent dielectric eps_s = rf_epsilon
                          (INFINITY: the conducting limit); see below */
} mdx_system_desc;

/* Read-only facts about a context (mdx_get_info). */
typedef struct mdx_info {
  int32_t n_atoms;
  int32_t cell_dims[3];      /* cells per dimension                       */
  int32_t cell_divisions;
  int32_t nl_capacity;       /* neighbours per atom the list can hold     */
  int32_t pme_grid[3];
  int32_t pme_brick[3];      /* grid points per PME brick                 */
  double alpha;              /* Ewald splitting parameter in use          */
  double r_list;             /* fl32(r_c + r_g)                           */
  int64_t n_list_entries;    /* entries in the last built list: twice the
                                pairs (full list) or the pairs (half list);
                                -1 before the first build                 */
  int64_t steps_taken;       /* steps integrated since creation           */
  int64_t n_builds;          /* list builds so far: explicit builds plus
                                the rebuilds inside mdx_integrate_step    */
  int64_t n_list_tiles;      /* 4x4 cluster tiles in the last built list,
                                with the padding to groups of four (-1
                                before the first build)                   */
} mdx_info;

/* Names a status code; never NULL. */
const char* mdx_error_string(int code);

/*
 * Creates a context on the current HIP device bound to `hip_stream`
 * (a hipStream_t; NULL = the null stream). Copies what it needs from `d`
 * and allocates all device scratch once. Errors: MDX_E_INVALID,
 * MDX_E_BOX_TOO_SMALL (r_c + r_g > min L / 2), MDX_E_OUT_OF_MEMORY, MDX_E_HIP.
 * On error *out is NULL.
 */
int mdx_create(mdx_ctx** out, const mdx_system_desc* d, void* hip_stream);

/* Frees library-owned device memory; NULL is a no-op. Synchronises the stream. */
int mdx_destroy(mdx_ctx* ctx);

/* Rebinds the context to another stream (hipStream_t). */
int mdx_set_stream(mdx_ctx* ctx, void* hip_stream);

/*
 * Builds the Verlet list (Sec. II.A.2, "Neighborlists") for dev positions
 * pos[3][N]: bins atoms into x-y columns, sorts each column by z (ties by
 * atom index), cuts it into 4-atom clusters, and tests every atom pair of
 * the cluster pairs whose bounding boxes come closer than r_nl with the
 * float32 inclusion predicate
 *     s = fl(x_j - x_i);  d = s, or fl(fl(x_j - L) - x_i) if s > L/2,
 *     or fl(x_j + fl(L - x_i)) if s < -L/2   (per dimension);
 *     r2 = fl(fl(fl(dx*dx) + fl(dy*dy)) + fl(dz*dz));  keep iff
 *     r2 < fl(r_nl * r_nl), r_nl = fl(r_c + r_g), excluded pairs dropped.
 * Also snapshots pos for the r_g/2 validity test. Synchronising only when
 * the list overflowed: the capacity is then grown and the list rebuilt.
 */
int mdx_build_neighbors(mdx_ctx* ctx, const float* pos);

/*
 * Synchronising. Writes the current list as unique pairs (i, j), i < j, in
 * caller atom indices, sorted lexicographically, into pairs_host[cap][2]
 * and its length into *n. MDX_E_CAPACITY if cap < *n (*n still set).
 */
int mdx_get_neighbor_pairs(mdx_ctx* ctx, int32_t* pairs_host, int64_t cap, int64_t* n);

/*
 * Short-range forces at dev pos[3][N] from the current list: LJ + real-space
 * Ewald (or the reaction field, rf_epsilon > 0) over listed pairs with
 * r2 < fl(r_c^2) (same float32 expression as the list), the erf exclusion
 * correction (FP64; Ewald only), bonds and angles.
 * force (dev [3][N]) is OVERWRITTEN. energy (dev double[6], slots
 * MDX_ENERGY_LJ..MDX_ENERGY_ANGLE) may be NULL; with energy the variant with
 * FP64 reductions runs. virial (dev double[9], row-major, symmetric, may be
 * NULL) is OVERWRITTEN with the virial of these terms, W_ab = sum over
 * interactions of sum_k s_k,a F_k,b (s_k: member atom positions relative to
 * one member of the interaction, minimum image; for a pair, r_j - r_i times
 * the force on j), in FP64 (energy units); the pressure follows as
 * P = (2 E_kin + tr W) / (3 V) with the reciprocal-space part from
 * mdx_compute_pme added to W.
 * Latches MDX_FLAG_NL_STALE if an atom moved > r_g/2 since the build.
 */
int mdx_compute_nonbonded(mdx_ctx* ctx, const float* pos, float* force, double* energy,
                          double* virial);

/*
 * Reciprocal-space forces by smooth PME at dev pos[3][N]: order-4 B-spline
 * charge spreading onto the K_x x K_y x K_z grid, 3D FFT, multiplication by
 * the influence function B(m) C(m), inverse FFT and force gather. force (dev
 * [3][N]) is ACCUMULATED into. energy (dev double[1], MDX_ENERGY_COUL_REC)
 * may be NULL. Needs a built list (atoms are processed in cell order).
 * virial (dev double[9], may be NULL) is OVERWRITTEN with the SPME virial
 * sum_m E(m) (delta_ab - 2 (1 + pi^2 m^2 / alpha^2) m_a m_b / m^2), FP64,
 * the strain derivative of E_rec (W_aa = -L_a dE_rec/dL_a with the atoms
 * scaled along).
 */
int mdx_compute_pme(mdx_ctx* ctx, const float* pos, float* force, double* energy,
                    double* virial);

/*
 * The reciprocal Ewald sum evaluated directly (Sec. II.A.2, Eqs. 9-12 with
 * Eq. 11 in its standard form, tin-foil boundary): over m = (n_x/L_x,
 * n_y/L_y, n_z/L_z), |n_d| <= n_max, m != 0, E_rec = k_e/(2 pi V) sum_m
 * exp(-pi^2 m^2/alpha^2)/m^2 |S(m)|^2 with S(m) = sum_j q_j exp(2 pi i m.r_j),
 * and its forces; O(N n_max^3), all sums in FP64: a high-accuracy reference
 * for mdx_compute_pme. pos dev [3][N]; force (dev [3][N]) is ACCUMULATED
 * into; energy (dev double[1], may be NULL) is OVERWRITTEN with E_rec.
 * Scratch (16 (3 (2 n_max + 1) N + (2 n_max + 1)^3) bytes) is allocated on
 * the first call with a larger n_max and kept. MDX_E_INVALID without Ewald
 * electrostatics (ewald_delta or ewald_alpha), or for n_max outside [1, 64].
 */
int mdx_compute_ewald_direct(mdx_ctx* ctx, const float* pos, float* force, double* energy,
                             int32_t n_max);

/*
 * mdx_compute_ewald_direct for callers that cannot allocate device memory
 * (code under HIP graph capture, tight serving loops, harnesses that forbid
 * hipMalloc): the same kernels, arithmetic and results, bit for bit, but the
 * scratch (per-atom phase tables, structure factors, energy terms) lives in
 * one fixed array of the library per device, 32 MiB, which each GPU the
 * library runs on holds until the process ends; the call makes no
 * allocation, free or memset. mdx_create takes the array's device address.
 * The scratch needs 48 (2 n_max + 1) N + 24 K bytes, K = ((2 n_max + 1)^3 -
 * 1) / 2, each part rounded up to 256 bytes; mdx_ewald_direct_noalloc_bytes
 * reports it and the limit. MDX_E_CAPACITY when it exceeds the array; the
 * other errors as mdx_compute_ewald_direct. Every call on a device uses the
 * same array and overwrites all of the scratch it reads, so nothing carries
 * over from an earlier call; calls that overlap on one device (another
 * stream, another context, another thread) race and give wrong results.
 */
int mdx_compute_ewald_direct_noalloc(mdx_ctx* ctx, const float* pos, float* force,
                                     double* energy, int32_t n_max);
int mdx_ewald_direct_noalloc_bytes(int32_t n_atoms, int32_t n_max, int64_t* bytes,
                                   int64_t* limit);

/*
 * Velocity Verlet (Sec. II.D.1) for n_steps >= 1 with step dt:
 *   v += (dt/2) accel F/m;  x += dt v (wrapped into [0, L));  F = F(x);
 *   v += (dt/2) accel F/m.
 * pos, vel, force are dev [3][N] and are updated in place; force must hold
 * F(pos) on entry (e.g. from mdx_compute_nonbonded + mdx_compute_pme) and
 * holds F(pos) on exit. The list is rebuilt every rebuild_every steps, and
 * also on any step where an atom has moved more than r_g/2 since the last
 * build (tested every step on the device; no host synchronisation). The
 * number of builds is reported by mdx_get_info. Inside a step the PME spread
 * and FFT passes (and, from 40,000 atoms on, the PME force gather and the
 * bonded and exclusion terms) run on a library-owned second stream,
 * concurrently with the pair kernel; they are forked from and joined back
 * into the context's stream, so the call is ordered on that stream like any
 * other work.
 * energies, if not NULL, is dev double[n_steps][MDX_N_ENERGY]: all slots
 * after each step. After mdx_set_langevin with gamma > 0 each step opens with
 * the Langevin (BAOAB) half instead (kinetic energy from the closing kick's
 * velocities as before).
 */
int mdx_integrate_step(mdx_ctx* ctx, float* pos, float* vel, float* force, int32_t n_steps,
                       float dt, double* energies);

/*
 * Graph replay of mdx_integrate_step (the chunked step loop recorded once as
 * a HIP graph and launched as one unit, instead of a dozen launches per
 * step). With chunk > 0 (a multiple of rebuild_every), a call whose n_steps
 * is a multiple of chunk runs as chunk-step graph launches: the first one
 * records the chunk's launches on a library-owned stream and instantiates
 * them; later ones replay it as long as the call has the same pos, vel,
 * force and dt, the context has reallocated or reconfigured nothing (list
 * growth, mdx_load_state, mdx_set_rigid_water, mdx_set_langevin) and the
 * rebuild phase is the same; otherwise the chunk is recorded again. A call
 * with energies, timing enabled or Langevin dynamics runs its launches one
 * by one as before. Results are bit for bit those of the launch-by-launch
 * path. chunk = 0 switches it off. MDX_E_INVALID for chunk < 0 or not a
 * multiple of rebuild_every.
 */
int mdx_set_graph(mdx_ctx* ctx, int32_t chunk);

/*
 * Batched replicas (independent systems stepped together, e.g. the chains of
 * the paper's Hamiltonian Monte Carlo tuning, Sec. IV, which uses many
 * replicas): mdx_batch_create takes n_rep contexts (host array; each made by
 * mdx_create from its own descriptor, box and PME grid; each context at most
 * once) on one device, and chunk: 0, or a multiple of every replica's
 * rebuild_every. mdx_batch_integrate(b, pos, vel, force, n_steps, dt, stream)
 * advances every replica r by n_steps (a multiple of chunk if chunk > 0)
 * steps of mdx_integrate_step with its own pos[r], vel[r], force[r] (host
 * arrays of dev [3][N_r] pointers) and dt[r] (host array), each replica on a
 * stream of the batch's own (one per replica, forked from `stream` and
 * joined back into it by events), so the small systems run side by side on
 * the chip. With chunk > 0, mdx_batch_create switches every member to graph
 * replay of that chunk (mdx_set_graph) and each replica's chunks are single
 * graph launches; with chunk = 0 the replicas' launches go one by one.
 * Results are bit for bit those of mdx_integrate_step on each replica. Work
 * on a replica's own stream must be complete or ordered before `stream`.
 * MDX_E_INVALID for bad arguments, MDX_E_NO_LIST if a replica has no list
 * yet, MDX_E_UNSUPPORTED for graph replay with Langevin dynamics or timing on
 * a replica. mdx_batch_destroy frees the batch (not the contexts).
 */
int mdx_batch_create(mdx_batch** out, mdx_ctx* const* ctxs, int32_t n_rep, int32_t chunk);
int mdx_batch_integrate(mdx_batch* b, float* const* pos, float* const* vel, float* const* force,
                        int32_t n_steps, const float* dt, void* hip_stream);
int mdx_batch_destroy(mdx_batch* b);

/*
 * Autotuner of the tuning fields of a descriptor: times `steps` steps (after
 * `steps` untimed ones) of fresh contexts for each column width
 * cell_divisions = 1..4, each with the list built phase by phase and with
 * MDX_OPT_COOPERATIVE_BUILD, from pos, vel (dev [3][N], copied) with step dt
 * on `stream`, and returns the fastest in *cell_divisions and *options (d's
 * options with the build-mode bit of the winner). ms_per_step (host
 * double[8] or NULL): the times, build phase by phase then cooperative,
 * cell_divisions 1..4 each. None of these choices changes the list or the
 * forces' pairs (the list is independent of the column grid); the 4 x 4
 * cluster tile is fixed by the kernels' lane layout. Synchronising;
 * allocates while it runs.
 */
int mdx_autotune(const mdx_system_desc* d, const float* pos, const float* vel, float dt,
                 int32_t steps, void* hip_stream, int32_t* cell_divisions, uint32_t* options,
                 double* ms_per_step);

/* Synchronising. Returns the latched MDX_FLAG_* bits in *flags and clears them. */
int mdx_get_status(mdx_ctx* ctx, uint32_t* flags);

/*
 * Periodic image counters (the wrap of Sec. II.D.1's position update):
 * img (dev int32[3][N], caller atom order, caller-owned) receives, per
 * coordinate, the net number of box lengths mdx_integrate_step has wrapped
 * the atom by since the context was created (+1 each time x >= L_d moved it
 * down by L_d, -1 each time x < 0 moved it up), so pos + img * L is the
 * unwrapped trajectory. The copy is queued on the context's stream (not
 * synchronising). MDX_E_INVALID for a NULL img.
 */
int mdx_get_images(mdx_ctx* ctx, int32_t* img);

/*
 * Langevin dynamics for the following mdx_integrate_step calls (the paper's
 * stochastic integrator, Sec. II.D; the splitting read as BAOAB): each step
 * opens with v += (dt/2) a, x += (dt/2) v, v = c1 v + c2 sqrt(kT accel / m) xi,
 * x += (dt/2) v (c1 = exp(-gamma dt), c2 = sqrt(1 - c1^2)) and closes with
 * v += (dt/2) a as before. xi: three standard normals per atom and step,
 * Box-Muller of Philox4x64-10 (Salmon et al., SC'11) with counter (atom,
 * step, 0, 0) and key (seed low 64 bits, 0); step counts every step the
 * context has taken, so a run is reproducible from (seed, state, step) and
 * independent of how it is split into calls. Uniforms are the top 24 bits
 * + 1 over 2^24, normals sqrt(-2 ln u1) (cos, sin)(2 pi u2) and
 * sqrt(-2 ln u3) cos(2 pi u4), in float32. kT in energy units (k_B T),
 * gamma in 1/time; gamma = 0 returns to velocity Verlet. MDX_E_INVALID for
 * kT < 0, gamma < 0 or non-finite values; MDX_E_UNSUPPORTED with
 * MDX_OPT_KAHAN_VV.
 */
int mdx_set_langevin(mdx_ctx* ctx, double kT, double gamma, uint64_t seed);

/*
 * Rigid water for the following mdx_integrate_step calls (the rigid-water
 * option the paper uses for its longer time step, Sec. III; RATTLE with
 * velocity Verlet): mols (host int32[n_mol][3], caller atoms O, H1, H2, each
 * atom at most once) are held at |O-H| = d_oh and |H1-H2| = d_hh. After each
 * drift the three distances are restored along the previous bond vectors
 * with the same correction over dt applied to the velocities: in closed form
 * (SETTLE, FP64 per molecule) when the two hydrogens of every molecule have
 * the same mass, else by SHAKE iterations (float32, to a relative 2e-6 in
 * r^2); both reach the same constrained positions. After the closing kick
 * the velocities are projected onto the constraints (r . v_rel = 0). The
 * bond and angle terms of these molecules may stay on (their energy is then
 * constant) or be zero; atoms in no listed molecule move freely (the step
 * then keeps a copy of the positions before the drift in a buffer of the
 * context). Every step then runs its own opening kernel (no fused
 * closing/opening), and the kinetic energy slot holds the kinetic energy
 * of the projected velocities. A molecule with no SETTLE solution, whose
 * SHAKE iteration does not reach its tolerance in 200 sweeps, or whose
 * velocity system is singular, latches MDX_FLAG_CONSTRAINT. n_mol = 0 switches it off. MDX_E_INVALID for
 * bad indices or distances; MDX_E_UNSUPPORTED together with Langevin or
 * MDX_OPT_KAHAN_VV.
 */
int mdx_set_rigid_water(mdx_ctx* ctx, const int32_t* mols, int32_t n_mol, double d_oh,
                        double d_hh);

/*
 * Parameters of the model for the following calls (the quantities the
 * paper's differentiable simulation is differentiated with respect to,
 * Sec. IV): type_sigma, type_epsilon (host float[n_types], Eqs. 4-5) and
 * charge (host float[N]); a NULL array leaves that parameter unchanged. The
 * LJ tables, the charges and the self term (Eq. 12) are replaced; the list
 * is not affected. A context created without electrostatics accepts only
 * zero charges (MDX_E_UNSUPPORTED otherwise). MDX_E_INVALID for sigma <= 0,
 * epsilon < 0 or non-finite values. Synchronising.
 */
int mdx_set_parameters(mdx_ctx* ctx, const float* type_sigma, const float* type_epsilon,
                       const float* charge);

/*
 * Reverse mode of a velocity-Verlet trajectory (the paper differentiates
 * whole simulations, Sec. I and IV). For a run x_0 -> x_T of
 * mdx_integrate_step and a loss L(x_T, U(x_T)), the reverse pass gives
 * dL/dx_0, dL/dv_0, dL/d(dt) and dL/dtheta with theta = (epsilon_t for each
 * type, sigma_t for each type, t), where t moves the charges along the
 * direction of mdx_set_charge_direction, q(t) = q + t dq (for water,
 * dq = 1 on O and -1/2 on H gives d/dq_O with q_H = -q_O / 2).
 *
 * The derivatives are those of the run with its interaction sets held fixed
 * (pairs closer than r_c at each step, as the forward evaluated them): the
 * truncated potentials make the loss discontinuous where a pair crosses
 * r_c, and these are the derivatives of its smooth pieces. Per step the pass
 * applies the transpose of the velocity-Verlet step with one Hessian-vector
 * product of the force field (pairs, exclusion corrections, bonds, angles,
 * smooth PME with its dipole grid) and the parameter derivatives of the
 * force, FP32 arithmetic with FP64 sums. An epsilon_t of 0 has no
 * derivative (Lorentz-Berthelot mixing): its entry stays 0. Supported for
 * velocity Verlet with the default (full) list and unswitched potentials
 * (MDX_E_UNSUPPORTED with MDX_OPT_HALF_LIST, a switch, Langevin dynamics or
 * rigid water).
 *
 * Use: run the trajectory in segments, saving the state (mdx_save_state)
 * and the positions, velocities and forces at each segment's start
 * (checkpoints); then
 *   mdx_adjoint_begin(ctx, pos_T, force_T, gx, gv, gU, q, p, grad)
 * with pos_T, force_T (dev [3][N]) the final state, gx = dL/dx_T (dev
 * [3][N], unwrapped coordinates) and gU = dL/dU_T (dev double[1]): it sets
 * q = gx - gU F(x_T), p = gv (or 0) and grad = gU dU/dtheta (dev double[2 T + 2]:
 * epsilon_t, sigma_t, t, dt); then, for each segment from the last to the
 * first, mdx_load_state of its checkpoint and
 *   mdx_adjoint_segment(ctx, x_s, v_s, f_s, n_steps, dt, flags, q, p, grad, gm)
 * which repeats the segment's n_steps forward from (x_s, v_s, f_s)
 * (dev [3][N]; bit for bit the forward's steps, recorded in library-owned
 * buffers) and runs the reverse steps over it, updating q, p and grad in
 * place (flags below). At the end
 * q = dL/dx_0, p = dL/dv_0 (through the trajectory; a loss term in x_0
 * itself is the caller's) and grad holds dL/dtheta and dL/d(dt). The
 * context's list state afterwards is that of the segment. Asynchronous.
 *
 * A loss that also depends on the final velocities passes gv = dL/dv_T
 * (dev [3][N], or NULL for none) to mdx_adjoint_begin and MDX_ADJ_LAST to
 * the first mdx_adjoint_segment call (the trajectory's last segment), which
 * then also takes the end state's half of the last step. flags:
 * MDX_ADJ_FIRST for the segment that starts the trajectory, MDX_ADJ_LAST for
 * the one that ends it (both for a single segment). grad_mass (dev
 * double[N] or NULL) accumulates dL/dm_i through the dynamics (a = c F / m);
 * a loss term in the masses themselves (the sampled initial velocities, the
 * kinetic energy) is the caller's.
 */
#define MDX_ADJ_FIRST 0x1
#define MDX_ADJ_LAST  0x2
/* A loss term on an intermediate state n joins the reverse pass between the
 * segments that end and start there: q += gx - gU F(x_n), p += gv (gx, gv:
 * dev [3][N]; gU dev double[1]; each may be NULL; force = F(x_n), needed
 * with gU). With one-step segments (flags MDX_ADJ_FIRST | MDX_ADJ_LAST each)
 * (q, p) are dL/dx_n and dL/dv_n between segments, so every state of the
 * trajectory can carry loss terms. The energy's parameter derivatives at an
 * intermediate state are not added. Asynchronous. */
int mdx_adjoint_inject(mdx_ctx* ctx, const float* force, const float* gx, const float* gv,
                       const double* gU, float* q, float* p);
int mdx_set_charge_direction(mdx_ctx* ctx, const float* dq);   /* host float[N]; synchronising */
int mdx_adjoint_begin(mdx_ctx* ctx, const float* pos, const float* force, const float* gx,
                      const float* gv, const double* gU, float* q, float* p, double* grad);
int mdx_adjoint_segment(mdx_ctx* ctx, const float* x0, const float* v0, const float* f0,
                        int32_t n_steps, float dt, int32_t flags, float* q, float* p,
                        double* grad, double* grad_mass);

/*
 * Masses for the following calls (host float[N], each > 0): the integrator's
 * accel / m, the Langevin noise amplitudes and the rigid-water closed form
 * follow. Mass repartitioning, as the paper's Hamiltonian Monte Carlo tuning
 * does it (Sec. IV), changes the dynamics but not the sampled positional
 * distribution. MDX_E_INVALID for a mass <= 0 or not finite. Synchronising.
 */
int mdx_set_masses(mdx_ctx* ctx, const float* mass);

/* Sets the periodic image counters (mdx_get_images) to zero. */
int mdx_reset_images(mdx_ctx* ctx);
/* out (dev [3][N]) = pos + img L: the positions unwrapped by the image
 * counters. */
int mdx_get_unwrapped(mdx_ctx* ctx, const float* pos, float* out);

/* Fills *info (host). Synchronising once a list exists: the list is copied
 * to the host to count its entries. */
int mdx_get_info(mdx_ctx* ctx, mdx_info* info);

/*
 * Checkpoint and resume of a trajectory (the paper's simulation object keeps
 * its state between step calls, Sec. II.D; these calls make that state
 * portable). Everything mdx_integrate_step carries from one step to the next
 * besides the caller's position, velocity and force arrays:
 *   - the step counter (it keys the Langevin noise) and the number of steps
 *     since the last list build (the rebuild cadence),
 *   - the periodic image counters,
 *   - the neighbour list as built (slot order, cluster boxes, tiles, the
 *     build positions) and the pruned list with the positions it was made at,
 *   - the rebuild and prune gates, the Kahan compensation terms
 *     (MDX_OPT_KAHAN_VV).
 * The latched status flags, timing records and configuration calls
 * (mdx_set_langevin, mdx_set_rigid_water) are not part of it.
 *
 * mdx_state_size: *bytes (host) receives the size of the state as it stands
 * (it grows when the list capacity grows).
 * mdx_save_state: writes it into state (dev, caller-owned, `capacity` bytes,
 * 8-byte aligned). MDX_E_CAPACITY if capacity < mdx_state_size.
 * mdx_load_state: reads a state written by mdx_save_state of a context made
 * from the same descriptor (atom count, box, cutoffs, PME grid, options);
 * the list capacities are grown or shrunk to the saved ones. MDX_E_INVALID if
 * the buffer is not such a state or `size` is short of it. After loading,
 * mdx_integrate_step from the saved positions, velocities and forces repeats
 * bit for bit the steps the saving context took next.
 * All three are synchronising.
 */
int mdx_state_size(mdx_ctx* ctx, int64_t* bytes);
int mdx_save_state(mdx_ctx* ctx, void* state, int64_t capacity);
int mdx_load_state(mdx_ctx* ctx, const void* state, int64_t size);

/* ---- diagnostics ---------------------------------------------------------
 * Kernel timing with HIP events recorded around the launches of a kernel
 * group, on the stream the group runs on. Groups: MDX_TIMING_PAIR (the
 * short-range pair kernel), MDX_TIMING_PME (spread .. gather in
 * mdx_compute_pme; in mdx_integrate_step from the spread to the last FFT
 * pass on the second stream, which overlaps the pair kernel), MDX_TIMING_BUILD
 * (list build). mdx_set_timing(ctx, groups) takes a bit mask of groups
 * (bit MDX_TIMING_x set = record group x; 0 stops all): it clears the
 * earlier records of the groups it enables and records at most 8192
 * launches per group. Event records add small gaps between kernels, so a
 * run meant to time the whole step enables only the groups it needs.
 * mdx_get_timing is synchronising and returns the mean duration in ms and
 * the number of recorded launches. MDX_E_INVALID for a mask outside 0..7. */
#define MDX_TIMING_PAIR  0
#define MDX_TIMING_PME   1
#define MDX_TIMING_BUILD 2
int mdx_set_timing(mdx_ctx* ctx, int groups);
int mdx_get_timing(mdx_ctx* ctx, int group, double* mean_ms, int64_t* launches);

#ifdef __cplusplus
}
#endif

#endif /* MDX_H */
