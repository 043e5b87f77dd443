/*
 * md.h -- C ABI of the MI355X (gfx950) short-range coarse-grained MD step.
 *
 * The operations follow the problem statement of ESPResSo++ (arXiv
 * 2608.14911), section "Example usage": a periodic orthorhombic box
 * (OrthorhombicBC), a Verlet list with a cutoff and a skin (VerletList,
 * system.skin) over linked cells (CellGrid, section "Software design"),
 * per-type-pair Lennard-Jones potentials with shift='auto' and an optional
 * capping radius (LennardJones, LennardJonesCapped), bonded interactions
 * (section "Functionality"; here FENE bonds and cosine bending angles),
 * VelocityVerlet with a LangevinThermostat extension, particles given as
 * (id, type, mass, pos, v) (storage.addParticles), integrator.run(n) and
 * computeEnergy().
 *
 * Units: reduced LJ units (sigma, epsilon, mass, tau); "all lengths are in
 * sigma" as the paper's example states.
 *
 * Memory ownership.  The caller owns every device buffer, including the
 * workspace whose size md_workspace_bytes() returns; the library never
 * allocates or frees device memory.  It owns only host-side bookkeeping and
 * HIP events/graphs, released by md_destroy().  Input arrays are copied in
 * by md_init()/md_set_state(); outputs are written to caller buffers.
 *
 * Streams.  Every device operation is enqueued on the hipStream_t passed to
 * md_init() and is asynchronous unless stated otherwise.  Only
 * md_observables(), md_history(), md_get_neighbors(), md_status_check() and
 * md_timing_read() synchronise that stream.
 *
 * Errors.  Every function returns md_status (0 = MD_OK, negative = error);
 * nothing is thrown across the ABI.  Argument and geometry errors are
 * reported synchronously.  Conditions found on the device (neighbour-list
 * overflow, a FENE bond stretched to R0, a non-finite position) are latched
 * in a sticky device status word and reported by the next synchronising
 * call; the state is then invalid until md_set_state() or a new md_init().
 * md_last_error() returns a message for the last error on a handle.
 */
#ifndef MD_H
#define MD_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef int32_t md_status;
enum {
    MD_OK = 0,
    MD_ERR_ARG = -1,            /* invalid argument (NULL, size, range)      */
    MD_ERR_HIP = -2,            /* a HIP runtime call failed                 */
    MD_ERR_BOX_TOO_SMALL = -3,  /* fewer than 3 cells of side >= rc+skin     */
    MD_ERR_NL_OVERFLOW = -4,    /* a particle has more neighbours than the
                                   list capacity; md_last_error() names the
                                   capacity needed                            */
    MD_ERR_BOND_BROKEN = -5,    /* FENE bond length reached R0               */
    MD_ERR_NONFINITE = -6,      /* a position or velocity became NaN/Inf     */
    MD_ERR_STATE = -7,          /* handle poisoned by an earlier device error */
    MD_ERR_WORKSPACE = -8,      /* workspace too small or misaligned         */
    MD_ERR_TOPOLOGY = -9        /* bonds/angles exceed the per-particle limits */
};

/* status-word bits (md_obs.status_flags) */
#define MD_FLAG_NL_OVERFLOW 0x1u
#define MD_FLAG_BOND_BROKEN 0x2u
#define MD_FLAG_NONFINITE 0x4u

/* md_config.integrator.  MD_DPD: the dissipative-particle-dynamics pair
 * thermostat (section "Functionality") instead of the Langevin friction and
 * noise: for each pair with r = |r_i - r_j| < dpd_rc, e = (r_i - r_j) / r,
 * v_ij = v_i - v_j and w = 1 - r / dpd_rc, the force on i is
 *   -gamma w^2 (e . v_ij) e + sqrt(2 gamma kT) w theta_ij e / sqrt(dt),
 * theta_ij = theta_ji ~ N(0,1) from Philox4x32-10 at counter (step low
 * word, step high word, min id, max id) with key (seed low word, seed high
 * word ^ 6), Box-Muller on its first two words as uniforms (w + 1/2) 2^-32;
 * v is the half-step velocity of velocity Verlet.  Needs MD_FP32. */
enum { MD_NVE = 0, MD_LANGEVIN = 1, MD_DPD = 2 };
enum { MD_FP64 = 0, MD_FP32 = 1 };       /* md_config.force_precision */

#define MD_MAX_TYPES 4
#define MD_MAX_BONDS_PER_PARTICLE 4
#define MD_MAX_ANGLES_PER_PARTICLE 8
#define MD_HISTORY_CAPACITY 8192

/* md_config.flags */
#define MD_CFG_VIRIAL_TENSOR 0x1  /* accumulate the 6-component virial every step */
#define MD_CFG_NO_GRAPH 0x2       /* md_step launches kernels one by one, no hipGraph */
#define MD_CFG_NL_PER_PARTICLE 0x4 /* build the Verlet list one particle per lane */
#define MD_CFG_NL_TILES 0x8        /* build it one wavefront per 64-particle tile.  Default:
                                      tiles when cells of side rc+skin hold >= 8 particles
                                      on average, else per particle.  Both builds give the
                                      same lists, entry for entry, for equal cells */

/* One type pair of the LennardJones / LennardJonesCapped potential
 * (section "Example usage"): u(r) = 4 eps [(sigma/r)^12 - (sigma/r)^6] - shift
 * for r < rc; shift = NaN means 'auto' (u(rc) = 0); caprad > 0 freezes u and
 * the force magnitude at their values at r = caprad for r < caprad.
 * eps = 0 switches the pair off. */
typedef struct md_pair_params {
    double eps, sigma, rc, shift, caprad;
} md_pair_params;

typedef struct md_config {
    uint32_t struct_size;      /* = sizeof(md_config); ABI version check */
    int32_t n_types;           /* 1 .. MD_MAX_TYPES */
    int64_t n_particles;       /* 1 .. 2^28 - 1 (32-bit byte offsets of 16-byte records) */
    double box[3];             /* periodic orthorhombic box lengths */
    double dt;                 /* > 0 */
    double skin;               /* > 0; Verlet list radius = max rc + skin */
    int32_t integrator;        /* MD_NVE or MD_LANGEVIN */
    int32_t force_precision;   /* MD_FP64 or MD_FP32 (pair and bonded math) */
    double temperature;        /* Langevin kT */
    double gamma;              /* Langevin friction */
    uint64_t seed;             /* Philox4x64-10 key word 0 (noise stream 0) */
    md_pair_params pair[MD_MAX_TYPES * MD_MAX_TYPES]; /* row-major [ti][tj], symmetric */
    int64_t n_bonds;           /* FENE bonds */
    int64_t n_angles;          /* cosine bending angles */
    double fene_K, fene_R0;    /* u = -K R0^2/2 ln(1 - r^2/R0^2) */
    double k_bend;             /* u = k (1 - cos theta), theta = 0 straight */
    int32_t cell_factor;       /* 1 or 2: cells of side >= (rc+skin)/cell_factor;
                                  2 is the half-cutoff sub-cell decomposition;
                                  0 = 1, or 2 when fewer than 3 cells of side
                                  rc+skin fit per side */
    int32_t nl_capacity;       /* neighbours per particle, rounded up to a multiple
                                  of 8 (rows are streamed in batches of 8 slots);
                                  0 = from density */
    int32_t block_size;        /* particles (threads) per block of the FP32 fast force
                                  kernels: 64, 128, 256 or 512; 0 = 256.  The other force
                                  kernels and batches keep 256.  Changes cost only: every
                                  particle's force is computed alone, and only the order
                                  of the FP64 energy/virial block sums follows it */
    int32_t flags;             /* MD_CFG_* */
    double list_cutoff;        /* Verlet list radius = max(list_cutoff, max rc) + skin;
                                  0 = max rc.  The surrogate needs >= MD_SUR_RCUT */
    int32_t surrogate;         /* 1: reserve workspace for the learned surrogate */
    int32_t pad_;
    double shear_rate;         /* Lees-Edwards boundaries (section "New Features") when
                                  != 0: flow along x, gradient along y.  The image one
                                  box above (y + Ly) is displaced by delta(t) = shear_rate
                                  Ly t (mod Lx), t = step dt, and moves with shear_rate Ly
                                  along x; a particle leaving through y = Ly re-enters at
                                  y - Ly with x - delta and v_x - shear_rate Ly (through
                                  y = 0 the opposite).  Needs MD_FP32 and a constant dt;
                                  the list is rebuilt when twice the largest displacement
                                  plus the offset's change since the last build reaches
                                  the skin */
    double dpd_rc;             /* DPD weight range (MD_DPD); the Verlet list radius
                                  covers max(dpd_rc, rc, list_cutoff) + skin */
    int32_t table_points;      /* points per pair / angle table reserved in the
                                  workspace (md_set_pair_table, md_set_angle_table);
                                  0 = no tables.  Tables need MD_FP32 */
    int32_t angle_kind;        /* MD_ANGLE_*; kinds other than MD_ANGLE_COSINE need MD_FP32 */
    double angle_K, angle_phi0; /* MD_ANGLE_COSINE_SQUARED: u = K (cos phi - cos phi0)^2 */
    int32_t adress;            /* 1: AdResS force interpolation (md_set_cg_table); needs
                                  table_points > 0 and MD_FP32 */
    int32_t pad2_;
    double adress_x0, adress_d_at, adress_d_hy; /* slab of the atomistic zone along x */
} md_config;

/* Angle potentials (bonded interactions, section "Functionality";
 * AngularCosineSquared and TabulatedSubEnsAngular, section "New Features"),
 * in the bond angle phi at the centre (pi for a straight chain):
 *   MD_ANGLE_COSINE          u = k_bend (1 + cos phi) = k_bend (1 - cos theta),
 *                            theta = pi - phi (the Kremer-Grest bending)
 *   MD_ANGLE_COSINE_SQUARED  u = angle_K (cos phi - cos angle_phi0)^2
 *   MD_ANGLE_TABULATED       a table of u and du/dphi (md_set_angle_table)
 *                            on phi_k = k pi / (n - 1), both interpolated
 *                            linearly in phi; the force takes
 *                            dU/dcos(phi) = -(du/dphi) / max(sin phi, 1e-8) */
enum { MD_ANGLE_COSINE = 0, MD_ANGLE_COSINE_SQUARED = 1, MD_ANGLE_TABULATED = 2 };

/* Observables of one step n (positions x_n, on-step velocities v_n). */
typedef struct md_obs {
    int64_t step;
    double e_pair, e_bond, e_angle, e_kin, e_total;
    double virial;              /* W = sum over pairs/bonds/angles of r_ij . f_ij */
    double virial_tensor[6];    /* xx yy zz xy xz yz (only with MD_CFG_VIRIAL_TENSOR
                                   or from md_observables) */
    double pressure;            /* (2 K + W) / (3 V) */
    double temperature;         /* 2 K / ndof; ndof = 3N-3 (NVE) or 3N (Langevin) */
    int64_t n_rebuilds;         /* neighbour-list builds since md_init */
    uint32_t status_flags;      /* MD_FLAG_* latched on the device */
    int32_t nl_max_count;       /* largest neighbour count at the last build */
} md_obs;

/* Per-kernel timing collected with HIP events on the handle's stream. */
typedef struct md_timing {
    int64_t n_step_kernels;     /* launches of the fused force+integrate kernel */
    double ms_step_kernels;     /* their summed duration */
    int64_t n_rebuild;          /* steps whose rebuild stage was timed */
    double ms_rebuild;          /* summed duration of the rebuild stage (gated kernels) */
    int64_t n_finalize;
    double ms_finalize;
    double ms_bin_sort;         /* of ms_rebuild: binning and the cell sort (the rest
                                   is the neighbour-list build) */
} md_timing;

typedef struct md_handle_s* md_handle;

/* Bytes of device workspace md_init needs for this configuration (host
 * arithmetic only, no device call).  Returns MD_ERR_ARG for an invalid
 * config and MD_ERR_BOX_TOO_SMALL when fewer than 3 cells fit per side. */
md_status md_workspace_bytes(const md_config* cfg, size_t* bytes);

/* What a configuration resolves to (host arithmetic only, no device call):
 * the cell grid of the binning (CellGrid) and the Verlet-list build, after
 * the automatic choices of cell_factor = 0, nl_capacity = 0 and the
 * MD_CFG_NL_* flags.  Returns the same errors as md_workspace_bytes. */
#define MD_NL_BUILD_PER_PARTICLE 0 /* one particle per lane */
#define MD_NL_BUILD_TILES 1        /* one wavefront per 64-particle tile */
typedef struct md_plan {
    int32_t cells[3];          /* cells per side */
    int32_t cell_factor;       /* 1 or 2: cells of side >= list_radius / cell_factor */
    int32_t nl_capacity;       /* list slots per particle */
    int32_t nl_build;          /* MD_NL_BUILD_* */
    double list_radius;        /* max(rc, list_cutoff) + skin */
} md_plan;
md_status md_plan_config(const md_config* cfg, md_plan* out);

/* Create a simulation (storage.addParticles + decompose of the paper).
 *   pos, vel      device, FP64 [N][3], particle-id (tag) order; positions may
 *                 lie outside the box, they are folded in with image counters
 *   type          device int32 [N] in 0..n_types-1, or NULL (all type 0)
 *   mass_by_type  host FP64 [n_types], > 0
 *   bonds         host int32 [n_bonds][2] particle ids, or NULL if n_bonds = 0
 *   angles        host int32 [n_angles][3] particle ids (centre in the middle),
 *                 or NULL if n_angles = 0
 *   workspace     device, >= md_workspace_bytes(), 256-byte aligned,
 *                 owned by the caller and kept alive until md_destroy
 *   stream        hipStream_t (NULL = default stream)
 * Builds cells and the Verlet list.  Velocities are on-step velocities.
 * Synchronises the stream once (topology upload).  */
md_status md_init(const md_config* cfg, const double* pos, const double* vel, const int32_t* type,
                  const double* mass_by_type, const int32_t* bonds, const int32_t* angles,
                  void* workspace, size_t ws_bytes, void* stream, md_handle* out);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture set-up, tight serving loops, harnesses that forbid hipMalloc):
 * md_init with the workspace taken from a static device array of
 * MD_STATIC_WORKSPACE_BYTES that the library holds on each GPU until the
 * process ends, instead of a caller-owned one.  Same arguments, layout and
 * errors as md_init otherwise; the handle is used and released exactly like
 * one from md_init.
 *   - Calls no hipMalloc / hipFree or other device-allocating routine (host
 *     bookkeeping is allocated as for md_init); synchronises the stream once.
 *   - The array of the calling thread's current device is used; the stream
 *     must belong to that device.
 *   - A configuration whose md_workspace_bytes() exceeds
 *     MD_STATIC_WORKSPACE_BYTES is rejected with MD_ERR_WORKSPACE.
 *   - One live handle per GPU: while a handle from md_init_static exists on a
 *     device, a further call there returns MD_ERR_STATE; md_destroy frees
 *     the array for the next call.  The array keeps the previous handle's
 *     contents; md_init_static clears what must start at zero.  Work that two
 *     threads enqueue on one GPU's array at the same time races. */
#define MD_STATIC_WORKSPACE_BYTES (64u << 20)
md_status md_init_static(const md_config* cfg, const double* pos, const double* vel, const int32_t* type,
                         const double* mass_by_type, const int32_t* bonds, const int32_t* angles, void* stream,
                         md_handle* out);

/* Change run parameters without touching the state: dt, temperature, gamma,
 * seed, integrator, force_precision, the pair table (e.g. switching
 * LennardJonesCapped to LennardJones as the paper's example does),
 * fene_K/R0, k_bend, flags.  n_particles, n_types, box, skin, n_bonds and
 * n_angles must equal those given to md_init (MD_ERR_ARG otherwise: the
 * list radius and the half-skin rebuild threshold are fixed at md_init); a
 * pair table whose cutoffs plus the skin exceed that list radius is
 * rejected. */
md_status md_set_params(md_handle h, const md_config* cfg);

/* Tabulated pair potential of types (ti, tj) (section "Functionality":
 * tabulated potentials), replacing that pair's Lennard-Jones form (its eps,
 * sigma, shift and caprad are ignored; its rc stays the cutoff):
 *   u, f   host FP64 [npoints]: the energy and the radial force f = -du/dr
 *          on r_k = rmin + k (rc - rmin) / (npoints - 1)
 * Both are interpolated linearly in r; below rmin they keep their rmin
 * values; from rc on the pair does not interact.  Stored as FP32.
 * npoints in 2 .. md_config.table_points; 0 <= rmin < rc.  Symmetric (sets
 * (tj, ti) as well).  Errors: MD_ERR_ARG. */
md_status md_set_pair_table(md_handle h, int32_t ti, int32_t tj, const double* u, const double* f, int32_t npoints,
                            double rmin);
/* The angle table of MD_ANGLE_TABULATED: u and du/dphi, host FP64
 * [npoints], phi_k = k pi / (npoints - 1); npoints in 2 .. table_points. */
md_status md_set_angle_table(md_handle h, const double* u, const double* dudphi, int32_t npoints);
/* TabulatedSubEnsAngular: the angle table of the weighted sum of ntables
 * tables on one grid, u and dudphi host FP64 [ntables][npoints], weights
 * host FP64 [ntables]; sets the table sum_m w_m (u_m, du_m/dphi). */
md_status md_set_angle_subens(md_handle h, int32_t ntables, const double* u, const double* dudphi,
                              const double* weights, int32_t npoints);

/* AdResS (adaptive resolution, sections "Statement of need" and
 * "Functionality") on single-site molecules: with md_config.adress = 1 every
 * pair force is interpolated between the atomistic one (the pair table, or
 * its tabulated form) and a coarse-grained one:
 *   F_ij = w_i w_j F^AT_ij + (1 - w_i w_j) F^CG_ij,
 *   w(x) = 1 for d < d_at, 0 for d >= d_at + d_hy, cos^2(pi (d - d_at) / (2 d_hy))
 *          between, d = |x - adress_x0| (minimum image along x);
 * the reported pair energy is the same interpolation of u (force
 * interpolation conserves no energy).  The coarse-grained potential of types
 * (ti, tj) is a table as md_set_pair_table's: u, f host FP64 [npoints] on
 * r_k = rmin + k (rc_cg - rmin) / (npoints - 1), zero from rc_cg on; rc_cg + skin
 * must not exceed the list radius (set md_config.list_cutoff).  Pairs
 * without a coarse-grained table have F^CG = 0. */
md_status md_set_cg_table(md_handle h, int32_t ti, int32_t tj, const double* u, const double* f, int32_t npoints,
                          double rmin, double rc_cg);

/* Force a cell sort and neighbour-list build at the current positions. */
md_status md_build_neighbors(md_handle h);

/* Conservative forces at the current positions (no thermostat term), FP64
 * [N][3] in tag order into device f_out (NULL: only observables update). */
md_status md_forces(md_handle h, double* f_out);

/* Advance nsteps of velocity Verlet (+ Langevin).  Each step: rebuild the
 * list when some particle moved more than skin/2 since the last build,
 * evaluate forces, integrate, reduce energy and virial in FP64 into the
 * history ring.  Asynchronous; no host synchronisation. */
md_status md_step(md_handle h, int64_t nsteps);

/* Energies, virial, pressure and temperature at the current step
 * (computeEnergy() of the paper), on-step velocities.  Synchronises. Returns
 * the error code of a latched device condition, with *out still filled. */
md_status md_observables(md_handle h, md_obs* out);

/* Copy the per-step observables recorded since the last md_history call
 * (at most MD_HISTORY_CAPACITY of the most recent steps) to host out[max];
 * *n receives the number written.  Synchronises. */
md_status md_history(md_handle h, md_obs* out, int64_t max, int64_t* n);

/* Raw state in tag order, device buffers: pos [N][3] FP64 in [0,L), vel
 * [N][3] FP64, image [N][3] int32, pos_build [N][3] FP64 = positions at the
 * last neighbour-list build (each may be NULL); *step and *vel_half host
 * (may be NULL).  vel_half = 1: vel holds v_{step-1/2}; 0: the on-step
 * v_step.  A pending list rebuild is carried out first.  Restoring the
 * tuple with md_set_state (pos_build included) continues the run bit for
 * bit: the cell order is a function of the build positions and the ids.  */
md_status md_get_state(md_handle h, double* pos, double* vel, int32_t* image, double* pos_build,
                       int64_t* step, int32_t* vel_half);
/* Replace the state (same particles, types, topology).  pos_build NULL:
 * the list is built at pos.  Clears the latched device status. */
md_status md_set_state(md_handle h, const double* pos, const double* vel, const int32_t* image,
                       const double* pos_build, int64_t step, int32_t vel_half);

/* Current Verlet list in tag space: count [N] and idx [N][cap] device int32
 * (rows unsorted; entries past count are untouched).  Returns
 * MD_ERR_NL_OVERFLOW if cap is smaller than the longest row.  Synchronises. */
md_status md_get_neighbors(md_handle h, int32_t* count, int32_t* idx, int32_t cap);

/* Synchronise and return the latched device status as an md_status. */
md_status md_status_check(md_handle h);

/* Enable (1) / disable (0) HIP-event timing of the kernels md_step launches
 * (forces kernel-by-kernel launches while enabled); read and reset it. */
md_status md_timing_enable(md_handle h, int32_t enable);
md_status md_timing_read(md_handle h, md_timing* out);

/* ------------------------------------------------------------------------
 * Learned surrogate of the non-bonded pair force.  The paper has no learned
 * model; this is an extension built on its pair-force step: a per-particle
 * radial-descriptor MLP trained by force matching against the plain
 * potential, which stays available as the fallback and as the reference for the
 * surrogate's error.  FENE and bending stay plain.
 *
 *   g_k(r)   = exp(-(r - mu_k)^2 / (2 w^2)) (cos(pi r / r_d) + 1) / 2,
 *              w = MD_SUR_WIDTH, mu_k = MD_SUR_MU0 + k (MD_SUR_MU1 - MD_SUR_MU0) / 31,
 *              r_d = MD_SUR_RCUT, k = 0..31
 *   G_k(i)   = sum over j != i with r_ij < r_d of g_k(r_ij)
 *   x_i      = (G(i) - mean) * istd          (fixed standardisation)
 *   E_i      = w3 . silu(W2 silu(W1 x_i + b1) + b2) + b3,   E = sum_i E_i
 *   F_i      = -dE/dr_i = sum_j ((a_i + a_j) . g'(r_ij)) (x_j - x_i) / r_ij,
 *              a_i = dE_i/dG(i)
 * Parameters theta: FP32 [MD_SUR_NPARAM] = W1 [64][32] row-major, b1 [64],
 * W2 [64][64], b2 [64], w3 [64], b3 [1].  Precision MD_SUR_FP32: all network
 * arithmetic in FP32; MD_SUR_BF16: weights and activations rounded to BF16
 * (round to nearest even) as matrix-core operands, FP32 accumulation.  The
 * descriptor and pair-force arithmetic is FP32 in both.
 * All surrogate calls need md_config.surrogate = 1; they return MD_ERR_ARG
 * otherwise.
 * ------------------------------------------------------------------------ */
#define MD_SUR_NBASIS 32
#define MD_SUR_HIDDEN 64
#define MD_SUR_NPARAM 6337
#define MD_SUR_RCUT 2.5
#define MD_SUR_WIDTH 0.1
#define MD_SUR_MU0 0.8
#define MD_SUR_MU1 2.5
#define MD_SUR_VAR_FLOOR 1e-6
enum { MD_SUR_FP32 = 0, MD_SUR_BF16 = 1 };
enum { MD_PAIR_PLAIN = 0, MD_PAIR_SURROGATE = 1 };

/* Load the network: theta device FP32 [MD_SUR_NPARAM]; g_mean, g_istd device
 * FP32 [32] (standardisation constants).  Resets the Adam moments.  The
 * handle keeps its own copy (the master weights that md_sur_adam updates). */
md_status md_sur_set(md_handle h, const float* theta, const float* g_mean, const float* g_istd,
                     int32_t precision);
/* Copy the handle's master weights to device theta [MD_SUR_NPARAM]. */
md_status md_sur_get(md_handle h, float* theta);
/* Non-bonded force model of md_step / md_forces / md_observables:
 * MD_PAIR_PLAIN (the pair table) or MD_PAIR_SURROGATE (the network; the list
 * radius minus the skin must reach MD_SUR_RCUT). */
md_status md_set_pair_mode(md_handle h, int32_t mode);
/* Descriptors G at the current positions: device FP32 [N][32], tag order. */
md_status md_sur_descriptors(md_handle h, float* G);
/* The fixed standardisation (mean, istd) of x_i above, fitted on training
 * frames (the paper has no learned model; this belongs to the extension
 * described at the head of this section): over the N descriptor rows of each of
 * the nf frames, g_mean_k = mean of G_k and g_istd_k = 1 / sqrt(var_k +
 * MD_SUR_VAR_FLOOR), population variance, sums in FP64.  frames device FP64
 * [nf][N][3] positions (tag order; folded into the box); g_mean, g_istd
 * device FP32 [32], ready for md_sur_set.  Needs no network.  The handle's
 * state is replaced as by md_sur_loss_grad (last frame, zero velocities,
 * step 0).  MD_ERR_ARG on NULL pointers, nf < 1 or a list radius below the
 * descriptor cutoff. */
md_status md_sur_desc_stats(md_handle h, const double* frames, int32_t nf, float* g_mean, float* g_istd);
/* The network on P given descriptor rows: G device FP32 [P][32] (raw, the
 * handle's standardisation is applied); e device FP32 [P] (may be NULL) and
 * dedg device FP32 [P][32] = dE_i/dG(i). */
md_status md_sur_mlp_eval(md_handle h, const float* G, int64_t P, float* e, float* dedg);
/* Surrogate pair forces at the current positions for given input gradients
 * a_i = dE_i/dG(i): F_i = sum_j ((a_i + a_j) . g'(r_ij)) (x_j - x_i) / r_ij.
 * dedg device FP32 [N][32] tag order; f_out device FP64 [N][3] tag order.
 * A constant a_i = c makes E a pair potential (a linear readout of G), whose
 * forces are linear in c. */
md_status md_sur_pair_forces(md_handle h, const float* dedg, double* f_out);
/* Force-matching loss L = mean over frames, particles and components of
 * (F - F_ref)^2 at the handle's weights, and (grad != NULL or for a later
 * md_sur_adam) its gradient dL/dtheta by the analytic double backward.
 *   frames  device FP64 [nf][N][3] positions (tag order; folded into the box)
 *   f_ref   device FP64 [nf][N][3] reference non-bonded forces
 *   grad    device FP32 [MD_SUR_NPARAM] or NULL; loss host (may be NULL)
 * The handle's state is replaced: positions of the last frame, zero
 * velocities, step 0.  Synchronises when loss != NULL. */
md_status md_sur_loss_grad(md_handle h, const double* frames, const double* f_ref, int32_t nf, float* grad,
                           double* loss);
/* One Adam update (Kingma and Ba 2015, bias-corrected, step t >= 1) of the
 * master weights with the gradient of the last md_sur_loss_grad. */
md_status md_sur_adam(md_handle h, int64_t t, double lr, double beta1, double beta2, double eps);

md_status md_destroy(md_handle h);

/* ------------------------------------------------------------------------
 * Batches: many independent periodic systems advanced together, one kernel
 * launch per stage for all of them (replicas of uneven size; the paper's
 * per-system step applied to each, with its load-balancing concern met by
 * tiles of 256 particles that never straddle systems).  Each member keeps
 * its own cells, list, rebuild trigger, thermostat stream and observables;
 * a member's trajectory is the one a standalone handle with the same
 * configuration computes.  Members need one particle type, FP32 pair math,
 * a cubic box, no capping radius, no surrogate, no DPD, no shear, no tables,
 * the cosine angle, no AdResS, and at most 262144 particles (MD_ERR_ARG
 * otherwise).
 * ------------------------------------------------------------------------ */
typedef struct md_batch_s* md_batch;

/* Workspace bytes for the batch cfgs[0..nsys-1] (host arithmetic only). */
md_status md_batch_workspace_bytes(const md_config* cfgs, int32_t nsys, size_t* bytes);
/* Create the batch.  pos[s], vel[s]: device FP64 [n_s][3]; mass_by_type[s]:
 * host FP64 [1]; bonds[s] / angles[s]: host int32 topology as for md_init, or
 * bonds / angles NULL for none; workspace: device, >= md_batch_workspace_bytes(),
 * 256-byte aligned, caller-owned.  Synchronises the stream. */
md_status md_batch_init(const md_config* cfgs, int32_t nsys, const double* const* pos, const double* const* vel,
                        const double* const* mass_by_type, const int32_t* const* bonds,
                        const int32_t* const* angles, void* workspace, size_t ws_bytes, void* stream,
                        md_batch* out);
/* Advance every member nsteps (asynchronous; replayed from a hipGraph of two
 * steps). */
md_status md_batch_step(md_batch b, int64_t nsteps);
/* Observables of every member at the current step into host out[nsys];
 * synchronises; returns the first member's latched device error, if any. */
md_status md_batch_observables(md_batch b, md_obs* out);
/* State of member sys, as md_get_state. */
md_status md_batch_get_state(md_batch b, int32_t sys, double* pos, double* vel, int32_t* image,
                             double* pos_build, int64_t* step, int32_t* vel_half);
/* HIP-event timing of the batch's stages, as md_timing_enable / md_timing_read. */
md_status md_batch_timing_enable(md_batch b, int32_t enable);
md_status md_batch_timing_read(md_batch b, md_timing* out);
md_status md_batch_destroy(md_batch b);
const char* md_batch_last_error(md_batch b);

const char* md_status_string(md_status s);
const char* md_last_error(md_handle h);

#ifdef __cplusplus
}
#endif
#endif /* MD_H */
