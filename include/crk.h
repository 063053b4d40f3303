/*
 * crk.h -- C ABI of the MI355X short-range step of CRK-HACC
 * (Frontiere et al., "Cosmological Hydrodynamics at Exascale: A
 * Trillion-Particle Leap in Capability").
 *
 * The step evaluates, for particles in periodic unit boxes, the short-range
 * gravitational force inside the handover scale r_c (Sec. IV-A: the force
 * is split into a spectral long-range part and a local short-range part)
 * and the CRKSPH hydrodynamics passes (Sec. IV-A: conservative
 * reproducing-kernel SPH), all as pairwise sums phi_i = sum_j phi_ij
 * (Eq. (1)) over leaf-leaf interaction lists of chaining-mesh bins and
 * per-bin k-d base leaves (Sec. IV-B.1).
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 * - Every particle pointer is a DEVICE pointer owned by the caller, in the
 *   caller's particle order.  Arrays hold float (context precision
 *   CRK_FP32) or double (CRK_FP64), except where a type is stated.
 * - Positions lie in [1, 2) (unit periodic box shifted by one).  In float32
 *   any two such values share one exponent, so their difference is exact.
 * - Vector fields are stored as planes: B and gradA hold 3 planes of n
 *   values (plane a at offset a*n), gradB holds 9 planes with plane
 *   (3*g + a) = d B^a / d x^g.
 * - Particles are grouped into n_boxes independent periodic boxes by the
 *   per-box offsets of the gas and dm arrays; boxes do not interact.
 * - All work is enqueued asynchronously on the context's stream; no entry
 *   point synchronises except build_tree / build_interaction_lists outside
 *   graph capture (they read back sizes), crk_sync, and the calls whose
 *   comment says so (crk_tree_set_active, crk_tree_refit, crk_count_pairs,
 *   crk_pass_times, crk_tree_get_info after a synchronising build).
 * - Return value: CRK_OK or a negative crk_status; the message of the last
 *   failure on the calling thread is returned by crk_last_error().
 *   Argument errors are detected on the host before anything is enqueued.
 *   Errors found on the device (non-finite or out-of-range inputs, a
 *   capacity fixed at graph capture being exceeded) are latched in the
 *   context and returned by crk_sync.
 * - The library never aborts, never throws across this boundary and keeps
 *   no global state besides the last-error message.
 */
#ifndef CRK_H
#define CRK_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    CRK_OK = 0,
    CRK_EINVAL = -1,    /* bad argument (host side) or bad input value      */
    CRK_ECAPACITY = -2, /* a capacity fixed at graph capture was exceeded    */
    CRK_EDEVICE = -3,   /* HIP runtime error                                 */
    CRK_ESTATE = -4,    /* call out of order (e.g. lists before tree)        */
    CRK_ESTALE = -5     /* the tree no longer covers the particles' motion:
                           rebuild it (crk_tree_refit)                       */
} crk_status;

typedef enum {
    CRK_FP64 = 0, /* plain double precision everywhere                       */
    CRK_FP32 = 1  /* float pair sums with compensated accumulation; double
                     moment-matrix solve and double integration             */
} crk_precision;

typedef struct crk_ctx crk_ctx;   /* opaque, library-owned */
typedef struct crk_tree crk_tree; /* opaque, library-owned */

/* Physical constants of the step.  The paper fixes none of them; these are
 * the method's usual choices: ideal gas gamma, Monaghan viscosity C_l, C_q
 * with denominator guard eps_Q, gravitational constant G. */
typedef struct {
    double gamma; /* adiabatic index (5/3)                 */
    double Cl;    /* linear viscosity coefficient (1)      */
    double Cq;    /* quadratic viscosity coefficient (2)   */
    double epsQ;  /* viscosity guard, times h^2 (0.01)     */
    double G;     /* gravitational constant (1)            */
} crk_params;

/* Host-side description of the boxes (all arrays are HOST memory, read
 * during build_tree only). */
typedef struct {
    int32_t n_boxes;       /* >= 1                                          */
    const int64_t *gas_off; /* n_boxes + 1 offsets into the gas arrays       */
    const int64_t *dm_off;  /* n_boxes + 1 offsets into the dm arrays        */
    const double *r_c;      /* per box: gravity cutoff, 0 < r_c < 0.5        */
    const double *eps;      /* per box: Plummer softening, 0 <= eps < r_c    */
    const double *h_max;    /* per box: upper bound of the gas smoothing
                               lengths, 0 < 2 h_max < 0.5 (checked on the
                               device; a larger h raises CRK_EINVAL at
                               crk_sync)                                     */
} crk_boxes;

/* Tunables of the tree and launch shape (results do not depend on them
 * beyond floating-point rounding order). */
typedef struct {
    int32_t leaf_max;   /* k-d leaf size bound, 16..256 (default 64)         */
    double cm_factor;   /* chaining-mesh bin width / max(r_c, 2 h_max), in
                           [1, 64]; 0 (default) widens the bins until each
                           holds about 4 leaf_max particles of the denser
                           species (never narrower than max(r_c, 2 h_max)) */
    int32_t grid_mult;  /* persistent grid = grid_mult x CU count
                           workgroups (four times that for the 64-thread
                           split form) popping items from a cost-ordered
                           atomic queue; 0 = one workgroup per leaf or
                           sub-leaf (default 0)                             */
    int32_t xcd_remap;  /* 1: with one workgroup per leaf or sub-leaf, give
                           each of the 8 XCDs a contiguous range of them
                           (default 1)                                       */
    int32_t walk_mask;  /* passes whose sweep walks per-lane hit lists:
                           bit 0 density, 1 coefficients, 2 hydro, 3 gravity;
                           one workgroup per leaf of <= 64 only (default 0) */
    int32_t sub_sweep;  /* sub-leaf sweeps (leaf_max <= 64, one workgroup per
                           leaf): the tree splits every leaf into <= 4
                           sub-leaves of <= 16, reordering the leaf's slots;
                           1: each 16-lane group sweeps only the candidates
                           near its sub-leaf; 2: one wavefront per sub-leaf,
                           culled against the sub-leaf box, four lanes per
                           particle (default); 3: four wavefronts per leaf
                           staging the leaf's candidates once in shared LDS,
                           each then culling them against its sub-leaf box
                           and sweeping as in 2; 0: whole-leaf sweep        */
    int32_t tree_lds;   /* 1: after one sort by bin, sort every bin along the
                           three axes and run its k-d levels in LDS (bins of
                           up to 4096 particles; larger bins fall back to
                           the per-axis global sorts); 0: always the global
                           sorts.  Both give the same tree (default 1)      */
    int32_t tile;       /* j-tile width of the split form (sub_sweep 2): the
                           LDS candidate buffer holds tile x 64 records
                           (capped per pass at 64 KiB); 0: the pass's own
                           width (default); 1, 2, 4 or 8                    */
    int32_t act_groups; /* with an active subset (crk_tree_set_active) and
                           sub-leaves, k > 0: when the active leaves hold on
                           average at least k active particles each, the
                           sub-leaf sweeps take, for each sub-leaf holding
                           an active particle, its active particles only,
                           boxed at their current positions (an active
                           group); otherwise, and with k = 0, the tree's
                           sub-leaves with all their particles and their
                           grown boxes, skipping those without an active
                           particle.  In [0, 4096]; default 1, groups
                           for every subset (with the sub-leaf sweep of one
                           wavefront per listed sub-leaf they measured
                           faster at every activity tried)                   */
} crk_tuning;

/* ------------------------------------------------------------------------ */
/* context                                                                   */
/* ------------------------------------------------------------------------ */

/* Creates a context on the current HIP device.  stream: a hipStream_t (or
 * NULL for the default stream) on which all work is enqueued.  params may
 * be NULL for the defaults above. */
int crk_ctx_create(crk_ctx **out, int precision, void *stream,
                   const crk_params *params);
int crk_ctx_destroy(crk_ctx *ctx);
int crk_set_tuning(crk_ctx *ctx, const crk_tuning *t);
int crk_get_tuning(const crk_ctx *ctx, crk_tuning *t);

/* Message of the last failed call on this thread ("" if none). */
const char *crk_last_error(void);

/* Waits for the context's stream and returns the first latched device-side
 * error (CRK_EINVAL for bad input values, CRK_ECAPACITY when a capacity
 * fixed at capture was exceeded), then clears it.  *required (may be NULL)
 * receives the list capacity, in entries, that the last build needed. */
int crk_sync(crk_ctx *ctx, int64_t *required);

/* ------------------------------------------------------------------------ */
/* the six operations of the short-range step                               */
/* ------------------------------------------------------------------------ */

/* Chaining-mesh bins and per-bin k-d base leaves (Sec. IV-B.1).
 * Each box is cut into n_cm^3 bins of width >= max(r_c, 2 h_max) (see
 * crk_tuning.cm_factor), so every interaction of a particle lies in its bin
 * or one of the 26 neighbours.  Particles are sorted by (species, box,
 * bin); inside each bin a k-d tree splits the widest extent (ties by caller
 * index) until leaves hold <= leaf_max particles, the left side taking
 * ceil(k/2) of the k leaves a node needs (the median for even k); only the
 * leaves are kept.
 * gx, gy, gz, gh: gas positions and smoothing lengths (n_gas values);
 * dx, dy, dz: dark-matter positions (n_dm values); n_gas = gas_off[n_boxes],
 * n_dm = dm_off[n_boxes]; boxes may be empty, but n_gas + n_dm = 0 is
 * rejected with CRK_EINVAL (there is nothing to build).  The positions and
 * h are copied into the tree (in tree order); later calls use the copies.
 * *tree is created on first use and reused (grown as needed) when
 * non-NULL. */
int build_tree(crk_ctx *ctx, const crk_boxes *boxes, const void *gx,
               const void *gy, const void *gz, const void *gh,
               const void *dx, const void *dy, const void *dz,
               crk_tree **tree);

/* Leaf-leaf interaction lists (Sec. IV-B.1): for every leaf, the leaves of
 * its own and the 26 neighbouring bins whose periodic bounding boxes come
 * closer than the interaction range, with the periodic image shift of each.
 * Gravity list: all species, range r_c.  Hydro list: gas leaves only, range
 * 2 max(h_max of either leaf).  Ranges are widened by 1e-5 relative so that
 * no pair accepted by float32 arithmetic is missed. */
int build_interaction_lists(crk_ctx *ctx, crk_tree *tree);

/* Volume and uncorrected density of every gas particle (CRKSPH, Sec. IV-A;
 * a pairwise sum of the form of Eq. (1)):
 *   V_i = 1 / sum_j W(r_ij, h_i),   rho~_i = sum_j m_j W(r_ij, h_i),
 * over gas j with r_ij < 2 h_i, j = i included; W is the cubic spline.
 * m: gas masses (n_gas); V, rho_tilde: outputs (n_gas). */
int crk_density(crk_ctx *ctx, crk_tree *tree, const void *m, void *V,
                void *rho_tilde);

/* crk_density that allocates nothing, for callers that cannot allocate
 * device memory: code under HIP graph capture, tight serving loops,
 * harnesses that forbid hipMalloc.  Same arguments, results and errors as
 * crk_density (bitwise the same outputs), but the masses in tree order, the
 * one scratch buffer of that pass, live in a static device array of the
 * library (CRK_NOALLOC_MAX_GAS values of the context precision, 16 MiB,
 * held on every GPU the library runs on until the process ends) instead of
 * library-allocated memory, and no timing events are recorded.  The tree
 * (built by build_tree) must already exist.  More than CRK_NOALLOC_MAX_GAS
 * gas particles: CRK_EINVAL.  Every call on one GPU shares that GPU's
 * array, which keeps the last call's contents: calls that overlap on one
 * GPU (several streams or threads at once) race and must be serialised by
 * the caller.  Nothing in the array needs to start at zero. */
#define CRK_NOALLOC_MAX_GAS 2097152
int crk_density_noalloc(crk_ctx *ctx, crk_tree *tree, const void *m, void *V,
                        void *rho_tilde);

/* Reproducing-kernel correction coefficients (CRKSPH, Sec. IV-A; the
 * paper's highest-throughput kernel, Sec. V-B).  Gathers the moments
 * m0, m1, m2 of V_j W(r_ij, h_i) and their gradients, then solves, per
 * particle in double precision,
 *   B = -m2^-1 m1,  A = 1/(m0 + B.m1),
 *   d_g B = -m2^-1 (d_g m1 + d_g m2 B),  d_g A = -A^2 (d_g m0 + d_g B.m1
 *   + B.d_g m1),
 * so that A(1 + B.x_ij) W reproduces constant and linear fields, then the
 * corrected density rho = A (rho~ + B.M1) with M1 = sum m_j x_ij W_ij, the
 * ideal-gas pressure P = (gamma - 1) rho u and sound speed
 * cs = sqrt(gamma (gamma - 1) u).  A singular m2 falls back to B = grad B = 0,
 * A = 1/m0, grad A = -grad m0 / m0^2.
 * Inputs m, V, u (n_gas); outputs A, rho, P, cs (n_gas), B and gradA
 * (3 planes), gradB (9 planes). */

int crk_coefficients(crk_ctx *ctx, crk_tree *tree, const void *m,
                     const void *V, const void *u, void *A, void *B,
                     void *gradA, void *gradB, void *rho, void *P, void *cs);

/* CRKSPH accelerations and specific-energy rates (Sec. IV-A; the
 * antisymmetric pair terms of Eq. (2)).  With the corrected-kernel gradient
 * g_k(y) = dA_k (1 + B_k.y) W_k + A_k (dB_k.y + B_k) W_k
 *          + A_k (1 + B_k.y) grad W_k   (W_k at h_k),
 * G_ij = g_i(x_ij) - g_j(x_ji) and the Monaghan viscosity
 * Q_ij = rho_i (-C_l cs_i mu_ij + C_q mu_ij^2),
 * mu_ij = min(0, h_i v_ij.x_ij / (r^2 + eps_Q h_i^2)), the pair force is
 *   F_ij = -1/2 V_i V_j [(P_i + P_j) G_ij + Q_ij g_i(x_ij) - Q_ji g_j(x_ji)]
 * = -F_ji, and a_i = sum_j F_ij / m_i, du_i/dt = -sum_j v_ij.F_ij / (2 m_i),
 * over gas j != i with r_ij < 2 max(h_i, h_j).
 * Inputs (n_gas each): m, vx, vy, vz, V, rho, P, cs, A; B, gradA (3 planes),
 * gradB (9 planes).  Outputs ax, ay, az, dudt (n_gas). */
int crk_hydro_forces(crk_ctx *ctx, crk_tree *tree, const void *m,
                     const void *vx, const void *vy, const void *vz,
                     const void *V, const void *rho, const void *P,
                     const void *cs, const void *A, const void *B,
                     const void *gradA, const void *gradB, void *ax,
                     void *ay, void *az, void *dudt);

/* Velocity gradient with the corrected kernel (the CRKSPH gradient of a
 * field, Sec. IV-A; the input of the reconstructed viscosity below):
 *   dv[a][b]_i = sum_j V_j (v_j^a - v_i^a) g_i(x_ij)_b
 * over gas j with r_ij < 2 h_i, g_i the corrected-kernel gradient at h_i
 * (as in crk_hydro_forces).  The corrected kernel reproduces linear fields,
 * so a linear velocity field returns its gradient exactly wherever the
 * moment matrix is regular.
 * Inputs (n_gas each): vx, vy, vz, V, A; B, gradA (3 planes), gradB
 * (9 planes), from crk_density and crk_coefficients.  Output dv: 9 planes
 * of n_gas, plane 3a + b = d v^a / d x^b.  Timed as index 7 of
 * crk_pass_times. */
int crk_velocity_gradient(crk_ctx *ctx, crk_tree *tree, const void *vx,
                          const void *vy, const void *vz, const void *V,
                          const void *A, const void *B, const void *gradA,
                          const void *gradB, void *dv);

/* crk_hydro_forces with the viscosity acting on a limited linear
 * reconstruction of the velocities at the pair midpoint (CRKSPH's
 * viscosity, Sec. IV-A; the limiter is a reading):
 *   v~_ij = v_ij - phi_ij/2 (dv_i + dv_j) x_ij,
 *   phi_ij = 4 s_i s_j / (s_i + s_j)^2 if s_i s_j > 0 else 0,
 *   s_k = x_ij . dv_k x_ij  (van Leer's limiter of the ratio s_i / s_j),
 * times exp(-((eta - eta_crit) / eta_fold)^2) when
 * eta = r_ij / max(h_i, h_j) < eta_crit; mu_ij takes v~_ij in place of
 * v_ij.  phi is symmetric in the pair, so F_ij = -F_ji still; du/dt keeps
 * the actual v_ij, so the energy rate is conserved.  A linear flow whose
 * pairs all lie beyond eta_crit gets no viscous force.
 * Arguments as crk_hydro_forces, plus dv (9 planes from
 * crk_velocity_gradient), eta_crit >= 0 and eta_fold > 0 (finite, else
 * CRK_EINVAL; usual values 0.8 and 0.2). */
int crk_hydro_forces_limited(crk_ctx *ctx, crk_tree *tree, const void *m,
                             const void *vx, const void *vy, const void *vz,
                             const void *V, const void *rho, const void *P,
                             const void *cs, const void *A, const void *B,
                             const void *gradA, const void *gradB,
                             const void *dv, double eta_crit, double eta_fold,
                             void *ax, void *ay, void *az, void *dudt);

/* Compatible specific-energy rate for the kick that crk_integrate applies
 * next (CRKSPH's energy-conserving update, Sec. IV-A; the form is a
 * reading): with the pair forces F_ij of the current state (exactly those
 * of crk_hydro_forces, or of crk_hydro_forces_limited when dv is given) and
 * the velocities after the kick v1 = v + dt (a_grav + a_hydro),
 *   du_i/dt = -sum_j F_ij . (v^c_i - v^c_j) / (2 m_i),  v^c = (v + v1)/2,
 * over the same pairs.  A kick v1, u1 = u + dt du/dt with the hydro forces
 * alone then conserves sum m (v^2/2 + u) to rounding (the plain rate, the
 * pair work at v, only to O(dt^2)); dt = 0 gives the plain rate.
 * Arguments as crk_hydro_forces_limited (dv may be NULL: plain viscosity;
 * eta_crit, eta_fold are checked only with dv), plus dt (finite) and the
 * accelerations of the kick: a_grav 3 planes (required), a_hydro 3 planes
 * or NULL.  Output dudt (n_gas) only; the accelerations are not rewritten.
 * Timed as index 8 of crk_pass_times. */
int crk_hydro_energy_compatible(crk_ctx *ctx, crk_tree *tree, const void *m,
                                const void *vx, const void *vy, const void *vz,
                                const void *V, const void *rho, const void *P,
                                const void *cs, const void *A, const void *B,
                                const void *gradA, const void *gradB,
                                const void *dv, double eta_crit,
                                double eta_fold, double dt,
                                const void *const a_grav[3],
                                const void *const a_hydro[3], void *dudt);

/* The compatible energy update inside the block kicks of a hierarchical
 * cycle (CRKSPH's energy conservation, Sec. IV-A, under the adaptive
 * integration of that section; the split of the kicks is this library's
 * reading).  The kick after substep `substep` of a cycle of 2^max_level
 * substeps moves each gas particle i by a width w_i from its bin b
 * (tau_b = dt / 2^b): substep -1, the opening half-kick of every particle
 * at the start of the interval, w = tau_b / 2; a particle ending a step
 * after `substep`, w = tau_b (its closing half-kick and the opening
 * half-kick of its next step, made with the same forces, as one kick), or
 * tau_b / 2 after the last substep; any other particle w = 0.  With
 * v1 = v + w (a_grav + a_hydro), the rate is that of
 * crk_hydro_energy_compatible with the pair work at (v + v1)/2, written for
 * the particles crk_tree_set_active selected; the caller's two half-kicks
 * (crk_kick phases 1 and 0) both apply it, so u gains w du/dt in all.
 * With one bin (or bins that differ only between particles that do not
 * interact) the hydro kicks conserve sum m (v^2/2 + u) to rounding.
 * The selection must be that of crk_tree_set_active(bins, max_level,
 * substep), or everything for substep -1 (CRK_ESTATE otherwise).
 * dt > 0 is the interval; bins_gas: n_gas int32 levels (device, caller
 * order, clamped to [0, max_level]); other arguments as
 * crk_hydro_energy_compatible.  Timed as index 8 of crk_pass_times. */
int crk_hydro_energy_compatible_block(
    crk_ctx *ctx, crk_tree *tree, const void *m, const void *vx,
    const void *vy, const void *vz, const void *V, const void *rho,
    const void *P, const void *cs, const void *A, const void *B,
    const void *gradA, const void *gradB, const void *dv, double eta_crit,
    double eta_fold, double dt, int32_t max_level, const int32_t *bins_gas,
    int64_t substep, const void *const a_grav[3], const void *const a_hydro[3],
    void *dudt);

/* Short-range gravity inside the handover scale (Sec. IV-A, with the
 * long-range part left to a spectral particle-mesh solver):
 *   a_i = -G sum_{j != i, r_ij < r_c} m_j g(r_ij) x_ij / r_ij,
 *   g(r) = r / (r^2 + eps^2)^(3/2) - R_S2(r; r_c),
 * where R_S2 is the force between two S2 clouds of diameter r_c (Hockney &
 * Eastwood), over both species of the particle's box.
 * m_gas (n_gas), m_dm (n_dm): masses; outputs ax/ay/az for gas (n_gas) and
 * dm (n_dm). */
int shortrange_gravity(crk_ctx *ctx, crk_tree *tree, const void *m_gas,
                       const void *m_dm, void *ax_gas, void *ay_gas,
                       void *az_gas, void *ax_dm, void *ay_dm, void *az_dm);

/* One kick-drift in double precision (the mixed-precision pattern of
 * Sec. IV-A: float short-range sums, double state):
 *   v += dt (a_grav + a_hydro), x += dt v wrapped into [1, 2), u += dt dudt,
 * then refreshes the context-precision copies of x, v and u.
 * n particles; x64, v64: 3 planes of doubles (in/out); u64: doubles or NULL
 * (dm); a_grav: 3 planes (context precision); a_hydro and dudt: 3 planes /
 * n values or NULL; x, v: 3 pointers each to the context-precision copies
 * (out); u: context-precision copy or NULL. */
int crk_integrate(crk_ctx *ctx, int64_t n, double dt, double *x64,
                  double *v64, double *u64, const void *const a_grav[3],
                  const void *const a_hydro[3], const void *dudt,
                  void *const x[3], void *const v[3], void *u);

/* ------------------------------------------------------------------------ */
/* hierarchical time steps on a tree kept for an interval                    */
/* ------------------------------------------------------------------------ */
/* The adaptive integration of Sec. IV-A groups particles into timestep bins
 * and subcycles them inside a long step; Sec. IV-B.1 keeps the tree for the
 * whole interval, lets the leaf bounding boxes grow, and updates only active
 * leaves at a substep.  The interval dt is cut into 2^max_level substeps;
 * a particle of bin b steps by tau_b = dt / 2^b, starting at substeps s with
 * s % 2^(max_level-b) == 0 and ending after substeps s with
 * (s + 1) % 2^(max_level-b) == 0.  One substep of a block kick-drift-kick
 * cycle: crk_kick (phase 0), crk_drift (no wrap), crk_tree_refit,
 * crk_tree_set_active (substep s), build_interaction_lists (lists of the
 * active leaves only), the four passes (they then run over the active
 * leaves and write only active particles; inactive ones keep their
 * outputs), crk_kick (phase 1); after the last substep every particle is
 * synchronised and crk_drift with delta 0 and wrap 1 wraps the positions.
 * All arrays are device memory in caller order unless stated. */

/* Timestep bin of n particles: the smallest b in [0, max_level] whose
 * tau_b = dt / 2^b satisfies tau_b^4 |a|^2 <= (2 eta eps)^2 (the criterion
 * tau <= sqrt(2 eta eps / |a|) with softening eps) and, when h and cs are
 * given (gas), the Courant condition tau_b cs <= c_cfl h; max_level when
 * none does.  |a|^2 = ((ax^2 + ay^2) + az^2) with a = a_grav + a_hydro
 * (a_hydro may be NULL), evaluated in double with every operation rounded
 * once in that order, so the integer result is reproducible.  a_grav,
 * a_hydro: 3 planes, h, cs: n values (context precision, or NULL for dark
 * matter); bins: n int32 (out).  dt > 0, 0 <= max_level <= 30. */
int crk_timestep_bins(crk_ctx *ctx, int64_t n, double dt, int32_t max_level,
                      double eps, double c_cfl, double eta,
                      const void *const a_grav[3], const void *const a_hydro[3],
                      const void *h, const void *cs, int32_t *bins);

/* Selects the particles ending a step after substep `substep` of a cycle
 * with 2^max_level substeps (bins_gas: n_gas, bins_dm: n_dm int32 levels,
 * clamped to [0, max_level]); the leaves holding any of them become the work
 * items of the pair passes, which then write outputs for those particles
 * only.  substep < 0 selects everything (the state after build_tree).
 * The lists must be rebuilt after every call (build_interaction_lists then
 * lists the active leaves only; the passes report CRK_ESTATE until then).
 * With sub-leaves, the call also lists the sub-leaves that hold an active
 * particle (the split sweep then runs one wavefront per listed sub-leaf)
 * and, as tuning act_groups decides, gathers the active particles of each
 * into a group (see crk_tuning), boxed at the tree's current positions,
 * which the sub-leaf sweeps then take as their i-sets.  The subset's sizes
 * are reported by crk_tree_get_info.  Synchronises (reads the active leaf
 * and particle counts back). */
int crk_tree_set_active(crk_ctx *ctx, crk_tree *tree, const int32_t *bins_gas,
                        const int32_t *bins_dm, int32_t max_level,
                        int64_t substep);

/* Copies the particles' current positions (caller order, context
 * precision; not wrapped inside an interval) into the tree and grows every
 * leaf and sub-leaf bounding box to contain them; boxes never shrink and the
 * smoothing lengths stay those of build_tree.  Returns CRK_ESTALE when a
 * leaf box reaches so far out of its chaining-mesh bin (by d) that the
 * 27-bin stencil could miss a pair (2 d + range > bin width): the tree must
 * then be rebuilt.  The lists must be rebuilt after a refit (the passes
 * report CRK_ESTATE until then), and an active subset's dense groups
 * (tuning act_groups) are dropped until the next crk_tree_set_active (the
 * passes then sweep the tree's sub-leaves).  Synchronises. */
int crk_tree_refit(crk_ctx *ctx, crk_tree *tree, const void *gx,
                   const void *gy, const void *gz, const void *dx,
                   const void *dy, const void *dz);

/* Block kick at substep s: the particles starting (phase 0) or ending
 * (phase 1) a step at s get v += (a_grav + a_hydro) tau_b / 2 and
 * u += dudt tau_b / 2 in double, then the context-precision copies v and u
 * are refreshed.  v64: 3 planes of doubles (in/out); u64: doubles or NULL;
 * a_grav: 3 planes, a_hydro: 3 planes or NULL, dudt (with u64); v: 3
 * pointers to the copies, u: copy or NULL. */
int crk_kick(crk_ctx *ctx, int64_t n, double dt, int32_t max_level,
             int64_t substep, int32_t phase, const int32_t *bins, double *v64,
             double *u64, const void *const a_grav[3],
             const void *const a_hydro[3], const void *dudt, void *const v[3],
             void *u);

/* Drift of every particle, x += v delta in double (x64, v64: 3 planes),
 * wrapped into [1, 2) when wrap != 0, then the context-precision copies x
 * (3 pointers) are refreshed. */
int crk_drift(crk_ctx *ctx, int64_t n, double delta, int32_t wrap,
              double *x64, const double *v64, void *const x[3]);

/* ------------------------------------------------------------------------ */
/* friends-of-friends groups                                                 */
/* ------------------------------------------------------------------------ */

/* Friends-of-friends groups of every box (the in-situ halo finding of
 * Sec. IV-B.3, here as a second pair workload over the same tree and
 * gravity lists): two particles of a box closer than the linking length b
 * (strictly; squared separations in double from the exact float32
 * separations) are friends; groups are the connected components, both
 * species together.  labels_gas (n_gas) and labels_dm (n_dm) receive, per
 * particle, the smallest combined caller index of its group (gas index, or
 * n_gas + dm index): deterministic whatever the order of the links.
 * Needs built lists, no active subset, 0 < b <= r_c of every box. */
int crk_fof(crk_ctx *ctx, crk_tree *tree, double b, int32_t *labels_gas,
            int32_t *labels_dm);

/* ------------------------------------------------------------------------ */
/* long-range gravity on a mesh                                              */
/* ------------------------------------------------------------------------ */

/* The spectral particle-mesh half of the force split of Sec. IV-A, for one
 * periodic unit box: the long-range acceleration that shortrange_gravity
 * leaves out, i.e. the force between S2 clouds of diameter r_c, so that the
 * two add up to the periodic Newtonian force (up to the mesh error, below
 * 1 % for r_c >= 6 mesh cells, tested against an Ewald sum).  Cloud-in-cell
 * deposit of all masses on the nodes j / n_mesh (double atomics), FFT,
 * multiplication by 4 pi G S2(k)^2 / (k^2 W(k)^2) with W the CIC window
 * prod_a sinc^2(k_a / (2 n_mesh)), spectral gradient i k (k = 0 and each
 * component's Nyquist plane removed), three inverse FFTs, cloud-in-cell
 * interpolation.  Positions (context precision, periodic, wrapped into the
 * box by the deposit), masses; outputs a_gas (3 pointers, n_gas values) and
 * a_dm (3 pointers, n_dm values), overwritten.  n_mesh even in [4, 2048];
 * the mesh workspace and FFT plans live in the context and are reused for
 * the same n_mesh. */
int crk_pm_gravity(crk_ctx *ctx, int32_t n_mesh, double r_c, int64_t n_gas,
                   const void *gx, const void *gy, const void *gz,
                   const void *m_gas, int64_t n_dm, const void *dx,
                   const void *dy, const void *dz, const void *m_dm,
                   void *const a_gas[3], void *const a_dm[3]);

/* ------------------------------------------------------------------------ */
/* tree queries, graph capture, release                                      */
/* ------------------------------------------------------------------------ */

/* Sizes of a built tree (host values; valid after a synchronising build). */
typedef struct {
    int64_t n_gas, n_dm;
    int64_t n_leaves, n_gas_leaves;
    int64_t n_bins;                 /* chaining-mesh bins over all boxes     */
    int64_t grav_entries, hydro_entries; /* list lengths (leaf pairs)        */
    int32_t kd_levels;              /* k-d levels run                        */
    /* the subset of the last crk_tree_set_active (0 after build_tree and
     * for substep < 0): its leaves and particles, and 1 when the sub-leaf
     * sweeps take active groups (tuning act_groups) */
    int64_t act_leaves, act_particles;
    int32_t act_grouped;
} crk_tree_info;
int crk_tree_get_info(const crk_tree *tree, crk_tree_info *info);

/* Group properties of a friends-of-friends labelling (the in-situ halo
 * finding of Sec. IV-B.3), for the labels crk_fof returns (group label =
 * smallest combined caller index of its members: gas index, or n_gas + dm
 * index).  Per index q of [0, n_gas + n_dm): count[q] members, mass[q]
 * their total mass and centre (3 planes of n_gas + n_dm doubles, plane a at
 * offset a (n_gas + n_dm)) the periodic centre of mass -- every member at
 * its minimum image about particle q, the mass-weighted mean of the images,
 * wrapped into [1, 2) -- at the indices that label a group; 0 elsewhere.
 * Sums in double with atomics (their order, so the last bits, may vary).
 * gas_x, dm_x: 3 pointers each to positions (context precision, caller
 * order); m_gas, m_dm: masses; labels: int32, caller order.  Labels outside
 * [0, n_gas + n_dm) are skipped and reported by crk_sync (CRK_EINVAL).
 * Outputs are overwritten (cleared by the call).  Needs no tree. */
int crk_fof_properties(crk_ctx *ctx, int64_t n_gas, int64_t n_dm,
                       const int32_t *labels_gas, const int32_t *labels_dm,
                       const void *const gas_x[3], const void *m_gas,
                       const void *const dm_x[3], const void *m_dm,
                       int32_t *count, double *mass, double *centre);

/* Pair counts under each pass's own pair test (a diagnostic for throughput
 * accounting; synchronises).  totals[0]: gas pairs with r_ij < 2 h_i, i = j
 * included (density and coefficients); totals[1]: gas pairs i != j with
 * r_ij < 2 max(h_i, h_j) (hydro forces); totals[2]: pairs with
 * 0 < r_ij < r_c (gravity).  totals[3..5]: the (i, candidate) pairs the
 * sweeps of those passes evaluate after culling against the leaf boxes. */
int crk_count_pairs(crk_ctx *ctx, crk_tree *tree, int64_t totals[6]);

/* Copies the tree-order permutation (caller index of each tree slot: gas
 * index, or n_gas + dm index) and the leaf table (start, count; host int64
 * arrays of n_leaves) to host memory; either pointer may be NULL. */
int crk_tree_get_leaves(crk_ctx *ctx, const crk_tree *tree, int64_t *perm,
                        int64_t *leaf_start, int64_t *leaf_count);

/* Captures everything enqueued on the context's stream between begin and
 * end into a HIP graph (build_tree and build_interaction_lists then use
 * the capacities of the previous eager build and read nothing back);
 * crk_graph_launch replays it.  Capacities exceeded during a replay are
 * reported by crk_sync as CRK_ECAPACITY; the recovery is an eager call at
 * the new size followed by a new capture.  The graph holds the addresses of
 * the library's buffers at capture time: once any library buffer of the
 * process has been grown (moved) or freed since then (an eager call that
 * needs more room, crk_tree_free, crk_ctx_destroy of any context),
 * crk_graph_launch returns CRK_ESTATE without launching anything, and the
 * caller captures again. */
int crk_graph_begin(crk_ctx *ctx);
int crk_graph_end(crk_ctx *ctx);
int crk_graph_launch(crk_ctx *ctx);
/* Drops the captured graph, if any (a later crk_graph_launch returns
 * CRK_ESTATE until the next capture). */
int crk_graph_reset(crk_ctx *ctx);

int crk_tree_free(crk_tree *tree);

/* Timing with HIP events on the context's stream (outside graph capture).
 * enable = 1 starts recording; crk_pass_times waits for the stream and
 * returns, per operation since the last query, the summed milliseconds of
 * the whole call (pass_ms) and of its main kernel alone (kernel_ms: the pair
 * kernel of each pass and the integrate kernel), and the number of
 * main-kernel launches.  Index order: 0 build_tree, 1 lists, 2 density,
 * 3 coefficients, 4 hydro, 5 gravity, 6 integrate, 7 velocity gradient,
 * 8 compatible energy rate.  Any array may be NULL. */
int crk_timing_enable(crk_ctx *ctx, int enable);
int crk_pass_times(crk_ctx *ctx, double pass_ms[9], double kernel_ms[9],
                   int64_t launches[9]);

#ifdef __cplusplus
}
#endif

#endif /* CRK_H */
