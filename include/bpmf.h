/*
 * bpmf.h -- C ABI of libbpmf, the MI355X (gfx950) hot path of grid-based
 * binding-potential-of-mean-force (BPMF) sampling, after D. D. L. Minh,
 * "Alchemical Grid Dock (AlGDock): Binding Free Energy Calculations between
 * Flexible Ligands and Rigid Receptors" (arXiv 1507.03703).
 *
 * The library samples a flexible ligand against a rigid receptor that is
 * represented by precomputed interaction grids, with replica-exchange
 * Hamiltonian Monte Carlo over a ladder of thermodynamic states, and builds
 * the reduced-energy matrix u_kn that MBAR turns into free energies.
 *
 * Conventions shared by every entry point
 *   Units      A, fs, amu, kJ/mol, elementary charge, K.
 *   Status     every function returns BPMF_OK (0) or a negative BPMF_E_* code;
 *              bpmf_last_error() returns the calling thread's last message.
 *              Nothing aborts and no C++ exception crosses this boundary.
 *   Memory     "host" pointers are read (or written) during the call only and
 *              stay owned by the caller.  "device" pointers are HIP device
 *              addresses owned by the caller; the library reads/writes them in
 *              stream order.  Persistent device state (grid, ligands,
 *              replicas, samples, scratch) is allocated through the allocator
 *              callback given to bpmf_create (hipMalloc if none) and released
 *              by bpmf_destroy.
 *   Streams    all device work is enqueued on the stream given to
 *              bpmf_create.  Calls that return host data synchronise that
 *              stream; the others return without waiting.
 *   Validation arguments are checked before anything is enqueued; a failed
 *              check leaves all state unchanged.  Asynchronous HIP failures
 *              surface as BPMF_E_HIP on a later call.
 *   Numerics   a non-finite Hamiltonian or exchange exponent is not an error:
 *              the move is rejected and counted (see bpmf_get_stats).
 *   Threads    one context per host thread.
 *   Determinism the same inputs, seed, build and GPU give bitwise-identical
 *              results (no floating-point atomics on any result path).
 */
#ifndef BPMF_H
#define BPMF_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#if defined(BPMF_BUILD)
#define BPMF_API __attribute__((visibility("default")))
#else
#define BPMF_API
#endif

enum {
  BPMF_OK = 0,
  BPMF_E_INVAL = -1,  /* invalid argument (message says which) */
  BPMF_E_NOMEM = -2,  /* allocation failed */
  BPMF_E_HIP = -3,    /* HIP runtime error */
  BPMF_E_STATE = -4,  /* call made in the wrong order */
  BPMF_E_UNIMPL = -5  /* option the library does not support */
};

/* Limits of the library. */
#define BPMF_MAX_ATOMS 128     /* atoms per ligand */
#define BPMF_MAX_CHANNELS 8    /* grid channels */
#define BPMF_MAX_STATES 1024   /* thermodynamic states per ligand */
#define BPMF_MAX_MBAR_STATES 128
#define BPMF_MAX_MBAR_BATCH 65535  /* problems per bpmf_mbar_batch call */
#define BPMF_MAX_EXCHANGE_SWEEPS 1024  /* exchange sweeps per due exchange */

typedef struct bpmf_ctx bpmf_ctx;
typedef void* (*bpmf_alloc_fn)(size_t bytes, void* user);
typedef void (*bpmf_free_fn)(void* ptr, void* user);

/* ------------------------------------------------------------------------
 * Lifecycle
 * ------------------------------------------------------------------------ */

/* Create a context on HIP device `device`.
 *   seed       key of the counter-based generator (Philox-4x32-10) that
 *              draws every random number of the run;
 *   hip_stream hipStream_t to enqueue on (NULL = the null stream);
 *   alloc/free device allocator for persistent state, or both NULL for
 *              hipMalloc/hipFree; alloc_user is passed through.
 * Errors: BPMF_E_INVAL (null out, one of alloc/free missing), BPMF_E_HIP. */
BPMF_API int bpmf_create(bpmf_ctx** out, int device, uint64_t seed, void* hip_stream,
                bpmf_alloc_fn alloc, bpmf_free_fn free_fn, void* alloc_user);

/* Synchronise the stream and release every allocation of the context. */
BPMF_API int bpmf_destroy(bpmf_ctx* ctx);

/* Message of the calling thread's most recent failure ("" if none). */
BPMF_API const char* bpmf_last_error(void);

/* ABI version of this header (major*100 + minor). */
BPMF_API int bpmf_version(void);

/* Wait for all work enqueued by the context. */
BPMF_API int bpmf_sync(bpmf_ctx* ctx);

/* ------------------------------------------------------------------------
 * Receptor grids
 *   The paper represents receptor-ligand interactions by one electrostatic
 *   and two van der Waals grids (Methodology, "Thermodynamic Cycle": grid
 *   interaction energy Psi_g = Psi_PBSA + Psi_vdW).  Each channel is
 *   trilinearly interpolated; a channel with transform 4 stores the quartic
 *   root of its values and is raised to the fourth power after
 *   interpolation (the repulsive grid's inverse transformation power of 4).
 *   Outside the grid the value of the nearest boundary point is used (clamp
 *   to edge), with zero normal gradient.
 * ------------------------------------------------------------------------ */
typedef struct {
  int nx, ny, nz;      /* nodes per axis, each 2..2^24 */
  int n_channels;      /* 1..BPMF_MAX_CHANNELS */
  double origin[3];    /* position of node (0,0,0) */
  double spacing;      /* node spacing, > 0 */
  const int* transform; /* host, n_channels entries: 0 = none, 4 = quartic root */
} bpmf_grid_desc;

/* Upload the grid: host_nodes is nz*ny*nx*n_channels floats, x fastest,
 * channel innermost (node (ix,iy,iz) channel c at
 * ((iz*ny + iy)*nx + ix)*n_channels + c).  Replaces a previous grid (only
 * allowed before the first ligand is set up).  The library keeps a
 * cell-major copy on the device: per cell the values of its 8 corners,
 * padded to 8, 16, 32 or 64 floats (128 bytes for 3 or 4 channels), so one
 * interpolation reads one aligned record; device memory is about 8x the
 * node grid (0.5 GB for 160^3 x 3, 2.1 GB for 256^3 x 3).
 * Errors: BPMF_E_INVAL (bad sizes, more than 64 GiB of cell records,
 * non-finite node, negative node on a transform-4 channel), BPMF_E_STATE
 * (ligands exist), BPMF_E_NOMEM. */
BPMF_API int bpmf_grid_upload(bpmf_ctx* ctx, const bpmf_grid_desc* desc,
                     const float* host_nodes);

/* ------------------------------------------------------------------------
 * Ligands, their force field and their ladder of thermodynamic states
 *   Intramolecular energy (the U_s(r_L) term of the alchemical protocol,
 *   GAFF functional forms): bonds K_r (r - r0)^2, angles
 *   K_theta (theta - theta0)^2, proper torsions (V/2)(1 + cos(n phi - gamma))
 *   with phi the IUPAC dihedral.  Binding-site restraint (Eq. binding_site):
 *   U_I = k (d - d0)^2 / 2 for d > d0, where d is the distance of the
 *   mass-weighted centre from site_center.  State k has temperature T_k and
 *   grid weights w_kc, so that
 *       U_k(x) = U_bond + U_angle + U_tors + U_I + sum_c w_kc Psi_c(x),
 *       Psi_c(x) = sum_i s_ic * interp_c(x_i)   (interp^4 for transform 4),
 *   and u_k = U_k / (R T_k) with R = 8.314462618e-3 kJ/(mol K)
 *   (reduced potential, Thermodynamic Cycle).
 * ------------------------------------------------------------------------ */
typedef struct {
  int n_atoms;                /* 1..BPMF_MAX_ATOMS */
  const double* mass;         /* host, n_atoms, > 0 (amu) */
  const double* scale;        /* host, n_atoms x n_channels factors s_ic */
  int n_bonds;
  const int* bond_ij;         /* host, n_bonds x 2 atom indices */
  const double* bond_k_r0;    /* host, n_bonds x 2: K_r, r0 */
  int n_angles;
  const int* angle_ijk;       /* host, n_angles x 3, j = vertex */
  const double* angle_k_t0;   /* host, n_angles x 2: K_theta, theta0 (rad) */
  int n_tors;
  const int* tors_ijkl;       /* host, n_tors x 4 */
  const double* tors_v_n_g;   /* host, n_tors x 3: V/2, n (integer 1..6),
                                 gamma (rad) */
  double site_center[3];
  double d0;                  /* restraint radius (A), >= 0 */
  double k_restraint;         /* kJ/(mol A^2), >= 0 */
  int n_states;               /* K = replicas of this ligand, 1..BPMF_MAX_STATES */
  const double* T;            /* host, K temperatures (K), > 0 */
  const double* w;            /* host, K x n_channels grid weights */
  const double* dt_fs;        /* host, K time steps (fs), > 0 */
  const float* x0;            /* host, K x n_atoms x 3 start of replica r (state r) */
  int sample_capacity;        /* recorded samples per state (>= 0) */
} bpmf_ligand_desc;

/* Copy a ligand to the device; replica r starts in state r at x0[r].
 * Returns its id (0, 1, ...) in *ligand_id.  The grid must exist.
 * Errors: BPMF_E_INVAL (any index out of range or repeated within a term,
 * non-positive mass/T/dt, non-finite parameter), BPMF_E_STATE (no grid),
 * BPMF_E_NOMEM. */
BPMF_API int bpmf_ligand_setup(bpmf_ctx* ctx, const bpmf_ligand_desc* desc,
                      int* ligand_id);

/* ------------------------------------------------------------------------
 * Sampling
 * ------------------------------------------------------------------------ */
typedef struct {
  int n_sweeps;        /* >= 0 */
  int n_leapfrog;      /* velocity-Verlet steps per HMC trial, >= 1 */
  int exchange_every;  /* 0 = never; else exchange when counter % every == 0 */
  int exchange_scheme; /* 0 = neighbour pairs, even/odd by counter parity;
                          1 = all pairs 1..max_sep apart, sequential */
  int max_sep;         /* scheme 1 only, >= 1 */
  int sample_every;    /* 0 = never; else record when (counter+1) % every == 0 */
  int pose_move_every; /* 0 = never; else after the call's sweeps P, 2P, ...
                          one pose move (bpmf_pose_move) of every ligand with
                          a proposal */
  int external_moves;  /* 0 = none; else after every unit (P sweeps, or one
                          sweep when pose_move_every = 0) this many external
                          moves (bpmf_external_move) of every ligand */
  int external_k_max;  /* states 0..external_k_max-1 take external moves */
  double external_sigma; /* translation per axis (A), > 0 when used */
  int exchange_sweeps; /* 0 or 1 = one exchange sweep when an exchange is
                          due; n > 1 (scheme 1 only, <= BPMF_MAX_EXCHANGE_
                          SWEEPS) = n sweeps in a row (Equilibration and
                          production: each iteration ends with 25) */
} bpmf_sweep_args;

/* Run n_sweeps sweeps over every ligand.  One sweep of a ligand with
 * per-ligand counter s is (the order of effects; with scheme 0 the kernels
 * apply steps 2-3 of a sweep at the start of the next one, and of the last
 * sweep before returning):
 *   1. one HMC move per replica (Sampling: velocity-Verlet trial moves):
 *      momenta v_i ~ N(0, R T_k / m_i * 1e-4) (A/fs), n_leapfrog steps of
 *      v += dt/2 a; x += dt v; v += dt/2 a with a = F/m * 1e-4, then accept
 *      iff ln u < -(H1 - H0) / (R T_k), H = U_k + sum m v^2/2 * 1e4,
 *      H summed in double; non-finite H or x => reject;
 *   2. if due, exchange_sweeps replica-exchange sweeps (see bpmf_exchange);
 *   3. if due, record one sample per state: the configuration and cached
 *      energy components of the replica currently in that state;
 *   4. s += 1.
 * With pose_move_every = P > 0 the call runs units of P sweeps, each
 * closed by one independence pose move per replica of every ligand that has
 * a proposal (the moves see the state after the unit's last exchange and
 * record); sweeps past the last whole unit run without a move.  With
 * external_moves = n > 0 every unit (of P sweeps, or of one sweep when P =
 * 0) is closed, after its pose move, by n external moves per replica in the
 * states below external_k_max (Sampling: the paper attempts them in the
 * states whose grid coupling is below 0.01, after each HMC move; here they
 * follow the unit's exchange, an equally valid order of moves that each
 * keep the target).  max(1, chunk / P) units (P = 1 without pose moves)
 * are captured as one hipGraph and replayed, the units left over launched
 * plainly (see bpmf_set_graph).
 * Random numbers: Philox-4x32-10 keyed by the context seed, counter
 * (index, ligand<<16 | replica, s, purpose) with purpose 1 = momenta
 * (index = atom), 2 = acceptance (index 0), 3 | sep<<8 = exchange
 * (index = lower state, replica field = exchange sweep j of the due
 * exchange, 0-based); uniforms (u32 + 1) 2^-32.
 * Errors: BPMF_E_INVAL (bad args, sample capacity would overflow),
 * BPMF_E_STATE (no ligand). */
BPMF_API int bpmf_hmc_sweep(bpmf_ctx* ctx, const bpmf_sweep_args* args);

/* n_sweeps (1..BPMF_MAX_EXCHANGE_SWEEPS) replica-exchange sweeps in a row
 * of ligand `ligand_id` (-1 = every ligand) at its current counter s (the
 * counter is not advanced; sweep j draws its uniforms with replica field j).  Each attempted pair
 * (a, b) with configuration x in state a and y in state b is accepted with
 * probability min(1, exp(-[u_a(y) + u_b(x) - u_a(x) - u_b(y)])) (Eq.
 * repXacc), evaluated in double from the cached components; acceptance swaps
 * the two state labels.  Scheme 0 attempts (a, a+1) for a = s mod 2, s mod
 * 2 + 2, ...; scheme 1 attempts every pair 1..max_sep apart, separation
 * ascending then a ascending, each decision seeing the previous ones
 * (Sampling: pairs 1..min(5, K) states apart). */
BPMF_API int bpmf_exchange(bpmf_ctx* ctx, int ligand_id, int scheme, int max_sep,
                           int n_sweeps);

/* ------------------------------------------------------------------------
 * Reduced-energy matrix and free energies (Estimation)
 * ------------------------------------------------------------------------ */

/* u_kn = U_k(x_n) / (R T_k) for every state k of the ligand and every sample
 * n, in double, written row-major with leading dimension ld >= n_samples to
 * device buffer dev_ukn (K x ld doubles, caller-owned).  dev_samples is a
 * device array of n_samples x n_atoms x 3 floats, or NULL to use the samples
 * recorded so far (n_samples must then equal K x records, round-major).
 * Energy components are computed once per sample; U_k is affine in them. */
BPMF_API int bpmf_energy_matrix(bpmf_ctx* ctx, int ligand_id, const float* dev_samples,
                       int64_t n_samples, double* dev_ukn, int64_t ld);

/* bpmf_energy_matrix for n ligands in one call (host arrays of n entries;
 * dev_samples may be NULL, or have NULL entries, for recorded samples).
 * Every sample of every listed ligand is evaluated by persistent launches
 * (ligands of up to 64 and of 65-128 atoms side by side, or in one launch
 * when the larger ones hold most of the work; each workgroup takes a
 * contiguous share of the samples of equal estimated cost), so many small
 * ligands fill the chip together; each entry's u_kn is the one
 * bpmf_energy_matrix writes.  Errors:
 * BPMF_E_INVAL naming the entry (nothing is launched). */
BPMF_API int bpmf_energy_matrix_batch(bpmf_ctx* ctx, int n,
                                      const int* ligand_ids,
                                      const float* const* dev_samples,
                                      const int64_t* n_samples,
                                      double* const* dev_ukn,
                                      const int64_t* ld);

/* bpmf_energy_matrix_batch for callers that cannot allocate memory (code
 * under HIP graph capture, tight serving loops, harnesses that forbid
 * allocation): the same validation, kernels and results (bit for bit), but
 * the call allocates nothing -- no device, pinned or staging memory, no
 * events.  Its job table (one entry per listed ligand with samples, plus
 * one per wavefront class) lives in a fixed device array of
 * BPMF_NOALLOC_MAX_JOBS + 4 entries (about 56 KB) that each device running
 * the library holds until the process ends; it is written by small kernels
 * on the context's stream, then read by the u_kn launches.  Every call on a
 * device shares that array: calls that overlap on one device (different
 * streams or contexts, not ordered by the caller) race and may compute
 * wrong results; calls ordered on one stream do not.  Its launches run one
 * after the other on the context's stream and are not covered by
 * bpmf_set_timing.  Errors: as bpmf_energy_matrix_batch, plus
 * BPMF_E_INVAL when n exceeds BPMF_NOALLOC_MAX_JOBS and BPMF_E_UNIMPL when
 * the device index is 64 or more (no table address kept for it). */
#define BPMF_NOALLOC_MAX_JOBS 1024
BPMF_API int bpmf_energy_matrix_batch_noalloc(bpmf_ctx* ctx, int n,
                                              const int* ligand_ids,
                                              const float* const* dev_samples,
                                              const int64_t* n_samples,
                                              double* const* dev_ukn,
                                              const int64_t* ld);

/* MBAR (Shirts & Chodera 2008, which the paper uses for f_BC,L and f_CD'):
 * solves f_i = -ln sum_n exp(-u_in) / sum_k N_k exp(f_k - u_kn) with f_0 = 0
 * by Newton iterations on the convex MBAR objective, in double on the
 * device.  dev_ukn: K x N (leading dimension ld) device doubles; N_k: host,
 * K sample counts (all > 0, summing to N).  Outputs (host): f[K], var[K]
 * with var[k] the asymptotic variance of f_k - f_0 (var[0] = 0; +inf when
 * the Hessian at the solution is singular, i.e. states without overlap),
 * *n_iter.  Each iteration is a Newton step with backtracking when the
 * gauge-fixed Hessian is numerically positive definite, else one step of
 * the fixed-point equation.  Stops when the largest change of f is below
 * tol or after max_iter iterations (then *n_iter = max_iter).  warm_start
 * != 0: f holds the initial guess on entry (shifted so that f_0 = 0; e.g.
 * the previous cycle's estimate), else the iteration starts from f = 0. */
BPMF_API int bpmf_mbar(bpmf_ctx* ctx, const double* dev_ukn, int K, int64_t N,
              int64_t ld, const int64_t* N_k, double tol, int max_iter,
              double* f, double* var, int* n_iter,
                       int warm_start);

/* MBAR for n_problems independent problems (e.g. every ligand of a batch)
 * in one call: problem p has K[p] states (1..BPMF_MAX_MBAR_STATES) and
 * N[p] samples in the device matrix dev_ukn[p] (K[p] x N[p], leading
 * dimension ld[p]).  dev_ukn, K, N and ld are host arrays of n_problems
 * entries; N_k, f and var hold the problems' K-vectors back to back (host,
 * sum of K entries; var may be NULL), n_iter n_problems ints (may be NULL).
 * Each problem gets exactly the iteration, stopping rule and result
 * bpmf_mbar gives it alone (bpmf_mbar is this call with one problem); the
 * batch advances every unfinished problem by one step per round, so the
 * host waits for the device about three times per iteration of the slowest
 * problem, not per problem.  Scratch grows with the sum over problems of
 * N + 8 (K + K^2) x (N / (4096 / Kp)) doubles (Kp = K rounded up to 16, 32,
 * 64 or 128).  Errors: BPMF_E_INVAL naming the offending problem (nothing is
 * computed). */
BPMF_API int bpmf_mbar_batch(bpmf_ctx* ctx, int n_problems,
                             const double* const* dev_ukn, const int* K,
                             const int64_t* N, const int64_t* ld,
                             const int64_t* N_k, double tol, int max_iter,
                             double* f, double* var, int* n_iter,
                             int warm_start);

/* ------------------------------------------------------------------------
 * Direct evaluation (the energy/force kernel the sampler runs, exposed)
 * ------------------------------------------------------------------------ */

/* For n_conf configurations dev_x (device, n_conf x n_atoms x 3 floats) and
 * per-configuration grid weights dev_w (device, n_conf x n_channels
 * doubles), write dev_terms (device, n_conf x (4 + n_channels) doubles:
 * U_bond, U_angle, U_tors, U_I, Psi_0..) and, unless NULL, dev_forces
 * (device, n_conf x n_atoms x 3 floats) = -grad(U_bond + U_angle + U_tors +
 * U_I + sum_c w_c Psi_c). */
BPMF_API int bpmf_evaluate(bpmf_ctx* ctx, int ligand_id, const float* dev_x,
                  int64_t n_conf, const double* dev_w, double* dev_terms,
                  float* dev_forces);

/* Grid term alone at n independent points: dev_pos (n x 3 floats),
 * dev_scale (n x n_channels floats), host w (n_channels doubles).  Writes
 * dev_energy (n x n_channels floats, e_ic = s_ic interp_c(x_i) after the
 * transform) and dev_force (n x 3 floats, -sum_c w_c grad e_ic); either
 * output may be NULL. */
BPMF_API int bpmf_grid_eval(bpmf_ctx* ctx, const float* dev_pos, const float* dev_scale,
                   int64_t n, const double* w, float* dev_energy,
                   float* dev_force);

/* ------------------------------------------------------------------------
 * Replica state, statistics, samples (checkpoint / resume)
 * ------------------------------------------------------------------------ */

/* Host copies of a ligand's replica state: x (K x n_atoms x 3 floats),
 * state_of_replica (K ints), comps (K x (1 + n_channels) doubles: U_bond +
 * U_angle + U_tors + U_I, then Psi_c), counter (sweeps done).  Any output
 * may be NULL.  Synchronises. */
BPMF_API int bpmf_get_replicas(bpmf_ctx* ctx, int ligand_id, float* x,
                      int* state_of_replica, double* comps, uint64_t* counter);

/* Restore replica state (inverse of bpmf_get_replicas).  state_of_replica
 * must be a permutation of 0..K-1.  comps may be NULL: then they are
 * recomputed from x.  Clears nothing else (statistics, the round-trip count
 * and recorded samples are kept; see bpmf_reset_samples); round-trip
 * tracking restarts from the given states. */
BPMF_API int bpmf_set_replicas(bpmf_ctx* ctx, int ligand_id, const float* x,
                      const int* state_of_replica, const double* comps,
                      uint64_t counter);

/* Counters since setup (host outputs, any may be NULL): hmc_acc/hmc_try per
 * state (K), ex_acc/ex_try per neighbour pair (a, a+1) (K-1), nonfinite =
 * trial moves rejected for a non-finite Hamiltonian or position. */
BPMF_API int bpmf_get_stats(bpmf_ctx* ctx, int ligand_id, int64_t* hmc_acc,
                   int64_t* hmc_try, int64_t* ex_acc, int64_t* ex_try,
                   int64_t* nonfinite);

/* Replica round trips since setup (Sampling: the replica-exchange walk
 * between the end states), *trips (host): the number of times a replica
 * that visited state K-1 since it was last in state 0 returned to state 0.
 * A replica starts on its way up only from state 0 (replica 0 at setup, or
 * the replica bpmf_set_replicas places there).  States are observed after
 * every exchange: with the all-separations scheme after the exchange
 * sweeps of each sweep, not after each of them.  0 for a single state.
 * Errors: BPMF_E_INVAL (null trips, bad ligand). */
BPMF_API int bpmf_get_round_trips(bpmf_ctx* ctx, int ligand_id,
                                  int64_t* trips);

/* Recorded samples: *n_records rounds so far; x (records x K x n_atoms x 3
 * floats) and comps (records x K x (1 + n_channels) doubles), round-major,
 * state-minor; either may be NULL.  Synchronises. */
BPMF_API int bpmf_get_samples(bpmf_ctx* ctx, int ligand_id, int64_t* n_records,
                     float* x, double* comps);

/* Forget recorded samples of a ligand (-1 = all). */
BPMF_API int bpmf_reset_samples(bpmf_ctx* ctx, int ligand_id);

/* ------------------------------------------------------------------------
 * Learned rigid-body pose proposal
 *   The paper's external-coordinate move proposes a random rotation about
 *   the centre of mass and a Gaussian translation and accepts by the
 *   Metropolis criterion (Sampling).  Here the proposal is an 8-component
 *   Gaussian mixture over the pose (t, omega) -- t = centre of mass minus
 *   site centre (A), omega = rotation vector of the body frame built from
 *   three frame atoms -- produced by an MLP 16 -> 256 -> 256 -> 104 (SiLU)
 *   from sin/cos of up to 8 conditioning torsions.  Internal coordinates are
 *   kept; the independence Metropolis-Hastings acceptance uses the mixture
 *   folded onto SE(3) (sum over the rotation-vector preimages
 *   (theta + 2 pi m) n, m = -3..3, with the Haar factor
 *   2 (1 - cos|omega|)/|omega|^2):
 *       ln alpha = -(E_k(x') - E_k(x)) / (R T_k) + ln q(xi) - ln q(xi').
 *   Network outputs per component j (13): logit, mu_t (3), raw mu_w (3) with
 *   mu_w = pi tanh(raw), raw sigma_t (3), raw sigma_w (3) with
 *   sigma = lo + (hi - lo) sigmoid(raw), sigma_t in [0.02, 3] A, sigma_w in
 *   [0.02, 1.5] rad.  Dense layers run on bf16 matrix cores with fp32
 *   accumulation; master weights are fp32.
 *   Parameter vector (BPMF_PROPOSAL_PARAMS floats): W1 (16 x 256, [in][out]),
 *   b1 (256), W2 (256 x 256), b2, W3 (256 x 104), b3 (104).
 * ------------------------------------------------------------------------ */
#define BPMF_PROPOSAL_PARAMS 96872
#define BPMF_PROPOSAL_OUT 104
#define BPMF_PROPOSAL_FEAT 16

/* Attach a proposal to a ligand: frame_atoms (host, 3 distinct atoms whose
 * positions define the body frame: e1 along a0->a1, e2 the part of a0->a2
 * orthogonal to e1, e3 = e1 x e2), n_cond <= 8 conditioning torsions
 * cond_ijkl (host, n_cond x 4 atom indices), initial params (host). */
BPMF_API int bpmf_proposal_setup(bpmf_ctx* ctx, int ligand_id,
                                 const int* frame_atoms, int n_cond,
                                 const int* cond_ijkl, const float* params);

/* Copy the fp32 parameters out (out != NULL) and/or in (in != NULL). */
BPMF_API int bpmf_proposal_params(bpmf_ctx* ctx, int ligand_id, float* out,
                                  const float* in);

/* Pose and features of N configurations dev_x (device, N x n_atoms x 3):
 * dev_feats (device, N x 16: sin, cos of each conditioning torsion, zero
 * padded), dev_poses (device, N x 6: t, omega with |omega| <= pi). */
BPMF_API int bpmf_pose_features(bpmf_ctx* ctx, int ligand_id,
                                const float* dev_x, int64_t N,
                                float* dev_feats, float* dev_poses);

/* Network outputs dev_out (device, N x 104) for dev_feats (device, N x 16). */
BPMF_API int bpmf_proposal_forward(bpmf_ctx* ctx, int ligand_id,
                                   const float* dev_feats, int64_t N,
                                   float* dev_out);

/* Gradient (device, BPMF_PROPOSAL_PARAMS floats) of the mean negative
 * log-likelihood of dev_poses under the mixture for dev_feats; *loss (host,
 * may be NULL) receives the loss (synchronises). */
BPMF_API int bpmf_proposal_grad(bpmf_ctx* ctx, int ligand_id,
                                const float* dev_feats, const float* dev_poses,
                                int64_t N, float* dev_grad, double* loss);

/* `steps` Adam steps (beta1 0.9, beta2 0.999, eps 1e-8, learning rate lr)
 * on minibatches of `batch` rows drawn with replacement (Philox) from the N
 * training pairs; loss_out (host, steps doubles, may be NULL) receives each
 * step's minibatch loss (synchronises every step when given). */
BPMF_API int bpmf_proposal_train(bpmf_ctx* ctx, int ligand_id,
                                 const float* dev_feats,
                                 const float* dev_poses, int64_t N, int batch,
                                 int steps, double lr, double* loss_out);

/* `rounds` independence MH pose moves of every replica of the ligand (-1 =
 * every ligand with a proposal) at the current sweep counter.  Random
 * numbers: Philox purpose 4, index 0 (component), 1 and 2 (normals of t and
 * omega), 3 (acceptance). */
BPMF_API int bpmf_pose_move(bpmf_ctx* ctx, int ligand_id, int rounds);

/* ------------------------------------------------------------------------
 * External-coordinate moves (Sampling: external coordinate Markov chain
 * Monte Carlo)
 * ------------------------------------------------------------------------ */

/* n_moves external moves in a row of every replica of the ligand (-1 =
 * every ligand) whose state is below k_max, at the current sweep counter s
 * (not advanced; calls at the same s repeat their random numbers).  A move
 * rotates the ligand rigidly about its (mass-weighted) centre of mass by
 * the rotation of a uniform random unit quaternion -- with uniforms u1, u2,
 * u3: (w, x, y, z) = (sqrt(u1) cos 2 pi u3, sqrt(1-u1) sin 2 pi u2,
 * sqrt(1-u1) cos 2 pi u2, sqrt(u1) sin 2 pi u3) -- translates it by sigma z
 * (z standard normal per axis; the paper uses 0.6 A) and is accepted iff
 * ln u < -(U_k(x') - U_k(x)) / (R T_k), energies in double; the proposal is
 * symmetric.  Accepted moves update the positions and cached components.
 * Random numbers: Philox purpose 6, index 3m (u1, u2, u3 of move m), 3m + 1
 * (the three normals), 3m + 2 (acceptance, first word).
 * Errors: BPMF_E_INVAL (n_moves < 0, k_max < 0, sigma not positive and
 * finite). */
BPMF_API int bpmf_external_move(bpmf_ctx* ctx, int ligand_id, int n_moves,
                                int k_max, double sigma);

/* Attempted and accepted external moves per state (host arrays of K, may
 * be NULL). */
BPMF_API int bpmf_get_external_stats(bpmf_ctx* ctx, int ligand_id,
                                     int64_t* accepted, int64_t* tried);

/* Pose-move counts per state (host, K each) and ln alpha of each replica's
 * last move (host, K); any output may be NULL. */
BPMF_API int bpmf_get_pose_stats(bpmf_ctx* ctx, int ligand_id, int64_t* acc,
                                 int64_t* tries, double* last_ln_alpha);

/* ------------------------------------------------------------------------
 * Intramolecular nonbonded and implicit-solvent terms of a ligand
 * (Thermodynamic Cycle: the ligand force field and its OBC generalised-
 * Born/surface-area solvent)
 * ------------------------------------------------------------------------ */
typedef struct {
  const double* charge;     /* host, n_atoms partial charges (e) */
  const double* lj_sigma;   /* host, n_atoms LJ sigma (A), > 0 */
  const double* lj_eps;     /* host, n_atoms LJ epsilon (kJ/mol), >= 0 */
  const double* gb_radius;  /* host, n_atoms intrinsic radii rho (A), > 0.09 */
  const double* gb_scale;   /* host, n_atoms HCT scale factors S, > 0 */
  int n_exclusions;         /* pairs without LJ and Coulomb (1-2, 1-3) */
  const int* exclusions;    /* host, n_exclusions x 2 atom indices */
  int n_pairs14;            /* 1-4 pairs (an excluded pair stays excluded) */
  const int* pairs14;       /* host, n_pairs14 x 2 */
  double lj14, el14;        /* 1-4 scale factors of LJ and Coulomb */
  double eps_solute;        /* dielectric inside (1) */
  double eps_solvent;       /* dielectric of the solvent (78.5) */
  double sa_gamma;          /* surface tension (kJ/mol/A^2), 0 = no SA term */
  double probe_radius;      /* solvent probe radius (A), 1.4 */
} bpmf_pair_desc;

/* Attach pair parameters to a ligand (up to 128 atoms; replaces earlier
 * ones).  Synchronises. */
BPMF_API int bpmf_pair_setup(bpmf_ctx* ctx, int ligand_id,
                             const bpmf_pair_desc* desc);

/* For n_conf configurations dev_x (device, n_conf x n_atoms x 3 floats)
 * write dev_terms (device, n_conf x 4 doubles):
 *   E_LJ   = sum over pairs not excluded of 4 eps_ij ((s/r)^12 - (s/r)^6),
 *            s = (sigma_i + sigma_j)/2, eps_ij = sqrt(eps_i eps_j), 1-4
 *            pairs x lj14;
 *   E_Coul = the same pairs' k_e q_i q_j / (eps_solute r), 1-4 x el14;
 *   E_GB   = -(k_e/2)(1/eps_solute - 1/eps_solvent) sum_i sum_j q_i q_j /
 *            f_ij, f_ij = sqrt(r^2 + R_i R_j exp(-r^2/(4 R_i R_j))), f_ii =
 *            R_i; Born radii 1/R_i = 1/rt_i - tanh(psi - 0.8 psi^2 + 4.85
 *            psi^3)/rho_i (OBC II), psi = I_i rt_i, rt = rho - 0.09, I_i
 *            the HCT descreening sum over j of the integral of r^-4/(4 pi)
 *            over the ball of radius S_j rt_j outside radius rt_i;
 *   E_SA   = sum_i 4 pi sa_gamma (rho_i + probe)^2 (rho_i / R_i)^6;
 * k_e = 1389.3546 kJ/mol A e^-2; and, unless NULL, dev_forces (device,
 * n_conf x n_atoms x 3 floats) = -grad of their sum.  Float32 arithmetic,
 * energies summed in double. */
BPMF_API int bpmf_pair_evaluate(bpmf_ctx* ctx, int ligand_id,
                                const float* dev_x, int64_t n_conf,
                                double* dev_terms, float* dev_forces);

/* Put the ligand's pair terms (bpmf_pair_setup) into its sampled energy
 * (on != 0) or take them out (on = 0): the Full pathway's ligand energy
 * with its intramolecular nonbonded and implicit-solvent terms
 * (Thermodynamic Cycle).  While on, U_k(x) of the sweeps (HMC moves,
 * exchange, recorded components), of bpmf_energy_matrix(_batch) and of the
 * external and pose moves (rigid moves: the terms do not change) includes
 * E_LJ + E_Coul + E_GB + E_SA, summed with the bonded terms in the first
 * cached component, and their force joins the HMC force; bpmf_evaluate
 * keeps evaluating the bonded, restraint and grid terms only.  The cached
 * components are recomputed, the stored start-of-trajectory forces
 * dropped and captured graphs recaptured.  Synchronises.  Errors:
 * BPMF_E_STATE (no pair parameters), BPMF_E_UNIMPL (the ligand's topology
 * and pair parameters exceed 64 KB of LDS per replica). */
BPMF_API int bpmf_pair_sample(bpmf_ctx* ctx, int ligand_id, int on);

/* ------------------------------------------------------------------------
 * Ligand information, state parameters, single-ligand sweeps
 * ------------------------------------------------------------------------ */

/* Sizes of a ligand (host outputs, any may be NULL). */
BPMF_API int bpmf_ligand_info(bpmf_ctx* ctx, int ligand_id, int* n_atoms,
                              int* n_states, int* n_channels,
                              int* sample_capacity);

/* Replace the K thermodynamic states of a ligand: T (K temperatures, > 0),
 * w (K x n_channels grid weights), dt_fs (K time steps, > 0), host arrays.
 * Replicas, cached energy components (which do not depend on the state),
 * statistics and samples are kept; captured sweep graphs stay valid.
 * Synchronises. */
BPMF_API int bpmf_set_states(bpmf_ctx* ctx, int ligand_id, const double* T,
                             const double* w, const double* dt_fs);

/* bpmf_hmc_sweep restricted to one ligand: only its replicas move, only its
 * counter, statistics and samples change. */
BPMF_API int bpmf_hmc_sweep_ligand(bpmf_ctx* ctx, int ligand_id,
                                   const bpmf_sweep_args* args);

/* ------------------------------------------------------------------------
 * Ladder initialisation (Initialization; state insertion and equilibration
 * detection from Equilibration and production)
 * ------------------------------------------------------------------------ */
#define BPMF_SCHEDULE_LINEAR 0 /* every channel weighted by alpha */
#define BPMF_SCHEDULE_SOFT 1   /* Thermodynamic Cycle: channels rep, att, ele
                                  weighted by alpha_g = (2a-1)^2 / (1 +
                                  exp(-1000 (a - 1/2))), soft rep and soft ele
                                  by alpha_sg = 1 - (2a-1)^2 */

/* Temperature T(alpha) = (T_cold - T_hot) alpha + T_hot and the n_channels
 * weights w of the state at alpha in [0, 1] (host outputs). */
BPMF_API int bpmf_protocol_state(double alpha, int kind, int n_channels,
                                 double T_hot, double T_cold, double* T,
                                 double* w);

/* Population standard deviations over n samples with cached components
 * comps (host, n x (1 + n_channels): U0, Psi_c) in the state at alpha:
 * sigma[0] of Psi_g (the original grids' channels summed), sigma[1] of
 * Psi_sg (the soft grids'; 0 for the linear schedule), sigma[2] of the
 * reduced energy u = (U0 + sum_c w_c Psi_c) / (R T). */
BPMF_API int bpmf_protocol_sigmas(const double* comps, int64_t n,
                                  int n_channels, double alpha, int kind,
                                  double T_hot, double T_cold, double* sigma);

/* Parameter selection (Initialization, thermodynamic length): the next
 * alpha = alpha + speed / [ |d alpha_sg / d alpha| sigma[1] / (R T) +
 * |d alpha_g / d alpha| sigma[0] / (R T) + |T_cold - T_hot| sigma[2] / T ]
 * (the linear schedule: d alpha_g / d alpha = 1, no soft term), never past
 * 1; 1 when the bracket is 0.  The paper's speed is 0.2. */
BPMF_API int bpmf_protocol_next_alpha(double alpha, const double* sigma,
                                      int kind, double speed, double T_hot,
                                      double T_cold, double* next);

/* Temperature-only path: T moves towards T_target by speed R T^2 /
 * sigma_U and stops there (the paper's speed is 20). */
BPMF_API int bpmf_protocol_next_temperature(double T, double sigma_U,
                                            double speed, double T_target,
                                            double* next);

/* Seed selection by sampling importance resampling: n_draw indices into n
 * samples (host idx), drawn with replacement with probability proportional
 * to exp(log_w) (non-finite log_w: weight 0).  Draw j inverts the
 * cumulative weights (summed in index order after subtracting the largest
 * log_w) at u_j times the total, u_j the Philox uniform (index j, ligand
 * ligand_id, replica 0, counter `state`, purpose 7). */
BPMF_API int bpmf_protocol_sir(const double* log_w, int64_t n, int n_draw,
                               uint64_t seed, int ligand_id, int state,
                               int64_t* idx);

/* Time-step rule: acceptance above 0.8: dt + 0.125 fs; below 0.1: dt -
 * 0.5 fs; below 0.4: dt - 0.25 fs (never below dt_min); *done = 1 when the
 * acceptance lies in [0.4, 0.8] or dt is already at dt_min. */
BPMF_API int bpmf_protocol_adapt_dt(double dt, double acc, double dt_min,
                                    double* new_dt, int* done);

/* Mean over n pairs of min(1, exp(-[u_k(y) + u_k+1(x) - u_k(x) -
 * u_k+1(y)])) (Eq. repXacc; a non-finite exponent counts 0), host arrays
 * of the four reduced energies per pair. */
BPMF_API int bpmf_protocol_mean_pacc(const double* uk_x, const double* uk1_x,
                                     const double* uk_y, const double* uk1_y,
                                     int64_t n, double* mean);

/* State insertion between cycles: out (host, up to max_out) is the ladder
 * alpha (K states) with a state at the midpoint of every neighbour pair
 * whose exchange acceptance pacc[k] (K - 1 values) is below threshold (the
 * paper: 0.4). */
BPMF_API int bpmf_protocol_insert(const double* alpha, int K,
                                  const double* pacc, double threshold,
                                  int max_out, double* out, int* K_out);

/* Equilibration detection (Chodera 2016): among the n_candidates starts
 * t0 = floor(i n / n_candidates) the one that maximises the number of
 * uncorrelated samples (n - t0) / g(a[t0:]) (ties: the earlier), g = 1 + 2
 * sum_t (1 - t/N) C_t / C_0 stopped at the first C_t <= 0. */
BPMF_API int bpmf_detect_equilibration(const double* a, int64_t n,
                                       int n_candidates, int64_t* t0,
                                       double* g, double* n_eff);

/* Random placements (Initialization: configurations put at random
 * centre-of-mass positions in the binding site with random orientations):
 * poses [first, first + count) of n_conf configurations dev_confs (device,
 * n_conf x n_atoms x 3) at n_com site positions x n_orient orientations,
 * pose (c * n_com + i) * n_orient + o, written to dev_out (device, count x
 * n_atoms x 3; count x n_atoms < 2^32).  Position i: the ligand's site
 * centre + d0 u^(1/3) (sin t cos p, sin t sin p, cos t), cos t = 2u - 1,
 * p = 2 pi u (Philox index i, purpose 7 | 1<<8); orientation o: the
 * rotation of the uniform unit quaternion of three uniforms (index o,
 * purpose 7 | 2<<8), applied about the configuration's mass-weighted
 * centre. */
BPMF_API int bpmf_place_poses(bpmf_ctx* ctx, int ligand_id,
                              const float* dev_confs, int n_conf, int n_com,
                              int n_orient, int64_t first, int64_t count,
                              float* dev_out);

typedef struct {
  int ligand_id;      /* ligand whose K replicas run the seeds of each state
                         (K seeds per state); its states, replicas and
                         samples are overwritten */
  int kind;           /* BPMF_SCHEDULE_LINEAR or BPMF_SCHEDULE_SOFT */
  double T_hot;       /* T at alpha = 0 (K) */
  double T_cold;      /* T at alpha = 1 (K) */
  double speed;       /* thermodynamic speed s (the paper: 0.2) */
  int n_trials;       /* HMC trials per seed and run, <= sample capacity */
  int n_leapfrog;     /* velocity-Verlet steps per trial */
  double dt_start;    /* time step of state 0 (fs) */
  double dt_min;      /* floor of the adapted time step (fs) */
  int max_dt_rounds;  /* runs per selection at most while adapting dt */
  int max_selections; /* selections per state at most (speed x 4/5 between) */
  int n_conf, n_com, n_orient; /* n_com > 0: state 0's sample set is the
                         placements (bpmf_place_poses) of the final
                         configurations of its first n_conf (<= K) replicas
                         at n_com positions x n_orient orientations (the
                         paper: 50 x 453 x 100); 0: its own samples */
  int max_states;     /* capacity of the result arrays, >= 2 */
} bpmf_init_args;

#define BPMF_TRACE_FIELDS 10
typedef struct {
  /* outputs */
  int n_states;       /* states in the ladder */
  int reached_target; /* 1 when the last state has alpha = 1 */
  int n_selections;   /* selections made, repeats included */
  int n_runs;         /* sampling runs made, time-step repeats included */
  int n_removed;      /* states dropped for p_acc above 0.99 */
  int n_trace;        /* trace records written */
  /* host arrays, sized by max_states */
  double* alpha;
  double* T;
  double* w;          /* max_states x n_channels */
  double* dt;         /* time step of the state's last run (fs) */
  double* acc;        /* HMC acceptance of that run */
  double* pacc;       /* verified mean exchange acceptance with the state it
                         was selected from (1 for state 0) */
  double* sigma;      /* may be NULL; max_states x 3 (bpmf_protocol_sigmas
                         of the state's sample set) */
  float* x;           /* may be NULL; max_states x K x n_atoms x 3 final
                         configurations of the state's last run */
  double* trace;      /* may be NULL; trace_cap x BPMF_TRACE_FIELDS, one
                         record per selection: alpha_from, its sigma[0..2],
                         speed, alpha_new, dt, acceptance, p_acc, outcome (0
                         appended, 1 repeated with speed x 4/5, 2 replaced
                         the state it came from) */
  int trace_cap;
} bpmf_init_result;

/* Initialise a ladder of states from alpha = 0 (T_hot, grids off) to alpha
 * = 1 (T_cold, grids on) (Initialization).  State 0 runs from the ligand's
 * current replicas.  Then, until alpha = 1 or max_states: the next alpha
 * by bpmf_protocol_next_alpha from the last state's sample set; K seeds by
 * bpmf_protocol_sir with weights exp[u_k - u_new] (counter = the new
 * state's index); K runs of n_trials HMC trials from the seeds, repeated
 * with the time step changed by bpmf_protocol_adapt_dt until it is done or
 * max_dt_rounds runs were made (the first run starts from the previous
 * state's time step); p_acc by bpmf_protocol_mean_pacc over pairs spread
 * evenly over both sample sets (sample i with sample i when the sets are
 * equal in size).  p_acc below 0.4: select again with speed x 4/5 (at most
 * max_selections times); above 0.99: the new state replaces the previous
 * one unless that is state 0.  A state's sample set is its last run's
 * recorded samples (n_trials x K).  Synchronises; leaves the ligand's
 * replicas, states and samples at the last state's last run. */
BPMF_API int bpmf_initialize_ladder(bpmf_ctx* ctx, const bpmf_init_args* args,
                                    bpmf_init_result* result);

/* ------------------------------------------------------------------------
 * Launch shape
 * ------------------------------------------------------------------------ */

/* Wavefronts per replica in the HMC sweep (and in bpmf_evaluate): 1, 2, 4
 * or 8, or 0 for the automatic choice (per ligand the smallest power of two,
 * at most 8, that gives every bonded term a thread -- each kind of term
 * starting on a wavefront boundary, and from four wavefronts on only the
 * wavefronts without atoms taking terms -- halved while replicas x
 * wavefronts over all ligands exceed 4096).  Never fewer than
 * ceil(n_atoms / 64).  Results depend on it only through the rounding of
 * the per-wavefront energy partial sums. */
BPMF_API int bpmf_set_waves(bpmf_ctx* ctx, int waves);

/* bpmf_hmc_sweep replays a hipGraph of `chunk` captured sweeps (default 64;
 * 0 = plain launches).  The graph is captured on a private stream once per
 * (sweep arguments, ligand set) and launched on the context's stream; the
 * kernels read every per-sweep quantity from device memory, so replays are
 * identical to plain launches.  Units closed by moves are captured
 * max(1, chunk / P) to a graph.  With timing enabled a graph launch is timed
 * as a whole and counts as the sweeps it holds. */
BPMF_API int bpmf_set_graph(bpmf_ctx* ctx, int chunk);

/* Autotuner: time `n_sweeps` sweeps of n_leapfrog steps for each launch
 * shape -- wavefronts per replica chosen automatically, or forced to 1, 2,
 * 4, 8 (raised per ligand to the minimum its atom count needs, as in
 * bpmf_set_waves) -- on the ligands set up, with HIP events (eager launches
 * below the graph chunk, graph replays from it on); keep the fastest and
 * report it in *chosen (0 = automatic).  ms_out (host, 5 doubles, may be
 * NULL) receives the mean sweep time of each candidate in that order.
 * Then, one atom-count class at a time (up to 16, 32, 48, 64, 96 and 128
 * atoms, largest first), the other wavefront counts are tried for that
 * class's ligands alone and kept (as per-ligand choices, see
 * bpmf_set_ligand_waves) where they save more than 2 % of the sweep; the
 * classes' launches run side by side.  bpmf_get_waves reports each
 * ligand's result.  The shapes are timed with workgroup order 1; with
 * several ligands order 0 is timed last and kept if it saves more than
 * 2 % (bpmf_get_task_order reports the result).  The sampler state
 * (positions, state maps, components,
 * counters, statistics) is snapshotted on the device before the trials and
 * restored after, so tuning does not change the run.  Per-ligand choices
 * made before the call are replaced. */
BPMF_API int bpmf_autotune(bpmf_ctx* ctx, int n_sweeps, int n_leapfrog,
                           double* ms_out, int* chosen);

/* A ligand's own wavefronts per replica (1, 2, 4 or 8, raised to the
 * minimum its atom count needs; 0 = none: the bpmf_set_waves choice
 * applies).  Results depend on it only through the rounding of the
 * per-wavefront energy partial sums.  Errors: BPMF_E_INVAL. */
BPMF_API int bpmf_set_ligand_waves(bpmf_ctx* ctx, int ligand_id, int waves);

/* Order of the sweep's workgroups within each wavefront class: 1 (the
 * default) the replicas of the ligands with the most work per sweep
 * (bonded terms and atoms) first, so that the longest workgroups start
 * earliest; 0 ligand by ligand, replicas in order.  A single ligand's
 * replicas keep their order either way.  Results do not depend on it.
 * Errors: BPMF_E_INVAL (order not 0 or 1; null order). */
BPMF_API int bpmf_set_task_order(bpmf_ctx* ctx, int order);
BPMF_API int bpmf_get_task_order(bpmf_ctx* ctx, int* order);

/* Wavefronts per replica the sweep currently uses for a ligand. */
BPMF_API int bpmf_get_waves(bpmf_ctx* ctx, int ligand_id, int* waves);

/* ------------------------------------------------------------------------
 * Kernel timing (HIP events on the context's stream)
 * ------------------------------------------------------------------------ */
enum {
  BPMF_TIMER_HMC = 0,
  BPMF_TIMER_COMPONENTS = 1,
  BPMF_TIMER_TAIL = 2,
  BPMF_TIMER_GRID_EVAL = 3
};

/* While enabled, every `every`-th launch of each timed kernel (HMC: the
 * kernels of one sweep, which with scheme 0 also apply the previous sweep's
 * exchange and record, with scheme 1 followed by the tail kernel; TAIL: the
 * kernel that closes a scheme-0 call; COMPONENTS: the launches of one
 * energy-matrix call, which run side by side, as one interval; GRID_EVAL:
 * the kernel of bpmf_grid_eval) is bracketed by a
 * pair of HIP events recorded on the context's stream (at most 8192 pairs
 * per kernel between reads).  Enabling clears earlier records. */
BPMF_API int bpmf_set_timing(bpmf_ctx* ctx, int enable, int every);

/* Mean duration in ms of the bracketed launches of `kernel` since timing
 * was enabled or last read, and their number; clears the records.
 * Synchronises. */
BPMF_API int bpmf_get_timing(bpmf_ctx* ctx, int kernel, double* mean_ms,
                             int64_t* n_timed);

#ifdef __cplusplus
}
#endif
#endif /* BPMF_H */
