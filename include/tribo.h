/*
 * tribo.h -- C ABI of the MI355X particle-step library (libtribo.so).
 *
 * One call of tf_step advances the Lagrangian particle phase of a wall-bounded
 * periodic channel, driven by a frozen carrier velocity field, by whole time
 * steps.  Per step and per ensemble (Wilms & Grosshans, Sec. 2.2-2.3):
 *   1. particles are binned by grid cell (cell = control volume, Sec. 2.2)
 *      and sorted by (cell, particle id);
 *   2. cell charge = sum of the particle charges in the cell (Sec. 2.2),
 *      accumulated exactly in fixed point (q * 2^48, round-to-nearest-even);
 *   3. the Poisson equation lap(phi) = -rho_el/eps (Sec. 2.2, eps = 1 in
 *      these units) is solved with grounded walls phi = 0 (Sec. 4.2) and
 *      periodic x, z (Sec. 3.1) on the second-order finite-volume grid
 *      (Sec. 3.1): Fourier transforms in x and z, one tridiagonal solve per
 *      Fourier mode in y;
 *   4. per particle: trilinear carrier velocity, cell-centred E = -grad(phi)
 *      (Gauss part, Eq. (2.9)) plus Coulomb's law, Eq. (2.8), between
 *      particles of the same cell (hybrid scheme, Sec. 2.2), Schiller-Naumann
 *      drag, Eq. (2.6)-(2.7), gravity/buoyancy, semi-implicit Euler for the
 *      equation of motion, Eq. (2.5);
 *   5. wall impact: hard-sphere rebound (Sec. 2.2) with restitution e and
 *      condenser-model charge transfer (Sec. 2.3.1, Eq. (2.13)-(2.19)) in
 *      the lumped normalised form dq = -f (dU + q), f = k_c (1+e)^(2/5) u_n^(4/5);
 *   6. periodic wrap, grid-cell histograms of concentration and charge
 *      (Sec. 4.1), impact counts, wall charge and impact-velocity histogram.
 *
 * Units: wall units (nu = u_tau = 1), half channel height h = Re_tau, charge in
 * units of q_sat.  All floating-point state is IEEE binary64.
 *
 * Memory and ownership.  Every device pointer passed in is owned by the
 * caller and must stay valid for the lifetime of the handle; the library
 * never allocates device memory.  All scratch (sorted particle buffers, cell
 * tables, spectra, statistics, recorded trajectories) lives in the caller's
 * workspace of tf_workspace_size() bytes.  The host-side handle is allocated
 * by tf_init and released by tf_destroy.
 *
 * Streams.  All device work of a handle is enqueued on the stream given to
 * tf_init, asynchronously.  tf_stats synchronises that stream before
 * returning host data; tf_init and tf_set_params synchronise it too.
 *
 * Errors.  Every int-returning call returns TF_OK (0) or a negative TF_E*
 * code; tf_last_error() describes the most recent failure of the calling
 * thread.  No C++ exception crosses the ABI.  Faults detected on the device
 * (non-finite state, fixed-point overflow, a particle outside the channel
 * after a rebound) are sticky per-ensemble flags reported by tf_stats.
 */
#ifndef TRIBO_H
#define TRIBO_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct tf_handle tf_handle;

/* return codes */
#define TF_OK 0
#define TF_EINVAL (-1)     /* invalid argument or configuration */
#define TF_ESIZE (-2)      /* workspace too small / size limit exceeded */
#define TF_EHIP (-3)       /* HIP runtime error */
#define TF_ESTATE (-4)     /* call not valid in the handle's current state */
#define TF_EOVERFLOW (-5)  /* fixed-point or counter overflow */

/* tf_init flags */
#define TF_INIT_KEEP_DEPOSIT 1u   /* also store each step's per-cell fixed-point charge */
#define TF_INIT_GRAPHS 2u         /* replay steps from captured HIP graphs */
#define TF_INIT_SOURCE 4u         /* also compute each step's 2-way coupling source (TF_FIELD_SOURCE) */

/* tf_step flags */
#define TF_STEP_RECORD 1u         /* record the steps for tf_adjoint_step (needs trajectory capacity) */

/* sticky device flags (tf_stats_out.flags); a step that raises one still runs
 * to completion on every particle:
 *   TF_FLAG_NONFINITE  a particle's new position, velocity or charge is not finite
 *   TF_FLAG_OVERFLOW   a fixed-point conversion (deposit q 2^48, charge profile
 *                      q 2^32, wall charge -dq 2^40) rounds to a magnitude of
 *                      2^62 or more, or is not finite; that entry contributes 0
 *   TF_FLAG_OUTSIDE    a particle is still outside [d/2, ly - d/2] in y after
 *                      its wall rebound (a penetration deeper than the channel) */
#define TF_FLAG_NONFINITE 1
#define TF_FLAG_OVERFLOW 2
#define TF_FLAG_OUTSIDE 4

/* fixed-point scales (powers of two) */
#define TF_FIX_DEPOSIT 48   /* cell charge and q_now: sum rne(q * 2^48) */
#define TF_FIX_WALL 40      /* wall charge: sum rne(-dq * 2^40) */
#define TF_FIX_QCUM 32      /* time-summed charge profile: sum rne(q * 2^32) */
#define TF_NBIN 64          /* impact-velocity histogram bins */

/*
 * One independent ensemble (channel + particles).
 *   nx, nz      cells in the periodic directions: even, of the form 2^a 3^b 5^c, 4..256
 *   ny          cells between the walls, 2..1024
 *   lx, lz      periodic lengths; cells are uniform, dx = lx/nx, dz = lz/nz
 *   y_faces     host array of ny+1 strictly increasing wall-normal faces,
 *               y_faces[0] = 0 (lower wall), y_faces[ny] = ly (upper wall);
 *               copied at tf_init
 *   dt          time step; density_ratio = rho_p/rho (> 1)
 *   k_c, delta_u, e   charge-transfer coefficient, normalised contact
 *               potential difference, restitution coefficient (0 < e <= 1)
 *   c_el        electric coupling: specific electric force = c_el q E / d^3
 *   g           gravitational acceleration vector (buoyancy applied inside)
 *   un_bin      bin width of the wall-normal impact-velocity histogram
 *   u_nodes     device pointer, carrier velocity at the mesh nodes,
 *               layout [3][ny+1][nz][nx] (component, y face, z, x), node
 *               (i, j, k) at (i dx, y_faces[j], k dz); borrowed (read by
 *               every step) until tf_set_carrier replaces it
 *   n_particles 0..2^30 (an empty ensemble still solves the field of zero
 *               charge and counts its steps)
 *   pp, k_pp    4-way coupling (pp = 1; 0 = off): binary hard-sphere
 *               collisions between particles sharing a grid cell (Sec. 2.2),
 *               resolved together on the state at the start of each step
 *               when a pair overlaps and approaches; fully elastic, masses
 *               ~ d^3; condenser charge exchange (Sec. 2.3.1)
 *               dq_i = -dq_j = (d_i q_j - d_j q_i)/(d_i + d_j) (1 - exp(-x)),
 *               x = k_pp (d_i d_j)^2 (d_i + d_j)^(-3/5) (d_i^3 + d_j^3)^(-4/5)
 *               |u_i - u_j|^(3/5) (the Hertz contact area and time with the
 *               material constants folded into k_pp >= 0).  The drag update
 *               and wall charging start from the changed velocity and charge;
 *               the step's electric forces use the deposited charges.  Not
 *               differentiated: TF_STEP_RECORD is refused while pp is on.
 *   charging    wall charging: 0 = condenser model (k_c, delta_u), 1 = the
 *               stochastic scaling model (Sec. 2.3.2): an impact gives the
 *               particle dq = mu_w - Dq_1, mu_w = ssm_dq0min N_w/N_w0 (the
 *               wall's sites, mean), Dq_1 a skew-normal number with mean
 *               (ssm_dq0min - ssm_mu0) N_i/N_0, standard deviation
 *               ssm_sigma0 sqrt(N_i/N_0), skewness -ssm_gamma0 N_0/N_i
 *               (limited to +-0.99); N_w/N_w0 = A/A_0 chi_w, N_i/N_0 = A/A_0
 *               chi_i, A/A_0 = (d/ssm_d0)^2 (u_n/ssm_un0)^(4/5),
 *               chi_w = 1 - sgn(ssm_dq0min) 4q/(ssm_csat d^2),
 *               chi_i = 1 + sgn(ssm_dq0min - ssm_mu0) 4q/(ssm_csat d^2), both
 *               clipped to [0, 1].  Random numbers: Philox4x32-10 at counter
 *               (particle id, step number since tf_init, 0, 0), key (seed,
 *               0x53534D31), Box-Muller on the first two words.  With
 *               ssm_sigma0 = ssm_gamma0 = 0 and ssm_mu0 = ssm_dq0min the model
 *               is deterministic.  Not differentiated (TF_STEP_RECORD refused).
 */
typedef struct {
  int32_t nx, ny, nz, n_particles;
  double lx, lz;
  const double* y_faces;
  double dt, density_ratio, k_c, delta_u, e, c_el;
  double g[3];
  double un_bin;
  const double* u_nodes;
  double k_pp;
  int32_t pp;
  int32_t charging;           /* wall charging model: 0 condenser, 1 SSM */
  uint32_t seed, reserved;    /* SSM random numbers */
  double ssm_dq0min, ssm_mu0, ssm_sigma0, ssm_gamma0, ssm_csat, ssm_d0, ssm_un0;
} tf_ensemble;

/* Particle arrays (device pointers, n_particles doubles each, indexed by
 * particle id).  d is the diameter (constant in time). */
typedef struct {
  double *x, *y, *z, *vx, *vy, *vz, *q, *d;
} tf_particles;

typedef struct {
  int64_t steps;              /* steps taken since tf_init */
  int32_t flags;              /* sticky TF_FLAG_* */
  int32_t ny;
  int64_t impacts[2];         /* wall impacts [lower, upper] */
  int64_t wall_q[2];          /* charge received by each wall, sum rne(-dq 2^40) */
  int64_t un_hist[TF_NBIN];   /* impacts per bin of u_n / un_bin (last bin open) */
  int64_t* crel_y;            /* optional host [ny]: time-summed particle count per y cell */
  int64_t* qcum_y;            /* optional host [ny]: time-summed sum rne(q 2^32) per y cell */
  int64_t* qnow_y;            /* optional host [ny]: sum rne(q 2^48) per y cell at the latest deposit */
  double q_sum;               /* total particle charge at the latest deposit */
  int64_t pp_pairs;           /* colliding particle pairs (4-way coupling) since tf_init */
} tf_stats_out;

/* Bytes of device workspace for these ensembles.  traj_steps > 0 reserves
 * room to record that many steps for tf_adjoint_step.  Returns 0 if the
 * configuration is invalid. */
size_t tf_workspace_size(const tf_ensemble* ens, int32_t n_ens, int32_t traj_steps);

/* Validate the configuration, carve the workspace, copy the initial
 * particles (one tf_particles per ensemble, read on the stream), bin them.
 * stream is a hipStream_t (NULL = default stream). */
int tf_init(const tf_ensemble* ens, int32_t n_ens, const tf_particles* init,
            void* workspace, size_t workspace_bytes, int32_t traj_steps,
            void* stream, uint32_t flags, tf_handle** out);

/* Advance every ensemble by n_steps >= 0 steps.  With TF_STEP_RECORD the
 * steps are appended to the recorded trajectory (at most traj_steps since the
 * last tf_adjoint_step or tf_set_state); a handle without any particles
 * records nothing (its derivatives are zero), so tf_adjoint_step then
 * returns TF_ESTATE. */
int tf_step(tf_handle* h, int32_t n_steps, uint32_t flags);

/* Copy the statistics of ensemble `ens` to the host (synchronises). */
int tf_stats(tf_handle* h, int32_t ens, tf_stats_out* out);

/* Copy the current particle state of ensemble `ens` into `out` (device
 * arrays, id order), or replace it from `in`.  Asynchronous on the stream.
 * tf_set_state also clears the recorded trajectory. */
int tf_get_state(tf_handle* h, int32_t ens, const tf_particles* out);
int tf_set_state(tf_handle* h, int32_t ens, const tf_particles* in);

/* Make ensemble `ens` read its carrier velocity from u_nodes (same layout
 * as tf_ensemble.u_nodes, device memory, borrowed) from the next step on: a
 * time-dependent carrier field.  Asynchronous, in stream order (steps queued
 * before the call read the previous field, which must stay valid until they
 * have run); captured step graphs stay valid.  Errors: TF_EINVAL (NULL,
 * ensemble out of range), TF_ESTATE (a recorded trajectory is pending), TF_EHIP. */
int tf_set_carrier(tf_handle* h, int32_t ens, const double* u_nodes);

/* Replace (k_c, delta_u, e) of every ensemble: host array [n_ens][3], each
 * finite with 0 < e <= 1 (else TF_EINVAL, nothing changed).  Steps queued
 * before the call use the old values.  TF_ESTATE while a recorded trajectory
 * is pending: its reverse step needs the parameters it was recorded with. */
int tf_set_params(tf_handle* h, const double* theta);

/*
 * Reverse-mode derivative of the recorded steps with the discrete events
 * (cell of each particle, wall impacts, periodic wraps) held fixed.
 *   lambda   device arrays, id order, one tf_particles per ensemble: on entry
 *            dJ/d(state) at the end of the recorded steps, on return dJ/d(state)
 *            at their start (the d member is ignored)
 *   w_wall   device [n_ens][2]: dJ/d(charge received by the lower/upper wall)
 *            over the recorded steps (the wall accumulators never feed back);
 *            read on the stream
 *   dtheta   device [n_ens][3]: dJ/d(k_c, delta_u, e) is ADDED to it on the stream
 * Asynchronous on the handle's stream: the caller's buffers must stay valid
 * until the queued work has run.  Consumes the recorded trajectory (a later
 * tf_step may record again).  The fixed-point deposit is treated as the
 * identity (its derivative is zero almost everywhere).  Errors: TF_EINVAL
 * (NULL pointer), TF_ESTATE (nothing recorded), TF_EHIP.
 */
int tf_adjoint_step(tf_handle* h, const tf_particles* lambda, const double* w_wall, double* dtheta);

/* Solve the Poisson problem of ensemble `ens` for a given per-cell
 * fixed-point charge q_fixed (device int64 [ncell], scale 2^48, cell index
 * (j*nz + k)*nx + i) into phi (device double [ncell]).  Uses the handle's
 * scratch; asynchronous on the stream. */
int tf_poisson(tf_handle* h, int32_t ens, const int64_t* q_fixed, double* phi);

/*
 * Allocation-free variant of tf_poisson, for callers that cannot allocate
 * device memory or that must make no allocating call (code under HIP graph
 * capture, tight serving loops, harnesses that forbid allocation).  Same
 * arguments, result and stream semantics as tf_poisson; the spectrum scratch
 * is a static device array of TF_NOALLOC_MAX_SPECTRUM_BYTES held by the
 * library on each GPU it runs on until the process ends (its address is taken
 * at tf_init).  The call allocates nothing, host or device.
 *   Limit: 16 ny nz nhp bytes of spectrum, nhp = nx/2 + 1 rounded up to a
 *   multiple of 8; larger ensembles give TF_ESIZE.
 *   Concurrency: every call on one GPU shares that GPU's scratch, which keeps
 *   the last call's contents (the result depends only on entries the call
 *   writes first, so no clearing is needed); calls whose queued work overlaps
 *   on one GPU (several streams or handles at once) race.
 * Errors: TF_EINVAL (NULL pointer, ensemble out of range), TF_ESIZE, TF_EHIP.
 */
#define TF_NOALLOC_MAX_SPECTRUM_BYTES (64u << 20)
int tf_poisson_noalloc(tf_handle* h, int32_t ens, const int64_t* q_fixed, double* phi);

/* Copy a field of the latest step of ensemble `ens` to device memory `out`:
 * TF_FIELD_PHI (double [ncell]); with TF_INIT_KEEP_DEPOSIT, TF_FIELD_DEPOSIT
 * (int64 [ncell]); with TF_INIT_SOURCE, TF_FIELD_SOURCE (double [3][ncell],
 * component-major): the momentum source F_s of the carrier equation
 * (Sec. 2.1, 2-way coupling), minus the aerodynamic forces on the particles
 * of each cell (cell of x^n) per unit cell volume, the force on a particle
 * being the step's implicit drag m_p (phi_D / tau_p)(u - v^{n+1}),
 * m_p = rho_r pi d^3 / 6, fluid density 1.  Asynchronous on the stream. */
#define TF_FIELD_PHI 0
#define TF_FIELD_DEPOSIT 1
#define TF_FIELD_SOURCE 2
int tf_field(tf_handle* h, int32_t ens, int32_t which, void* out);

/*
 * Per-phase timing with HIP events on the handle's stream.  After
 * tf_profile_begin, the next max_steps steps are launched eagerly with events
 * at the boundaries of the phases in phase_mask (bit p = phase p; 0 = all);
 * tf_profile_end synchronises and returns the summed milliseconds of each
 * bracketed phase over the profiled steps (0 for the others).  Every event
 * costs a few microseconds of the step.  Phases:
 *   0 sort: the row-count prefix sum (after init or tf_set_state: the full
 *     counting sort)
 *   1 deposit + forward FFT along x (the incremental sort runs fused here)
 *   2 forward FFT along z
 *   3 tridiagonal y-solves              4 inverse FFT along z
 *   5 inverse FFT along x               6 particle push
 */
#define TF_NPHASE 7
int tf_profile_begin(tf_handle* h, int32_t max_steps, uint32_t phase_mask);
/* The same with events on every `every`-th step only (the first, the
 * (every+1)-th, ...) until max_steps steps carry them; every >= 1.  The steps
 * in between run eagerly without events: fewer events in a timed stretch. */
int tf_profile_begin_every(tf_handle* h, int32_t max_steps, uint32_t phase_mask, int32_t every);
int tf_profile_end(tf_handle* h, double* phase_ms /* [TF_NPHASE] */, int32_t* n_steps);

/*
 * Tile shapes of the sort and Poisson kernels, used by every later tf_init /
 * tf_workspace_size of the calling process (0 = built-in choice):
 *   sort_cap   members held in LDS by the fused sort's list (a row pair with
 *              more is listed one row at a time when each row fits, else it
 *              takes a second pass through global memory); 0 = twice the
 *              mean pair rounded up to 64, -1 = none (always two passes),
 *              else 1..4096 (clamped to what fits 64 KiB of LDS per block)
 *   fz_cols    spectral columns per block of the z transforms (1..64, and
 *              fz_cols nz <= 2048)
 *   tri_modes  Fourier modes per block of the tridiagonal solves: 4, 8, 16
 *              or 32 (the block's 256 threads split evenly among them; a
 *              mode's lanes must cover ny with at most 16 rows each)
 *   inv_plane  inverse z and x transforms: 1 = one block per y plane (the
 *              plane's half spectrum in LDS), 2 = two blocks per y plane (even
 *              and odd z rows; needs nz % 4 == 0), 4 = four blocks per y plane
 *              (z rows by residue mod 4; needs nz % 8 == 0), 3 = a z kernel
 *              then an x kernel through global memory; 0 = 2 when it fits and
 *              2 ny does not exceed the GPU's CU count, else 1 when the plane
 *              fits a block, else 4 when a quarter plane does, else 3
 *   push_order order of the push's blocks over the GPU's XCDs (each with its
 *              own L2): 1 = consecutive slot ranges per XCD (an XCD's L2
 *              keeps the carrier and phi rows that neighbouring cells share),
 *              2 = the hardware's round robin (every XCD on neighbouring
 *              slots: shared rows come from the memory-side cache, work near
 *              the walls and in the middle of the channel spread evenly);
 *              0 = 1 for a handle of one mesh class, 2 for several
 * Values whose LDS need exceeds a block's LDS are rejected at tf_init.
 * Results do not depend on sort_cap, fz_cols or push_order (bitwise); tri_modes and
 * inv_plane set the association order of the tridiagonal scans or of the
 * inverse transforms, so they change results at the rounding level only.
 */
typedef struct {
  int32_t sort_cap, fz_cols, tri_modes, inv_plane, push_order;
} tf_tuning;
int tf_set_tuning(const tf_tuning* t);

/* Tile shapes for the ensembles of one mesh-size class (nx, ny, nz); they take
 * precedence over tf_set_tuning for those ensembles (t == NULL removes the
 * entry).  Ensembles of different classes in one handle keep their own tiles
 * within the same launches.  The sort's member capacity and the push's block
 * order are one per handle: the class's sort_cap (>= 0 here, 0 = no choice)
 * and push_order apply when every ensemble of the handle has that mesh and
 * tf_set_tuning set none; a handle with several mesh classes takes the
 * built-in rules. */
int tf_set_tuning_class(int32_t nx, int32_t ny, int32_t nz, const tf_tuning* t);

void tf_destroy(tf_handle* h);
const char* tf_error_string(int code);
const char* tf_last_error(void);

#ifdef __cplusplus
}
#endif
#endif /* TRIBO_H */
