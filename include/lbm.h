/*
 * lbm.h -- C ABI of the MI355X (gfx950) lattice Boltzmann library for the
 * thermodynamically consistent, conservative Allen-Cahn / Navier-Stokes
 * surfactant model with solid adsorption (Huang, Chai, Liu, Huang).
 *
 * One time step advances three coupled D2Q9 populations in lattice units
 * (dx = dt = 1, c_s^2 = 1/3):
 *   f  hydrodynamics, pressure-based equilibrium      (Sec. 3, f_eq of lattice 1)
 *   g  phase field phi, conservative Allen-Cahn with the weighted nonlinear
 *      Lagrange multiplier lambda_phi h_phi'(phi)     (Sec. 2.1, eq15 and AC_phi)
 *   h  surfactant psi, linear constraint mubar_psi    (Sec. 2.1, AC_psi)
 * with the chemical potentials (eq_muphi, eq_mupsi), the potential-form
 * surface-tension / Marangoni force F = -phi grad mu_phi - psi grad mu_psi + G
 * (eq_Fs0), the isotropic gradient and Laplacian stencils and backward time
 * differences (end of Sec. 3), the wetting and solid-adsorption natural
 * boundary conditions (Sec. 2.1, eq "boundary", wall energy eq8) and the two
 * global FP64 reductions that set the multipliers every step.
 *
 * Conventions for every entry point:
 *  - Return value: LBM_OK (0) or a negative lbm_status.  lbm_last_error()
 *    gives a message owned by the handle, valid until the next call on it.
 *  - Host pointers are caller-owned; the library reads or writes exactly the
 *    stated number of elements and keeps no reference after returning.
 *  - Fields crossing the boundary are FP64, row-major [ny][nx], x fastest,
 *    whatever the storage precision; node (x, y) sits at position (x, y), the
 *    bottom wall at y = -1/2 and the top wall at y = ny - 1/2.
 *  - Calls on one handle are ordered on its HIP stream.  One handle must not
 *    be used from two host threads at once.
 */
#ifndef LBM_H
#define LBM_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define LBM_ABI_VERSION 4

typedef struct lbm_handle lbm_handle; /* opaque, owned by the library */

typedef enum {
  LBM_OK = 0,
  LBM_E_ARG = -1,          /* invalid argument or parameter set */
  LBM_E_UNSUPPORTED = -2,  /* valid request this library does not implement */
  LBM_E_OOM = -3,          /* device or host allocation failed */
  LBM_E_DEVICE = -4,       /* no usable gfx950 device, or a HIP runtime error */
  LBM_E_NONFINITE = -5,    /* a non-finite value appeared in the fields */
  LBM_E_RANGE = -6,        /* psi left the open interval (0, 1) */
  LBM_E_STATE = -7         /* call not allowed in the handle's current state */
} lbm_status;

/* Boundary kinds for the bottom and top walls; x is always periodic.
 *  PERIODIC  periodic in y (both walls must then be PERIODIC)
 *  WALL_WET  half-way bounce-back no-slip wall (tangential speed u_wall_*)
 *            carrying the wetting and solid-adsorption conditions
 *  NOSLIP    half-way bounce-back no-slip wall (tangential speed u_wall_*),
 *            zero normal flux of phi and psi
 *  FREESLIP  specular reflection for f, zero normal flux of phi and psi */
enum { LBM_BC_PERIODIC = 0, LBM_BC_WALL_WET = 1, LBM_BC_NOSLIP = 2, LBM_BC_FREESLIP = 3 };
/* Storage precision of the populations.  Collisions run in FP64 (FP64) or
 * FP32 (FP32, FP16_SHIFTED); the multiplier sums are always FP64. */
enum { LBM_FP64 = 0, LBM_FP32 = 1, LBM_FP16_SHIFTED = 2 };
/* Constraint for phi: weighted nonlinear map h = 1/2 + g(phi) (AC_phi) or the
 * classical linear map h = phi. */
enum { LBM_CONSTRAINT_NONLINEAR = 0, LBM_CONSTRAINT_LINEAR = 1 };
/* Initial geometry: drop (liquid disc of radius R0 at (x0,y0)), slab (liquid
 * for |x - x0| < a/2), bubble (gas disc).  The profile is the equilibrium
 * phi_b tanh(2 phi_b sqrt(1 - psi_b) d / eps) of Sec. 2.2, d the signed
 * distance (minimum image in periodic directions), psi = psi_b, u = 0, p = 0. */
enum { LBM_INIT_DROP = 0, LBM_INIT_SLAB = 1, LBM_INIT_BUBBLE = 2 };

/* Model parameters in lattice units, named as in Sec. 2 and Sec. 3.
 * Entries marked "derive" take the stated default when set to the sentinel. */
typedef struct {
  int32_t abi_version;      /* must be LBM_ABI_VERSION */
  int32_t nx, ny;           /* grid, both >= 3 */
  int32_t bc_bottom, bc_top;
  int32_t precision;
  int32_t constraint_phi;
  int32_t init_kind;
  int32_t adv_raw;          /* 0 (default): phi and psi are advected by the mean (u(n) + u(n-1))/2 of the
                               velocity of this and the previous step; 1: by u(n) itself (literal
                               reading, excites the D2Q9 staggered-momentum mode on long runs) */
  int32_t tile_rows;        /* height of the 64-wide tiles of the fused step kernel: 0 chooses from the grid
                               size and precision (4 to 16 rows, up to 32 in FP64), a multiple of 4
                               up to 4096 forces it (a tuning knob: results differ only in the
                               summation order of the global multiplier sums) */
  int32_t phi_hold;         /* 0 (default): lambda_phi as eq15 gives it, S1/S2, which holds d/dt of
                               sum h_phi at zero in continuous time; the discrete step then lets sum h_phi
                               drift (about 1e-7 of it per step in a 64^2 drop).  1: lambda_phi also
                               returns sum h_phi to its value in the initial state (or the last
                               lbm_load_fields), adding (m0 - S4)/(M_phi S2), S4 = sum h_phi now */
  int32_t sat_cap;          /* Remark 1 (Sec. 2.1): 0 (default) the smooth Langmuir-Szyszkowski
                               tensions sigma_sa0 (1 + beta_sa ln(1 - psi)) the paper computes with;
                               1: each held at half its clean value or more, sigma_sa0 max(1/2,
                               1 + beta_sa ln(1 - psi)), in the wall energy and both wall fluxes (the
                               psi derivative is zero where the hold acts).  Other values: LBM_E_ARG */
  double sigma_gl0, eps;    /* clean gas-liquid tension, thickness: kappa = 3 eps sigma/8, beta = 3 sigma/(4 eps) */
  double M_phi, M_psi;      /* mobilities (>= 0) */
  double lambda_s;          /* psi gradient coefficient; < 0 derive: kappa/2 with a wetting wall, else 0 */
  double kBT, W;            /* <= 0 derive: kBT = 4 beta Pi, W = 4 beta / Ex */
  double Ex, Pi;            /* solubility and entropy groups (Sec. 4) */
  double psi_b;             /* bulk surfactant in [0,1); 0 switches the surfactant off */
  double phi_b;             /* <= 0 derive: phi_b^2 = 1 - W psi_b / (4 beta (1 - psi_b)) (Sec. 2.2) */
  double theta0_deg;        /* clean Young angle, (0,180) on a wetting wall */
  double sigma_sg0, sigma_sl0; /* < 0 derive: difference sigma cos theta0, sum 16 sigma / 15 */
  double beta_sg, beta_sl;  /* Langmuir-Szyszkowski elasticities (eq "langmuir") */
  double rho_l, rho_g, mu_l, mu_g; /* rho and dynamic viscosity linear in (1 + phi/phi_b)/2 */
  double gx, gy;            /* body acceleration, G = rho (gx, gy) */
  double u_wall_bottom, u_wall_top; /* tangential speed of no-slip walls */
  double eta_phi, eta_psi;  /* <= 0 derive: eta = D / (c_s^2 (1/s1 - 1/2)), D_phi = M_phi kappa, D_psi = M_psi lambda_s + M0 */
  double M0;                /* < 0 derive: 0 if lambda_s > 0, else M_phi kappa */
  double s_f[5], s_g[5], s_h[5]; /* MRT rates by moment order 0..4 (<= 0: 1); s_f[2] <= 0: local 1/(3 mu/rho + 1/2) */
  double x0, y0, R0, a, b;  /* initial geometry */
  double mms_dx;            /* 0 (default): off.  > 0: the accuracy test of Sec. 4.1 on the unit square
                               with grid spacing mms_dx (nx mms_dx = ny mms_dx = 1, periodic, FP64
                               storage, linear constraint, surfactant on): the step prescribes the
                               velocity (0.05, -0.03) (lattice units: times dt/dx, dt = dx^2/0.15) and
                               p = 0, and adds dt times the test's manufactured sources S_phi, S_psi
                               at time t = n dt of step n to R_phi and R_psi; steps run eagerly (the
                               step index is a launch argument), without captured graphs */
} lbm_params;

typedef struct {
  int64_t step;             /* completed steps */
  int64_t nonfinite;        /* nodes with a non-finite phi, psi, u or p */
  int64_t psi_out_of_range; /* nodes with psi outside (0,1) (surfactant runs) */
  int64_t cap_violations;   /* wetting-wall nodes where 1 + beta_sa ln(1 - psi) <= 1/2 (Remark 1) */
  double mass_psi;          /* sum psi, conserved by the linear constraint */
  double m_phi_h;           /* sum (1/2 + g(phi)), the nonlinear phase measure */
  double sum_phi;           /* sum phi */
  double area_phi_pos;      /* area of phi > 0, two-triangle reconstruction (Sec. 4.1) */
  double kinetic;           /* sum rho |u|^2 / 2 */
  double free_energy;       /* discrete E_f (eq1) including the wall energy */
  double umax;              /* max |u| */
  double lambda_phi;        /* multiplier of the current state (eq15 with h_phi) */
  double mubar_psi;         /* mean chemical potential of the current state */
  double contact_width;     /* bottom wall: length of phi > 0 on the first two rows, extrapolated to the wall */
  double cap_height;        /* bottom wall: highest phi = 0 crossing above the wall */
  double theta_app_deg;     /* 2 atan(2 H / L), 180 when detached (L = 0) */
} lbm_invariants;

/* Field mask bits for lbm_fetch_fields / lbm_load_fields; planes are laid
 * out one after another in increasing bit order. */
enum { LBM_F_PHI = 1, LBM_F_PSI = 2, LBM_F_UX = 4, LBM_F_UY = 8, LBM_F_P = 16,
       LBM_F_RHO = 32, LBM_F_MU_PHI = 64, LBM_F_MU_PSI = 128 };

/* Number of derived constants reported by lbm_derived, in this order:
 * kappa, beta, W, kBT, phi_b, sigma_sg0, sigma_sl0, lambda_s, M0, eta_phi, eta_psi, psi_c. */
#define LBM_N_DERIVED 12

/* Bytes of device memory a handle with these parameters needs. */
int lbm_required_bytes(const lbm_params* p, size_t* bytes);

/* Validate p, derive the lattice constants, place the state and build the
 * initial fields (Sec. 2.2 profile, equilibrium populations, u = 0, p = 0).
 * dev_buf: NULL to let the library allocate, or caller-owned device memory of
 * at least lbm_required_bytes (it must outlive the handle; never freed here).
 * hip_stream: a hipStream_t to order all work on, or NULL for a library
 * stream.  On error *out is NULL and the status says why (LBM_E_ARG for a bad
 * parameter set; the message is available from lbm_last_error(NULL)). */
int lbm_init(const lbm_params* p, void* dev_buf, size_t buf_bytes, void* hip_stream, lbm_handle** out);

/* Enqueue n time steps (n >= 0).  One step is the scheme of Sec. 3 for all
 * three populations: zeroth moments (macroscopic recovery), the wall values of
 * the natural boundary conditions (eq "boundary" with the wall energy eq8),
 * the chemical potentials (eq_muphi, eq_mupsi) with the isotropic stencils of
 * the end of Sec. 3, the multiplier sums of eq15 and AC_psi in FP64, the force
 * (eq_Fs0), velocity and pressure, the sources R_phi, R_psi with their
 * backward differences, the three MRT collisions (unified MRT equation, f_eq of
 * the three lattices, F_{i,1..3}) and streaming with the walls.
 * Asynchronous: returns once the work is on the stream.  Faults in the fields
 * surface at the next synchronising call.  Runs are replayed from HIP graphs
 * of 2, 4, 8, 16 or 32 steps the handle captures on first use (a run is split
 * into the longest such pieces; same results bit for bit; on grids of at most
 * 1024 workgroups the captured steps reduce the previous step's multiplier
 * sums themselves, in the same order); the first step after (re)initialisation,
 * an odd last step and steps while kernel timing is active are launched one
 * by one.  For a given tile_rows the step kernel's schedule (lbm_step_kernel)
 * does not change the results in FP32 and FP16 storage (bit for bit); in FP64
 * storage the kernels contract multiply-adds differently (last bits);
 * tile_rows itself groups the multiplier sums, so it changes their last bits.  Errors: LBM_E_ARG for n < 0, LBM_E_STATE
 * after a latched fault, LBM_E_DEVICE when a launch fails. */
int lbm_step(lbm_handle* h, int64_t n);

/* Diagnostics of the current state: the conserved sums of Sec. 2.1 (sum psi of
 * AC_psi, sum h_phi of eq15), the two-triangle area of phi > 0 (Sec. 4.1), the
 * kinetic and free energy with the wall energy (eq1, eq8; the energy law of
 * Sec. 2.4), max |u|, the multipliers, and at a bottom wall the contact width,
 * cap height and apparent angle of a circular cap (eq "a", Sec. 4.3).  FP64
 * sums on the device, then one small device-to-host copy; synchronises the
 * stream.  *out is caller-owned.  Returns LBM_E_RANGE when psi left (0,1),
 * else LBM_E_NONFINITE when a field is not finite (*out filled in both cases);
 * either latches the handle so that lbm_step returns LBM_E_STATE until
 * lbm_load_fields or lbm_load_state replaces the state. */
int lbm_reduce_invariants(lbm_handle* h, lbm_invariants* out);

/* Macroscopic fields of the current state (time n, before its collision):
 * phi and psi as the zeroth moments, u and p as Sec. 3 recovers them (rho u =
 * sum c_i f_i + F/2, p from sum_{i != 0} f_i), rho(phi), and mu_phi, mu_psi
 * (eq_muphi, eq_mupsi, without the multiplier terms).  Written to the
 * caller-owned host buffer as FP64 [popcount(mask)][ny][nx], planes in
 * increasing bit order; n_doubles must be at least that size (LBM_E_ARG
 * otherwise, or for a mask outside the LBM_F_* bits).  Synchronises the
 * stream. */
int lbm_fetch_fields(lbm_handle* h, uint32_t mask, double* host, size_t n_doubles);

/* Replace the state by equilibrium populations of the given fields: mask must
 * contain LBM_F_PHI and LBM_F_PSI, and may contain LBM_F_UX | LBM_F_UY;
 * pressure is set to 0 and the backward-difference history restarts. */
int lbm_load_fields(lbm_handle* h, uint32_t mask, const double* host, size_t n_doubles);

/* Raw state for checkpoint / restart: populations, history planes, the
 * pending multipliers, phi_hold's reference sum and the step count
 * (restarting from a blob continues the run bit for bit).  lbm_state_bytes
 * gives the size; load_state only accepts a blob from a handle with identical
 * parameters (LBM_E_ARG otherwise). */
int lbm_state_bytes(lbm_handle* h, size_t* bytes);
int lbm_save_state(lbm_handle* h, void* host, size_t bytes);
int lbm_load_state(lbm_handle* h, const void* host, size_t bytes);

/* Derived lattice constants (LBM_N_DERIVED doubles, order above). */
int lbm_derived(lbm_handle* h, double* out);

/* Populations of the current state as FP64 [27][ny][nx] (f0..f8, g0..g8,
 * h0..h8, post-streaming at time n).  Synchronises the stream. */
int lbm_fetch_populations(lbm_handle* h, double* host, size_t n_doubles);

/* Kernel timing with HIP events on the handle's stream.  lbm_timing_begin
 * creates event pairs for up to max_steps steps; every following lbm_step
 * brackets each of its kernels (LBM_K_* below: the fused step kernel and the
 * one-block reduction that forms the multipliers) with an event pair until the
 * pairs run out.  lbm_timing_end synchronises the
 * stream and writes, per kernel kind, the summed duration in ms
 * (ms[LBM_N_KERNELS]) and the number of launches timed
 * (launches[LBM_N_KERNELS]); it releases the events. */
enum { LBM_K_STEP = 0, LBM_K_FINISH = 1, LBM_N_KERNELS = 2 };
int lbm_timing_begin(lbm_handle* h, int64_t max_steps);
int lbm_timing_end(lbm_handle* h, double* ms, int64_t* launches);

/* Bytes of HBM state one step of this handle must read and write per node:
 * the 27 populations, the FP64 phi/psi planes and the velocity and source
 * history (the algorithmic traffic of the step). */
int lbm_bytes_per_node_step(lbm_handle* h, double* bytes);

/* Achievable-bandwidth probe (a measurement aid for the roofline; not part of
 * the method).  One kernel moves, per node of an nx x ny periodic grid, exactly
 * the bytes lbm_bytes_per_node_step counts for a step with surfactant in the
 * given storage precision, in the step's access pattern and without its
 * arithmetic: the 27 populations pulled from the neighbours that streaming
 * reads (FP16 storage: the rest populations of g and h from FP32 planes), six
 * history planes in the collision type and two FP64 planes, each read once
 * and written once.  lbm_probe_bytes gives the device bytes the probe needs
 * (nx * ny <= 2^28); lbm_probe_stream runs it on dev_buf (caller-owned,
 * 256-byte aligned, contents overwritten) on hip_stream (NULL: the null
 * stream): two warm-up launches, then `reps` launches (1..10000) timed with
 * HIP events; *ms_out is their mean duration.  It synchronises the stream.
 * Errors go to lbm_last_error(NULL). */
int lbm_probe_bytes(int32_t nx, int32_t ny, int32_t precision, size_t* bytes);
int lbm_probe_stream(int32_t nx, int32_t ny, int32_t precision, int32_t reps, void* dev_buf, size_t buf_bytes,
                     void* hip_stream, float* ms_out);

/* The device's streaming-copy ceiling (a measurement aid beside the probe):
 * copies `bytes` from src to dst (device memory, caller-owned, 16-byte
 * aligned, bytes a positive multiple of 16, the regions not overlapping) with
 * 16-byte non-temporal loads and stores, two warm-up copies and `reps` timed
 * ones (1..10000) on hip_stream (NULL: the null stream); *ms_out is their mean
 * duration (the rate counts bytes read plus bytes written).  Synchronises the
 * stream.  Errors go to lbm_last_error(NULL). */
int lbm_probe_copy(const void* src, void* dst, size_t bytes, int32_t reps, void* hip_stream, float* ms_out);

/* Which kernel this handle's steps launch (the results are the same for
 * each; only the schedule differs), chosen from the number of workgroups
 * against the device's compute units:
 *   LBM_KV_SMALL   one-pass 4-row tiles of eight waves (at most one workgroup per CU)
 *   LBM_KV_MID     one-pass 4-row tiles of four waves (up to three per CU; FP32, FP16)
 *   LBM_KV_SWEEP   the upward row sweep, built for one workgroup per CU
 *   LBM_KV_SWEEP_PACKED  the row sweep of walled grids built for three workgroups per CU
 * *workgroups is the step launch's workgroup count and *cus the CU count the
 * choice used: the device's, unless the environment variable LBM_KERNEL_CUS
 * (read by lbm_init; 1..65536) overrides it, which tests use to run every
 * variant on one device. */
enum { LBM_KV_SMALL = 0, LBM_KV_MID = 1, LBM_KV_SWEEP = 2, LBM_KV_SWEEP_PACKED = 3 };
int lbm_step_kernel(lbm_handle* h, int32_t* variant, int32_t* workgroups, int32_t* cus);

/* Release the handle and any library-owned device memory and stream. */
int lbm_destroy(lbm_handle* h);

/* Message of the last failed call on h (or of the last failed lbm_init when
 * h is NULL).  Never NULL. */
const char* lbm_last_error(const lbm_handle* h);

/* ------------------------------------------------------------ batched sweep
 * Many independent cases (each its own lbm_params: grid, physics, walls)
 * advanced together: one kernel launch per step covers the workgroups of all
 * cases, a second forms each case's multipliers (the per-case reductions of
 * eq15 and the psi constraint).  The cases of a batch share one storage
 * precision and one kind of y boundary (all walled or all periodic); their
 * results equal, bit for bit, those of single handles with the same segment
 * height.  A case can be retired (not stepped) and its slot refilled with new
 * parameters of the same grid.  Runs replay from HIP graphs of 1, 2, 4, 8, 16
 * or 32 steps (a run is split into the longest such pieces). */
typedef struct lbm_batch lbm_batch; /* opaque, owned by the library */

/* Device bytes for the batch's state (cases[0..count-1]); validates every case
 * (LBM_E_ARG with the case index in the message). */
int lbm_batch_required_bytes(const lbm_params* cases, int32_t count, size_t* bytes);

/* Create a batch and initialise every case as lbm_init does.  seg_rows is the
 * row-segment height of the step workgroups for all cases (a multiple of 4; 0
 * chooses one from the total size); dev_buf / hip_stream as for lbm_init (the
 * caller's buffer must hold lbm_batch_required_bytes, 256-byte aligned). */
int lbm_batch_init(const lbm_params* cases, int32_t count, int32_t seg_rows, void* dev_buf, size_t buf_bytes,
                   void* hip_stream, lbm_batch** out);

/* Enqueue n steps of every active case (asynchronous, as lbm_step).  Returns
 * LBM_E_STATE while an active case is latched faulted by a diagnostic. */
int lbm_batch_step(lbm_batch* b, int64_t n);

/* Activity of every case (active[count]: 0 retires a case, which then keeps
 * its state; nonzero steps it).  Synchronises the stream. */
int lbm_batch_set_active(lbm_batch* b, const int32_t* active);

/* lbm_reduce_invariants for every case into out[count] (synchronises).
 * Returns the first case's error code, after filling every entry. */
int lbm_batch_reduce_invariants(lbm_batch* b, lbm_invariants* out);

/* lbm_fetch_fields of case index (synchronises). */
int lbm_batch_fetch_fields(lbm_batch* b, int32_t index, uint32_t mask, double* host, size_t n_doubles);

/* Refill slot index with a new case of any grid whose state fits the slot
 * (lbm_required_bytes(p) <= lbm_batch_slot_bytes of the slot), with the
 * batch's precision and kind of y boundary; initialised as lbm_init does, and
 * made active.  The other cases keep their state.  A grid of another size
 * changes the batch's workgroup map, which is rebuilt (and the step graphs
 * captured again) at the next call that steps or sets activity; results do not
 * depend on the slot a case runs in.  LBM_E_ARG if the case does not fit or
 * does not match the batch (the slot keeps its case); if initialising the new
 * case fails on the device the slot is retired and the error returned. */
int lbm_batch_replace_case(lbm_batch* b, int32_t index, const lbm_params* p);

/* Bytes of device memory slot index holds (set by the case it was created
 * with): a refill with lbm_batch_replace_case must need no more. */
int lbm_batch_slot_bytes(lbm_batch* b, int32_t index, size_t* bytes);

/* Autotuner: for each segment height of {4, 8, 16, 32, 64} steps the batch
 * 1 + trial_steps times from its initial state, timing the last trial_steps,
 * and checks the result: every active case's sum psi, sum phi, sum h_phi and
 * lambda_phi must lie within a relative 1e-10 (FP64 storage), 1e-6 (FP32) or
 * 1e-4 (FP16) of the first candidate's, with no non-finite field (the
 * candidates change only how the FP64 multiplier sums are grouped).  Keeps the
 * fastest candidate that passes (written to *seg_rows_out) and puts every case
 * back to its initial state.  Only before the first step.  LBM_E_NONFINITE if
 * no candidate passes (the batch keeps its previous height). */
int lbm_batch_autotune(lbm_batch* b, int32_t trial_steps, int32_t* seg_rows_out);

/* The last autotune's candidates, in the order tried: segment height, time of
 * the trial steps (ms), largest relative deviation of the checked sums from
 * the first candidate's (0 for the first), and 1 when the candidate passed the
 * check.  Caller-owned arrays of max_rows entries; *rows receives the number of
 * candidates (0 before any autotune).  LBM_E_ARG when max_rows is smaller. */
int lbm_batch_autotune_report(lbm_batch* b, int32_t max_rows, int32_t* seg_rows, double* ms, double* max_rel_dev,
                              int32_t* passed, int32_t* rows);

/* Cases, segment height, workgroups of one step launch and total nodes. */
int lbm_batch_info(lbm_batch* b, int32_t* count, int32_t* seg_rows, int32_t* workgroups, int64_t* nodes);

/* Kernel timing of the batch's step and finishing kernels, as lbm_timing_*. */
int lbm_batch_timing_begin(lbm_batch* b, int64_t max_steps);
int lbm_batch_timing_end(lbm_batch* b, double* ms, int64_t* launches);

/* Release the batch, its cases and any library-owned memory and stream. */
int lbm_batch_destroy(lbm_batch* b);

/* Message of the last failed call on b (of the last failed lbm_batch_init or
 * lbm_batch_required_bytes when b is NULL).  Never NULL. */
const char* lbm_batch_last_error(const lbm_batch* b);

#ifdef __cplusplus
}
#endif
#endif
