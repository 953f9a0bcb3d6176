/*
 * lbm3d.h -- C ABI of the three-dimensional (D3Q19) lattice Boltzmann step of
 * the conservative Allen-Cahn / Navier-Stokes surfactant model with solid
 * adsorption (Huang, Chai, Liu, Huang), on gfx950.
 *
 * The model of Sec. 2 is stated for d = 2 and 3, and the unified MRT scheme of
 * Sec. 3 for any velocity set with a moment matrix M and a diagonal relaxation
 * matrix.  This library runs it on D3Q19 (weights 1/3, 1/18, 1/36) with the 19
 * raw moments c_x^a c_y^b c_z^c grouped by order and relaxed by
 * diag(s0, s1, s2, s3, s4): one time step advances the three populations
 *   f  hydrodynamics, pressure-based equilibrium (Sec. 3, f_eq of lattice 1)
 *   g  phase field phi, weighted nonlinear multiplier  (eq15, AC_phi)
 *   h  surfactant psi, linear multiplier               (AC_psi)
 * with the chemical potentials (eq_muphi, eq_mupsi), the force
 * F = -phi grad mu_phi - psi grad mu_psi + G (eq_Fs0), the isotropic D3Q19
 * stencils and backward time differences (end of Sec. 3), the wetting and
 * solid-adsorption conditions at walls (Sec. 2.1, eq "boundary", eq8) and the
 * FP64 multiplier sums every step.  The readings of the 2-D library hold:
 * phi and psi are advected by the mean of this and the previous step's velocity
 * (adv_raw = 1: the step's own velocity), rho and mu are linear in the liquid
 * fraction held to [0, 1], walls are half-way bounce-back with a ghost layer.
 *
 * Geometry: x and y are periodic; z is periodic (both kinds LBM_BC_PERIODIC) or
 * bounded by walls at z = -1/2 and z = nz - 1/2 (the LBM_BC_* kinds of lbm.h).
 * Node (x, y, z) sits at that position.
 *
 * Conventions as in lbm.h: every entry point returns LBM_OK (0) or a negative
 * lbm_status; lbm3d_last_error gives the message.  Fields crossing the boundary
 * are FP64 [nz][ny][nx], x fastest, whatever the storage precision.  Host
 * buffers are caller-owned.  Calls on one handle are ordered on its stream.
 */
#ifndef LBM3D_H
#define LBM3D_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define LBM3D_ABI_VERSION 2

typedef struct lbm3d_handle lbm3d_handle; /* opaque, owned by the library */

/* Model parameters in lattice units, as lbm_params (lbm.h) with a third axis.
 * precision: LBM_FP64 or LBM_FP32 (storage of the populations; the
 * macroscopic fields, the sums and the collisions run in FP64). */
typedef struct {
  int32_t abi_version;      /* LBM3D_ABI_VERSION */
  int32_t nx, ny, nz;       /* each >= 3, nx ny nz < 2^31 */
  int32_t bc_bottom, bc_top;  /* walls in z: LBM_BC_PERIODIC (both), WALL_WET, NOSLIP, FREESLIP */
  int32_t precision;
  int32_t constraint_phi;   /* LBM_CONSTRAINT_NONLINEAR or _LINEAR */
  int32_t init_kind;        /* LBM_INIT_DROP (sphere), _SLAB (|x - x0| < a/2), _BUBBLE */
  int32_t adv_raw;          /* 0: two-step mean advecting velocity; 1: the step's own */
  int32_t phi_hold;         /* 1: lambda also returns sum h_phi to its initial value */
  int32_t solid_wet;        /* 1: solid nodes (lbm3d_set_solid) carry the wetting and adsorption
                               conditions of theta0, beta_sg, beta_sl; 0: neutral no-flux solids */
  double sigma_gl0, eps, M_phi, M_psi, lambda_s, kBT, W, Ex, Pi, psi_b, phi_b;
  double theta0_deg, sigma_sg0, sigma_sl0, beta_sg, beta_sl;
  double rho_l, rho_g, mu_l, mu_g;
  double gx, gy, gz;
  double u_wall_bottom, u_wall_top;   /* x speed of the z walls */
  double eta_phi, eta_psi, M0;
  double s_f[5], s_g[5], s_h[5];      /* rates by moment order; s_f[2] <= 0: local viscosity */
  double x0, y0, z0, R0, a;
} lbm3d_params;

typedef struct {
  int64_t step, nonfinite, psi_out_of_range;
  double mass_psi, m_phi_h, sum_phi, kinetic, umax, lambda_phi, mubar_psi;
} lbm3d_invariants;

/* Field mask bits of lbm3d_fetch_fields (planes in increasing bit order). */
enum { LBM3D_F_PHI = 1, LBM3D_F_PSI = 2, LBM3D_F_UX = 4, LBM3D_F_UY = 8, LBM3D_F_UZ = 16, LBM3D_F_P = 32,
       LBM3D_F_RHO = 64, LBM3D_F_MU_PHI = 128, LBM3D_F_MU_PSI = 256 };

/* Device bytes a handle with these parameters needs (LBM_E_ARG for a bad set). */
int lbm3d_required_bytes(const lbm3d_params* p, size_t* bytes);

/* Validate, derive the constants as lbm_init does, place the state and build
 * the initial fields (the tanh profile of Sec. 2.2 around a sphere, a slab or
 * a spherical bubble; u = 0, p = 0; equilibrium populations).  dev_buf: NULL
 * or caller-owned device memory of lbm3d_required_bytes, 256-byte aligned
 * (never freed here); hip_stream: NULL for a library stream.  LBM_E_ARG for
 * invalid parameters and for grids of 2^29 nodes or more. */
int lbm3d_init(const lbm3d_params* p, void* dev_buf, size_t buf_bytes, void* hip_stream, lbm3d_handle** out);

/* Enqueue n >= 0 time steps of Sec. 3 (five kernels each: chemical potentials
 * with the multiplier sums; the multipliers; force, velocity, pressure,
 * sources, the flow lattice's MRT collision and push streaming with the walls;
 * the phase-field and surfactant collisions and streaming; the zeroth moments
 * of the new state).  Asynchronous. */
int lbm3d_step(lbm3d_handle* h, int64_t n);

/* Conserved sums (sum psi of AC_psi, sum h_phi of eq15, sum phi), kinetic
 * energy, max |u|, the multipliers of the current state and fault counts, as
 * FP64 sums on the device; synchronises.  LBM_E_RANGE / LBM_E_NONFINITE when
 * psi left (0,1) or a field is not finite (*out filled in both cases). */
int lbm3d_reduce_invariants(lbm3d_handle* h, lbm3d_invariants* out);

/* Macroscopic fields of the current state (phi, psi, u, p, rho, mu_phi,
 * mu_psi as Sec. 3 recovers them) into host[popcount(mask)][nz][ny][nx]
 * (n_doubles at least that size, else LBM_E_ARG); synchronises. */
int lbm3d_fetch_fields(lbm3d_handle* h, uint32_t mask, double* host, size_t n_doubles);

/* Replace the state by equilibrium populations of phi, psi and, if with_u,
 * u (host: [2 or 5][nz][ny][nx] FP64: phi, psi[, ux, uy, uz]); p = 0, the
 * history restarts and phi_hold's reference becomes this state's sum. */
int lbm3d_load_fields(lbm3d_handle* h, int32_t with_u, const double* host, size_t n_doubles);

/* Complex walls: mark solid nodes (mask[nz][ny][nx], nonzero = solid; n at
 * least nx ny nz; caller-owned, read once).  A link from a fluid node into a
 * solid node is a half-way bounce-back wall for all three lattices; the
 * stencils see a ghost value there taken at the fluid node itself, link by link
 * (mirror values for psi and the potentials; with solid_wet, phi + J_phi/kappa
 * and the wall term (2 w_i / c_s^2) J of eq. "boundary" per link), and sums and
 * the mean potential run over fluid nodes.  The state is rebuilt as equilibrium
 * populations of the current phi, psi at the fluid nodes (history restarts,
 * phi_hold's reference is retaken).  LBM_E_ARG if no fluid node is left. */
int lbm3d_set_solid(lbm3d_handle* h, const uint8_t* mask, size_t n);

/* Bytes of HBM state one step moves per node by design (all four kernels). */
int lbm3d_bytes_per_node_step(lbm3d_handle* h, double* bytes);

/* Release the handle and library-owned memory and stream. */
int lbm3d_destroy(lbm3d_handle* h);

/* Message of the last failed call on h (of lbm3d_init when h is NULL). */
const char* lbm3d_last_error(const lbm3d_handle* h);

#ifdef __cplusplus
}
#endif
#endif
