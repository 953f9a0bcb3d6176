/*
 * lbm3d_oracle.h -- plain FP64 CPU oracle of the coupled conservative
 * Allen-Cahn / Navier-Stokes surfactant lattice Boltzmann step in three
 * dimensions (D3Q19).
 *
 * TEST INFRASTRUCTURE ONLY.  This library exists to check the HIP path.  Only
 * the test suite, the smoke entry point and the CPU-baseline leg of the
 * benchmark may load it.  It shares no code, header, table or constant with
 * the HIP library.  The model (Sec. 2) is stated for d = 2 and 3; the scheme
 * (Sec. 3) is written for any velocity set with a moment matrix and a
 * diagonal relaxation matrix grouped by moment order.
 *
 * Units: lattice units throughout (dx = dt = 1, c_s^2 = 1/3).
 * Layout of every field handed in or out: FP64 [nz][ny][nx], x fastest.
 * x and y are periodic; z is periodic or bounded by walls at z = -1/2 and
 * z = nz - 1/2.
 */
#ifndef LBM3D_ORACLE_H
#define LBM3D_ORACLE_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* Same wall kinds, constraint and initial geometries as the 2-D oracle. */
enum { ORC3_PERIODIC = 0, ORC3_WALL_WET = 1, ORC3_NOSLIP = 2, ORC3_FREESLIP = 3 };
enum { ORC3_NONLINEAR = 0, ORC3_LINEAR = 1 };
enum { ORC3_INIT_DROP = 0, ORC3_INIT_SLAB = 1, ORC3_INIT_BUBBLE = 2 };

typedef struct {
  int32_t nx, ny, nz;
  int32_t bc_bottom, bc_top;     /* z walls */
  int32_t constraint_phi;
  int32_t init_kind;
  int32_t adv_raw;               /* 1: advect with u(n); 0: with (u(n) + u(n-1))/2 */
  int32_t phi_hold;              /* 1: lambda also returns sum h_phi to its initial value */
  int32_t solid_wet;             /* 1: solid nodes (orc3_set_solid) carry the wetting and adsorption BCs */
  double sigma_gl0, eps, M_phi, M_psi, lambda_s, kBT, W, Ex, Pi, psi_b, phi_b;
  double theta0_deg, sigma_sg0, sigma_sl0, beta_sg, beta_sl;
  double rho_l, rho_g, mu_l, mu_g;
  double gx, gy, gz;
  double u_wall_bottom, u_wall_top;   /* x speed of no-slip walls */
  double eta_phi, eta_psi, M0;
  double s_f[5], s_g[5], s_h[5];      /* rates by moment order 0..4; s_f[2] <= 0: local viscosity */
  double x0, y0, z0, R0, a;           /* drop centre and radius; slab width a (slab: |x - x0| < a/2) */
} orc3_params;

typedef struct {
  int64_t step, nonfinite, psi_out_of_range;
  double mass_psi, m_phi_h, sum_phi, kinetic, umax, lambda_phi, mubar_psi, sum_R_psi, orthogonality;
} orc3_inv;

enum { ORC3_F_PHI = 1, ORC3_F_PSI = 2, ORC3_F_UX = 4, ORC3_F_UY = 8, ORC3_F_UZ = 16, ORC3_F_P = 32,
       ORC3_F_RHO = 64, ORC3_F_MU_PHI = 128, ORC3_F_MU_PSI = 256 };
#define ORC3_N_DERIVED 12   /* kappa, beta, W, kBT, phi_b, sigma_sg0, sigma_sl0, lambda_s, M0, eta_phi, eta_psi, psi_c */

typedef struct orc3_sim orc3_sim;

orc3_sim* orc3_create(const orc3_params* p, char* err, int errlen);
void      orc3_destroy(orc3_sim* s);
void      orc3_step(orc3_sim* s, int64_t n);
void      orc3_derived(const orc3_sim* s, double* out);
void      orc3_fields(orc3_sim* s, uint32_t mask, double* out);
void      orc3_invariants(orc3_sim* s, orc3_inv* out);
/* Replace phi, psi (and u, may be NULL: three planes ux, uy, uz) by
 * equilibrium populations; the history restarts. */
void      orc3_load_fields(orc3_sim* s, const double* phi, const double* psi, const double* u);
/* Mark solid nodes (mask[N], nonzero = solid) and rebuild equilibrium
 * populations from the current phi, psi at the fluid nodes (history restarts).
 * Returns -1 if no fluid node is left. */
int       orc3_set_solid(orc3_sim* s, const unsigned char* mask);
/* Populations of the current state: 57 planes [f0..f18, g0..g18, h0..h18]. */
void      orc3_get_populations(const orc3_sim* s, double* out);
/* The velocity set in the oracle's own order (19 x 3 ints) and weights. */
void      orc3_lattice(int* c, double* w);

#ifdef __cplusplus
}
#endif
#endif
