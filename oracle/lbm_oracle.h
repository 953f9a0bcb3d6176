/*
 * lbm_oracle.h -- plain FP64 CPU oracle of the coupled conservative
 * Allen-Cahn / Navier-Stokes surfactant lattice Boltzmann step.
 *
 * TEST INFRASTRUCTURE ONLY.  This library exists to check the HIP path.  Only
 * the test suite, the smoke entry point and the CPU-baseline leg of the
 * benchmark may load it.  It shares no code, header, table or constant with
 * the HIP library; both follow the paper (model: Section 2, scheme: Section 3)
 * and the same readings of its open points (listed in lbm_oracle.c).
 *
 * Units: lattice units throughout (dx = dt = 1, c_s^2 = 1/3).
 * Layout of every field handed in or out: FP64, row-major [ny][nx], x fastest.
 */
#ifndef LBM_ORACLE_H
#define LBM_ORACLE_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* Wall kinds for the bottom (y = -1/2) and top (y = ny - 1/2) boundaries. */
enum { ORC_PERIODIC = 0, ORC_WALL_WET = 1, ORC_NOSLIP = 2, ORC_FREESLIP = 3 };
/* Conservation constraint applied to phi (Section 2.1): weighted nonlinear
 * map h = 1/2 + g(phi), or the classical linear one h = phi. */
enum { ORC_NONLINEAR = 0, ORC_LINEAR = 1 };
/* Initial phase-field geometry. */
enum { ORC_INIT_DROP = 0, ORC_INIT_SLAB = 1, ORC_INIT_BUBBLE = 2 };

typedef struct {
  int32_t nx, ny;
  int32_t bc_bottom, bc_top;
  int32_t constraint_phi;
  int32_t init_kind;
  int32_t mms;            /* 1: manufactured-solution mode (Section 4.1), see orc_mms_* */
  int32_t adv_raw;        /* 1: advect phi, psi with the step's own velocity u (literal);
                             0: with the two-step mean (u(n) + u(n-1))/2 (default reading) */
  int32_t phi_hold;       /* 1: the phi multiplier also returns sum h_phi to its initial value
                             (see orc_step); 0: eq15 as printed (default) */
  int32_t sat_cap;        /* 1: Remark-1 saturation, sigma_sa(psi) = sigma_sa0 max(1/2, 1 + beta_sa ln(1 - psi));
                             0: the smooth Langmuir-Szyszkowski form the paper computes with (default) */
  double sigma_gl0, eps;  /* clean tension and interface-thickness parameter */
  double M_phi, M_psi;    /* mobilities */
  double lambda_s;        /* psi gradient coefficient; <0: kappa/2 with a wetting wall, else 0 */
  double kBT, W;          /* <=0: from Pi and Ex */
  double Ex, Pi;          /* solubility and entropy groups (Section 4) */
  double psi_b;           /* bulk surfactant; 0 switches surfactant off */
  double phi_b;           /* <=0: from psi_b (Section 2.2) */
  double theta0_deg;      /* clean Young angle */
  double sigma_sg0, sigma_sl0; /* <0: from Young's law and sum 16 sigma/15 */
  double beta_sg, beta_sl;     /* Langmuir-Szyszkowski elasticities */
  double rho_l, rho_g, mu_l, mu_g;
  double gx, gy;               /* body acceleration, G = rho g */
  double u_wall_bottom, u_wall_top; /* tangential wall speeds (no-slip walls) */
  double eta_phi, eta_psi;     /* <=0: from the diffusivity with s1 */
  double M0;                   /* <0: 0 if lambda_s>0 else M_phi kappa */
  double s_f[5], s_g[5], s_h[5]; /* rates by moment order 0..4; s_f[2]<=0: from local viscosity */
  double x0, y0, R0, a, b;     /* initial geometry */
  double mms_dx;               /* manufactured mode: grid spacing in [0,1]^2 */
} orc_params;

typedef struct {
  int64_t step, nonfinite, psi_out_of_range, cap_violations;
  double mass_psi, m_phi_h, sum_phi, area_phi_pos, kinetic, free_energy, umax;
  double lambda_phi, mubar_psi, contact_width, cap_height, theta_app_deg;
  double sum_R_psi, orthogonality;   /* per-step identities of the last step */
} orc_inv;

/* Derived lattice constants, in this order:
 * kappa, beta, W, kBT, phi_b, sigma_sg0, sigma_sl0, lambda_s, M0, eta_phi, eta_psi, psi_c */
#define ORC_N_DERIVED 12

/* Field mask bits for orc_fields (output planes in increasing bit order). */
enum { ORC_F_PHI = 1, ORC_F_PSI = 2, ORC_F_UX = 4, ORC_F_UY = 8, ORC_F_P = 16,
       ORC_F_RHO = 32, ORC_F_MU_PHI = 64, ORC_F_MU_PSI = 128 };

typedef struct orc_sim orc_sim;

/* Returns NULL and writes a message into err (size errlen) on invalid input. */
orc_sim* orc_create(const orc_params* p, char* err, int errlen);
void     orc_destroy(orc_sim* s);
void     orc_step(orc_sim* s, int64_t n);
void     orc_derived(const orc_sim* s, double* out /* ORC_N_DERIVED */);
/* Macroscopic fields of the current state (time n, before its collision). */
void     orc_fields(orc_sim* s, uint32_t mask, double* out);
void     orc_invariants(orc_sim* s, orc_inv* out);
/* Replace phi, psi (and u, may be NULL) and rebuild equilibrium populations;
 * the backward-difference history restarts. */
void     orc_load_fields(orc_sim* s, const double* phi, const double* psi,
                         const double* ux, const double* uy);
/* Populations of the current state: out holds 27 planes [f0..f8, g0..g8, h0..h8][ny][nx]. */
void     orc_get_populations(const orc_sim* s, double* out);
/* Manufactured-solution mode: relative L2 errors (phi, psi) against the exact
 * solution at the current time, and the conserved sums. */
void     orc_mms_errors(orc_sim* s, double* e_phi, double* e_psi);
/* Diagnostics on an arbitrary field (pinned on synthetic inputs). */
double   orc_area_positive(const double* phi, int nx, int ny, int wall_bottom, int wall_top, int periodic_y);
void     orc_contact(const double* phi, int nx, int ny, double* width, double* height, double* theta_deg);
/* Number of OpenMP threads the node loops use (1 without OpenMP). */
int      orc_threads(void);
/* 0: run every node loop on the calling thread (for timing one case per
 * thread, or one thread alone); 1 (default): OpenMP on large grids. */
void     orc_set_parallel(int on);

#ifdef __cplusplus
}
#endif
#endif
