/*
 * lbm_oracle.c -- plain FP64 CPU oracle of one lattice Boltzmann time step of
 * the thermodynamically consistent, conservative Allen-Cahn / Navier-Stokes
 * surfactant model with solid adsorption (Huang, Chai, Liu, Huang).
 *
 * TEST INFRASTRUCTURE ONLY: it is the yardstick the HIP path is checked
 * against.  Only the test suite, the smoke entry point and the CPU-baseline leg
 * of the benchmark may load it.  It shares no code with the HIP path.
 *
 * The code takes the scheme's steps in the paper's order and notation:
 *   O1  phi = sum_i g_i, psi = sum_i h_i                     (Sec. 3, macroscopic recovery)
 *   O2  wall values from the natural wetting / adsorption BCs (Sec. 2.1, eq. "boundary")
 *   O3  chemical potentials mu_phi, mu_psi                    (Sec. 2.1, eq_muphi / eq_mupsi)
 *   O4  Lagrange multipliers lambda_phi, mubar_psi            (Sec. 2.1, eq15, AC_psi, AC_phi)
 *   O5  force F = -phi grad mu_phi - psi grad mu_psi + G      (Sec. 2.1, eq_Fs0)
 *   O6  velocity and pressure                                  (Sec. 3, macroscopic recovery)
 *   O7  sources R_phi, R_psi and their backward differences    (Sec. 3, source terms)
 *   O8  MRT collision of the three populations                 (Sec. 3, unified MRT LBE)
 *   O9  streaming with periodic / bounce-back / moving / free-slip walls
 *   O10 history for the backward differences
 * Where the paper leaves a point open it is read as follows: D2Q9 with raw
 * moments grouped by order; relaxation rates not tied to transport are 1,
 * the f shear rate follows the local viscosity, g and h use s1 = 1 so that
 * eta = 6 D; M0 = 0 when lambda_s > 0, else M_phi kappa; rho and mu are
 * linear in (1 + phi/phi_b)/2 held to [0, 1]; every lattice bounces back half-way at a
 * wall, whose ghost row carries phi + J_phi/kappa and whose flux J_psi enters
 * mu_psi and the source; on the first step the backward differences vanish;
 * phi and psi are advected by the mean of the velocities of this and the
 * previous step (adv_raw selects the step's own velocity).
 *
 * Plain loops, FP64, a generic 9x9 moment matrix and its numerically computed
 * inverse; global sums are sequential in row-major order.
 */
#include "lbm_oracle.h"

#include <math.h>
#ifdef _OPENMP
#include <omp.h>
#endif
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#define Q 9
/* Node loops run on OpenMP threads only on grids large enough to pay for the
 * fork and join (smaller grids are faster on one thread); results do not
 * depend on it, every threaded loop writes per-node values only. */
#define ORC_PAR_MIN_NODES 1024
static int g_parallel = 1;   /* orc_set_parallel(0): every loop on the calling thread */
/* D2Q9 velocities c_i, weights w_i, opposite and y-mirrored directions. */
static const int EX[Q] = {0, 1, 0, -1, 0, 1, -1, -1, 1};
static const int EY[Q] = {0, 0, 1, 0, -1, 1, 1, -1, -1};
static const double WQ[Q] = {4.0 / 9.0,  1.0 / 9.0,  1.0 / 9.0,  1.0 / 9.0, 1.0 / 9.0,
                             1.0 / 36.0, 1.0 / 36.0, 1.0 / 36.0, 1.0 / 36.0};
static const int OPP[Q] = {0, 3, 4, 1, 2, 7, 8, 5, 6};
static const int MIRY[Q] = {0, 1, 4, 3, 2, 8, 7, 6, 5};
static const double CS2 = 1.0 / 3.0;
/* Exponents (a,b) of the raw moments c_x^a c_y^b, grouped by order; the
 * relaxation matrix is diag(s0, s1, s1, s2, s2, s2, s3, s3, s4). */
static const int MA[Q] = {0, 1, 0, 2, 1, 0, 2, 1, 2};
static const int MB[Q] = {0, 0, 1, 0, 1, 2, 1, 2, 2};
static const int MORDER[Q] = {0, 1, 1, 2, 2, 2, 3, 3, 4};

struct orc_sim {
  orc_params p;
  int nx, ny, N, periodic_y, surf;
  double kappa, beta, W, kBT, phib, sg0, sl0, lambda_s, M0, eta_phi, eta_psi, psi_c;
  double Mm[Q][Q], Mi[Q][Q];
  double *f, *g, *h, *fn, *gn, *hn;                       /* [Q][N] */
  double *phi_h, *psi_h, *ux_h, *uy_h, *Rphi_h, *Rpsi_h;  /* step n-1 */
  double *vx_h, *vy_h;                                    /* advecting velocity of step n-1 */
  int have_hist;
  int64_t step;
  double sumRpsi_last, orth_last;
  /* per-step work fields */
  double *phi, *psi, *mu_phi, *mu_psi, *lap0_psi, *Tphi, *Tpsi, *rho, *ux, *uy, *pr;
  double *Fx, *Fy, *grx, *gry, *Rphi, *Rpsi, *vx, *vy;
  double *Jphi_b, *Jpsi_b, *Jphi_t, *Jpsi_t; /* per-column wall fluxes */
  double lambda, mubar;
  double m_ref;   /* sum of h_phi(phi) of the initial (or loaded) state */
};

/* ------------------------------------------------------------------ helpers */
static int wrapi(int a, int n) { a %= n; return a < 0 ? a + n : a; }
static double powi(int c, int e) { double r = 1.0; for (int k = 0; k < e; ++k) r *= c; return r; }

/* Wall switching function g(phi) = 3 phi/(4 phi_b) - phi^3/(4 phi_b^3) and its
 * derivative (Sec. 2.1, below eq8). */
static double gsw(const orc_sim* s, double ph) {
  double b = s->phib;
  return 3.0 * ph / (4.0 * b) - ph * ph * ph / (4.0 * b * b * b);
}
static double gsw_d(const orc_sim* s, double ph) {
  double b = s->phib;
  return 3.0 / (4.0 * b) * (1.0 - ph * ph / (b * b));
}
/* h_phi(phi) itself: 1/2 + g (AC_phi) or phi. */
static double hval(const orc_sim* s, double ph) {
  return s->p.constraint_phi == ORC_LINEAR ? ph : 0.5 + gsw(s, ph);
}
static double sum_h(const orc_sim* s, const double* phi) {
  double m = 0.0;
  for (int n = 0; n < s->N; ++n) m += hval(s, phi[n]);
  return m;
}
/* h_phi'(phi): weighted nonlinear constraint h = 1/2 + g (AC_phi) or linear h = phi. */
static double hprime(const orc_sim* s, double ph) {
  return s->p.constraint_phi == ORC_LINEAR ? 1.0 : gsw_d(s, ph);
}
/* Density and dynamic viscosity: linear in the liquid fraction (1 + phi/phi_b)/2,
 * which is held to [0, 1] (the paper gives no rho(phi); unbounded, a phi just past
 * -phi_b would drive the light phase's density through zero at large ratios). */
static double liquid_frac(const orc_sim* s, double ph) {
  double w = 0.5 * (1.0 + ph / s->phib);
  return w < 0.0 ? 0.0 : (w > 1.0 ? 1.0 : w);
}
static double rho_of(const orc_sim* s, double ph) {
  return s->p.rho_g + (s->p.rho_l - s->p.rho_g) * liquid_frac(s, ph);
}
static double mud_of(const orc_sim* s, double ph) {
  return s->p.mu_g + (s->p.mu_l - s->p.mu_g) * liquid_frac(s, ph);
}
/* Remark 1: the factor by which surfactant lowers a solid-fluid tension,
 * 1 + beta ln(1 - psi) (eq "langmuir"), held at 1/2 or more, and its psi
 * derivative, -beta/(1 - psi) on the smooth side and zero where the hold acts.
 * Used only with sat_cap; the default is the smooth form below. */
static double sat_factor(double beta, double ps) {
  double q = 1.0 + beta * log(1.0 - ps);
  return q < 0.5 ? 0.5 : q;
}
static double sat_factor_d(double beta, double ps) {
  double q = 1.0 + beta * log(1.0 - ps);
  return q <= 0.5 ? 0.0 : -beta / (1.0 - ps);
}
/* The wall energy is f_w = (s_sg + s_sl)/2 - (s_sg - s_sl) g(phi), with
 * s_sa = sigma_sa0 (factor of psi) and the clean difference sigma cos(theta0). */
static double wall_diff_sat(const orc_sim* s, double ps) {
  double cth = cos(s->p.theta0_deg * M_PI / 180.0);
  return s->p.sigma_gl0 * cth + s->sg0 * (sat_factor(s->p.beta_sg, ps) - 1.0)
       - s->sl0 * (sat_factor(s->p.beta_sl, ps) - 1.0);
}
/* -df_w/dphi and -df_w/dpsi of the wall energy (eq8, boundary). */
static double wall_Jphi(const orc_sim* s, double ph, double ps) {
  if (s->surf && s->p.sat_cap) return wall_diff_sat(s, ps) * gsw_d(s, ph);
  double cth = cos(s->p.theta0_deg * M_PI / 180.0);
  double a = s->p.sigma_gl0 * cth;
  if (s->surf) a += log(1.0 - ps) * (s->sg0 * s->p.beta_sg - s->sl0 * s->p.beta_sl);
  return a * gsw_d(s, ph);
}
static double wall_Jpsi(const orc_sim* s, double ph, double ps) {
  if (s->p.sat_cap) {
    double dsg = s->sg0 * sat_factor_d(s->p.beta_sg, ps), dsl = s->sl0 * sat_factor_d(s->p.beta_sl, ps);
    return -(0.5 * (dsg + dsl) - (dsg - dsl) * gsw(s, ph));
  }
  double d = s->sg0 * s->p.beta_sg - s->sl0 * s->p.beta_sl;
  double m = s->sg0 * s->p.beta_sg + s->sl0 * s->p.beta_sl;
  return -(d * gsw(s, ph) - 0.5 * m) / (1.0 - ps);
}
static double wall_fw(const orc_sim* s, double ph, double ps) {
  if (s->surf && s->p.sat_cap)
    return 0.5 * (s->sg0 * sat_factor(s->p.beta_sg, ps) + s->sl0 * sat_factor(s->p.beta_sl, ps))
         - wall_diff_sat(s, ps) * gsw(s, ph);
  double cth = cos(s->p.theta0_deg * M_PI / 180.0);
  double l = s->surf ? log(1.0 - ps) : 0.0;
  double d = s->sg0 * s->p.beta_sg - s->sl0 * s->p.beta_sl;
  double m = s->sg0 * s->p.beta_sg + s->sl0 * s->p.beta_sl;
  return -(s->p.sigma_gl0 * cth + l * d) * gsw(s, ph) + 0.5 * l * m + 0.5 * (s->sg0 + s->sl0);
}

static int is_wall(int bc) { return bc != ORC_PERIODIC; }

/* Value of field a at the neighbour x+c_i of (x,y).  Beyond a wall the ghost
 * takes the value of the fluid node next to it in the same column (mirror). */
static double nb_mirror(const orc_sim* s, const double* a, int x, int y, int i) {
  int xx = wrapi(x + EX[i], s->nx), yy = y + EY[i];
  if (s->periodic_y) yy = wrapi(yy, s->ny);
  else if (yy < 0 || yy >= s->ny) yy = y;
  return a[yy * s->nx + xx];
}
/* Sum over directions pointing into a wetting wall of 2 w_i / c_s^2 * J(column). */
static double wall_T(const orc_sim* s, const double* Jb, const double* Jt, int x, int y) {
  if (s->periodic_y) return 0.0;
  double t = 0.0;
  for (int i = 1; i < Q; ++i) {
    int yy = y + EY[i];
    int xx = wrapi(x + EX[i], s->nx);
    if (yy < 0) t += 2.0 * WQ[i] / CS2 * Jb[xx];
    else if (yy >= s->ny) t += 2.0 * WQ[i] / CS2 * Jt[xx];
  }
  return t;
}
/* Density at neighbour x+c_i; beyond a wetting wall rho(phi_hat) with the
 * ghost phase field phi_hat = phi_f + J_phi / kappa. */
static double nb_rho(const orc_sim* s, int x, int y, int i) {
  int xx = wrapi(x + EX[i], s->nx), yy = y + EY[i];
  if (s->periodic_y) yy = wrapi(yy, s->ny);
  else if (yy < 0 || yy >= s->ny) {
    double ph = s->phi[y * s->nx + xx];
    double J = yy < 0 ? s->Jphi_b[xx] : s->Jphi_t[xx];
    return rho_of(s, ph + J / s->kappa);
  }
  return s->rho[yy * s->nx + xx];
}

/* Gauss-Jordan inverse with partial pivoting. */
static int invert9(double A[Q][Q], double Ainv[Q][Q]) {
  double a[Q][2 * Q];
  for (int r = 0; r < Q; ++r)
    for (int c = 0; c < 2 * Q; ++c) a[r][c] = c < Q ? A[r][c] : (c - Q == r ? 1.0 : 0.0);
  for (int c = 0; c < Q; ++c) {
    int piv = c;
    for (int r = c + 1; r < Q; ++r)
      if (fabs(a[r][c]) > fabs(a[piv][c])) piv = r;
    if (fabs(a[piv][c]) < 1e-14) return -1;
    if (piv != c)
      for (int k = 0; k < 2 * Q; ++k) { double t = a[c][k]; a[c][k] = a[piv][k]; a[piv][k] = t; }
    double d = a[c][c];
    for (int k = 0; k < 2 * Q; ++k) a[c][k] /= d;
    for (int r = 0; r < Q; ++r)
      if (r != c) {
        double m = a[r][c];
        for (int k = 0; k < 2 * Q; ++k) a[r][k] -= m * a[c][k];
      }
  }
  for (int r = 0; r < Q; ++r)
    for (int c = 0; c < Q; ++c) Ainv[r][c] = a[r][Q + c];
  return 0;
}

/* MRT collision (Sec. 3): out = x - M^-1 S M (x - x_eq) + M^-1 (I - S/2) M v
 * [+ w_i * extra].  rates[k] is the rate of moment row k. */
static void mrt_collide(const orc_sim* s, const double* x, const double* xeq, const double* v,
                        const double* rates, double extra, double* out) {
  double m[Q], me[Q], mv[Q], ms[Q];
  for (int k = 0; k < Q; ++k) {
    m[k] = me[k] = mv[k] = 0.0;
    for (int i = 0; i < Q; ++i) {
      m[k] += s->Mm[k][i] * x[i];
      me[k] += s->Mm[k][i] * xeq[i];
      mv[k] += s->Mm[k][i] * v[i];
    }
  }
  for (int k = 0; k < Q; ++k) ms[k] = m[k] - rates[k] * (m[k] - me[k]) + (1.0 - 0.5 * rates[k]) * mv[k];
  for (int i = 0; i < Q; ++i) {
    double acc = 0.0;
    for (int k = 0; k < Q; ++k) acc += s->Mi[i][k] * ms[k];
    out[i] = acc + WQ[i] * extra;
  }
}

/* Equilibria (Sec. 3): pressure-based f_eq and the eta-weighted g_eq / h_eq. */
static void feq_flow(double pr, double rho, double ux, double uy, double* out) {
  for (int i = 0; i < Q; ++i) {
    double cu = EX[i] * ux + EY[i] * uy, uu = ux * ux + uy * uy;
    double su = cu / CS2 + cu * cu / (2.0 * CS2 * CS2) - uu / (2.0 * CS2);
    out[i] = pr / CS2 * (WQ[i] - (i == 0 ? 1.0 : 0.0)) + rho * WQ[i] * su;
  }
}
static void feq_scalar(double c, double eta, double cux, double cuy, double* out) {
  out[0] = c + (WQ[0] - 1.0) * eta * c;
  for (int i = 1; i < Q; ++i) out[i] = WQ[i] * eta * c + WQ[i] * (EX[i] * cux + EY[i] * cuy) / CS2;
}

/* ------------------------------------------------------- manufactured case */
/* Exact solution of the accuracy test (Sec. 4.1) on [0,1]^2 at physical time t. */
static double mms_phi(double x, double y, double t) {
  return 0.5 * exp(-t) * sin(2.0 * M_PI * (x - 0.05 * t)) * cos(2.0 * M_PI * (y + 0.03 * t));
}
static double mms_psi(double x, double y, double t) {
  return 0.5 + 0.05 * exp(-2.0 * t) * cos(2.0 * M_PI * (x - 0.05 * t)) * sin(2.0 * M_PI * (y + 0.03 * t));
}
static double mms_dt(const orc_sim* s) { return s->p.mms_dx * s->p.mms_dx / 0.15; }
/* Lattice-unit source dt*S for phi and psi at node (x,y), step n: the exact
 * chemical potentials (Laplacian of the exact phi is -8 pi^2 phi) and their
 * stated spatial means, with physical mobility M = M_lu / dt. */
static void mms_source(const orc_sim* s, int x, int y, int64_t n, double* sphi, double* spsi) {
  double dx = s->p.mms_dx, dt = mms_dt(s), t = (double)n * dt;
  double X = x * dx, Y = y * dx;
  double ph = mms_phi(X, Y, t), ps = mms_psi(X, Y, t);
  double kap_phys = s->kappa * dx * dx;
  double mu_phi = 4.0 * s->beta * (1.0 - ps) * (ph * ph * ph - ph) + kap_phys * 8.0 * M_PI * M_PI * ph + s->W * ps * ph;
  double mu_psi = s->kBT * log(ps / (1.0 - ps)) - s->beta * (1.0 - ph * ph) * (1.0 - ph * ph) + 0.5 * s->W * ph * ph;
  double a = 0.5 * exp(-t);
  double mubar_psi = -s->beta * (1.0 - a * a / 2.0 + 9.0 * a * a * a * a / 64.0) + s->W * a * a / 8.0;
  *sphi = -dt * ph + s->p.M_phi * (mu_phi - 0.0);
  *spsi = -dt * 2.0 * (ps - 0.5) + s->p.M_psi * (mu_psi - mubar_psi);
}
static double mms_u_lattice(const orc_sim* s, double u_phys) { return u_phys * mms_dt(s) / s->p.mms_dx; }

/* ------------------------------------------------------------ construction */
static void set_err(char* err, int errlen, const char* msg) {
  if (err && errlen > 0) { strncpy(err, msg, (size_t)errlen - 1); err[errlen - 1] = 0; }
}
static double rate_or(double v, double dflt) { return v > 0.0 ? v : dflt; }

static int derive(orc_sim* s, char* err, int errlen) {
  const orc_params* p = &s->p;
  int wet = p->bc_bottom == ORC_WALL_WET || p->bc_top == ORC_WALL_WET;
  s->surf = p->psi_b > 0.0;
  s->kappa = 3.0 * p->eps * p->sigma_gl0 / 8.0;
  s->beta = 3.0 * p->sigma_gl0 / (4.0 * p->eps);
  s->W = p->W > 0.0 ? p->W : 4.0 * s->beta / (p->Ex > 0.0 ? p->Ex : 0.5);
  s->kBT = p->kBT > 0.0 ? p->kBT : 4.0 * s->beta * (p->Pi > 0.0 ? p->Pi : 1.35);
  if (p->phi_b > 0.0) s->phib = p->phi_b;
  else if (s->surf) {
    double b2 = 1.0 - s->W * p->psi_b / (4.0 * s->beta * (1.0 - p->psi_b));
    if (!(b2 > 0.0)) { set_err(err, errlen, "bulk surfactant too large: phi_b^2 <= 0"); return -1; }
    s->phib = sqrt(b2);
  } else s->phib = 1.0;
  if (p->sigma_sg0 >= 0.0 && p->sigma_sl0 >= 0.0) { s->sg0 = p->sigma_sg0; s->sl0 = p->sigma_sl0; }
  else {
    double c = p->sigma_gl0 * cos(p->theta0_deg * M_PI / 180.0), sum = 16.0 * p->sigma_gl0 / 15.0;
    s->sg0 = 0.5 * (sum + c);
    s->sl0 = 0.5 * (sum - c);
  }
  s->lambda_s = p->lambda_s >= 0.0 ? p->lambda_s : (wet ? 0.5 * s->kappa : 0.0);
  s->M0 = p->M0 >= 0.0 ? p->M0 : (s->lambda_s > 0.0 ? 0.0 : p->M_phi * s->kappa);
  double s1g = rate_or(p->s_g[1], 1.0), s1h = rate_or(p->s_h[1], 1.0);
  s->eta_phi = p->eta_phi > 0.0 ? p->eta_phi : p->M_phi * s->kappa / (CS2 * (1.0 / s1g - 0.5));
  s->eta_psi = p->eta_psi > 0.0 ? p->eta_psi : (p->M_psi * s->lambda_s + s->M0) / (CS2 * (1.0 / s1h - 0.5));
  s->psi_c = exp(-(s->beta + 0.5 * s->W) / s->kBT);
  if (wet && s->surf && s->lambda_s == 0.0 && (p->beta_sg != 0.0 || p->beta_sl != 0.0)) {
    set_err(err, errlen, "lambda_s = 0 cannot carry the solid-adsorption boundary condition");
    return -1;
  }
  return 0;
}

static int validate(const orc_params* p, char* err, int errlen) {
  if (p->nx < 3 || p->ny < 3) { set_err(err, errlen, "nx and ny must be >= 3"); return -1; }
  if (p->bc_bottom < 0 || p->bc_bottom > 3 || p->bc_top < 0 || p->bc_top > 3) { set_err(err, errlen, "bad boundary kind"); return -1; }
  if ((p->bc_bottom == ORC_PERIODIC) != (p->bc_top == ORC_PERIODIC)) { set_err(err, errlen, "periodic y needs both boundaries periodic"); return -1; }
  if (!(p->sigma_gl0 > 0.0) || !(p->eps > 0.0)) { set_err(err, errlen, "sigma_gl0 and eps must be > 0"); return -1; }
  if (!(p->M_phi >= 0.0) || !(p->M_psi >= 0.0)) { set_err(err, errlen, "mobilities must be >= 0"); return -1; }
  if (!(p->psi_b >= 0.0 && p->psi_b < 1.0)) { set_err(err, errlen, "psi_b must lie in [0,1)"); return -1; }
  if (!(p->rho_l > 0.0 && p->rho_g > 0.0 && p->mu_l > 0.0 && p->mu_g > 0.0)) { set_err(err, errlen, "densities and viscosities must be > 0"); return -1; }
  int wet = p->bc_bottom == ORC_WALL_WET || p->bc_top == ORC_WALL_WET;
  if (wet && !(p->theta0_deg > 0.0 && p->theta0_deg < 180.0)) { set_err(err, errlen, "theta0 must lie in (0,180)"); return -1; }
  const double* rs[3] = {p->s_f, p->s_g, p->s_h};
  for (int l = 0; l < 3; ++l)
    for (int k = 0; k < 5; ++k)
      if (rs[l][k] >= 2.0) { set_err(err, errlen, "relaxation rates must lie in (0,2)"); return -1; }
  if (p->constraint_phi != ORC_NONLINEAR && p->constraint_phi != ORC_LINEAR) { set_err(err, errlen, "bad constraint"); return -1; }
  if (p->mms && (p->bc_bottom != ORC_PERIODIC || !(p->mms_dx > 0.0))) { set_err(err, errlen, "manufactured mode needs periodic boundaries and mms_dx"); return -1; }
  return 0;
}

static double* zalloc(size_t n) { return (double*)calloc(n, sizeof(double)); }

static void init_fields(orc_sim* s) {
  int nx = s->nx, ny = s->ny;
  double* ph = zalloc(s->N);
  double* ps = zalloc(s->N);
  double* ux = zalloc(s->N);
  double* uy = zalloc(s->N);
  const orc_params* p = &s->p;
  for (int y = 0; y < ny; ++y)
    for (int x = 0; x < nx; ++x) {
      int n = y * nx + x;
      if (p->mms) {
        double X = x * p->mms_dx, Y = y * p->mms_dx;
        ph[n] = mms_phi(X, Y, 0.0);
        ps[n] = mms_psi(X, Y, 0.0);
        ux[n] = mms_u_lattice(s, 0.05);
        uy[n] = mms_u_lattice(s, -0.03);
        continue;
      }
      /* signed distance, positive inside the liquid, minimum image in periodic directions */
      double dx = x - p->x0, dy = y - p->y0;
      dx -= nx * floor(dx / nx + 0.5);
      if (s->periodic_y) dy -= ny * floor(dy / ny + 0.5);
      double d;
      if (p->init_kind == ORC_INIT_SLAB) d = 0.5 * p->a - fabs(dx);
      else if (p->init_kind == ORC_INIT_BUBBLE) d = sqrt(dx * dx + dy * dy) - p->R0;
      else d = p->R0 - sqrt(dx * dx + dy * dy);
      /* equilibrium profile with bulk surfactant (Sec. 2.2) */
      double sq = s->surf ? sqrt(1.0 - p->psi_b) : 1.0;
      ph[n] = s->phib * tanh(2.0 * s->phib * sq * d / p->eps);
      ps[n] = s->surf ? p->psi_b : 0.0;
    }
  orc_load_fields(s, ph, ps, p->mms ? ux : NULL, p->mms ? uy : NULL);
  free(ph); free(ps); free(ux); free(uy);
}

orc_sim* orc_create(const orc_params* p, char* err, int errlen) {
  if (validate(p, err, errlen)) return NULL;
  orc_sim* s = (orc_sim*)calloc(1, sizeof(orc_sim));
  s->p = *p;
  s->nx = p->nx; s->ny = p->ny; s->N = p->nx * p->ny;
  s->periodic_y = p->bc_bottom == ORC_PERIODIC;
  if (derive(s, err, errlen)) { free(s); return NULL; }
  for (int k = 0; k < Q; ++k)
    for (int i = 0; i < Q; ++i) s->Mm[k][i] = powi(EX[i], MA[k]) * powi(EY[i], MB[k]);
  if (invert9(s->Mm, s->Mi)) { set_err(err, errlen, "moment matrix singular"); free(s); return NULL; }
  size_t N = (size_t)s->N;
  s->f = zalloc(Q * N); s->g = zalloc(Q * N); s->h = zalloc(Q * N);
  s->fn = zalloc(Q * N); s->gn = zalloc(Q * N); s->hn = zalloc(Q * N);
  double** work[] = {&s->phi_h, &s->psi_h, &s->ux_h, &s->uy_h, &s->Rphi_h, &s->Rpsi_h,
                     &s->phi, &s->psi, &s->mu_phi, &s->mu_psi, &s->lap0_psi, &s->Tphi, &s->Tpsi,
                     &s->rho, &s->ux, &s->uy, &s->pr, &s->Fx, &s->Fy, &s->grx, &s->gry,
                     &s->Rphi, &s->Rpsi, &s->vx, &s->vy, &s->vx_h, &s->vy_h};
  for (size_t k = 0; k < sizeof(work) / sizeof(work[0]); ++k) *work[k] = zalloc(N);
  s->Jphi_b = zalloc(s->nx); s->Jpsi_b = zalloc(s->nx); s->Jphi_t = zalloc(s->nx); s->Jpsi_t = zalloc(s->nx);
  init_fields(s);   /* also sets m_ref */
  return s;
}

void orc_destroy(orc_sim* s) {
  if (!s) return;
  double* ptrs[] = {s->f, s->g, s->h, s->fn, s->gn, s->hn, s->phi_h, s->psi_h, s->ux_h, s->uy_h,
                    s->Rphi_h, s->Rpsi_h, s->phi, s->psi, s->mu_phi, s->mu_psi, s->lap0_psi,
                    s->Tphi, s->Tpsi, s->rho, s->ux, s->uy, s->pr, s->Fx, s->Fy, s->grx, s->gry,
                    s->Rphi, s->Rpsi, s->Jphi_b, s->Jpsi_b, s->Jphi_t, s->Jpsi_t, s->vx, s->vy, s->vx_h, s->vy_h};
  for (size_t k = 0; k < sizeof(ptrs) / sizeof(ptrs[0]); ++k) free(ptrs[k]);
  free(s);
}

void orc_derived(const orc_sim* s, double* out) {
  double v[ORC_N_DERIVED] = {s->kappa, s->beta, s->W, s->kBT, s->phib, s->sg0, s->sl0,
                             s->lambda_s, s->M0, s->eta_phi, s->eta_psi, s->psi_c};
  memcpy(out, v, sizeof(v));
}

void orc_load_fields(orc_sim* s, const double* phi, const double* psi, const double* ux, const double* uy) {
  int N = s->N;
  double fe[Q], ge[Q], he[Q];
  for (int n = 0; n < N; ++n) {
    double u = ux ? ux[n] : 0.0, v = uy ? uy[n] : 0.0;
    feq_flow(0.0, rho_of(s, phi[n]), u, v, fe);
    if (!ux) for (int i = 0; i < Q; ++i) fe[i] = 0.0; /* u = 0, p = 0 gives f = 0 */
    feq_scalar(phi[n], s->eta_phi, phi[n] * u, phi[n] * v, ge);
    feq_scalar(s->surf ? psi[n] : 0.0, s->eta_psi, psi[n] * u, psi[n] * v, he);
    for (int i = 0; i < Q; ++i) {
      s->f[i * N + n] = fe[i];
      s->g[i * N + n] = ge[i];
      s->h[i * N + n] = s->surf ? he[i] : 0.0;
    }
  }
  s->have_hist = 0;
  s->m_ref = sum_h(s, phi);
}

void orc_get_populations(const orc_sim* s, double* out) {
  size_t N = (size_t)s->N;
  memcpy(out, s->f, Q * N * sizeof(double));
  memcpy(out + Q * N, s->g, Q * N * sizeof(double));
  memcpy(out + 2 * Q * N, s->h, Q * N * sizeof(double));
}

/* -------------------------------------------------------------- the step */
/* O1-O6 at the current state: everything the collision needs except the
 * multipliers, plus the multipliers themselves (O4). */
static void macro(orc_sim* s) {
  int nx = s->nx, ny = s->ny, N = s->N;
  /* O1: zeroth moments */
#pragma omp parallel for if (g_parallel && s->N >= ORC_PAR_MIN_NODES)
  for (int n = 0; n < N; ++n) {
    double a = 0.0, b = 0.0;
    for (int i = 0; i < Q; ++i) { a += s->g[i * N + n]; b += s->h[i * N + n]; }
    s->phi[n] = a;
    s->psi[n] = s->surf ? b : 0.0;
    s->rho[n] = rho_of(s, a);
  }
  /* O2: wall fluxes J = -df_w/dphi, -df_w/dpsi at the fluid node next to a wetting wall */
  for (int x = 0; x < nx; ++x) {
    s->Jphi_b[x] = s->Jpsi_b[x] = s->Jphi_t[x] = s->Jpsi_t[x] = 0.0;
    if (s->p.bc_bottom == ORC_WALL_WET) {
      double ph = s->phi[x], ps = s->psi[x];
      s->Jphi_b[x] = wall_Jphi(s, ph, ps);
      s->Jpsi_b[x] = s->surf ? wall_Jpsi(s, ph, ps) : 0.0;
    }
    if (s->p.bc_top == ORC_WALL_WET) {
      double ph = s->phi[(ny - 1) * nx + x], ps = s->psi[(ny - 1) * nx + x];
      s->Jphi_t[x] = wall_Jphi(s, ph, ps);
      s->Jpsi_t[x] = s->surf ? wall_Jpsi(s, ph, ps) : 0.0;
    }
  }
  /* O3: chemical potentials; Laplacian = zero-flux part L0 plus the wall term T */
#pragma omp parallel for if (g_parallel && s->N >= ORC_PAR_MIN_NODES)
  for (int y = 0; y < ny; ++y)
    for (int x = 0; x < nx; ++x) {
      int n = y * nx + x;
      double ph = s->phi[n], ps = s->psi[n];
      double l0p = 0.0, l0s = 0.0;
      for (int i = 1; i < Q; ++i) {
        l0p += 2.0 * WQ[i] / CS2 * (nb_mirror(s, s->phi, x, y, i) - ph);
        l0s += 2.0 * WQ[i] / CS2 * (nb_mirror(s, s->psi, x, y, i) - ps);
      }
      double tp = wall_T(s, s->Jphi_b, s->Jphi_t, x, y);
      double ts = wall_T(s, s->Jpsi_b, s->Jpsi_t, x, y);
      s->Tphi[n] = tp;
      s->Tpsi[n] = ts;
      s->lap0_psi[n] = l0s;
      s->mu_phi[n] = 4.0 * s->beta * (1.0 - ps) * (ph * ph * ph - ph) - s->kappa * l0p - tp + s->W * ps * ph;
      if (s->surf)
        s->mu_psi[n] = s->kBT * log(ps / (1.0 - ps)) - s->lambda_s * l0s - ts
                     - s->beta * (1.0 - ph * ph) * (1.0 - ph * ph) + 0.5 * s->W * ph * ph;
      else s->mu_psi[n] = 0.0;
    }
  /* O4: global multipliers, sequential FP64 sums in row-major order */
  double S1 = 0.0, S2 = 0.0, S3 = 0.0, S4 = 0.0;
  for (int n = 0; n < N; ++n) {
    double hp = hprime(s, s->phi[n]);
    S1 += hp * s->mu_phi[n];
    S2 += hp * hp;
    S3 += s->mu_psi[n];
    S4 += hval(s, s->phi[n]);
  }
  s->lambda = S2 > 0.0 ? S1 / S2 : 0.0;
  /* Optional reading: eq15 keeps d/dt of sum h_phi at zero in continuous time,
   * but the discrete step lets sum h_phi drift (the phi lattice's own diffusion
   * is not the stencil Laplacian inside mu_phi that eq15 sees).  With phi_hold
   * the multiplier also takes back the accumulated drift, (m_ref - S4) / (M S2),
   * so that sum h_phi stays at its initial value as the paper states it does. */
  if (s->p.phi_hold && S2 > 0.0 && s->p.M_phi > 0.0) s->lambda += (s->m_ref - S4) / (s->p.M_phi * S2);
  s->mubar = S3 / N;
  /* O5, O6: gradients, force, velocity, pressure */
#pragma omp parallel for if (g_parallel && s->N >= ORC_PAR_MIN_NODES)
  for (int y = 0; y < ny; ++y)
    for (int x = 0; x < nx; ++x) {
      int n = y * nx + x;
      double grx = 0, gry = 0, gmpx = 0, gmpy = 0, gmsx = 0, gmsy = 0;
      for (int i = 1; i < Q; ++i) {
        double r = nb_rho(s, x, y, i);
        double mp = nb_mirror(s, s->mu_phi, x, y, i), ms = nb_mirror(s, s->mu_psi, x, y, i);
        grx += WQ[i] * EX[i] * r / CS2;  gry += WQ[i] * EY[i] * r / CS2;
        gmpx += WQ[i] * EX[i] * mp / CS2; gmpy += WQ[i] * EY[i] * mp / CS2;
        gmsx += WQ[i] * EX[i] * ms / CS2; gmsy += WQ[i] * EY[i] * ms / CS2;
      }
      double ph = s->phi[n], ps = s->psi[n], rho = s->rho[n];
      double Fx = -ph * gmpx - ps * gmsx + rho * s->p.gx;
      double Fy = -ph * gmpy - ps * gmsy + rho * s->p.gy;
      s->grx[n] = grx; s->gry[n] = gry; s->Fx[n] = Fx; s->Fy[n] = Fy;
      if (s->p.mms) {
        s->ux[n] = mms_u_lattice(s, 0.05);
        s->uy[n] = mms_u_lattice(s, -0.03);
        s->pr[n] = 0.0;
        continue;
      }
      double jx = 0, jy = 0, sum_nz = 0;
      for (int i = 0; i < Q; ++i) {
        double fi = s->f[i * N + n];
        jx += EX[i] * fi; jy += EY[i] * fi;
        if (i) sum_nz += fi;
      }
      double ux = (jx + 0.5 * Fx) / rho, uy = (jy + 0.5 * Fy) / rho;
      s->ux[n] = ux; s->uy[n] = uy;
      s->pr[n] = CS2 / (1.0 - WQ[0]) * (sum_nz + 0.5 * (ux * grx + uy * gry) - rho * WQ[0] * (ux * ux + uy * uy) / (2.0 * CS2));
    }
}

static void step_once(orc_sim* s) {
  int nx = s->nx, ny = s->ny, N = s->N;
  macro(s);
  /* O7: sources (with the wall-flux terms on wall rows), then the identities'
   * sums in node order */
#pragma omp parallel for if (g_parallel && s->N >= ORC_PAR_MIN_NODES)
  for (int n = 0; n < N; ++n) {
    double ph = s->phi[n], ps = s->psi[n], hp = hprime(s, ph);
    s->Rphi[n] = s->p.M_phi * (-4.0 * s->beta * (1.0 - ps) * (ph * ph * ph - ph) - s->W * ps * ph + s->lambda * hp)
               + s->p.M_phi * s->Tphi[n];
    if (s->surf)
      s->Rpsi[n] = -s->M0 * s->lap0_psi[n]
                 + s->p.M_psi * (-s->kBT * log(ps / (1.0 - ps)) + s->beta * (1.0 - ph * ph) * (1.0 - ph * ph)
                                 - 0.5 * s->W * ph * ph + s->mubar)
                 + s->p.M_psi * s->Tpsi[n];
    else s->Rpsi[n] = 0.0;
    if (s->p.mms) {
      int x = n % nx, y = n / nx;
      double sp, ss;
      mms_source(s, x, y, s->step, &sp, &ss);
      s->Rphi[n] += sp;
      s->Rpsi[n] += ss;
    }
  }
  double sumR = 0.0, orth = 0.0;
  for (int n = 0; n < N; ++n) {
    double hp = hprime(s, s->phi[n]);
    sumR += s->Rpsi[n];
    orth += hp * (s->mu_phi[n] - s->lambda * hp);
  }
  s->sumRpsi_last = sumR;
  s->orth_last = orth;
  /* O8: collisions */
#pragma omp parallel for if (g_parallel && s->N >= ORC_PAR_MIN_NODES)
  for (int n = 0; n < N; ++n) {
    double ph = s->phi[n], ps = s->psi[n], rho = s->rho[n], ux = s->ux[n], uy = s->uy[n];
    double x[Q], xe[Q], v[Q], out[Q], rates[Q];
    /* velocity that advects phi and psi (reading: mean of this and the
     * previous step, which removes the lattice's period-2 staggered
     * momentum from the scalar transport; the literal reading uses u) */
    double vx = ux, vy = uy;
    if (!s->p.adv_raw && s->have_hist) { vx = 0.5 * (ux + s->ux_h[n]); vy = 0.5 * (uy + s->uy_h[n]); }
    s->vx[n] = vx;
    s->vy[n] = vy;
    /* backward differences of phi v, psi v and R (first step: zero) */
    double dpx = 0, dpy = 0, dsx = 0, dsy = 0, dRp = 0, dRs = 0;
    if (s->have_hist) {
      dpx = ph * vx - s->phi_h[n] * s->vx_h[n];
      dpy = ph * vy - s->phi_h[n] * s->vy_h[n];
      dsx = ps * vx - s->psi_h[n] * s->vx_h[n];
      dsy = ps * vy - s->psi_h[n] * s->vy_h[n];
      dRp = s->Rphi[n] - s->Rphi_h[n];
      dRs = s->Rpsi[n] - s->Rpsi_h[n];
    }
    /* flow lattice */
    if (!s->p.mms) {
      double s2 = s->p.s_f[2] > 0.0 ? s->p.s_f[2] : 1.0 / (3.0 * mud_of(s, ph) / rho + 0.5);
      double sf[5] = {rate_or(s->p.s_f[0], 1.0), rate_or(s->p.s_f[1], 1.0), s2,
                      rate_or(s->p.s_f[3], 1.0), rate_or(s->p.s_f[4], 1.0)};
      for (int k = 0; k < Q; ++k) rates[k] = sf[MORDER[k]];
      for (int i = 0; i < Q; ++i) x[i] = s->f[i * N + n];
      feq_flow(s->pr[n], rho, ux, uy, xe);
      double ugr = ux * s->grx[n] + uy * s->gry[n];
      for (int i = 0; i < Q; ++i) {
        double cu = EX[i] * ux + EY[i] * uy, cg = EX[i] * s->grx[n] + EY[i] * s->gry[n];
        double cF = EX[i] * s->Fx[n] + EY[i] * s->Fy[n];
        v[i] = WQ[i] * (ugr + cF / CS2 + (cu * cg - CS2 * ugr) / CS2);
      }
      mrt_collide(s, x, xe, v, rates, 0.0, out);
      for (int i = 0; i < Q; ++i) s->f[i * N + n] = out[i];
    }
    /* phase-field lattice */
    {
      double sg[5];
      for (int k = 0; k < 5; ++k) sg[k] = rate_or(s->p.s_g[k], 1.0);
      for (int k = 0; k < Q; ++k) rates[k] = sg[MORDER[k]];
      for (int i = 0; i < Q; ++i) x[i] = s->g[i * N + n];
      feq_scalar(ph, s->eta_phi, ph * vx, ph * vy, xe);
      for (int i = 0; i < Q; ++i) v[i] = WQ[i] * (EX[i] * dpx + EY[i] * dpy) / CS2;
      mrt_collide(s, x, xe, v, rates, s->Rphi[n] + 0.5 * dRp, out);
      for (int i = 0; i < Q; ++i) s->g[i * N + n] = out[i];
    }
    /* surfactant lattice */
    if (s->surf) {
      double sh[5];
      for (int k = 0; k < 5; ++k) sh[k] = rate_or(s->p.s_h[k], 1.0);
      for (int k = 0; k < Q; ++k) rates[k] = sh[MORDER[k]];
      for (int i = 0; i < Q; ++i) x[i] = s->h[i * N + n];
      feq_scalar(ps, s->eta_psi, ps * vx, ps * vy, xe);
      for (int i = 0; i < Q; ++i) v[i] = WQ[i] * (EX[i] * dsx + EY[i] * dsy) / CS2;
      mrt_collide(s, x, xe, v, rates, s->Rpsi[n] + 0.5 * dRs, out);
      for (int i = 0; i < Q; ++i) s->h[i * N + n] = out[i];
    }
  }
  /* O9: streaming (a permutation of the population slots: rows write disjoint targets) */
#pragma omp parallel for if (g_parallel && s->N >= ORC_PAR_MIN_NODES)
  for (int y = 0; y < ny; ++y)
    for (int x = 0; x < nx; ++x) {
      int n = y * nx + x;
      for (int i = 0; i < Q; ++i) {
        int xx = wrapi(x + EX[i], nx), yy = y + EY[i];
        if (s->periodic_y || (yy >= 0 && yy < ny)) {
          int m = wrapi(yy, ny) * nx + xx;
          s->fn[i * N + m] = s->f[i * N + n];
          s->gn[i * N + m] = s->g[i * N + n];
          s->hn[i * N + m] = s->h[i * N + n];
          continue;
        }
        int bc = yy < 0 ? s->p.bc_bottom : s->p.bc_top;
        double uw = yy < 0 ? s->p.u_wall_bottom : s->p.u_wall_top;
        s->gn[OPP[i] * N + n] = s->g[i * N + n];
        s->hn[OPP[i] * N + n] = s->h[i * N + n];
        if (bc == ORC_FREESLIP) {
          s->fn[MIRY[i] * N + y * nx + xx] = s->f[i * N + n];
        } else {
          s->fn[OPP[i] * N + n] = s->f[i * N + n] - 2.0 * WQ[i] * s->rho[n] * (EX[i] * uw) / CS2;
        }
      }
    }
  double* t;
  t = s->f; s->f = s->fn; s->fn = t;
  t = s->g; s->g = s->gn; s->gn = t;
  t = s->h; s->h = s->hn; s->hn = t;
  /* O10: history */
  memcpy(s->phi_h, s->phi, N * sizeof(double));
  memcpy(s->psi_h, s->psi, N * sizeof(double));
  memcpy(s->ux_h, s->ux, N * sizeof(double));
  memcpy(s->uy_h, s->uy, N * sizeof(double));
  memcpy(s->vx_h, s->vx, N * sizeof(double));
  memcpy(s->vy_h, s->vy, N * sizeof(double));
  memcpy(s->Rphi_h, s->Rphi, N * sizeof(double));
  memcpy(s->Rpsi_h, s->Rpsi, N * sizeof(double));
  s->have_hist = 1;
  s->step += 1;
}

void orc_step(orc_sim* s, int64_t n) {
  for (int64_t k = 0; k < n; ++k) step_once(s);
}

void orc_fields(orc_sim* s, uint32_t mask, double* out) {
  macro(s);
  const double* src[8] = {s->phi, s->psi, s->ux, s->uy, s->pr, s->rho, s->mu_phi, s->mu_psi};
  size_t N = (size_t)s->N, k = 0;
  for (int b = 0; b < 8; ++b)
    if (mask & (1u << b)) memcpy(out + (k++) * N, src[b], N * sizeof(double));
}

/* -------------------------------------------------------------- diagnostics */
/* Fraction of a linear triangle where the interpolant is positive. */
static double tri_frac(double a, double b, double c) {
  int np = (a > 0) + (b > 0) + (c > 0);
  if (np == 3) return 1.0;
  if (np == 0) return 0.0;
  double v[3] = {a, b, c};
  if (np == 1) {
    int k = a > 0 ? 0 : (b > 0 ? 1 : 2);
    double p = v[k], q = v[(k + 1) % 3], r = v[(k + 2) % 3];
    return p * p / ((p - q) * (p - r));
  }
  int k = a <= 0 ? 0 : (b <= 0 ? 1 : 2);
  double m = v[k], q = v[(k + 1) % 3], r = v[(k + 2) % 3];
  return 1.0 - m * m / ((m - q) * (m - r));
}
/* Positive length fraction of a linear segment. */
static double seg_frac(double a, double b) {
  if (a > 0 && b > 0) return 1.0;
  if (a <= 0 && b <= 0) return 0.0;
  return a > 0 ? a / (a - b) : b / (b - a);
}

/* Area of {phi > 0} from the two-triangle linear reconstruction of each cell
 * (Sec. 4.1); with walls, the half cells between a wall and the first fluid
 * row count by the 1-D reconstruction along that row. */
double orc_area_positive(const double* phi, int nx, int ny, int wall_bottom, int wall_top, int periodic_y) {
  double A = 0.0;
  int ycells = periodic_y ? ny : ny - 1;
  for (int y = 0; y < ycells; ++y)
    for (int x = 0; x < nx; ++x) {
      int x1 = (x + 1) % nx, y1 = (y + 1) % ny;
      double a = phi[y * nx + x], b = phi[y * nx + x1], c = phi[y1 * nx + x1], d = phi[y1 * nx + x];
      A += 0.5 * tri_frac(a, b, c) + 0.5 * tri_frac(a, c, d);
    }
  if (!periodic_y) {
    for (int x = 0; x < nx; ++x) {
      int x1 = (x + 1) % nx;
      if (wall_bottom) A += 0.5 * seg_frac(phi[x], phi[x1]);
      if (wall_top) A += 0.5 * seg_frac(phi[(ny - 1) * nx + x], phi[(ny - 1) * nx + x1]);
    }
  }
  return A;
}

/* Contact width at the bottom wall (y = -1/2): the positive length of the
 * first and second rows (zero crossings by linear interpolation) extrapolated
 * linearly to the wall; cap height above the wall of the highest phi = 0
 * crossing of a liquid column; apparent angle 2 atan(2H/L) of a circular cap
 * (Sec. 4.3, eq. a).  A drop that left the wall has L = 0 and angle 180. */
void orc_contact(const double* phi, int nx, int ny, double* width, double* height, double* theta_deg) {
  double L0 = 0.0, L1 = 0.0, H = 0.0;
  for (int x = 0; x < nx; ++x) {
    L0 += seg_frac(phi[x], phi[(x + 1) % nx]);
    L1 += seg_frac(phi[nx + x], phi[nx + (x + 1) % nx]);
  }
  double L = L0 > 0.0 ? L0 + 0.5 * (L0 - L1) : 0.0;
  if (L < 0.0) L = 0.0;
  for (int x = 0; x < nx; ++x) {
    if (!(phi[x] > 0)) continue;
    double hx = ny - 0.5;
    for (int y = 0; y + 1 < ny; ++y) {
      double a = phi[y * nx + x], b = phi[(y + 1) * nx + x];
      if (a > 0 && b <= 0) { hx = y + a / (a - b) + 0.5; break; }
    }
    if (hx > H) H = hx;
  }
  *width = L;
  *height = H;
  *theta_deg = L > 0.0 ? 2.0 * atan(2.0 * H / L) * 180.0 / M_PI : 180.0;
}

void orc_invariants(orc_sim* s, orc_inv* out) {
  int nx = s->nx, ny = s->ny;
  macro(s);
  memset(out, 0, sizeof(*out));
  out->step = s->step;
  double Ef = 0.0;
  for (int y = 0; y < ny; ++y)
    for (int x = 0; x < nx; ++x) {
      int n = y * nx + x;
      double ph = s->phi[n], ps = s->psi[n], ux = s->ux[n], uy = s->uy[n];
      if (!isfinite(ph) || !isfinite(ps) || !isfinite(ux) || !isfinite(uy) || !isfinite(s->pr[n])) out->nonfinite++;
      if (s->surf && !(ps > 0.0 && ps < 1.0)) out->psi_out_of_range++;
      out->mass_psi += ps;
      out->m_phi_h += 0.5 + gsw(s, ph);
      out->sum_phi += ph;
      double u2 = ux * ux + uy * uy;
      out->kinetic += 0.5 * s->rho[n] * u2;
      if (sqrt(u2) > out->umax) out->umax = sqrt(u2);
      /* free-energy density with isotropic gradients; ghosts from the wall BCs */
      double gpx = 0, gpy = 0, gsx = 0, gsy = 0;
      for (int i = 1; i < Q; ++i) {
        int xx = wrapi(x + EX[i], nx), yy = y + EY[i];
        double vp, vs;
        if (s->periodic_y || (yy >= 0 && yy < ny)) {
          int m = wrapi(yy, ny) * nx + xx;
          vp = s->phi[m]; vs = s->psi[m];
        } else {
          int m = y * nx + xx;
          double Jp = yy < 0 ? s->Jphi_b[xx] : s->Jphi_t[xx];
          double Js = yy < 0 ? s->Jpsi_b[xx] : s->Jpsi_t[xx];
          vp = s->phi[m] + Jp / s->kappa;
          vs = s->psi[m] + (s->lambda_s > 0.0 ? Js / s->lambda_s : 0.0);
        }
        gpx += WQ[i] * EX[i] * vp / CS2; gpy += WQ[i] * EY[i] * vp / CS2;
        gsx += WQ[i] * EX[i] * vs / CS2; gsy += WQ[i] * EY[i] * vs / CS2;
      }
      double e = s->beta * (ph * ph - 1.0) * (ph * ph - 1.0) + 0.5 * s->kappa * (gpx * gpx + gpy * gpy);
      if (s->surf)
        e += s->kBT * (ps * log(ps) + (1.0 - ps) * log(1.0 - ps)) + 0.5 * s->lambda_s * (gsx * gsx + gsy * gsy)
           - s->beta * ps * (1.0 - ph * ph) * (1.0 - ph * ph) + 0.5 * s->W * ps * ph * ph;
      Ef += e;
    }
  for (int x = 0; x < nx; ++x) {
    int rows[2] = {0, ny - 1};
    int bcs[2] = {s->p.bc_bottom, s->p.bc_top};
    for (int w = 0; w < 2; ++w) {
      if (bcs[w] != ORC_WALL_WET) continue;
      int n = rows[w] * nx + x;
      Ef += wall_fw(s, s->phi[n], s->psi[n]);
      if (s->surf) {
        double l = log(1.0 - s->psi[n]);
        if (s->p.beta_sg > 0.0 && 1.0 + s->p.beta_sg * l <= 0.5) out->cap_violations++;
        if (s->p.beta_sl > 0.0 && 1.0 + s->p.beta_sl * l <= 0.5) out->cap_violations++;
      }
    }
  }
  out->free_energy = Ef;
  out->area_phi_pos = orc_area_positive(s->phi, nx, ny, is_wall(s->p.bc_bottom), is_wall(s->p.bc_top), s->periodic_y);
  out->lambda_phi = s->lambda;
  out->mubar_psi = s->mubar;
  if (is_wall(s->p.bc_bottom)) orc_contact(s->phi, nx, ny, &out->contact_width, &out->cap_height, &out->theta_app_deg);
  out->sum_R_psi = s->sumRpsi_last;
  out->orthogonality = s->orth_last;
}

void orc_mms_errors(orc_sim* s, double* e_phi, double* e_psi) {
  int nx = s->nx, ny = s->ny, N = s->N;
  double t = (double)s->step * mms_dt(s);
  double np = 0, dp = 0, ns = 0, ds = 0;
  for (int y = 0; y < ny; ++y)
    for (int x = 0; x < nx; ++x) {
      int n = y * nx + x;
      double a = 0, b = 0;
      for (int i = 0; i < Q; ++i) { a += s->g[i * N + n]; b += s->h[i * N + n]; }
      double pe = mms_phi(x * s->p.mms_dx, y * s->p.mms_dx, t), se = mms_psi(x * s->p.mms_dx, y * s->p.mms_dx, t);
      np += (a - pe) * (a - pe); dp += pe * pe;
      ns += (b - se) * (b - se); ds += se * se;
    }
  *e_phi = sqrt(np / dp);
  *e_psi = sqrt(ns / ds);
}

void orc_set_parallel(int on) { g_parallel = on ? 1 : 0; }

int orc_threads(void) {
#ifdef _OPENMP
  return omp_get_max_threads();
#else
  return 1;
#endif
}
