/*
 * lbm3d_oracle.c -- plain FP64 CPU oracle of one lattice Boltzmann time step
 * of the conservative Allen-Cahn / Navier-Stokes surfactant model with solid
 * adsorption (Huang, Chai, Liu, Huang) in three dimensions, on D3Q19.
 *
 * TEST INFRASTRUCTURE ONLY: the yardstick the HIP path is checked against.
 * Only the test suite, the smoke entry point and the CPU-baseline leg of the
 * benchmark may load it.  It shares no code with the HIP path.
 *
 * The model of Sec. 2 is stated for d = 2 and 3 and the unified MRT scheme of
 * Sec. 3 for a general velocity set: the steps are those of the 2-D oracle,
 *   O1  phi = sum_i g_i, psi = sum_i h_i                     (Sec. 3, macroscopic recovery)
 *   O2  wall values from the wetting / adsorption BCs        (Sec. 2.1, eq. "boundary")
 *   O3  chemical potentials                                   (eq_muphi, eq_mupsi)
 *   O4  multipliers lambda_phi, mubar_psi                     (eq15, AC_psi, AC_phi)
 *   O5  force F = -phi grad mu_phi - psi grad mu_psi + G      (eq_Fs0)
 *   O6  velocity and pressure                                 (Sec. 3)
 *   O7  sources and their backward differences                (Sec. 3)
 *   O8  MRT collision of the three populations                (Sec. 3)
 *   O9  streaming with periodic x, y and walls in z
 *   O10 history
 * on the D3Q19 velocity set with its isotropic weights (1/3, 1/18, 1/36), the
 * isotropic gradient and Laplacian of the end of Sec. 3 over its 18 moving
 * directions, and 19 raw moments c_x^a c_y^b c_z^c grouped by order (0; 1 x3;
 * 2 x6; 3 x6: the c_a^2 c_b with a != b; 4 x3: the c_a^2 c_b^2), relaxed with
 * diag(s0, s1, s2, s3, s4) by order.  Every open point is read as in the 2-D
 * oracle (advection by the two-step mean velocity unless adv_raw; rho and mu
 * linear in the liquid fraction held to [0, 1]; half-way bounce-back with a
 * ghost layer carrying phi + J_phi/kappa and the wall flux J_psi).
 *
 * Complex walls (orc3_set_solid): nodes marked solid hold no fluid.  A link
 * from a fluid node x to a solid node x + c_i is a half-way bounce-back wall for
 * all three lattices, and the stencils see a ghost value there taken at x
 * itself, link by link: mirror values for psi, mu_phi and mu_psi, and, on a
 * wetting solid, phi(x) + J_phi(x)/kappa with the wall flux J of x's own phi and
 * psi (eq. "boundary"); the wall term of a node is (2 w_i / c_s^2) J(x) summed
 * over its links into the solid.  Sums and means run over fluid nodes.  (The
 * flat z walls keep the column rule: a ghost takes the values of the fluid node
 * in its own column.)
 *
 * Plain loops, FP64, the generic 19x19 moment matrix and its numerically
 * computed inverse; global sums sequential in [z][y][x] order.
 */
#include "lbm3d_oracle.h"

#include <math.h>
#ifdef _OPENMP
#include <omp.h>
#endif
#include <stdlib.h>
#include <string.h>

#define Q 19
#define PAR_MIN_NODES 512   /* node loops on OpenMP threads from this size on (results do not depend on it) */

static int CV[Q][3];
static double WQ[Q];
static int OPP[Q], MIRZ[Q];
static const double CS2 = 1.0 / 3.0;
static int MEXP[Q][3], MORD[Q];
static int g_tables_ready = 0;

static void build_tables(void) {
  if (g_tables_ready) return;
  int k = 0;
  CV[k][0] = CV[k][1] = CV[k][2] = 0; WQ[k++] = 1.0 / 3.0;
  for (int a = 0; a < 3; ++a)
    for (int sgn = 1; sgn >= -1; sgn -= 2) {
      CV[k][0] = CV[k][1] = CV[k][2] = 0;
      CV[k][a] = sgn;
      WQ[k++] = 1.0 / 18.0;
    }
  for (int a = 0; a < 3; ++a)
    for (int b = a + 1; b < 3; ++b)
      for (int sa = 1; sa >= -1; sa -= 2)
        for (int sb = 1; sb >= -1; sb -= 2) {
          CV[k][0] = CV[k][1] = CV[k][2] = 0;
          CV[k][a] = sa;
          CV[k][b] = sb;
          WQ[k++] = 1.0 / 36.0;
        }
  for (int i = 0; i < Q; ++i)
    for (int j = 0; j < Q; ++j) {
      if (CV[j][0] == -CV[i][0] && CV[j][1] == -CV[i][1] && CV[j][2] == -CV[i][2]) OPP[i] = j;
      if (CV[j][0] == CV[i][0] && CV[j][1] == CV[i][1] && CV[j][2] == -CV[i][2]) MIRZ[i] = j;
    }
  /* raw moments grouped by order */
  static const int E[Q][3] = {{0, 0, 0}, {1, 0, 0}, {0, 1, 0}, {0, 0, 1},
                              {2, 0, 0}, {0, 2, 0}, {0, 0, 2}, {1, 1, 0}, {1, 0, 1}, {0, 1, 1},
                              {2, 1, 0}, {2, 0, 1}, {1, 2, 0}, {0, 2, 1}, {1, 0, 2}, {0, 1, 2},
                              {2, 2, 0}, {2, 0, 2}, {0, 2, 2}};
  for (int m = 0; m < Q; ++m) {
    for (int d = 0; d < 3; ++d) MEXP[m][d] = E[m][d];
    MORD[m] = E[m][0] + E[m][1] + E[m][2];
  }
  g_tables_ready = 1;
}

void orc3_lattice(int* c, double* w) {
  build_tables();
  for (int i = 0; i < Q; ++i) {
    for (int d = 0; d < 3; ++d) c[3 * i + d] = CV[i][d];
    w[i] = WQ[i];
  }
}

struct orc3_sim {
  orc3_params p;
  int nx, ny, nz, N, periodic_z, surf;
  double kappa, beta, W, kBT, phib, sg0, sl0, lambda_s, M0, eta_phi, eta_psi, psi_c;
  double Mm[Q][Q], Mi[Q][Q];
  double *f, *g, *h, *fn, *gn, *hn;
  double *phi_h, *psi_h, *vx_h, *vy_h, *vz_h, *ux_h, *uy_h, *uz_h, *Rphi_h, *Rpsi_h;
  int have_hist;
  int64_t step;
  double sumRpsi_last, orth_last;
  double *phi, *psi, *mu_phi, *mu_psi, *lap0_psi, *Tphi, *Tpsi, *rho, *ux, *uy, *uz, *pr;
  double *Fx, *Fy, *Fz, *grx, *gry, *grz, *Rphi, *Rpsi, *vx, *vy, *vz;
  double *Jphi_b, *Jpsi_b, *Jphi_t, *Jpsi_t;   /* per (x, y) column of the wall layer */
  double lambda, mubar, m_ref;
  unsigned char* solid;   /* [N] 1 = solid node (orc3_set_solid), NULL: none */
  int Nf;                 /* fluid nodes */
};

static int wrapi(int a, int n) { a %= n; return a < 0 ? a + n : a; }
static double powi(int c, int e) { double r = 1.0; for (int k = 0; k < e; ++k) r *= c; return r; }

/* g(phi) of the wall energy and h_phi (Sec. 2.1) */
static double gsw(const orc3_sim* s, double ph) {
  double b = s->phib;
  return 3.0 * ph / (4.0 * b) - ph * ph * ph / (4.0 * b * b * b);
}
static double gsw_d(const orc3_sim* s, double ph) {
  double b = s->phib;
  return 3.0 / (4.0 * b) * (1.0 - ph * ph / (b * b));
}
static double hval(const orc3_sim* s, double ph) { return s->p.constraint_phi == ORC3_LINEAR ? ph : 0.5 + gsw(s, ph); }
static double hprime(const orc3_sim* s, double ph) { return s->p.constraint_phi == ORC3_LINEAR ? 1.0 : gsw_d(s, ph); }
static double liquid_frac(const orc3_sim* s, double ph) {
  double w = 0.5 * (1.0 + ph / s->phib);
  return w < 0.0 ? 0.0 : (w > 1.0 ? 1.0 : w);
}
static double rho_of(const orc3_sim* s, double ph) { return s->p.rho_g + (s->p.rho_l - s->p.rho_g) * liquid_frac(s, ph); }
static double mud_of(const orc3_sim* s, double ph) { return s->p.mu_g + (s->p.mu_l - s->p.mu_g) * liquid_frac(s, ph); }
/* -df_w/dphi and -df_w/dpsi of the wall energy (eq8, boundary) */
static double wall_Jphi(const orc3_sim* s, double ph, double ps) {
  double a = s->p.sigma_gl0 * cos(s->p.theta0_deg * M_PI / 180.0);
  if (s->surf) a += log(1.0 - ps) * (s->sg0 * s->p.beta_sg - s->sl0 * s->p.beta_sl);
  return a * gsw_d(s, ph);
}
static double wall_Jpsi(const orc3_sim* s, double ph, double ps) {
  double d = s->sg0 * s->p.beta_sg - s->sl0 * s->p.beta_sl;
  double m = s->sg0 * s->p.beta_sg + s->sl0 * s->p.beta_sl;
  return -(d * gsw(s, ph) - 0.5 * m) / (1.0 - ps);
}

static int idx(const orc3_sim* s, int x, int y, int z) { return (z * s->ny + y) * s->nx + x; }

/* Neighbour x + c_i of node (x, y, z); beyond a wall: -1 (bottom) or -2 (top),
 * with the column (xx, yy) of the neighbour in *col. */
static int nb(const orc3_sim* s, int x, int y, int z, int i, int* col) {
  int xx = wrapi(x + CV[i][0], s->nx), yy = wrapi(y + CV[i][1], s->ny), zz = z + CV[i][2];
  *col = yy * s->nx + xx;
  if (s->periodic_z) zz = wrapi(zz, s->nz);
  else if (zz < 0) return -1;
  else if (zz >= s->nz) return -2;
  int m = idx(s, xx, yy, zz);
  if (s->solid && s->solid[m]) return -3;
  return m;
}
static int is_solid(const orc3_sim* s, int n) { return s->solid && s->solid[n]; }
/* value of a at x + c_i; beyond a wall the fluid node of the same column next
 * to it (mirror) */
static double nb_mirror(const orc3_sim* s, const double* a, int x, int y, int z, int i) {
  int col, m = nb(s, x, y, z, i, &col);
  if (m >= 0) return a[m];
  if (m == -3) return a[idx(s, x, y, z)];   /* link-wise mirror at a solid node */
  return a[z * s->nx * s->ny + col];
}
static double wall_T(const orc3_sim* s, const double* Jb, const double* Jt, int x, int y, int z) {
  if (s->periodic_z) return 0.0;
  double t = 0.0;
  for (int i = 1; i < Q; ++i) {
    int col, m = nb(s, x, y, z, i, &col);
    if (m == -1) t += 2.0 * WQ[i] / CS2 * Jb[col];
    else if (m == -2) t += 2.0 * WQ[i] / CS2 * Jt[col];
  }
  return t;
}
/* wall term of the links of (x, y, z) into solid nodes (wetting solids only) */
static double solid_T(const orc3_sim* s, int x, int y, int z, double J) {
  if (!s->solid || !s->p.solid_wet) return 0.0;
  double t = 0.0;
  for (int i = 1; i < Q; ++i) {
    int col;
    if (nb(s, x, y, z, i, &col) == -3) t += 2.0 * WQ[i] / CS2 * J;
  }
  return t;
}
static double nb_rho(const orc3_sim* s, int x, int y, int z, int i) {
  int col, m = nb(s, x, y, z, i, &col);
  if (m >= 0) return s->rho[m];
  if (m == -3) {
    int n = idx(s, x, y, z);
    double ph = s->phi[n];
    return rho_of(s, s->p.solid_wet ? ph + wall_Jphi(s, ph, s->psi[n]) / s->kappa : ph);
  }
  double ph = s->phi[z * s->nx * s->ny + col];
  double J = m == -1 ? s->Jphi_b[col] : s->Jphi_t[col];
  return rho_of(s, ph + J / s->kappa);
}

static int invert(double A[Q][Q], double Ainv[Q][Q]) {
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

/* x* = x - M^-1 S M (x - x_eq) + M^-1 (I - S/2) M v + w_i extra */
static void mrt_collide(const orc3_sim* s, const double* x, const double* xeq, const double* v, const double* rates,
                        double extra, double* out) {
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
static double cdot(int i, double ax, double ay, double az) { return CV[i][0] * ax + CV[i][1] * ay + CV[i][2] * az; }
static void feq_flow(double pr, double rho, double ux, double uy, double uz, double* out) {
  double uu = ux * ux + uy * uy + uz * uz;
  for (int i = 0; i < Q; ++i) {
    double cu = cdot(i, ux, uy, uz);
    double su = cu / CS2 + cu * cu / (2.0 * CS2 * CS2) - uu / (2.0 * CS2);
    out[i] = pr / CS2 * (WQ[i] - (i == 0 ? 1.0 : 0.0)) + rho * WQ[i] * su;
  }
}
static void feq_scalar(double c, double eta, double jx, double jy, double jz, double* out) {
  out[0] = c + (WQ[0] - 1.0) * eta * c;
  for (int i = 1; i < Q; ++i) out[i] = WQ[i] * eta * c + WQ[i] * cdot(i, jx, jy, jz) / CS2;
}

static void set_err(char* err, int errlen, const char* msg) {
  if (err && errlen > 0) { strncpy(err, msg, (size_t)errlen - 1); err[errlen - 1] = 0; }
}
static double rate_or(double v, double dflt) { return v > 0.0 ? v : dflt; }

static int derive(orc3_sim* s, char* err, int errlen) {
  const orc3_params* p = &s->p;
  int wet = p->bc_bottom == ORC3_WALL_WET || p->bc_top == ORC3_WALL_WET;
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

static int validate(const orc3_params* p, char* err, int errlen) {
  if (p->nx < 3 || p->ny < 3 || p->nz < 3) { set_err(err, errlen, "nx, ny and nz must be >= 3"); return -1; }
  if (p->bc_bottom < 0 || p->bc_bottom > 3 || p->bc_top < 0 || p->bc_top > 3) { set_err(err, errlen, "bad boundary kind"); return -1; }
  if ((p->bc_bottom == ORC3_PERIODIC) != (p->bc_top == ORC3_PERIODIC)) { set_err(err, errlen, "periodic z needs both walls periodic"); return -1; }
  if (!(p->sigma_gl0 > 0.0) || !(p->eps > 0.0)) { set_err(err, errlen, "sigma_gl0 and eps must be > 0"); return -1; }
  if (!(p->psi_b >= 0.0 && p->psi_b < 1.0)) { set_err(err, errlen, "psi_b must lie in [0,1)"); return -1; }
  if (!(p->rho_l > 0.0 && p->rho_g > 0.0 && p->mu_l > 0.0 && p->mu_g > 0.0)) { set_err(err, errlen, "densities and viscosities must be > 0"); return -1; }
  return 0;
}

static double* zalloc(size_t n) { return (double*)calloc(n, sizeof(double)); }

void orc3_load_fields(orc3_sim* s, const double* phi, const double* psi, const double* u) {
  int N = s->N;
  double fe[Q], ge[Q], he[Q];
  for (int n = 0; n < N; ++n) {
    if (is_solid(s, n)) {
      for (int i = 0; i < Q; ++i) s->f[(size_t)i * N + n] = s->g[(size_t)i * N + n] = s->h[(size_t)i * N + n] = 0.0;
      continue;
    }
    double ux = u ? u[n] : 0.0, uy = u ? u[N + n] : 0.0, uz = u ? u[2 * N + n] : 0.0;
    double ps = s->surf ? psi[n] : 0.0;
    feq_flow(0.0, rho_of(s, phi[n]), ux, uy, uz, fe);
    if (!u) for (int i = 0; i < Q; ++i) fe[i] = 0.0;
    feq_scalar(phi[n], s->eta_phi, phi[n] * ux, phi[n] * uy, phi[n] * uz, ge);
    feq_scalar(ps, s->eta_psi, ps * ux, ps * uy, ps * uz, he);
    for (int i = 0; i < Q; ++i) {
      s->f[(size_t)i * N + n] = fe[i];
      s->g[(size_t)i * N + n] = ge[i];
      s->h[(size_t)i * N + n] = s->surf ? he[i] : 0.0;
    }
  }
  s->have_hist = 0;
  double m = 0.0;
  for (int n = 0; n < N; ++n)
    if (!is_solid(s, n)) m += hval(s, phi[n]);
  s->m_ref = m;
}

static void init_fields(orc3_sim* s) {
  const orc3_params* p = &s->p;
  double* ph = zalloc(s->N);
  double* ps = zalloc(s->N);
  for (int z = 0; z < s->nz; ++z)
    for (int y = 0; y < s->ny; ++y)
      for (int x = 0; x < s->nx; ++x) {
        double dx = x - p->x0, dy = y - p->y0, dz = z - p->z0;
        dx -= s->nx * floor(dx / s->nx + 0.5);
        dy -= s->ny * floor(dy / s->ny + 0.5);
        if (s->periodic_z) dz -= s->nz * floor(dz / s->nz + 0.5);
        double r = sqrt(dx * dx + dy * dy + dz * dz), d;
        if (p->init_kind == ORC3_INIT_SLAB) d = 0.5 * p->a - fabs(dx);
        else if (p->init_kind == ORC3_INIT_BUBBLE) d = r - p->R0;
        else d = p->R0 - r;
        double sq = s->surf ? sqrt(1.0 - p->psi_b) : 1.0;
        int n = idx(s, x, y, z);
        ph[n] = s->phib * tanh(2.0 * s->phib * sq * d / p->eps);
        ps[n] = s->surf ? p->psi_b : 0.0;
      }
  orc3_load_fields(s, ph, ps, NULL);
  free(ph);
  free(ps);
}

orc3_sim* orc3_create(const orc3_params* p, char* err, int errlen) {
  build_tables();
  if (validate(p, err, errlen)) return NULL;
  orc3_sim* s = (orc3_sim*)calloc(1, sizeof(orc3_sim));
  s->p = *p;
  s->nx = p->nx; s->ny = p->ny; s->nz = p->nz; s->N = p->nx * p->ny * p->nz;
  s->periodic_z = p->bc_bottom == ORC3_PERIODIC;
  s->Nf = s->N;
  if (derive(s, err, errlen)) { free(s); return NULL; }
  for (int k = 0; k < Q; ++k)
    for (int i = 0; i < Q; ++i)
      s->Mm[k][i] = powi(CV[i][0], MEXP[k][0]) * powi(CV[i][1], MEXP[k][1]) * powi(CV[i][2], MEXP[k][2]);
  if (invert(s->Mm, s->Mi)) { set_err(err, errlen, "moment matrix singular"); free(s); return NULL; }
  size_t N = (size_t)s->N;
  s->f = zalloc(Q * N); s->g = zalloc(Q * N); s->h = zalloc(Q * N);
  s->fn = zalloc(Q * N); s->gn = zalloc(Q * N); s->hn = zalloc(Q * N);
  double** work[] = {&s->phi_h, &s->psi_h, &s->vx_h, &s->vy_h, &s->vz_h, &s->ux_h, &s->uy_h, &s->uz_h, &s->Rphi_h,
                     &s->Rpsi_h, &s->phi, &s->psi, &s->mu_phi, &s->mu_psi, &s->lap0_psi, &s->Tphi, &s->Tpsi, &s->rho,
                     &s->ux, &s->uy, &s->uz, &s->pr, &s->Fx, &s->Fy, &s->Fz, &s->grx, &s->gry, &s->grz, &s->Rphi,
                     &s->Rpsi, &s->vx, &s->vy, &s->vz};
  for (size_t k = 0; k < sizeof(work) / sizeof(work[0]); ++k) *work[k] = zalloc(N);
  size_t cols = (size_t)s->nx * s->ny;
  s->Jphi_b = zalloc(cols); s->Jpsi_b = zalloc(cols); s->Jphi_t = zalloc(cols); s->Jpsi_t = zalloc(cols);
  init_fields(s);
  return s;
}

void orc3_destroy(orc3_sim* s) {
  if (!s) return;
  double* ptrs[] = {s->f, s->g, s->h, s->fn, s->gn, s->hn, s->phi_h, s->psi_h, s->vx_h, s->vy_h, s->vz_h, s->ux_h,
                    s->uy_h, s->uz_h, s->Rphi_h, s->Rpsi_h, s->phi, s->psi, s->mu_phi, s->mu_psi, s->lap0_psi, s->Tphi,
                    s->Tpsi, s->rho, s->ux, s->uy, s->uz, s->pr, s->Fx, s->Fy, s->Fz, s->grx, s->gry, s->grz, s->Rphi,
                    s->Rpsi, s->vx, s->vy, s->vz, s->Jphi_b, s->Jpsi_b, s->Jphi_t, s->Jpsi_t};
  for (size_t k = 0; k < sizeof(ptrs) / sizeof(ptrs[0]); ++k) free(ptrs[k]);
  free(s->solid);
  free(s);
}

void orc3_derived(const orc3_sim* s, double* out) {
  double v[ORC3_N_DERIVED] = {s->kappa, s->beta, s->W, s->kBT, s->phib, s->sg0, s->sl0,
                              s->lambda_s, s->M0, s->eta_phi, s->eta_psi, s->psi_c};
  memcpy(out, v, sizeof(v));
}

void orc3_get_populations(const orc3_sim* s, double* out) {
  size_t N = (size_t)s->N;
  memcpy(out, s->f, Q * N * sizeof(double));
  memcpy(out + Q * N, s->g, Q * N * sizeof(double));
  memcpy(out + 2 * Q * N, s->h, Q * N * sizeof(double));
}

/* O1-O6 at the current state */
static void macro(orc3_sim* s) {
  int nx = s->nx, ny = s->ny, nz = s->nz, N = s->N, cols = nx * ny;
#pragma omp parallel for if (N >= PAR_MIN_NODES)
  for (int n = 0; n < N; ++n) {
    double a = 0.0, b = 0.0;
    for (int i = 0; i < Q; ++i) { a += s->g[(size_t)i * N + n]; b += s->h[(size_t)i * N + n]; }
    s->phi[n] = a;
    s->psi[n] = s->surf ? b : 0.0;
    s->rho[n] = rho_of(s, a);   /* solid nodes: zero populations, never read as fluid */
  }
  /* O2: wall fluxes at the first fluid layer of each wetting wall */
  for (int c = 0; c < cols; ++c) {
    s->Jphi_b[c] = s->Jpsi_b[c] = s->Jphi_t[c] = s->Jpsi_t[c] = 0.0;
    if (s->p.bc_bottom == ORC3_WALL_WET) {
      double ph = s->phi[c], ps = s->psi[c];
      s->Jphi_b[c] = wall_Jphi(s, ph, ps);
      s->Jpsi_b[c] = s->surf ? wall_Jpsi(s, ph, ps) : 0.0;
    }
    if (s->p.bc_top == ORC3_WALL_WET) {
      double ph = s->phi[(nz - 1) * cols + c], ps = s->psi[(nz - 1) * cols + c];
      s->Jphi_t[c] = wall_Jphi(s, ph, ps);
      s->Jpsi_t[c] = s->surf ? wall_Jpsi(s, ph, ps) : 0.0;
    }
  }
  /* O3 */
#pragma omp parallel for if (N >= PAR_MIN_NODES)
  for (int z = 0; z < nz; ++z)
    for (int y = 0; y < ny; ++y)
      for (int x = 0; x < nx; ++x) {
        int n = idx(s, x, y, z);
        if (is_solid(s, n)) { s->mu_phi[n] = s->mu_psi[n] = s->Tphi[n] = s->Tpsi[n] = s->lap0_psi[n] = 0.0; continue; }
        double ph = s->phi[n], ps = s->psi[n], l0p = 0.0, l0s = 0.0;
        for (int i = 1; i < Q; ++i) {
          l0p += 2.0 * WQ[i] / CS2 * (nb_mirror(s, s->phi, x, y, z, i) - ph);
          l0s += 2.0 * WQ[i] / CS2 * (nb_mirror(s, s->psi, x, y, z, i) - ps);
        }
        double tp = wall_T(s, s->Jphi_b, s->Jphi_t, x, y, z), ts = wall_T(s, s->Jpsi_b, s->Jpsi_t, x, y, z);
        tp += solid_T(s, x, y, z, wall_Jphi(s, ph, ps));
        if (s->surf) ts += solid_T(s, x, y, z, wall_Jpsi(s, ph, ps));
        s->Tphi[n] = tp;
        s->Tpsi[n] = ts;
        s->lap0_psi[n] = l0s;
        s->mu_phi[n] = 4.0 * s->beta * (1.0 - ps) * (ph * ph * ph - ph) - s->kappa * l0p - tp + s->W * ps * ph;
        s->mu_psi[n] = s->surf ? s->kBT * log(ps / (1.0 - ps)) - s->lambda_s * l0s - ts
                                   - s->beta * (1.0 - ph * ph) * (1.0 - ph * ph) + 0.5 * s->W * ph * ph
                               : 0.0;
      }
  /* O4 */
  double S1 = 0.0, S2 = 0.0, S3 = 0.0, S4 = 0.0;
  for (int n = 0; n < N; ++n) {
    if (is_solid(s, n)) continue;
    double hp = hprime(s, s->phi[n]);
    S1 += hp * s->mu_phi[n];
    S2 += hp * hp;
    S3 += s->mu_psi[n];
    S4 += hval(s, s->phi[n]);
  }
  s->lambda = S2 > 0.0 ? S1 / S2 : 0.0;
  if (s->p.phi_hold && S2 > 0.0 && s->p.M_phi > 0.0) s->lambda += (s->m_ref - S4) / (s->p.M_phi * S2);
  s->mubar = S3 / s->Nf;
  /* O5, O6 */
#pragma omp parallel for if (N >= PAR_MIN_NODES)
  for (int z = 0; z < nz; ++z)
    for (int y = 0; y < ny; ++y)
      for (int x = 0; x < nx; ++x) {
        int n = idx(s, x, y, z);
        if (is_solid(s, n)) {
          s->grx[n] = s->gry[n] = s->grz[n] = s->Fx[n] = s->Fy[n] = s->Fz[n] = 0.0;
          s->ux[n] = s->uy[n] = s->uz[n] = s->pr[n] = 0.0;
          continue;
        }
        double gr[3] = {0, 0, 0}, gmp[3] = {0, 0, 0}, gms[3] = {0, 0, 0};
        for (int i = 1; i < Q; ++i) {
          double r = nb_rho(s, x, y, z, i);
          double mp = nb_mirror(s, s->mu_phi, x, y, z, i), ms = nb_mirror(s, s->mu_psi, x, y, z, i);
          for (int d = 0; d < 3; ++d) {
            gr[d] += WQ[i] * CV[i][d] * r / CS2;
            gmp[d] += WQ[i] * CV[i][d] * mp / CS2;
            gms[d] += WQ[i] * CV[i][d] * ms / CS2;
          }
        }
        double ph = s->phi[n], ps = s->psi[n], rho = s->rho[n];
        double G[3] = {s->p.gx, s->p.gy, s->p.gz}, F[3];
        for (int d = 0; d < 3; ++d) F[d] = -ph * gmp[d] - ps * gms[d] + rho * G[d];
        s->grx[n] = gr[0]; s->gry[n] = gr[1]; s->grz[n] = gr[2];
        s->Fx[n] = F[0]; s->Fy[n] = F[1]; s->Fz[n] = F[2];
        double j[3] = {0, 0, 0}, sum_nz = 0.0;
        for (int i = 0; i < Q; ++i) {
          double fi = s->f[(size_t)i * N + n];
          for (int d = 0; d < 3; ++d) j[d] += CV[i][d] * fi;
          if (i) sum_nz += fi;
        }
        double ux = (j[0] + 0.5 * F[0]) / rho, uy = (j[1] + 0.5 * F[1]) / rho, uz = (j[2] + 0.5 * F[2]) / rho;
        s->ux[n] = ux; s->uy[n] = uy; s->uz[n] = uz;
        double ugr = ux * gr[0] + uy * gr[1] + uz * gr[2];
        s->pr[n] = CS2 / (1.0 - WQ[0]) * (sum_nz + 0.5 * ugr - rho * WQ[0] * (ux * ux + uy * uy + uz * uz) / (2.0 * CS2));
      }
}

static void step_once(orc3_sim* s) {
  int nx = s->nx, ny = s->ny, nz = s->nz, N = s->N;
  macro(s);
  /* O7 (the identities' sums afterwards, in node order) */
#pragma omp parallel for if (N >= PAR_MIN_NODES)
  for (int n = 0; n < N; ++n) {
    if (is_solid(s, n)) { s->Rphi[n] = s->Rpsi[n] = 0.0; continue; }
    double ph = s->phi[n], ps = s->psi[n], hp = hprime(s, ph);
    s->Rphi[n] = s->p.M_phi * (-4.0 * s->beta * (1.0 - ps) * (ph * ph * ph - ph) - s->W * ps * ph + s->lambda * hp)
               + s->p.M_phi * s->Tphi[n];
    s->Rpsi[n] = s->surf ? -s->M0 * s->lap0_psi[n]
                             + s->p.M_psi * (-s->kBT * log(ps / (1.0 - ps)) + s->beta * (1.0 - ph * ph) * (1.0 - ph * ph)
                                             - 0.5 * s->W * ph * ph + s->mubar)
                             + s->p.M_psi * s->Tpsi[n]
                         : 0.0;
  }
  double sumR = 0.0, orth = 0.0;
  for (int n = 0; n < N; ++n) {
    if (is_solid(s, n)) continue;
    double hp = hprime(s, s->phi[n]);
    sumR += s->Rpsi[n];
    orth += hp * (s->mu_phi[n] - s->lambda * hp);
  }
  s->sumRpsi_last = sumR;
  s->orth_last = orth;
  /* O8 */
#pragma omp parallel for if (N >= PAR_MIN_NODES)
  for (int n = 0; n < N; ++n) {
    if (is_solid(s, n)) continue;
    double ph = s->phi[n], ps = s->psi[n], rho = s->rho[n], u[3] = {s->ux[n], s->uy[n], s->uz[n]};
    double x[Q], xe[Q], v[Q], out[Q], rates[Q];
    double vv[3] = {u[0], u[1], u[2]};
    if (!s->p.adv_raw && s->have_hist) {
      vv[0] = 0.5 * (u[0] + s->ux_h[n]);
      vv[1] = 0.5 * (u[1] + s->uy_h[n]);
      vv[2] = 0.5 * (u[2] + s->uz_h[n]);
    }
    s->vx[n] = vv[0]; s->vy[n] = vv[1]; s->vz[n] = vv[2];
    double dp[3] = {0, 0, 0}, ds[3] = {0, 0, 0}, dRp = 0.0, dRs = 0.0;
    if (s->have_hist) {
      double vh[3] = {s->vx_h[n], s->vy_h[n], s->vz_h[n]};
      for (int d = 0; d < 3; ++d) {
        dp[d] = ph * vv[d] - s->phi_h[n] * vh[d];
        ds[d] = ps * vv[d] - s->psi_h[n] * vh[d];
      }
      dRp = s->Rphi[n] - s->Rphi_h[n];
      dRs = s->Rpsi[n] - s->Rpsi_h[n];
    }
    /* flow */
    double s2 = s->p.s_f[2] > 0.0 ? s->p.s_f[2] : 1.0 / (3.0 * mud_of(s, ph) / rho + 0.5);
    double sf[5] = {rate_or(s->p.s_f[0], 1.0), rate_or(s->p.s_f[1], 1.0), s2, rate_or(s->p.s_f[3], 1.0),
                    rate_or(s->p.s_f[4], 1.0)};
    for (int k = 0; k < Q; ++k) rates[k] = sf[MORD[k]];
    for (int i = 0; i < Q; ++i) x[i] = s->f[(size_t)i * N + n];
    feq_flow(s->pr[n], rho, u[0], u[1], u[2], xe);
    double gr[3] = {s->grx[n], s->gry[n], s->grz[n]}, F[3] = {s->Fx[n], s->Fy[n], s->Fz[n]};
    double ugr = u[0] * gr[0] + u[1] * gr[1] + u[2] * gr[2];
    for (int i = 0; i < Q; ++i) {
      double cu = cdot(i, u[0], u[1], u[2]), cg = cdot(i, gr[0], gr[1], gr[2]), cF = cdot(i, F[0], F[1], F[2]);
      v[i] = WQ[i] * (ugr + cF / CS2 + (cu * cg - CS2 * ugr) / CS2);
    }
    mrt_collide(s, x, xe, v, rates, 0.0, out);
    for (int i = 0; i < Q; ++i) s->f[(size_t)i * N + n] = out[i];
    /* phase field */
    double sg[5];
    for (int k = 0; k < 5; ++k) sg[k] = rate_or(s->p.s_g[k], 1.0);
    for (int k = 0; k < Q; ++k) rates[k] = sg[MORD[k]];
    for (int i = 0; i < Q; ++i) x[i] = s->g[(size_t)i * N + n];
    feq_scalar(ph, s->eta_phi, ph * vv[0], ph * vv[1], ph * vv[2], xe);
    for (int i = 0; i < Q; ++i) v[i] = WQ[i] * cdot(i, dp[0], dp[1], dp[2]) / CS2;
    mrt_collide(s, x, xe, v, rates, s->Rphi[n] + 0.5 * dRp, out);
    for (int i = 0; i < Q; ++i) s->g[(size_t)i * N + n] = out[i];
    /* surfactant */
    if (s->surf) {
      double sh[5];
      for (int k = 0; k < 5; ++k) sh[k] = rate_or(s->p.s_h[k], 1.0);
      for (int k = 0; k < Q; ++k) rates[k] = sh[MORD[k]];
      for (int i = 0; i < Q; ++i) x[i] = s->h[(size_t)i * N + n];
      feq_scalar(ps, s->eta_psi, ps * vv[0], ps * vv[1], ps * vv[2], xe);
      for (int i = 0; i < Q; ++i) v[i] = WQ[i] * cdot(i, ds[0], ds[1], ds[2]) / CS2;
      mrt_collide(s, x, xe, v, rates, s->Rpsi[n] + 0.5 * dRs, out);
      for (int i = 0; i < Q; ++i) s->h[(size_t)i * N + n] = out[i];
    }
  }
  /* O9: push streaming; walls in z (a permutation of the population slots: layers write disjoint targets) */
#pragma omp parallel for if (N >= PAR_MIN_NODES)
  for (int z = 0; z < nz; ++z)
    for (int y = 0; y < ny; ++y)
      for (int x = 0; x < nx; ++x) {
        int n = idx(s, x, y, z);
        if (is_solid(s, n)) {
          for (int i = 0; i < Q; ++i) s->fn[(size_t)i * N + n] = s->gn[(size_t)i * N + n] = s->hn[(size_t)i * N + n] = 0.0;
          continue;
        }
        for (int i = 0; i < Q; ++i) {
          size_t src = (size_t)i * N + n;
          int xx = wrapi(x + CV[i][0], nx), yy = wrapi(y + CV[i][1], ny), zz = z + CV[i][2];
          if ((s->periodic_z || (zz >= 0 && zz < nz)) && is_solid(s, idx(s, xx, yy, wrapi(zz, nz)))) {
            /* half-way bounce-back at a solid node (at rest) */
            s->fn[(size_t)OPP[i] * N + n] = s->f[src];
            s->gn[(size_t)OPP[i] * N + n] = s->g[src];
            s->hn[(size_t)OPP[i] * N + n] = s->h[src];
            continue;
          }
          if (s->periodic_z || (zz >= 0 && zz < nz)) {
            size_t dst = (size_t)i * N + idx(s, xx, yy, wrapi(zz, nz));
            s->fn[dst] = s->f[src];
            s->gn[dst] = s->g[src];
            s->hn[dst] = s->h[src];
            continue;
          }
          int bc = zz < 0 ? s->p.bc_bottom : s->p.bc_top;
          double uw = zz < 0 ? s->p.u_wall_bottom : s->p.u_wall_top;
          s->gn[(size_t)OPP[i] * N + n] = s->g[src];
          s->hn[(size_t)OPP[i] * N + n] = s->h[src];
          if (bc == ORC3_FREESLIP) s->fn[(size_t)MIRZ[i] * N + idx(s, xx, yy, z)] = s->f[src];
          else s->fn[(size_t)OPP[i] * N + n] = s->f[src] - 2.0 * WQ[i] * s->rho[n] * (CV[i][0] * uw) / CS2;
        }
      }
  double* t;
  t = s->f; s->f = s->fn; s->fn = t;
  t = s->g; s->g = s->gn; s->gn = t;
  t = s->h; s->h = s->hn; s->hn = t;
  /* O10 */
  size_t bytes = (size_t)N * sizeof(double);
  memcpy(s->phi_h, s->phi, bytes); memcpy(s->psi_h, s->psi, bytes);
  memcpy(s->ux_h, s->ux, bytes); memcpy(s->uy_h, s->uy, bytes); memcpy(s->uz_h, s->uz, bytes);
  memcpy(s->vx_h, s->vx, bytes); memcpy(s->vy_h, s->vy, bytes); memcpy(s->vz_h, s->vz, bytes);
  memcpy(s->Rphi_h, s->Rphi, bytes); memcpy(s->Rpsi_h, s->Rpsi, bytes);
  s->have_hist = 1;
  s->step += 1;
}

int orc3_set_solid(orc3_sim* s, const unsigned char* mask) {
  int nf = 0;
  for (int n = 0; n < s->N; ++n) nf += mask[n] ? 0 : 1;
  if (nf == 0) return -1;
  if (!s->solid) s->solid = (unsigned char*)calloc((size_t)s->N, 1);
  for (int n = 0; n < s->N; ++n) s->solid[n] = mask[n] ? 1 : 0;
  s->Nf = nf;
  /* rebuild the state from the current fields, fluid nodes only */
  double* ph = zalloc(s->N);
  double* ps = zalloc(s->N);
  macro(s);
  memcpy(ph, s->phi, (size_t)s->N * sizeof(double));
  memcpy(ps, s->psi, (size_t)s->N * sizeof(double));
  orc3_load_fields(s, ph, ps, NULL);
  free(ph);
  free(ps);
  return 0;
}

void orc3_step(orc3_sim* s, int64_t n) {
  for (int64_t k = 0; k < n; ++k) step_once(s);
}

void orc3_fields(orc3_sim* s, uint32_t mask, double* out) {
  macro(s);
  const double* src[9] = {s->phi, s->psi, s->ux, s->uy, s->uz, s->pr, s->rho, s->mu_phi, s->mu_psi};
  size_t N = (size_t)s->N, k = 0;
  for (int b = 0; b < 9; ++b)
    if (mask & (1u << b)) memcpy(out + (k++) * N, src[b], N * sizeof(double));
}

void orc3_invariants(orc3_sim* s, orc3_inv* out) {
  macro(s);
  memset(out, 0, sizeof(*out));
  out->step = s->step;
  for (int n = 0; n < s->N; ++n) {
    if (is_solid(s, n)) continue;
    double ph = s->phi[n], ps = s->psi[n], u2 = s->ux[n] * s->ux[n] + s->uy[n] * s->uy[n] + s->uz[n] * s->uz[n];
    if (!isfinite(ph) || !isfinite(ps) || !isfinite(u2) || !isfinite(s->pr[n])) out->nonfinite++;
    if (s->surf && !(ps > 0.0 && ps < 1.0)) out->psi_out_of_range++;
    out->mass_psi += ps;
    out->m_phi_h += 0.5 + gsw(s, ph);
    out->sum_phi += ph;
    out->kinetic += 0.5 * s->rho[n] * u2;
    if (sqrt(u2) > out->umax) out->umax = sqrt(u2);
  }
  out->lambda_phi = s->lambda;
  out->mubar_psi = s->mubar;
  out->sum_R_psi = s->sumRpsi_last;
  out->orthogonality = s->orth_last;
}
