// lbm_kernels.hip -- gfx950 kernels of the coupled three-population lattice
// Boltzmann step (phase field phi, surfactant psi, hydrodynamics f).
//
// Layout: structure of arrays.  Populations are 27 planes [f0..f8 g0..g8
// h0..h8] of N = nx*ny nodes, x fastest, in the storage type S; macroscopic
// planes likewise.  The stored value of population i at node z is its
// post-collision value at z ("pull" streaming): a step gathers
// f_i(x) = stored_i(x - c_i), so every load and store of a wavefront touches 64
// consecutive nodes of one plane.
//
// Precision design.  phi and psi are sums dominated by the rest populations
// g_0 ~ phi and h_0 ~ psi, whose storage rounding would feed the Laplacian in
// the chemical potential.  The rest populations are therefore stored shifted,
// g_0 - phi(n) and h_0 - psi(n), against FP64 planes holding phi(n), psi(n);
// the moving populations are small and stored as they are.  All macroscopic
// work (phi, psi, stencils, chemical potentials, force, velocity, pressure,
// sources, reductions) runs in FP64; the three MRT collisions run in the
// compute type C of the storage precision (FP64 or FP32).
//
// One step (Sec. 3 of the paper) is two launches:
//   k_step         fused step on 64 x TY tiles (see its comment): phi, psi
//                  (macroscopic recovery), chemical potentials with the wall
//                  terms (eq_muphi, eq_mupsi), per-tile FP64 sums of
//                  h'(phi) mu_phi, h'(phi)^2, mu_psi (eq15), force, velocity,
//                  pressure, sources, MRT collision of f, g, h, wall
//                  corrections; writes post-collision populations and the
//                  history for the backward differences
//   k_step_finish  lambda_phi = S1/S2, mubar_psi = S3/N            (eq15, AC_psi)
// The multiplier terms of a step's sources are applied by the next step (or by
// the diagnostic kernels below), so one pass over the grid suffices.
// Diagnostics (fields, invariants) recompute the macroscopic state with
//   k_moments      phi = sum g_i, psi = sum h_i plus the pending terms
//   k_mu_partials  mu_phi, mu_psi and the multiplier sums
//   k_multipliers  lambda_phi, mubar_psi of the current state
// No MFMA: the step moves ~300 B/node in FP32 storage and does ~1.3k VALU
// operations per node, no dense contraction; HBM bandwidth bounds it.

#include <type_traits>

#include "lbm_internal.h"
#include "../../include/lbm.h"

namespace lbm {
namespace {

constexpr double kPi = 3.14159265358979323846;

// ---------------------------------------------------------------- D2Q9 tables
// Directions: 0 rest, 1 (+x), 2 (+y), 3 (-x), 4 (-y), 5 (+x+y), 6 (-x+y),
// 7 (-x-y), 8 (+x-y).  Written as constexpr functions so unrolled loops fold.
__host__ __device__ constexpr int CX(int i) { return (i == 1 || i == 5 || i == 8) ? 1 : ((i == 3 || i == 6 || i == 7) ? -1 : 0); }
__host__ __device__ constexpr int CY(int i) { return (i == 2 || i == 5 || i == 6) ? 1 : ((i == 4 || i == 7 || i == 8) ? -1 : 0); }
__host__ __device__ constexpr int OPP(int i) { return i == 0 ? 0 : (i <= 4 ? ((i + 1) % 4) + 1 : ((i - 3) % 4) + 5); }
__host__ __device__ constexpr int MIRY(int i) { return i == 2 ? 4 : i == 4 ? 2 : i == 5 ? 8 : i == 8 ? 5 : i == 6 ? 7 : i == 7 ? 6 : i; }
template <class C> __device__ __forceinline__ constexpr C WQ(int i) { return i == 0 ? C(4.0 / 9.0) : (i <= 4 ? C(1.0 / 9.0) : C(1.0 / 36.0)); }
static_assert(OPP(1) == 3 && OPP(2) == 4 && OPP(3) == 1 && OPP(4) == 2, "opp");
static_assert(OPP(5) == 7 && OPP(6) == 8 && OPP(7) == 5 && OPP(8) == 6, "opp");

// ------------------------------------------------------------ storage codec
// FP16 ("shifted") storage keeps each population as its deviation from the
// u-independent part of its equilibrium at the node that wrote it, scaled by
// 2^10 into FP16's normal range: f_i (pressure based, already near zero) as
// f_i 2^10; g_i as (g_i - wt_i phi(z)) 2^10 with wt_0 = 1 - (1 - w_0) eta_phi
// and wt_i = w_i eta_phi, the rest-state equilibrium of Sec. 3; h_i likewise
// with psi and eta_psi.  The reference phi(z), psi(z) is the FP64 plane the
// writing step outputs, rounded to FP32 identically by writer and reader.
// Decoding returns the FP32/FP64 storage convention: the rest populations of
// g and h less phi (psi) of their own node, moving populations as they are.
// FP32 and FP64 storage encode and decode as the identity.
// Rounding to FP16 is coherent where the fields are uniform (every bulk node
// rounds the same deviation the same way), which would drift the phi and psi
// masses linearly in time.  So in FP16 storage the rest populations of g and h
// live in two FP32 planes (after the 27 FP16 planes), in the FP32 convention,
// and each writing node adds to its rest value the FP16 rounding residuals of
// its eight moving populations: what a node stores then decodes to exactly its
// post-collision zeroth moment (to FP32 rounding), and the masses are conserved.
template <class S> inline constexpr bool kHalf = std::is_same<S, _Float16>::value;
constexpr float kHalfScale = 1024.0f, kHalfInv = 1.0f / 1024.0f;
__host__ __device__ constexpr size_t rest_offset(size_t N) { return (27 * N * 2 + 255) / 256 * 256; }   // bytes
// FP32 rest plane of lattice lat (1 = g, 2 = h) in an FP16 population buffer
__device__ __forceinline__ float* rest_plane(void* P, size_t N, int lat) {
  return (float*)((char*)P + rest_offset(N)) + (size_t)(lat - 1) * N;
}
__device__ __forceinline__ const float* rest_plane(const void* P, size_t N, int lat) {
  return (const float*)((const char*)P + rest_offset(N)) + (size_t)(lat - 1) * N;
}

// v: population in the FP32 convention; c: reference (phi or psi) of the writing node
template <class S, class C>
__device__ __forceinline__ S encode(const DevParams& p, int lat, int i, C v, C c) {
  if constexpr (kHalf<S>) {
    if (lat == 0) return (S)(v * kHalfScale);
    const C eta = (C)(lat == 1 ? p.eta_phi : p.eta_psi);
    const C shift = i == 0 ? C(1.0 - 4.0 / 9.0) * eta * c : -WQ<C>(i) * eta * c;
    return (S)((v + shift) * kHalfScale);
  } else {
    return (S)v;
  }
}
// t: stored value; c: reference of the node that wrote it (the emitter; the
// node itself for i = 0 and at a bounce-back)
template <class S, class C>
__device__ __forceinline__ C decode(const DevParams& p, int lat, int i, S t, C c) {
  if constexpr (kHalf<S>) {
    const C v = (C)t * kHalfInv;
    if (lat == 0) return v;
    const C eta = (C)(lat == 1 ? p.eta_phi : p.eta_psi);
    return i == 0 ? v - C(1.0 - 4.0 / 9.0) * eta * c : v + WQ<C>(i) * eta * c;
  } else {
    return (C)t;
  }
}

__device__ __forceinline__ int wrap(int a, int n) { return a < 0 ? a + n : (a >= n ? a - n : a); }

// Neighbour x + (dx,dy) of (x,y) for the stencils.  Beyond a wall the ghost
// reads the fluid node next to it in the same column (index returned) and
// side tells which wall (-1 bottom, +1 top, 0 inside).
struct Nb { int idx; int side; };
__device__ __forceinline__ Nb nbr(const DevParams& p, int x, int y, int dx, int dy) {
  int xx = wrap(x + dx, p.nx), yy = y + dy;
  if (p.periodic_y) return {wrap(yy, p.ny) * p.nx + xx, 0};
  if (yy < 0) return {y * p.nx + xx, -1};
  if (yy >= p.ny) return {y * p.nx + xx, 1};
  return {yy * p.nx + xx, 0};
}
__device__ __forceinline__ bool wet_side(const DevParams& p, int side) { return side < 0 ? p.wet_bottom : p.wet_top; }

// Gather population i of lattice lat (0 f, 1 g, 2 h) at (x,y): the value that
// left x - c_i last step.  Sources beyond a wall: half-way bounce-back (the
// population that left x towards the wall), or for f at a free-slip wall the
// specular image that left x - (c_x, 0).  For i = 0 of g and h this is the
// shifted value g_0 - phi(n) (h_0 - psi(n)).
template <class S, class C>
__device__ __forceinline__ C pull(const DevParams& p, const S* __restrict__ P, int lat, int i, int x, int y,
                                  const double* __restrict__ ref) {
  const size_t N = (size_t)p.N;
  int sx = wrap(x - CX(i), p.nx), sy = y - CY(i);
  size_t at, em;   // element read and the node that wrote it
  if (p.periodic_y) sy = wrap(sy, p.ny);
  if (!p.periodic_y && (sy < 0 || sy >= p.ny)) {
    const int bc = sy < 0 ? p.bc_bottom : p.bc_top;
    em = (size_t)y * p.nx + x;
    if (lat == 0 && bc == LBM_BC_FREESLIP) at = (size_t)(9 * lat + MIRY(i)) * N + (size_t)y * p.nx + sx;
    else at = (size_t)(9 * lat + OPP(i)) * N + em;
  } else {
    em = (size_t)sy * p.nx + sx;
    at = (size_t)(9 * lat + i) * N + em;
  }
  if constexpr (kHalf<S>) {
    if (lat > 0 && i == 0) return (C)rest_plane(P, N, lat)[em];
    const C c = lat ? (C)ref[(size_t)(lat - 1) * N + em] : C(0);
    return decode<S, C>(p, lat, i, P[at], c);
  } else {
    return (C)P[at];
  }
}

// ------------------------------------------------------------------- physics
// All in FP64.  Wall switching function g(phi) and g'(phi), u = phi/phi_b (Sec. 2.1).
__device__ __forceinline__ double gsw(const DevParams& p, double ph) {
  const double u = ph * p.inv_phib;
  return 0.75 * u - 0.25 * u * u * u;
}
__device__ __forceinline__ double gsw_d(const DevParams& p, double ph) {
  const double u = ph * p.inv_phib;
  return 0.75 * p.inv_phib * (1.0 - u * u);
}
__device__ __forceinline__ double hprime(const DevParams& p, double ph) { return p.linear ? 1.0 : gsw_d(p, ph); }
// Density and dynamic viscosity: linear in the liquid fraction (1 + phi/phi_b)/2
// held to [0, 1], so that a phase field a little past -phi_b (a contact line,
// the bulk shift of a curved interface) cannot take the light phase's density
// through zero at large density ratios.
__device__ __forceinline__ double liquid_frac(const DevParams& p, double ph) {
  return fmin(fmax(0.5 * (1.0 + ph * p.inv_phib), 0.0), 1.0);
}
// h_phi(phi): 1/2 + g(phi) (AC_phi) or phi (linear constraint).
__device__ __forceinline__ double hval(const DevParams& p, double ph) {
  if (p.linear) return ph;
  const double u = ph * p.inv_phib;
  return 0.5 + 0.75 * u - 0.25 * u * u * u;
}
// lambda_phi from the sums (eq15), with the optional return of sum h_phi to m_ref.
__device__ __forceinline__ double lambda_of(const DevParams& p, double S1, double S2, double S4) {
  double lam = S2 > 0.0 ? S1 / S2 : 0.0;
  if (p.phi_hold && S2 > 0.0 && p.M_phi > 0.0) lam += (p.m_ref - S4) / (p.M_phi * S2);
  return lam;
}
__device__ __forceinline__ double rho_of(const DevParams& p, double ph) {
  return p.rho_g + (p.rho_l - p.rho_g) * liquid_frac(p, ph);
}
__device__ __forceinline__ double mud_of(const DevParams& p, double ph) {
  return p.mu_g + (p.mu_l - p.mu_g) * liquid_frac(p, ph);
}
// Wall energy f_w = (s_sg + s_sl)/2 - (s_sg - s_sl) g(phi) with s_sa =
// sigma_sa0 (1 + beta_sa L), L = ln(1 - psi).  Under Remark 1's saturation each
// beta_sa L is held at -1/2 or more; returns the surfactant parts of s_sg - s_sl
// and of s_sg + s_sl.
__device__ __forceinline__ double2 wall_surf_terms(const DevParams& p, double L) {
  if (!p.sat_cap) return make_double2(L * p.dsb, L * p.msb);
  const double a = p.sg0 * fmax(-0.5, p.beta_sg * L), b = p.sl0 * fmax(-0.5, p.beta_sl * L);
  return make_double2(a - b, a + b);
}
// J_phi = -df_w/dphi, J_psi = -df_w/dpsi at a wall node (eq8, boundary).
__device__ __forceinline__ double Jphi(const DevParams& p, double ph, double ps) {
  double a = p.sig_cos;
  if (p.surf) a += wall_surf_terms(p, log(1.0 - ps)).x;
  return a * gsw_d(p, ph);
}
__device__ __forceinline__ double Jpsi(const DevParams& p, double ph, double ps) {
  double d = p.dsb, m = p.msb;
  if (p.sat_cap) {   // each tension's psi derivative vanishes where its hold acts
    const double L = log(1.0 - ps);
    const double cg = p.beta_sg * L > -0.5 ? p.sg0 * p.beta_sg : 0.0;
    const double cl = p.beta_sl * L > -0.5 ? p.sl0 * p.beta_sl : 0.0;
    d = cg - cl;
    m = cg + cl;
  }
  return -(d * gsw(p, ph) - 0.5 * m) / (1.0 - ps);
}

// Laplacian pieces at (x,y): zero-flux part L0 of phi and psi, and the wall
// terms T = sum over directions into a wetting wall of 2 w_i/c_s^2 J(column),
// so that the Laplacian with wetting ghosts is L0 + T/kappa (phi) and
// L0 + T/lambda_s (psi).
struct Lap { double l0p, l0s, Tp, Ts; };
__device__ __forceinline__ Lap laplace(const DevParams& p, const double* __restrict__ phi, const double* __restrict__ psi, int x, int y) {
  const int n = y * p.nx + x;
  const double ph = phi[n], ps = psi[n];
  Lap r{0.0, 0.0, 0.0, 0.0};
#pragma unroll
  for (int i = 1; i < 9; ++i) {
    const Nb b = nbr(p, x, y, CX(i), CY(i));
    const double w2 = 6.0 * WQ<double>(i);  // 2 w_i / c_s^2
    const double pn = phi[b.idx], sn = psi[b.idx];
    r.l0p += w2 * (pn - ph);
    r.l0s += w2 * (sn - ps);
    if (b.side && wet_side(p, b.side)) {
      r.Tp += w2 * Jphi(p, pn, sn);
      if (p.surf) r.Ts += w2 * Jpsi(p, pn, sn);
    }
  }
  return r;
}

// Chemical potentials (eq_muphi, eq_mupsi) from the local values and stencil.
__device__ __forceinline__ double mu_phi_of(const DevParams& p, double ph, double ps, const Lap& L) {
  return 4.0 * p.beta * (1.0 - ps) * (ph * ph * ph - ph) - p.kappa * L.l0p - L.Tp + p.W * ps * ph;
}
__device__ __forceinline__ double mu_psi_of(const DevParams& p, double ph, double ps, const Lap& L) {
  if (!p.surf) return 0.0;
  const double q = 1.0 - ph * ph;
  return p.kBT * log(ps / (1.0 - ps)) - p.lambda_s * L.l0s - L.Ts - p.beta * q * q + 0.5 * p.W * ph * ph;
}

// Raw moments c_x^a c_y^b grouped by order: m00 m10 m01 m20 m11 m02 m21 m12 m22.
// m00 is not formed here: for g and h it is the exact phi / psi.
template <class C> __device__ __forceinline__ void moments_noncons(const C* f, C* m) {
  m[1] = f[1] - f[3] + f[5] - f[6] - f[7] + f[8];
  m[2] = f[2] - f[4] + f[5] + f[6] - f[7] - f[8];
  m[3] = f[1] + f[3] + f[5] + f[6] + f[7] + f[8];
  m[4] = f[5] - f[6] + f[7] - f[8];
  m[5] = f[2] + f[4] + f[5] + f[6] + f[7] + f[8];
  m[6] = f[5] + f[6] - f[7] - f[8];
  m[7] = f[5] - f[6] - f[7] + f[8];
  m[8] = f[5] + f[6] + f[7] + f[8];
}
// Inverse of the raw-moment transform for the moving directions 1..8.
template <class C> __device__ __forceinline__ void moving_populations(const C* m, C* f) {
  f[1] = C(0.5) * (m[1] + m[3] - m[7] - m[8]);
  f[2] = C(0.5) * (m[2] + m[5] - m[6] - m[8]);
  f[3] = C(0.5) * (-m[1] + m[3] + m[7] - m[8]);
  f[4] = C(0.5) * (-m[2] + m[5] + m[6] - m[8]);
  f[5] = C(0.25) * (m[4] + m[6] + m[7] + m[8]);
  f[6] = C(0.25) * (-m[4] + m[6] - m[7] + m[8]);
  f[7] = C(0.25) * (m[4] - m[6] - m[7] + m[8]);
  f[8] = C(0.25) * (-m[4] - m[6] + m[7] + m[8]);
}

// Pressure-based equilibrium of lattice 1 (Sec. 3), direction d.
__device__ __forceinline__ double feq_flow(int d, double pr, double rho, double ux, double uy) {
  const double cu = CX(d) * ux + CY(d) * uy, uu = ux * ux + uy * uy;
  const double su = 3.0 * cu + 4.5 * cu * cu - 1.5 * uu;
  return 3.0 * pr * (WQ<double>(d) - (d == 0 ? 1.0 : 0.0)) + rho * WQ<double>(d) * su;
}
// eta-weighted equilibrium of lattices 2 and 3 (Sec. 3), moving direction d >= 1.
__device__ __forceinline__ double feq_scalar_moving(int d, double c, double eta, double cux, double cuy) {
  return WQ<double>(d) * eta * c + 3.0 * WQ<double>(d) * (CX(d) * cux + CY(d) * cuy);
}

// Block-wide FP64 reduction (wave64 shuffles, then LDS across the four
// waves); the result is valid in thread 0.  Fixed order: bitwise reproducible.
__device__ __forceinline__ double wave_red(double v, bool is_max) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) {
    const double o = __shfl_down(v, off, 64);
    v = is_max ? fmax(v, o) : v + o;
  }
  return v;
}
__device__ double block_reduce(double v, bool is_max) {
  __shared__ double sh[kBlock / 64];
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  v = wave_red(v, is_max);
  if (lane == 0) sh[wid] = v;
  __syncthreads();
  if (threadIdx.x == 0) {
    double r = sh[0];
    for (int k = 1; k < kBlock / 64; ++k) r = is_max ? fmax(r, sh[k]) : r + sh[k];
    v = r;
  }
  __syncthreads();
  return v;
}

// ------------------------------------------------------------------- kernels
// Node (x, y) of the source of gathered population i (its emitter): x - c_i
// inside the fluid, the node itself for a bounce-back at a wall.
__device__ __forceinline__ int emitter(const DevParams& p, int i, int x, int y) {
  int sx = wrap(x - CX(i), p.nx), sy = y - CY(i);
  if (p.periodic_y) sy = wrap(sy, p.ny);
  else if (sy < 0 || sy >= p.ny) return y * p.nx + x;
  return sy * p.nx + sx;
}

// phi(n+1) = phi(n) + [stored g_0 shift + sum of the gathered moving g_i]
// + the pending multiplier term cdef M_phi lambda(n) sum_i w_i h'(phi(n)(emitter_i));
// psi likewise with the uniform term cdef M_psi (mubar(n) - mu_ref).
template <class S, class C>
__global__ __launch_bounds__(kBlock) void k_moments(DevParams p, const S* __restrict__ P, const double* __restrict__ prev,
                                                    const DevScalars* __restrict__ pend, double* __restrict__ phipsi) {
  const int n = blockIdx.x * kBlock + threadIdx.x;
  if (n >= p.N) return;
  const int x = n % p.nx, y = n / p.nx;
  const double lam = pend->cdef * p.M_phi * pend->lambda_phi;
  C a = C(0), b = C(0);
  double corr = 0.0;
#pragma unroll
  for (int i = 0; i < 9; ++i) {
    a += pull<S, C>(p, P, 1, i, x, y, prev);
    corr += WQ<double>(i) * hprime(p, prev[emitter(p, i, x, y)]);
  }
  phipsi[n] = prev[n] + (double)a + lam * corr;
  if (p.surf) {
#pragma unroll
    for (int i = 0; i < 9; ++i) b += pull<S, C>(p, P, 2, i, x, y, prev);
    phipsi[(size_t)p.N + n] = prev[(size_t)p.N + n] + (double)b + pend->cdef * p.M_psi * (pend->mubar_psi - p.mu_ref);
  } else {
    phipsi[(size_t)p.N + n] = 0.0;
  }
}

__global__ __launch_bounds__(kBlock) void k_mu_partials(DevParams p, const double* __restrict__ phipsi, double* __restrict__ mu,
                                                        double* __restrict__ partials) {
  const double* phi = phipsi;
  const double* psi = phipsi + p.N;
  double s1 = 0.0, s2 = 0.0, s3 = 0.0, s4 = 0.0;
  for (int n = blockIdx.x * kBlock + threadIdx.x; n < p.N; n += gridDim.x * kBlock) {
    const int x = n % p.nx, y = n / p.nx;
    const double ph = phi[n], ps = psi[n];
    const Lap L = laplace(p, phi, psi, x, y);
    const double mp = mu_phi_of(p, ph, ps, L), ms = mu_psi_of(p, ph, ps, L);
    mu[n] = mp;
    mu[(size_t)p.N + n] = ms;
    const double hp = hprime(p, ph);
    s1 += hp * mp;
    s2 += hp * hp;
    s3 += ms;
    s4 += hval(p, ph);
  }
  s1 = block_reduce(s1, false);
  s2 = block_reduce(s2, false);
  s3 = block_reduce(s3, false);
  s4 = block_reduce(s4, false);
  if (threadIdx.x == 0) {
    partials[kSums * blockIdx.x + 0] = s1;
    partials[kSums * blockIdx.x + 1] = s2;
    partials[kSums * blockIdx.x + 2] = s3;
    partials[kSums * blockIdx.x + 3] = s4;
  }
}

__global__ __launch_bounds__(kBlock) void k_multipliers(DevParams p, int nblk, const double* __restrict__ partials,
                                                        DevScalars* __restrict__ sc) {
  double s[kSums] = {0.0, 0.0, 0.0, 0.0};
  for (int b = threadIdx.x; b < nblk; b += kBlock)
    for (int k = 0; k < kSums; ++k) s[k] += partials[kSums * b + k];
  for (int k = 0; k < kSums; ++k) s[k] = block_reduce(s[k], false);
  if (threadIdx.x == 0) {
    sc->lambda_phi = lambda_of(p, s[0], s[1], s[3]);
    sc->mubar_psi = s[2] / (double)p.N;
  }
}

// Force, velocity and pressure at (x,y) from the phi/psi and mu planes and the
// gathered f (O5, O6 of the step), in FP64.
struct Macro { double rho, ux, uy, pr, Fx, Fy, grx, gry; };
template <class C>
__device__ __forceinline__ Macro macro_node(const DevParams& p, const double* __restrict__ phi, const double* __restrict__ psi,
                                            const double* __restrict__ mup, const double* __restrict__ mus, const C* f, int x, int y) {
  const int n = y * p.nx + x;
  const double ph = phi[n], ps = psi[n];
  Macro M;
  M.rho = rho_of(p, ph);
  double grx = 0, gry = 0, gpx = 0, gpy = 0, gsx = 0, gsy = 0;
#pragma unroll
  for (int i = 1; i < 9; ++i) {
    const Nb b = nbr(p, x, y, CX(i), CY(i));
    const double w3 = 3.0 * WQ<double>(i);  // w_i / c_s^2
    const double pn = phi[b.idx];
    double rn;
    if (b.side && wet_side(p, b.side)) rn = rho_of(p, pn + Jphi(p, pn, psi[b.idx]) / p.kappa);
    else rn = rho_of(p, pn);
    grx += w3 * CX(i) * rn;
    gry += w3 * CY(i) * rn;
    const double mpn = mup[b.idx], msn = mus[b.idx];
    gpx += w3 * CX(i) * mpn;
    gpy += w3 * CY(i) * mpn;
    gsx += w3 * CX(i) * msn;
    gsy += w3 * CY(i) * msn;
  }
  M.grx = grx;
  M.gry = gry;
  M.Fx = -ph * gpx - ps * gsx + M.rho * p.gx;
  M.Fy = -ph * gpy - ps * gsy + M.rho * p.gy;
  const double jx = (double)(f[1] - f[3] + f[5] - f[6] - f[7] + f[8]);
  const double jy = (double)(f[2] - f[4] + f[5] + f[6] - f[7] - f[8]);
  M.ux = (jx + 0.5 * M.Fx) / M.rho;
  M.uy = (jy + 0.5 * M.Fy) / M.rho;
  const double snz = (double)(f[1] + f[2] + f[3] + f[4] + f[5] + f[6] + f[7] + f[8]);
  // c_s^2/(1 - w0) = 3/5, w0/(2 c_s^2) = 2/3
  M.pr = 0.6 * (snz + 0.5 * (M.ux * grx + M.uy * gry) - M.rho * (2.0 / 3.0) * (M.ux * M.ux + M.uy * M.uy));
  return M;
}

// MRT collision of a scalar lattice (g or h) in moment space, given the
// gathered moving populations c[1..8], the exact zeroth moment c0 (phi or
// psi), advecting velocity v, the backward difference dq of c0 v, the
// source Rt = R + dR/2 and the rates; writes the shifted rest value
// (post-collision c_0 minus c0) and the moving values.
template <class C>
__device__ __forceinline__ void collide_scalar(const C* c, C c0, C eta, C vx, C vy, C dqx, C dqy, C Rt,
                                               const double* sr, C* o) {
  C m[9];
  moments_noncons(c, m);
  const C third = C(1.0 / 3.0);
  const C meq[9] = {c0, c0 * vx, c0 * vy, eta * c0 * third, C(0), eta * c0 * third, c0 * vy * third, c0 * vx * third,
                    eta * c0 * C(1.0 / 9.0)};
  const C mv[9] = {C(0), dqx, dqy, C(0), C(0), C(0), dqy * third, dqx * third, C(0)};
  const C src[9] = {Rt, C(0), C(0), Rt * third, C(0), Rt * third, C(0), C(0), Rt * C(1.0 / 9.0)};
  const C rt[9] = {(C)sr[0], (C)sr[1], (C)sr[1], (C)sr[2], (C)sr[2], (C)sr[2], (C)sr[3], (C)sr[3], (C)sr[4]};
#pragma unroll
  for (int k = 1; k < 9; ++k) m[k] = m[k] - rt[k] * (m[k] - meq[k]) + (C(1) - C(0.5) * rt[k]) * mv[k] + src[k];
  moving_populations(m, o);
  // rest population: m00 relaxes to c0 exactly, plus the source
  o[0] = Rt - m[3] - m[5] + m[8];
}

// XCD-aware order of the tiles: the hardware hands consecutive workgroups to
// the eight XCDs in turn; remapping gives each XCD one contiguous band of tiles
// so that the halo rows a tile re-reads sit in that XCD's own L2.
__device__ __forceinline__ int xcd_tile(int b, int nb) {
  const int q = nb / 8, r = nb % 8, xcd = b % 8, idx = b / 8;
  return xcd < r ? xcd * (q + 1) + idx : r * (q + 1) + (xcd - r) * q + idx;
}
__device__ __forceinline__ int modp(int a, int n) { a %= n; return a < 0 ? a + n : a; }

struct StepArgs {
  const void* Pin;
  void* Pout;
  const double* ref;        // phi(n-1), psi(n-1): FP64 planes, shift reference of the stored rest populations
  double* out;              // phi(n), psi(n)
  const void* hin;          // u, v (advecting), R_phi, R_psi of step n-1: 6 planes, compute type
  void* hout;               // the same for step n
  const DevScalars* pend;   // multipliers pending on Pin (from step n-1)
  DevScalars* next;         // multipliers of step n, written by k_step_finish
  double* partials;         // [ntiles][kSums]: S1, S2, S3, S4 (S4 only under phi_hold, else 0)
  int have_hist, nstrips, seg_rows, ntiles;
  // Non-null: the multipliers pending on Pin are reduced here, by every
  // workgroup, from step n-1's partials ([ntiles][kSums], the same tiling; step
  // n-1 had a history iff prev_have_hist) instead of being read from pend;
  // k_step_finish did not run for step n-1.
  const double* prev_partials;
  int prev_have_hist;
  int split_walls;          // walled sweep: wall-free segments take the periodic form
};

// lambda(n) = S1/S2, mubar(n) = S3/N from the per-tile partial sums of
// k_step (eq15 and the psi constraint), in a fixed order: bitwise
// reproducible.  A separate launch rather than a last-tile-done reduction
// inside k_step: the agent-scope release fence that pattern needs on every
// tile writes back the XCD's L2 and cost more than the whole step.
// lambda(n) = S1/S2 and mubar(n) = S3/N from the per-workgroup sums, in a
// fixed order (every thread of the block gets the result); cdef weights the
// multiplier terms step n+1 applies (1.5 from R + dR/2, 1 on a first step).
// In two parts, so that a step can issue the loads of the previous step's
// partial sums ahead of its own gathers and reduce them once those are in
// flight: each thread's share (the first kBlock threads, as in k_step_finish),
// then the block's three sums in one pass (each: a wave reduction, then thread 0
// adds the waves' results in wave order) and the multipliers.
__device__ __forceinline__ void multipliers_load(const double* __restrict__ partials, int ntiles, double* t) {
#pragma unroll
  for (int c = 0; c < kSums; ++c) t[c] = 0.0;
  if (threadIdx.x < kBlock) {
#pragma unroll 4
    for (int b = threadIdx.x; b < ntiles; b += kBlock) {
#pragma unroll
      for (int c = 0; c < kSums; ++c) t[c] += partials[kSums * (size_t)b + c];
    }
  }
}
__device__ __forceinline__ DevScalars multipliers_reduce(const double* t, const DevParams& p, int have_hist) {
  __shared__ double sh[kSums][kBlock / 64];
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  double w[kSums];
#pragma unroll
  for (int c = 0; c < kSums - 1; ++c) w[c] = wave_red(t[c], false);
  w[kSums - 1] = p.phi_hold ? wave_red(t[kSums - 1], false) : 0.0;   // S4 serves the hold only
  if (lane == 0 && wid < kBlock / 64) {
#pragma unroll
    for (int c = 0; c < kSums; ++c) sh[c][wid] = w[c];
  }
  __syncthreads();
  __shared__ DevScalars res;
  if (threadIdx.x == 0) {
    double r[kSums];
#pragma unroll
    for (int c = 0; c < kSums; ++c) {
      r[c] = sh[c][0];
      for (int k = 1; k < kBlock / 64; ++k) r[c] = r[c] + sh[c][k];
    }
    res.lambda_phi = lambda_of(p, r[0], r[1], r[3]);
    res.mubar_psi = r[2] / (double)p.N;
    res.cdef = have_hist ? 1.5 : 1.0;
  }
  __syncthreads();
  return res;
}
__device__ __forceinline__ DevScalars multipliers_of(const double* __restrict__ partials, int ntiles, const DevParams& p,
                                                    int have_hist) {
  double t[kSums];
  multipliers_load(partials, ntiles, t);
  return multipliers_reduce(t, p, have_hist);
}
__device__ __forceinline__ void finish_body(const double* __restrict__ partials, int ntiles, const DevParams& p,
                                            int have_hist, DevScalars* __restrict__ next) {
  const DevScalars r = multipliers_of(partials, ntiles, p, have_hist);
  if (threadIdx.x == 0) *next = r;
}

__global__ __launch_bounds__(kBlock) void k_step_finish(const DevParams* __restrict__ pp, const double* __restrict__ partials,
                                                        int ntiles, int have_hist, DevScalars* __restrict__ next) {
  finish_body(partials, ntiles, *pp, have_hist, next);
}

// Element at byte offset b (32-bit, per lane) from a row base pointer (64-bit,
// usually wave-uniform): the form the hardware addresses as a scalar base plus a
// vector offset, with no 64-bit address arithmetic per lane.
template <class T> __device__ __forceinline__ T* byte_at(T* base, unsigned b) { return (T*)((char*)base + b); }
template <class T> __device__ __forceinline__ const T* byte_at(const T* base, unsigned b) {
  return (const T*)((const char*)base + b);
}

// Gather of population i of lattice lat at the column whose byte offset (in
// storage elements) is b0 in row y; bm, bp are the byte offsets of the
// columns x - 1 and x + 1 (wrapped).  For a wave whose lanes share y the plane
// and row form a wave-uniform base.  Wall sources as in pull().
template <class S, class C, bool WALLS, int lat>
__device__ __forceinline__ C pull_row(const DevParams& p, const S* __restrict__ P, size_t N, int i, int y,
                                      unsigned bm, unsigned b0, unsigned bp) {
  // f is gathered once per step (g and h twice: for phi/psi and for the
  // collision), so its loads stream past the L2 instead of evicting g and h.
  auto ld = [&](const S* rowbase, unsigned b) {
    const S* q = byte_at(rowbase, b);
    if constexpr (lat == 0) return (C)__builtin_nontemporal_load(q);
    else return (C)*q;
  };
  if constexpr (kHalf<S> && lat > 0) {
    if (i == 0) return (C)*byte_at(rest_plane(P, N, lat) + (size_t)y * p.nx, 2 * b0);
  }
  const unsigned sb = CX(i) > 0 ? bm : (CX(i) < 0 ? bp : b0);
  int sy = y - CY(i);
  if (!WALLS) {
    sy = sy < 0 ? sy + p.ny : (sy >= p.ny ? sy - p.ny : sy);
  } else if (sy < 0 || sy >= p.ny) {
    const int bc = sy < 0 ? p.bc_bottom : p.bc_top;
    if (lat == 0 && bc == LBM_BC_FREESLIP) return ld(P + (size_t)MIRY(i) * N + (size_t)y * p.nx, sb);
    return ld(P + (size_t)(9 * lat + OPP(i)) * N + (size_t)y * p.nx, b0);
  }
  return ld(P + (size_t)(9 * lat + i) * N + (size_t)sy * p.nx, sb);
}

__device__ __forceinline__ int wave_uniform(int v) { return __builtin_amdgcn_readfirstlane(v); }
// Outputs of a step are not read again by it: streaming stores keep them from
// evicting the populations the tile's phases re-read from L2.
template <bool NT, class T> __device__ __forceinline__ void store_hint(T* p, T v) {
  if constexpr (NT) __builtin_nontemporal_store(v, p);
  else *p = v;
}
// A wave-uniform value the optimiser cannot see through: what is derived from
// it inside a loop stays in the loop instead of being hoisted into registers.
template <class T> __device__ __forceinline__ T opaque(T v) {
  asm volatile("" : "+s"(v));
  return v;
}
template <class T> __device__ __forceinline__ T opaque_v(T v) {   // the same for a value held in VGPRs
  asm volatile("" : "+v"(v));
  return v;
}

// One fused time step for a strip of kStripW = 60 columns and a segment of
// rows, swept upward (256 threads = 4 waves).  The 64 lanes of a wave cover the
// columns X0-2 .. X0+61 of one row: the strip plus the two halo columns on
// each side that the stencils need, so no phase needs a second pass for its
// x halo.  Per iteration every wave handles one row of each phase:
//  H  h'(phi(n-1)) of a row four iterations ahead of its use
//  A  phi(n), psi(n) of row r+2 from the gathered g, h, the FP64 reference
//     planes and the pending multiplier term (the segment's rows go to the
//     output planes)
//  B  mu_phi, mu_psi of row r+1 (wall terms from the first fluid row); FP64
//     sums of h' mu_phi, h'^2, mu_psi over the segment's nodes
//  C  force, velocity, pressure, sources and collision of row r; the
//     multiplier terms of this step's sources are left out of the stored
//     populations and of the stored source history (deferred to step n+1)
// The rows live in LDS rings indexed by row: each halo row of the segment is
// computed once, and the g_i, h_i (i >= 1) that A gathers for a row of the
// segment wait in LDS (as stored) for that row's collision, so C gathers
// only f from memory.  At a wall the ghost rows beyond it hold the nearest
// fluid row's values (computed again, not copied).
// k_step_finish then reduces the block sums to lambda(n), mubar(n) (or, on
// small grids inside a captured run, the next step's workgroups do).
// Schedules of step_body: the sweep, or one tile of four rows in one pass with
// eight waves (kOneShot8) or four (kOneShot4).
enum { kSweep = 0, kOneShot8 = 1, kOneShot4 = 2 };
// Manufactured source of the accuracy test (Sec. 4.1) at node (x, y) of step
// n, in lattice units (dt times the physical source): the exact fields
// phi^e = e^-t sin(2 pi (x - 0.05 t)) cos(2 pi (y + 0.03 t)) / 2 and psi^e =
// 1/2 + e^-2t cos(2 pi (x - 0.05 t)) sin(2 pi (y + 0.03 t)) / 20 solve the
// phi and psi equations with the prescribed velocity when S_phi = -phi^e +
// M (mu_phi^e - 0) and S_psi = -2 (psi^e - 1/2) + M (mu_psi^e - mubar_psi^e),
// mu^e the chemical potentials (eq_muphi, eq_mupsi; the Laplacian of phi^e
// is -8 pi^2 phi^e, lambda_s = 0) and mubar_psi^e = -beta (1 - a^2/2 + 9 a^4
// / 64) + W a^2 / 8, a = e^-t / 2, their stated means.  The lattice mobility
// is M dt, so dt S = -dt phi^e + M_lattice mu^e; kappa in physical units is
// the lattice kappa times dx^2.
__device__ __forceinline__ void manufactured_source(const DevParams& p, unsigned x, int y, int n, double& sphi,
                                                    double& spsi) {
  const double dx = p.mms_dx, dt = p.mms_dt, t = (double)n * dt, tp = 2.0 * 3.14159265358979323846;
  const double X = tp * ((double)x * dx - 0.05 * t), Y = tp * ((double)y * dx + 0.03 * t);
  const double a = 0.5 * exp(-t);
  const double ph = a * sin(X) * cos(Y), ps = 0.5 + 0.05 * exp(-2.0 * t) * cos(X) * sin(Y);
  const double kap = p.kappa * dx * dx;
  const double mu_phi = 4.0 * p.beta * (1.0 - ps) * (ph * ph * ph - ph) + kap * tp * tp * 2.0 * ph + p.W * ps * ph;
  const double mu_psi = p.kBT * log(ps / (1.0 - ps)) - p.beta * (1.0 - ph * ph) * (1.0 - ph * ph) + 0.5 * p.W * ph * ph;
  const double a2 = a * a, mubar = -p.beta * (1.0 - 0.5 * a2 + 9.0 * a2 * a2 / 64.0) + p.W * a2 / 8.0;
  sphi = -dt * ph + p.M_phi * mu_phi;
  spsi = -dt * 2.0 * (ps - 0.5) + p.M_psi * (mu_psi - mubar);
}

// LDS of one step workgroup, shared by the walled and the periodic form of a
// schedule (a kernel that holds both allocates it once; WK: a kernel with the
// walled form).
template <class S, class C, int SCHED, bool WK>
struct StepLds {
  // The walled form of the row sweep in FP32 and FP16 storage keeps each
  // thread's three FP64 sums (h' mu_phi, h'^2, mu_psi) here instead of in
  // registers: held in registers they are spilled to scratch there, and every
  // reload waits for all the row's gathers in flight.  The wall-free form keeps
  // them in registers; both add the same terms in the same order.
  static constexpr bool LSUM = sizeof(S) <= 4 && SCHED == kSweep && WK;
  // Ring rows: h' 16 (H writes at most 15 rows ahead of the oldest row C
  // reads); (phi, psi) 16, or 12 where LDS is short (FP64 storage, and the
  // sums above): A writes at most 10 rows ahead of the oldest row C reads;
  // (mu_phi, mu_psi) 8, or 6 beside the sums: B writes rows up to 4 ahead of
  // the oldest row C reads, after the barrier that ends C's reads of the rows
  // it replaces.  Row gy lives in slot gy mod rows (a mask for 16 and 8: the
  // remainder costs the periodic 4096^2 FP32 step 0.5%).
  static constexpr int RP = 16, RPP = (sizeof(S) == 8 || LSUM) ? 12 : 16, RM = LSUM ? 6 : 8;
  static constexpr bool H16 = kHalf<S>;
  // g_1..g_8, h_1..h_8 of a segment row from A to C, in storage form (FP64
  // storage: 48 KB, with the 12-slot (phi, psi) ring two workgroups per CU
  // still fit; C then gathers only f).  Six slots: the row wave w's A handles
  // at iteration k (Y0+4k+2+w) takes the slot of the row its C handled at
  // iteration k-1 (Y0+4k-4+w), which no other wave reads; C reads a row at
  // least one barrier after A wrote it.
  static constexpr int RS = 6;
  C hp[RP][kStripW + 6];                             // h'(phi(n-1)), columns X0-3 .. X0+62
  double2 pp[RPP][64];                               // (phi, psi)(n), columns X0-2 .. X0+61
  double2 mu[RM][64];                                // (mu_phi, mu_psi), columns X0-2 .. X0+61 (lanes 1..62 used)
  float2 ref[H16 ? RP : 1][H16 ? kStripW + 6 : 1];   // FP16 storage: (phi, psi)(n-1) as in hp
  S gh[RS][16][64];
  double2 u[SCHED == kOneShot8 ? 4 : 1][SCHED == kOneShot8 ? 64 : 1];   // velocity of the split collision
  double sacc[LSUM ? 3 : 1][LSUM ? kBlock : 1];
};
template <class S, class C, int SCHED, bool WK>
__device__ __forceinline__ StepLds<S, C, SCHED, WK>& step_lds() {
  __shared__ StepLds<S, C, SCHED, WK> lds;
  return lds;
}
template <class S, class C, bool WALLS, int SCHED = kSweep, bool MMS = false, bool WK = WALLS>
__device__ __forceinline__ void step_body(const DevParams& p, const StepArgs& a, const int tile, const int mms_step = 0) {
  // Store hint, as measured on MI355X.  FP32 and FP16 storage store plainly on
  // the row sweep and the four-wave tile: the lines of neighbouring strips
  // combine in the L2 before they are written back (at 4096^2 WRITE_SIZE falls
  // by 7% and the step takes 1.28 instead of 1.52 ms; the 512-case batch 1.57
  // instead of 1.65 ms).  FP64 storage, whose wider rows fill whole lines, and
  // the eight-wave tile of small grids keep the non-temporal hint (FP64 4096^2:
  // 2.35 against 2.45 ms).
  constexpr bool NTS = SCHED == kOneShot8 || sizeof(S) == 8;
  using L = StepLds<S, C, SCHED, WK>;
  constexpr int RP = L::RP, RM = L::RM, RS = L::RS, RPP = L::RPP;
  constexpr bool LS = L::LSUM && WALLS;
  // ring slots of a (wave-uniform) row index, which may lie below 0 (halo rows)
  auto pslot = [](int gy) {
    if constexpr ((RPP & (RPP - 1)) == 0) return gy & (RPP - 1);
    else return wave_uniform(((gy % RPP) + RPP) % RPP);
  };
  auto mslot = [](int gy) {
    if constexpr ((RM & (RM - 1)) == 0) return gy & (RM - 1);
    else return wave_uniform(((gy % RM) + RM) % RM);
  };
  constexpr bool H16 = L::H16;
  L& lds = step_lds<S, C, SCHED, WK>();
  auto& sHp = lds.hp;
  auto& sPP = lds.pp;
  auto& sMU = lds.mu;
  auto& sRef = lds.ref;
  auto& sGH = lds.gh;

  const int X0 = (tile % a.nstrips) * kStripW, Y0 = (tile / a.nstrips) * a.seg_rows;
  const int Yend = min(Y0 + a.seg_rows, p.ny);
  auto gh_slot = [&](int gy) { return (gy - Y0 + 2 * RS) % RS; };   // gy >= Y0 - 2
  const size_t N = (size_t)p.N;
  const S* __restrict__ Pin = (const S*)a.Pin;
  S* __restrict__ Pout = (S*)a.Pout;
  const double* __restrict__ ref = a.ref;
  // The multipliers pending on Pin and their weights in the pending terms,
  // set by set_pend() before phase A first runs: reduced from the previous
  // step's sums (small grids inside a captured run) or as k_step_finish left
  // them.
  // pend_load() issues the loads, pend_set() reduces and sets the terms.
  DevScalars pend;
  double lam1_ = 0.0, mub1_ = 0.0, pt_[kSums];
  auto pend_load = [&]() {
    if (a.prev_partials) multipliers_load(a.prev_partials, a.ntiles, pt_);
    else pend = *a.pend;
  };
  auto pend_set = [&]() {
    if (a.prev_partials) pend = multipliers_reduce(pt_, p, a.prev_have_hist);
    lam1_ = pend.cdef * p.M_phi * pend.lambda_phi;
    mub1_ = pend.cdef * p.M_psi * (pend.mubar_psi - p.mu_ref);
  };
  auto set_pend = [&]() {
    pend_load();
    pend_set();
  };
  const int lane = threadIdx.x & 63;
  const int wave = wave_uniform(threadIdx.x >> 6);
  // fluid row of a (possibly ghost or wrapped) row index
  auto row_of = [&](int gy) { return WALLS ? (gy < 0 ? 0 : (gy >= p.ny ? p.ny - 1 : gy)) : modp(gy, p.ny); };
  // ring row of the stencil centre: at a wall a ghost row is its fluid row's copy
  auto centre = [&](int gy) { return WALLS ? row_of(gy) : gy; };
  auto colm = [&](unsigned x) { return x == 0 ? (unsigned)p.nx - 1 : x - 1; };
  auto colp = [&](unsigned x) { return x + 1 == (unsigned)p.nx ? 0u : x + 1; };
  const unsigned xcol = (unsigned)modp(X0 - 2 + lane, p.nx);   // this lane's column
  // The phases take the lane and its column as arguments, opaque copies made per
  // iteration: what they derive from them (byte offsets, LDS addresses) is then
  // recomputed per row instead of being hoisted out of the sweep and held in
  // registers for its whole length.
  auto is_interior = [&](int ln) { return ln >= 2 && ln < kStripW + 2 && X0 + ln - 2 < p.nx; };

  // ---- H: h'(phi(n-1)) of row gy into ring slot gy; lanes 0 and 1 also take
  // the outer columns X0-3 and X0+62.  gather_H loads (phi, psi)(n-1) of the
  // lane's column into v[0], v[1] and of the outer column into v[2], v[3]
  // (psi for FP16 storage only); row_H fills the rings.
  auto gather_H = [&](int gy, int ln, unsigned x, double* v) {
    const double* r = ref + (size_t)row_of(gy) * p.nx;
    v[0] = *byte_at(r, x * (unsigned)sizeof(double));
    if constexpr (H16) v[1] = *byte_at(r + N, x * (unsigned)sizeof(double));
    if (ln < 2) {
      const unsigned xk = (unsigned)modp(X0 - 3 + (ln ? kStripW + 5 : 0), p.nx);
      v[2] = r[xk];
      if constexpr (H16) v[3] = r[N + xk];
    }
  };
  auto row_H = [&](int gy, int ln, const double* v) {
    sHp[gy & (RP - 1)][ln + 1] = (C)hprime(p, v[0]);
    if constexpr (H16) sRef[gy & (RP - 1)][ln + 1] = make_float2((float)v[0], (float)v[1]);
    if (ln < 2) {
      const int k = ln ? kStripW + 5 : 0;
      sHp[gy & (RP - 1)][k] = (C)hprime(p, v[2]);
      if constexpr (H16) sRef[gy & (RP - 1)][k] = make_float2((float)v[2], (float)v[3]);
    }
  };

  // ---- A: (phi, psi)(n) of row gy into ring slot gy
  // gather_A loads the streamed g, h of the row (tg, th) and (phi, psi)(n-1)
  // of the node (r0[0], r0[1]); row_A sums them.
  auto gather_A = [&](int gy, unsigned x, C* tg, C* th, double* r0) {
    const int y = wave_uniform(row_of(gy));
    const unsigned xs = x * sizeof(S), xsm = colm(x) * sizeof(S), xsp = colp(x) * sizeof(S), xd = x * sizeof(double);
    const size_t row = (size_t)y * p.nx;
    r0[0] = *byte_at(ref + row, xd);
    r0[1] = *byte_at(ref + N + row, xd);
#pragma unroll
    for (int i = 0; i < 9; ++i) {
      tg[i] = pull_row<S, C, WALLS, 1>(p, Pin, N, i, y, xsm, xs, xsp);
      th[i] = p.surf ? pull_row<S, C, WALLS, 2>(p, Pin, N, i, y, xsm, xs, xsp) : C(0);
    }
  };
  auto row_A = [&](int gy, int ln, unsigned x, const C* tg, const C* th, const double* r0) {
    const int y = wave_uniform(row_of(gy)), yc = centre(gy);
    const bool keep = gy >= Y0 && gy < Yend;   // a row C collides
    const int ks = gh_slot(gy);
    const unsigned xd = x * sizeof(double);
    C sg = C(0), sh = C(0), corr = C(0);
    const size_t row = (size_t)y * p.nx;
#pragma unroll
    for (int i = 0; i < 9; ++i) {
      // emitter of g_i: x - c_i, or the node itself at a wall
      const int sy = y - CY(i);
      const bool bb = WALLS && (sy < 0 || sy >= p.ny);
      const int er = bb ? yc & (RP - 1) : (yc - CY(i)) & (RP - 1), ec = bb ? ln + 1 : ln + 1 - CX(i);
      const C t = tg[i];
      if (i && keep) sGH[ks][i - 1][ln] = (S)t;
      if constexpr (H16) sg += i ? decode<S, C>(p, 1, i, (S)t, (C)sRef[er][ec].x) : t;   // rest: FP32 plane
      else sg += t;
      corr += WQ<C>(i) * sHp[er][ec];
    }
    const double ph = r0[0] + (double)sg + lam1_ * (double)corr;
    double ps = 0.0;
    if (p.surf) {
#pragma unroll
      for (int i = 0; i < 9; ++i) {
        const C t = th[i];
        if (i && keep) sGH[ks][7 + i][ln] = (S)t;
        if constexpr (H16) {
          const int sy = y - CY(i);
          const bool bb = WALLS && (sy < 0 || sy >= p.ny);
          const int er = bb ? yc & (RP - 1) : (yc - CY(i)) & (RP - 1), ec = bb ? ln + 1 : ln + 1 - CX(i);
          sh += i ? decode<S, C>(p, 2, i, (S)t, (C)sRef[er][ec].y) : t;
        } else {
          sh += t;
        }
      }
      ps = r0[1] + (double)sh + mub1_;
    }
    sPP[pslot(gy)][ln] = make_double2(ph, ps);
    if (is_interior(ln) && gy >= Y0 && gy < Yend) {
      store_hint<NTS>(byte_at(a.out + row, xd), ph);
      store_hint<NTS>(byte_at(a.out + N + row, xd), ps);
    }
  };

  // ---- B: (mu_phi, mu_psi) of row gy into ring slot gy (lanes 1..62)
  double s1 = 0.0, s2 = 0.0, s3 = 0.0, s4 = 0.0;
  auto row_B = [&](int gy, int ln) {
    const int y = wave_uniform(row_of(gy)), yc = centre(gy);
    const int l = min(max(ln, 1), 62);   // lanes 0 and 63 have no neighbour column: computed, unused
    const double2 c = sPP[pslot(yc)][l];
    const double ph = c.x, ps = c.y;
    // Next to a wetting wall the wall values J of this row's columns l - 1,
    // l, l + 1 enter: each lane evaluates them at its own column, the
    // neighbours' come by lane shuffle (the row is wave-uniform).
    const int wside = !WALLS ? 0 : (y == 0 ? -1 : (y == p.ny - 1 ? 1 : 0));
    const bool wet = wside != 0 && wet_side(p, wside);
    double jp = 0.0, js = 0.0;
    if (wet) {
      const double2 o = sPP[pslot(yc)][ln];
      jp = Jphi(p, o.x, o.y);
      if (p.surf) js = Jpsi(p, o.x, o.y);
    }
    Lap L{0.0, 0.0, 0.0, 0.0};
#pragma unroll
    for (int i = 1; i < 9; ++i) {
      const double w2 = 6.0 * WQ<double>(i);
      const double2 nb = sPP[pslot((yc + CY(i)))][l + CX(i)];
      L.l0p += w2 * (nb.x - ph);
      L.l0s += w2 * (nb.y - ps);
      if (wet && CY(i) == wside) {   // the fluid node next to the ghost: column x + c_x of this row
        L.Tp += w2 * __shfl(jp, l + CX(i));
        if (p.surf) L.Ts += w2 * __shfl(js, l + CX(i));
      }
    }
    const double mp = mu_phi_of(p, ph, ps, L), ms = mu_psi_of(p, ph, ps, L);
    sMU[mslot(gy)][ln] = make_double2(mp, ms);
    if (is_interior(ln) && gy >= Y0 && gy < Yend) {
      const double hp = hprime(p, ph);
      if constexpr (LS) {
        double* q = &lds.sacc[0][threadIdx.x];
        q[0] = fma(hp, mp, q[0]);
        q[kBlock] = fma(hp, hp, q[kBlock]);
        q[2 * kBlock] += ms;
      } else {
        s1 = fma(hp, mp, s1);
        s2 = fma(hp, hp, s2);
        s3 += ms;
      }
      if (p.phi_hold) s4 += hval(p, ph);   // S4 serves the hold only
    }
  };

  // ---- C: collide row gy (a fluid row of the segment)
  const C* __restrict__ hin = (const C*)a.hin;
  C* __restrict__ hout = (C*)a.hout;
  // the gathers of a collision row (f only: g and h come from A through LDS),
  // issued an iteration phase ahead of their use
  auto gather_C = [&](int gy, unsigned x, C* f) {
    const size_t N = opaque((size_t)p.N);
    const unsigned xs = x * sizeof(S), xsm = colm(x) * sizeof(S), xsp = colp(x) * sizeof(S);
#pragma unroll
    for (int i = 0; i < 9; ++i) f[i] = pull_row<S, C, WALLS, 0>(p, Pin, N, i, gy, xsm, xs, xsp);
  };
  auto row_C = [&](int gy, int ln, unsigned x, C* f, C* g, C* h) {
    const size_t row = (size_t)gy * p.nx;
    const int lc = min(max(ln, 2), kStripW + 1);   // halo lanes compute a copy and store nothing
    const bool interior = is_interior(ln);
    const unsigned xs = x * sizeof(S), xd = x * sizeof(double), xc = x * sizeof(C);
    // An opaque copy of N and of the rates per row keeps the compiler from
    // hoisting the plane offsets and converted constants out of the sweep
    // loop into registers.
    const size_t N = opaque((size_t)p.N);
    const double lam1 = opaque_v(lam1_), mub1 = opaque_v(mub1_);
    double rf[5], rg[5], rh[5];
#pragma unroll
    for (int k = 0; k < 5; ++k) {
      rf[k] = opaque(p.sf[k]);
      rg[k] = opaque(p.sg[k]);
      rh[k] = opaque(p.sh[k]);
    }
    const double2 c = sPP[pslot(gy)][lc];
    const double ph = c.x, ps = c.y;
    const double2 mc = sMU[mslot(gy)][lc];
    const double ph0 = *byte_at(ref + row, xd);   // phi(n-1)

    {   // g_i, h_i (i >= 1) as A gathered them
      g[0] = h[0] = C(0);
      const int ks = gh_slot(gy);
#pragma unroll
      for (int i = 1; i < 9; ++i) {
        g[i] = (C)sGH[ks][i - 1][ln];
        h[i] = p.surf ? (C)sGH[ks][7 + i][ln] : C(0);
      }
    }
    // decoded (FP16 storage) gathers plus the pending multiplier terms of g_i, h_i
    if constexpr (H16) {
#pragma unroll
      for (int i = 0; i < 9; ++i) f[i] = decode<S, C>(p, 0, i, (S)f[i], C(0));
    }
#pragma unroll
    for (int i = 1; i < 9; ++i) {
      const int sy = gy - CY(i);
      const bool bb = WALLS && (sy < 0 || sy >= p.ny);
      const int er = bb ? gy & (RP - 1) : (gy - CY(i)) & (RP - 1), ec = bb ? lc + 1 : lc + 1 - CX(i);
      if constexpr (H16) {
        const float2 re = sRef[er][ec];
        g[i] = decode<S, C>(p, 1, i, (S)g[i], (C)re.x);
        if (p.surf) h[i] = decode<S, C>(p, 2, i, (S)h[i], (C)re.y);
      }
      g[i] += (C)(lam1 * WQ<double>(i) * (double)sHp[er][ec]);
      if (p.surf) h[i] += (C)(mub1 * WQ<double>(i));
    }
    // gradients of phi (wetting ghosts), mu_phi, mu_psi; Laplacians of phi, psi.
    // Next to a wetting wall the ghost row's phi takes J_phi / kappa: each lane
    // evaluates J_phi at its own column of the ghost row, the neighbours' come
    // by lane shuffle.
    const int wside = !WALLS ? 0 : (gy == 0 ? -1 : (gy == p.ny - 1 ? 1 : 0));
    const bool wet = wside != 0 && wet_side(p, wside);
    double jg = 0.0;
    if (wet) {
      const double2 o = sPP[pslot((gy + wside))][ln];
      jg = Jphi(p, o.x, o.y);
    }
    double gfx = 0, gfy = 0, gpx = 0, gpy = 0, gsx = 0, gsy = 0, l0p = 0, l0s = 0;
#pragma unroll
    for (int i = 1; i < 9; ++i) {
      const double w3 = 3.0 * WQ<double>(i), w2 = 2.0 * w3;
      const double2 nb = sPP[pslot((gy + CY(i)))][lc + CX(i)];
      double q = nb.x;
      if (wet && CY(i) == wside) q += __shfl(jg, lc + CX(i)) / p.kappa;
      l0p += w2 * (nb.x - ph);
      l0s += w2 * (nb.y - ps);
      const double rq = rho_of(p, q);   // grad rho from the neighbours' densities (ghost phi at a wall)
      if (CX(i)) gfx += (CX(i) * w3) * rq;
      if (CY(i)) gfy += (CY(i) * w3) * rq;
      const double2 mn = sMU[mslot(gy + CY(i))][lc + CX(i)];
      if (CX(i)) { gpx += (CX(i) * w3) * mn.x; gsx += (CX(i) * w3) * mn.y; }
      if (CY(i)) { gpy += (CY(i) * w3) * mn.x; gsy += (CY(i) * w3) * mn.y; }
    }
    const double grx = gfx, gry = gfy;
    const double rho = rho_of(p, ph);
    const double Fx = -ph * gpx - ps * gsx + rho * p.gx, Fy = -ph * gpy - ps * gsy + rho * p.gy;
    double ux = ((double)(f[1] - f[3] + f[5] - f[6] - f[7] + f[8]) + 0.5 * Fx) / rho;
    double uy = ((double)(f[2] - f[4] + f[5] + f[6] - f[7] - f[8]) + 0.5 * Fy) / rho;
    const double snz = (double)(f[1] + f[2] + f[3] + f[4] + f[5] + f[6] + f[7] + f[8]);
    double pr = 0.6 * (snz + 0.5 * (ux * grx + uy * gry) - rho * (2.0 / 3.0) * (ux * ux + uy * uy));
    if constexpr (MMS) {   // the accuracy test prescribes u and p
      ux = p.mms_ux;
      uy = p.mms_uy;
      pr = 0.0;
    }

    // Sources without this step's multiplier terms (those are deferred).  With
    // the chemical potentials of phase B: R_phi = -M_phi (mu_phi + kappa L0(phi))
    // and R_psi = -M_psi mu_psi - (M0 + M_psi lambda_s) L0(psi), identical to the
    // bulk terms plus the wall terms of eq_muphi / eq_mupsi.
    double Rp0 = -p.M_phi * (mc.x + p.kappa * l0p);
    double Rs0 = p.surf ? -p.M_psi * mc.y - (p.M0 + p.M_psi * p.lambda_s) * l0s : 0.0;
    if constexpr (MMS) {
      double sp, ss;
      manufactured_source(p, x, gy, mms_step, sp, ss);
      Rp0 += sp;
      Rs0 += ss;
    }
    // the psi source the collision carries includes M_psi mu_ref (the rest of the multiplier term is pending)
    const double Rs0c = p.surf ? Rs0 + p.M_psi * p.mu_ref : 0.0;
    double vx = ux, vy = uy, dpx = 0, dpy = 0, dsx = 0, dsy = 0, Rtp = Rp0, Rts = Rs0c;
    if (a.have_hist) {
      const C* hr = hin + row;
      if (!p.adv_raw) {
        vx = 0.5 * (ux + (double)*byte_at(hr, xc));
        vy = 0.5 * (uy + (double)*byte_at(hr + N, xc));
      }
      const double vxh = *byte_at(hr + 2 * N, xc), vyh = *byte_at(hr + 3 * N, xc), ps0 = *byte_at(ref + N + row, xd);
      dpx = ph * vx - ph0 * vxh;
      dpy = ph * vy - ph0 * vyh;
      dsx = ps * vx - ps0 * vxh;
      dsy = ps * vy - ps0 * vyh;
      // R(n-1) in full: stored part plus its multiplier term
      const double Rp_prev = (double)*byte_at(hr + 4 * N, xc) + p.M_phi * pend.lambda_phi * hprime(p, ph0);
      const double Rs_prev = (double)*byte_at(hr + 5 * N, xc) + p.M_psi * pend.mubar_psi;
      Rtp = 1.5 * Rp0 - 0.5 * Rp_prev;
      Rts = 1.5 * Rs0c - 0.5 * Rs_prev;
    }

    // ---- lattice 1: MRT with the pressure-based equilibrium and A^1 forcing
    {
      C m[9], o[9];
      m[0] = f[0] + f[1] + f[2] + f[3] + f[4] + f[5] + f[6] + f[7] + f[8];
      moments_noncons(f, m);
      const double uu = ux * ux + uy * uy, third = 1.0 / 3.0, av = ux * grx + uy * gry;
      const C meq[9] = {C(0), (C)(rho * ux), (C)(rho * uy), (C)(pr + rho * ux * ux), (C)(rho * ux * uy), (C)(pr + rho * uy * uy),
                        (C)(rho * uy * third), (C)(rho * ux * third), (C)((pr + rho * uu) * third)};
      const C mv[9] = {(C)av, (C)Fx, (C)Fy, (C)(ux * grx + uy * gry * third), (C)((ux * gry + uy * grx) * third),
                       (C)(uy * gry + ux * grx * third), (C)(Fy * third), (C)(Fx * third), (C)(av * third)};
      const C s2 = p.s2_local ? (C)(1.0 / (3.0 * mud_of(p, ph) / rho + 0.5)) : (C)rf[2];
      const C rt[9] = {(C)rf[0], (C)rf[1], (C)rf[1], s2, s2, s2, (C)rf[3], (C)rf[3], (C)rf[4]};
#pragma unroll
      for (int k = 0; k < 9; ++k) m[k] = m[k] - rt[k] * (m[k] - meq[k]) + (C(1) - C(0.5) * rt[k]) * mv[k];
      moving_populations(m, o);
      o[0] = m[0] - m[3] - m[5] + m[8];
      const bool wb = WALLS && gy == 0 && p.bc_bottom != LBM_BC_FREESLIP;
      const bool wt = WALLS && gy == p.ny - 1 && p.bc_top != LBM_BC_FREESLIP;
#pragma unroll
      for (int i = 0; i < 9; ++i) {
        C v = o[i];
        if (wb && CY(i) < 0) v -= (C)(6.0 * WQ<double>(i) * rho * CX(i) * p.uw_bottom);
        if (wt && CY(i) > 0) v -= (C)(6.0 * WQ<double>(i) * rho * CX(i) * p.uw_top);
        if (interior) store_hint<NTS>(byte_at(Pout + (size_t)i * N + row, xs), encode<S, C>(p, 0, i, v, C(0)));
      }
    }
    // store the populations of lattice lat (1 g, 2 h) with reference c
    auto store_scalar = [&](int lat, const C* o, C c) {
      if constexpr (H16) {
        C rest = o[0];
#pragma unroll
        for (int i = 1; i < 9; ++i) {
          const S t = encode<S, C>(p, lat, i, o[i], c);
          rest += o[i] - decode<S, C>(p, lat, i, t, c);   // what the FP16 value loses
          if (interior) store_hint<NTS>(byte_at(Pout + (size_t)(9 * lat + i) * N + row, xs), t);
        }
        if (interior) store_hint<NTS>(byte_at(rest_plane(Pout, N, lat) + row, 2 * xs), (float)rest);
      } else {
#pragma unroll
        for (int i = 0; i < 9; ++i)
          if (interior) store_hint<NTS>(byte_at(Pout + (size_t)(9 * lat + i) * N + row, xs), (S)o[i]);
      }
    };
    {
      C o[9];
      collide_scalar<C>(g, (C)ph, (C)p.eta_phi, (C)vx, (C)vy, (C)dpx, (C)dpy, (C)Rtp, rg, o);
      store_scalar(1, o, (C)ph);
    }
    if (p.surf) {   // without surfactant the h planes hold the zeros they were loaded with
      C o[9];
      collide_scalar<C>(h, (C)ps, (C)p.eta_psi, (C)vx, (C)vy, (C)dsx, (C)dsy, (C)Rts, rh, o);
      store_scalar(2, o, (C)ps);
    }
    if (interior) {
      C* ho = hout + row;
      store_hint<NTS>(byte_at(ho, xc), (C)ux);
      store_hint<NTS>(byte_at(ho + N, xc), (C)uy);
      store_hint<NTS>(byte_at(ho + 2 * N, xc), (C)vx);
      store_hint<NTS>(byte_at(ho + 3 * N, xc), (C)vy);
      store_hint<NTS>(byte_at(ho + 4 * N, xc), (C)Rp0);
      store_hint<NTS>(byte_at(ho + 5 * N, xc), (C)Rs0);
    }
  };

  // ---- C split over two waves per row (the eight-wave tile): wave w < 4 takes
  // the force, velocity, pressure and f collision of row Y0 + w, wave w + 4 the
  // g and h collisions of the same row, so that every SIMD interleaves two
  // waves through the heaviest phase.  The velocity goes through LDS across
  // one barrier that every wave of the workgroup reaches once (active or not).
  // The arithmetic is row_C's, term for term.
  auto& sU = lds.u;
  auto gather_Cf = [&](int gy, unsigned x, C* f) {
    const size_t N = opaque((size_t)p.N);
    const unsigned xs = x * sizeof(S), xsm = colm(x) * sizeof(S), xsp = colp(x) * sizeof(S);
#pragma unroll
    for (int i = 0; i < 9; ++i) f[i] = pull_row<S, C, WALLS, 0>(p, Pin, N, i, gy, xsm, xs, xsp);
  };
  // the history a collision row reads (its g, h come from A through LDS):
  // phi, psi(n-1); u, v and the stored R of step n-1
  auto gather_Cgh = [&](int gy, unsigned x, double* hv) {
    const size_t N = opaque((size_t)p.N);
    const size_t row = (size_t)gy * p.nx;
    const unsigned xd = x * sizeof(double), xc = x * sizeof(C);
    hv[0] = *byte_at(ref + row, xd);
    if (a.have_hist) {
      const C* hr = hin + row;
      hv[1] = (double)*byte_at(hr, xc);
      hv[2] = (double)*byte_at(hr + N, xc);
      hv[3] = (double)*byte_at(hr + 2 * N, xc);
      hv[4] = (double)*byte_at(hr + 3 * N, xc);
      hv[5] = *byte_at(ref + N + row, xd);
      hv[6] = (double)*byte_at(hr + 4 * N, xc);
      hv[7] = (double)*byte_at(hr + 5 * N, xc);
    }
  };
  auto row_Cf = [&](bool active, int gy, int ln, unsigned x, C* f) {
    const size_t row = (size_t)gy * p.nx;
    const int lc = min(max(ln, 2), kStripW + 1);
    const bool interior = is_interior(ln);
    const unsigned xs = x * sizeof(S), xc = x * sizeof(C);
    const size_t N = opaque((size_t)p.N);
    double ph = 0.0, rho = 1.0, ux = 0.0, uy = 0.0, pr = 0.0, Fx = 0.0, Fy = 0.0, grx = 0.0, gry = 0.0;
    if (active) {
      const double2 c = sPP[pslot(gy)][lc];
      ph = c.x;
      const double ps = c.y;
      if constexpr (H16) {
#pragma unroll
        for (int i = 0; i < 9; ++i) f[i] = decode<S, C>(p, 0, i, (S)f[i], C(0));
      }
      const int wside = !WALLS ? 0 : (gy == 0 ? -1 : (gy == p.ny - 1 ? 1 : 0));
      const bool wet = wside != 0 && wet_side(p, wside);
      double jg = 0.0;
      if (wet) {
        const double2 o = sPP[pslot((gy + wside))][ln];
        jg = Jphi(p, o.x, o.y);
      }
      double gfx = 0, gfy = 0, gpx = 0, gpy = 0, gsx = 0, gsy = 0;
#pragma unroll
      for (int i = 1; i < 9; ++i) {
        const double w3 = 3.0 * WQ<double>(i);
        const double2 nb = sPP[pslot((gy + CY(i)))][lc + CX(i)];
        double q = nb.x;
        if (wet && CY(i) == wside) q += __shfl(jg, lc + CX(i)) / p.kappa;
        const double rq = rho_of(p, q);   // as in row_C
        if (CX(i)) gfx += (CX(i) * w3) * rq;
        if (CY(i)) gfy += (CY(i) * w3) * rq;
        const double2 mn = sMU[mslot(gy + CY(i))][lc + CX(i)];
        if (CX(i)) { gpx += (CX(i) * w3) * mn.x; gsx += (CX(i) * w3) * mn.y; }
        if (CY(i)) { gpy += (CY(i) * w3) * mn.x; gsy += (CY(i) * w3) * mn.y; }
      }
      grx = gfx;
      gry = gfy;
      rho = rho_of(p, ph);
      Fx = -ph * gpx - ps * gsx + rho * p.gx;
      Fy = -ph * gpy - ps * gsy + rho * p.gy;
      ux = ((double)(f[1] - f[3] + f[5] - f[6] - f[7] + f[8]) + 0.5 * Fx) / rho;
      uy = ((double)(f[2] - f[4] + f[5] + f[6] - f[7] - f[8]) + 0.5 * Fy) / rho;
      const double snz = (double)(f[1] + f[2] + f[3] + f[4] + f[5] + f[6] + f[7] + f[8]);
      pr = 0.6 * (snz + 0.5 * (ux * grx + uy * gry) - rho * (2.0 / 3.0) * (ux * ux + uy * uy));
      sU[gy - Y0][ln] = make_double2(ux, uy);
    }
    __syncthreads();
    if (!active) return;
    double rf[5];
#pragma unroll
    for (int k = 0; k < 5; ++k) rf[k] = opaque(p.sf[k]);
    C m[9], o[9];
    m[0] = f[0] + f[1] + f[2] + f[3] + f[4] + f[5] + f[6] + f[7] + f[8];
    moments_noncons(f, m);
    const double uu = ux * ux + uy * uy, third = 1.0 / 3.0, av = ux * grx + uy * gry;
    const C meq[9] = {C(0), (C)(rho * ux), (C)(rho * uy), (C)(pr + rho * ux * ux), (C)(rho * ux * uy), (C)(pr + rho * uy * uy),
                      (C)(rho * uy * third), (C)(rho * ux * third), (C)((pr + rho * uu) * third)};
    const C mv[9] = {(C)av, (C)Fx, (C)Fy, (C)(ux * grx + uy * gry * third), (C)((ux * gry + uy * grx) * third),
                     (C)(uy * gry + ux * grx * third), (C)(Fy * third), (C)(Fx * third), (C)(av * third)};
    const C s2 = p.s2_local ? (C)(1.0 / (3.0 * mud_of(p, ph) / rho + 0.5)) : (C)rf[2];
    const C rt[9] = {(C)rf[0], (C)rf[1], (C)rf[1], s2, s2, s2, (C)rf[3], (C)rf[3], (C)rf[4]};
#pragma unroll
    for (int k = 0; k < 9; ++k) m[k] = m[k] - rt[k] * (m[k] - meq[k]) + (C(1) - C(0.5) * rt[k]) * mv[k];
    moving_populations(m, o);
    o[0] = m[0] - m[3] - m[5] + m[8];
    const bool wb = WALLS && gy == 0 && p.bc_bottom != LBM_BC_FREESLIP;
    const bool wt = WALLS && gy == p.ny - 1 && p.bc_top != LBM_BC_FREESLIP;
#pragma unroll
    for (int i = 0; i < 9; ++i) {
      C v = o[i];
      if (wb && CY(i) < 0) v -= (C)(6.0 * WQ<double>(i) * rho * CX(i) * p.uw_bottom);
      if (wt && CY(i) > 0) v -= (C)(6.0 * WQ<double>(i) * rho * CX(i) * p.uw_top);
      if (interior) store_hint<NTS>(byte_at(Pout + (size_t)i * N + row, xs), encode<S, C>(p, 0, i, v, C(0)));
    }
    if (interior) {
      C* ho = hout + row;
      store_hint<NTS>(byte_at(ho, xc), (C)ux);
      store_hint<NTS>(byte_at(ho + N, xc), (C)uy);
    }
  };
  auto row_Cgh = [&](bool active, int gy, int ln, unsigned x, C* g, C* h, const double* hv) {
    const size_t row = (size_t)gy * p.nx;
    const int lc = min(max(ln, 2), kStripW + 1);
    const bool interior = is_interior(ln);
    const unsigned xs = x * sizeof(S), xc = x * sizeof(C);
    const size_t N = opaque((size_t)p.N);
    double ph = 0.0, ps = 0.0, ph0 = 0.0, Rp0 = 0.0, Rs0 = 0.0, Rtp = 0.0, Rts = 0.0;
    double uxh = 0.0, uyh = 0.0, vxh = 0.0, vyh = 0.0, ps0 = 0.0;
    if (active) {
      const double lam1 = opaque_v(lam1_), mub1 = opaque_v(mub1_);
      const double2 c = sPP[pslot(gy)][lc];
      ph = c.x;
      ps = c.y;
      const double2 mc = sMU[mslot(gy)][lc];
      ph0 = hv[0];
      {   // g_i, h_i (i >= 1) as A gathered them
        g[0] = h[0] = C(0);
        const int ks = gh_slot(gy);
#pragma unroll
        for (int i = 1; i < 9; ++i) {
          g[i] = (C)sGH[ks][i - 1][ln];
          h[i] = p.surf ? (C)sGH[ks][7 + i][ln] : C(0);
        }
      }
#pragma unroll
      for (int i = 1; i < 9; ++i) {
        const int sy = gy - CY(i);
        const bool bb = WALLS && (sy < 0 || sy >= p.ny);
        const int er = bb ? gy & (RP - 1) : (gy - CY(i)) & (RP - 1), ec = bb ? lc + 1 : lc + 1 - CX(i);
        if constexpr (H16) {
          const float2 re = sRef[er][ec];
          g[i] = decode<S, C>(p, 1, i, (S)g[i], (C)re.x);
          if (p.surf) h[i] = decode<S, C>(p, 2, i, (S)h[i], (C)re.y);
        }
        g[i] += (C)(lam1 * WQ<double>(i) * (double)sHp[er][ec]);
        if (p.surf) h[i] += (C)(mub1 * WQ<double>(i));
      }
      double l0p = 0, l0s = 0;
#pragma unroll
      for (int i = 1; i < 9; ++i) {
        const double w3 = 3.0 * WQ<double>(i), w2 = 2.0 * w3;
        const double2 nb = sPP[pslot((gy + CY(i)))][lc + CX(i)];
        l0p += w2 * (nb.x - ph);
        l0s += w2 * (nb.y - ps);
      }
      Rp0 = -p.M_phi * (mc.x + p.kappa * l0p);
      Rs0 = p.surf ? -p.M_psi * mc.y - (p.M0 + p.M_psi * p.lambda_s) * l0s : 0.0;
      const double Rs0c = p.surf ? Rs0 + p.M_psi * p.mu_ref : 0.0;   // as in row_C
      Rtp = Rp0;
      Rts = Rs0c;
      if (a.have_hist) {
        uxh = hv[1];
        uyh = hv[2];
        vxh = hv[3];
        vyh = hv[4];
        ps0 = hv[5];
        const double Rp_prev = hv[6] + p.M_phi * pend.lambda_phi * hprime(p, ph0);
        const double Rs_prev = hv[7] + p.M_psi * pend.mubar_psi;
        Rtp = 1.5 * Rp0 - 0.5 * Rp_prev;
        Rts = 1.5 * Rs0c - 0.5 * Rs_prev;
      }
    }
    __syncthreads();
    if (!active) return;
    const double2 u = sU[gy - Y0][ln];
    const double ux = u.x, uy = u.y;
    double vx = ux, vy = uy, dpx = 0, dpy = 0, dsx = 0, dsy = 0;
    if (a.have_hist) {
      if (!p.adv_raw) {
        vx = 0.5 * (ux + uxh);
        vy = 0.5 * (uy + uyh);
      }
      dpx = ph * vx - ph0 * vxh;
      dpy = ph * vy - ph0 * vyh;
      dsx = ps * vx - ps0 * vxh;
      dsy = ps * vy - ps0 * vyh;
    }
    double rg[5], rh[5];
#pragma unroll
    for (int k = 0; k < 5; ++k) {
      rg[k] = opaque(p.sg[k]);
      rh[k] = opaque(p.sh[k]);
    }
    auto store_lat = [&](int lat, const C* o, C cref) {
      if constexpr (H16) {
        C rest = o[0];
#pragma unroll
        for (int i = 1; i < 9; ++i) {
          const S t = encode<S, C>(p, lat, i, o[i], cref);
          rest += o[i] - decode<S, C>(p, lat, i, t, cref);
          if (interior) store_hint<NTS>(byte_at(Pout + (size_t)(9 * lat + i) * N + row, xs), t);
        }
        if (interior) store_hint<NTS>(byte_at(rest_plane(Pout, N, lat) + row, 2 * xs), (float)rest);
      } else {
#pragma unroll
        for (int i = 0; i < 9; ++i)
          if (interior) store_hint<NTS>(byte_at(Pout + (size_t)(9 * lat + i) * N + row, xs), (S)o[i]);
      }
    };
    {
      C o[9];
      collide_scalar<C>(g, (C)ph, (C)p.eta_phi, (C)vx, (C)vy, (C)dpx, (C)dpy, (C)Rtp, rg, o);
      store_lat(1, o, (C)ph);
    }
    if (p.surf) {
      C o[9];
      collide_scalar<C>(h, (C)ps, (C)p.eta_psi, (C)vx, (C)vy, (C)dsx, (C)dsy, (C)Rts, rh, o);
      store_lat(2, o, (C)ps);
    }
    if (interior) {
      C* ho = hout + row;
      store_hint<NTS>(byte_at(ho + 2 * N, xc), (C)vx);
      store_hint<NTS>(byte_at(ho + 3 * N, xc), (C)vy);
      store_hint<NTS>(byte_at(ho + 4 * N, xc), (C)Rp0);
      store_hint<NTS>(byte_at(ho + 5 * N, xc), (C)Rs0);
    }
  };

  if constexpr (SCHED == kOneShot8) {
    // ---- one tile of four rows [Y0, Yend) with eight waves (small grids):
    // every phase takes all its rows at once -- wave w: h' of rows Y0-3+w
    // (and Y0+5+w for w < 2), phi, psi of row Y0-2+w, mu of row Y0-1+w
    // (w < 6), the collision of row Y0+(w&3) split between waves w and w+4 -- and every load is issued
    // before the first wait.  The phases are those of the sweep on the same
    // rows, and the tile's sums are added in the order of the sweep's waves
    // (rows Y0+1, Y0+2, Y0+3, Y0), so the results equal the sweep's bit for bit.
    C f[9], g[9], h[9], tg[9], th[9];
    double r0[2], v0[4], v1[4], hv[8];
    const int rc = Y0 + (wave & 3);   // the collision row of this wave's half of C
    const bool collide = rc < Yend, fwave = wave < 4;
    pend_load();   // first: the multipliers are reduced while the gathers are in flight
    gather_H(Y0 - 3 + wave, lane, xcol, v0);
    if (wave < 2) gather_H(Y0 + 5 + wave, lane, xcol, v1);
    gather_A(Y0 - 2 + wave, xcol, tg, th, r0);
    if (collide) {
      if (fwave) gather_Cf(rc, xcol, f);
      else gather_Cgh(rc, xcol, hv);
    }
    pend_set();
    row_H(Y0 - 3 + wave, lane, v0);
    if (wave < 2) row_H(Y0 + 5 + wave, lane, v1);
    __syncthreads();
    row_A(Y0 - 2 + wave, lane, xcol, tg, th, r0);
    __syncthreads();
    if (wave < 6) row_B(Y0 - 1 + wave, lane);
    __syncthreads();
    if (fwave) row_Cf(collide, rc, lane, xcol, f);
    else row_Cgh(collide, rc, lane, xcol, g, h, hv);
    __shared__ double sR[kSums][8];
    const double q[kSums] = {wave_red(s1, false), wave_red(s2, false), wave_red(s3, false),
                             p.phi_hold ? wave_red(s4, false) : 0.0};
    if (lane == 0) {
#pragma unroll
      for (int c = 0; c < kSums; ++c) sR[c][wave] = q[c];
    }
    __syncthreads();
    if (threadIdx.x == 0) {
#pragma unroll
      for (int c = 0; c < kSums; ++c) {
        double r = sR[c][2];   // rows Y0+1, Y0+2, Y0+3, Y0 are those of waves 2, 3, 4, 1
        r = r + sR[c][3];
        r = r + sR[c][4];
        r = r + sR[c][1];
        a.partials[kSums * (size_t)tile + c] = r;
      }
    }
    return;
  }

  if constexpr (SCHED == kOneShot4) {
    // ---- one tile of four rows with four waves, each taking in every phase
    // the rows the sweep gives it for a 4-row segment (h' rows Y0-3+w, Y0+1+w,
    // Y0+5+w (w < 2); phi, psi rows Y0-2+w and Y0+2+w; mu rows Y0-3+w (w >= 2)
    // and Y0+1+w; the collision of row Y0+w), in the same order, but with all
    // loads issued before the first wait and no pipelining across rows: the
    // same results bit for bit, three dependent phases less.
    C f[9], g[9], h[9], tg0[9], th0[9], tg1[9], th1[9];
    double r00[2], r01[2], v0[4], v1[4], v2[4];
    const int rc = Y0 + wave;
    const bool collide = rc < Yend;
    pend_load();   // first, as in the eight-wave tile
    gather_H(Y0 - 3 + wave, lane, xcol, v0);
    gather_H(Y0 + 1 + wave, lane, xcol, v1);
    if (wave < 2) gather_H(Y0 + 5 + wave, lane, xcol, v2);
    gather_A(Y0 - 2 + wave, xcol, tg0, th0, r00);
    gather_A(Y0 + 2 + wave, xcol, tg1, th1, r01);
    if (collide) gather_C(rc, xcol, f);
    pend_set();
    row_H(Y0 - 3 + wave, lane, v0);
    row_H(Y0 + 1 + wave, lane, v1);
    if (wave < 2) row_H(Y0 + 5 + wave, lane, v2);
    __syncthreads();
    row_A(Y0 - 2 + wave, lane, xcol, tg0, th0, r00);
    row_A(Y0 + 2 + wave, lane, xcol, tg1, th1, r01);
    __syncthreads();
    if (wave >= 2) row_B(Y0 - 3 + wave, lane);
    row_B(Y0 + 1 + wave, lane);
    __syncthreads();
    if (collide) row_C(rc, lane, xcol, f, g, h);
    s1 = block_reduce(s1, false);
    s2 = block_reduce(s2, false);
    s3 = block_reduce(s3, false);
    if (p.phi_hold) s4 = block_reduce(s4, false);
    if (threadIdx.x == 0) {
      a.partials[kSums * (size_t)tile + 0] = s1;
      a.partials[kSums * (size_t)tile + 1] = s2;
      a.partials[kSums * (size_t)tile + 2] = s3;
      a.partials[kSums * (size_t)tile + 3] = s4;
    }
    return;
  }

  set_pend();
  if constexpr (LS) {
#pragma unroll
    for (int c = 0; c < 3; ++c) lds.sacc[c][threadIdx.x] = 0.0;   // each thread's own slots
  }
  // ---- the sweep.  Iteration k collides rows Y0+4k .. Y0+4k+3 (k = -1 only
  // fills the rings).  Ring lifetimes: H writes rows <= 15 ahead of the oldest
  // h' row C still reads; A writes <= 10 rows ahead of the oldest (phi, psi)
  // row C reads; B's writes follow the barrier after every wave's C.
#pragma unroll 1
  for (int j = wave; j < 10; j += NWAVE) {   // rows Y0-3 .. Y0+6
    double v[4];
    gather_H(Y0 - 3 + j, lane, xcol, v);
    row_H(Y0 - 3 + j, lane, v);
  }
  __syncthreads();
  // FP64 storage runs at two waves per SIMD with registers to spare: its A
  // gathers are issued one iteration ahead, behind that iteration's H and C
  // gathers, so that they land while B and C run.
  constexpr bool PREA = sizeof(S) == 8 && !MMS;
  C tgn[PREA ? 9 : 1], thn[PREA ? 9 : 1];
  double r0n[PREA ? 2 : 1];
  if constexpr (PREA) gather_A(Y0 - 4 + 2 + wave, xcol, tgn, thn, r0n);
#pragma unroll 1
  for (int k = -1; 4 * k < Yend - Y0; ++k) {
    const int ln = opaque_v(lane);
    const unsigned x = opaque_v(xcol);
    const int rc = wave_uniform(Y0 + 4 * k + wave);
    const bool collide = k >= 0 && rc < Yend;
    const int ra = rc + 2, rh = rc + 7;
    // All loads of the iteration are issued here, in the order of their use
    // (their counter drains in order): A's and H's gathers, then C's, which
    // stay in flight during A, H, B and the barriers.  H may follow A: A reads
    // h' of rows up to ra + 1, written by earlier iterations.
    C f[9], g[9], h[9], tg[9], th[9];
    double r0[2], v[4];
    if constexpr (PREA) {
#pragma unroll
      for (int i = 0; i < 9; ++i) {
        tg[i] = tgn[i];
        th[i] = thn[i];
      }
      r0[0] = r0n[0];
      r0[1] = r0n[1];
    } else {
      gather_A(ra, x, tg, th, r0);
    }
    if (k >= 0) gather_H(rh, ln, x, v);
    if (collide) gather_C(rc, x, f);
    if constexpr (PREA) {
      if (4 * (k + 1) < Yend - Y0) gather_A(ra + 4, x, tgn, thn, r0n);
    }
    row_A(ra, ln, x, tg, th, r0);
    if (k >= 0) row_H(rh, ln, v);
    __syncthreads();
    if (k >= 0 || wave >= 2) row_B(Y0 + 4 * k + 1 + wave, ln);   // k = -1: rows Y0-1 and Y0 only
    __syncthreads();
    if (collide) row_C(rc, ln, x, f, g, h);
  }
  if constexpr (LS) {
    s1 = lds.sacc[0][threadIdx.x];
    s2 = lds.sacc[1][threadIdx.x];
    s3 = lds.sacc[2][threadIdx.x];
  }
  s1 = block_reduce(s1, false);
  s2 = block_reduce(s2, false);
  s3 = block_reduce(s3, false);
  if (p.phi_hold) s4 = block_reduce(s4, false);
  if (threadIdx.x == 0) {
    a.partials[kSums * (size_t)tile + 0] = s1;
    a.partials[kSums * (size_t)tile + 1] = s2;
    a.partials[kSums * (size_t)tile + 2] = s3;
    a.partials[kSums * (size_t)tile + 3] = s4;
  }
}

// Workgroups per CU a step kernel is compiled for (MINB): the walled FP32 and
// FP16 variants need a few more registers than three workgroups (12 waves)
// per CU leave.  Compiled for three, they spill about a dozen values: faster
// on grids of more workgroups than CUs (a 512 x 256 sheared drop: 24.4
// against 30.5 us per step), slower when each CU holds one workgroup anyway
// (the 256 x 128 sessile drop: 16.1 against 15.2 us).  The launch picks.
template <class S> inline constexpr int kStepMinBlocks = sizeof(S) <= 4 ? 3 : 1;

// The parameter block is read from device memory (a copy the handle keeps),
// as the batched kernel reads it: scalar loads on demand instead of a kernel
// argument block held in (spilled) scalar registers, and the same code as the
// batched step, hence the same results bit for bit.
// A segment of a walled grid whose rows lie three or more rows inside both
// walls touches no wall: every row it reads or computes for its collisions
// (halo rows, stencil and gather sources) is a fluid row, so the periodic form
// of the sweep computes it exactly as the walled form does, with fewer
// registers and no wall branches.
__device__ __forceinline__ bool wall_free_segment(int tile, int nstrips, int seg_rows, int ny) {
  const int y0 = (tile / nstrips) * seg_rows;
  return y0 >= 3 && min(y0 + seg_rows, ny) <= ny - 3;
}

template <class S, class C, bool WALLS, int MINB>
__global__ __launch_bounds__(kBlock, MINB) void k_step(const DevParams* __restrict__ pp, StepArgs a) {
  const int t = xcd_tile(blockIdx.x, gridDim.x);
  if constexpr (WALLS) {
    if (a.split_walls && wall_free_segment(t, a.nstrips, a.seg_rows, pp->ny)) {
      step_body<S, C, false, kSweep, false, true>(*pp, a, t);
      return;
    }
  }
  step_body<S, C, WALLS>(*pp, a, t);
}

// The accuracy test of Sec. 4.1 (periodic grid, FP64): the row sweep with the
// prescribed velocity and the manufactured sources of step `step`.
__global__ __launch_bounds__(kBlock) void k_step_mms(const DevParams* __restrict__ pp, StepArgs a, int step) {
  step_body<double, double, false, kSweep, true>(*pp, a, xcd_tile(blockIdx.x, gridDim.x), step);
}

// Small grids (at most one workgroup of four rows per CU): the one-shot
// schedule of a tile with eight waves.
template <class S, class C, bool WALLS>
__global__ __launch_bounds__(2 * kBlock) void k_step_small(const DevParams* __restrict__ pp, StepArgs a) {
  step_body<S, C, WALLS, kOneShot8>(*pp, a, xcd_tile(blockIdx.x, gridDim.x));
}
// Grids of up to three such workgroups per CU: the same tile with four waves.
template <class S, class C, bool WALLS>
__global__ __launch_bounds__(kBlock, kStepMinBlocks<S>) void k_step_mid(const DevParams* __restrict__ pp, StepArgs a) {
  step_body<S, C, WALLS, kOneShot4>(*pp, a, xcd_tile(blockIdx.x, gridDim.x));
}

// Batched step: one launch over the workgroups of every case of a batch
// (wg_case maps a workgroup to its case); each case carries its own
// parameters, buffers, buffer parity and activity, so retired cases are
// skipped and a captured graph of the launch stays valid.
template <class S, class C, bool WALLS>
__global__ __launch_bounds__(kBlock, WALLS ? kStepMinBlocks<S> : 1) void k_step_batch(const BatchCase* __restrict__ cases,
                                                                                    const int* __restrict__ wg_case) {
  const int b = xcd_tile(blockIdx.x, gridDim.x);
  const int c = wave_uniform(wg_case[b]);
  const BatchCase& bc = cases[c];
  if (!bc.active) return;
  const int par = bc.parity;
  StepArgs a;
  a.Pin = bc.pops[par];
  a.Pout = bc.pops[par ^ 1];
  a.ref = bc.phipsi[par ^ 1];
  a.out = bc.phipsi[par];
  a.hin = bc.uhist[par ^ 1];
  a.hout = bc.uhist[par];
  a.pend = bc.scalars + par;
  a.next = bc.scalars + (par ^ 1);
  a.partials = bc.partials;
  a.have_hist = bc.have_hist;
  a.nstrips = bc.nstrips;
  a.seg_rows = bc.seg_rows;
  a.ntiles = bc.ntiles;
  a.prev_partials = nullptr;
  a.prev_have_hist = 0;
  a.split_walls = 1;
  const int t = b - bc.tile_begin;
  if constexpr (WALLS) {
    if (wall_free_segment(t, bc.nstrips, bc.seg_rows, bc.p.ny)) {
      step_body<S, C, false, kSweep, false, true>(bc.p, a, t);
      return;
    }
  }
  step_body<S, C, WALLS>(bc.p, a, t);
}

// One workgroup per case: the multipliers of the step just taken, then the
// case's buffer parity flips.
__global__ __launch_bounds__(kBlock) void k_step_finish_batch(BatchCase* __restrict__ cases) {
  BatchCase& bc = cases[blockIdx.x];
  if (!bc.active) return;
  const int par = bc.parity, hh = bc.have_hist;
  finish_body(bc.partials, bc.ntiles, bc.p, hh, bc.scalars + (par ^ 1));
  __syncthreads();
  if (threadIdx.x == 0) {
    bc.parity = par ^ 1;
    bc.have_hist = 1;
    bc.step += 1;
  }
}

// Initial fields (Sec. 2.2 equilibrium profile) into the FP64 staging buffer.
__global__ __launch_bounds__(kBlock) void k_init_fields(DevParams p, double* __restrict__ F) {
  const int n = blockIdx.x * kBlock + threadIdx.x;
  if (n >= p.N) return;
  const int x = n % p.nx, y = n / p.nx;
  double dx = x - p.x0, dy = y - p.y0;
  dx -= p.nx * floor(dx / p.nx + 0.5);
  if (p.periodic_y) dy -= p.ny * floor(dy / p.ny + 0.5);
  double d;
  if (p.init_kind == LBM_INIT_SLAB) d = 0.5 * p.a - fabs(dx);
  else if (p.init_kind == LBM_INIT_BUBBLE) d = sqrt(dx * dx + dy * dy) - p.R0;
  else d = p.R0 - sqrt(dx * dx + dy * dy);
  const size_t N = (size_t)p.N;
  F[n] = p.phib * tanh(p.init_scale * d);
  F[N + n] = p.surf ? p.psi_b : 0.0;
  F[2 * N + n] = 0.0;
  F[3 * N + n] = 0.0;
}

// Equilibrium populations of the staged fields (phi, psi, ux, uy), stored in
// the pull layout (the stored value at z for direction j is the population a
// gather will deliver, the inverse of `pull`), with the rest populations of
// g and h shifted by phi and psi, which go to the FP64 reference planes.
template <class S>
__global__ __launch_bounds__(kBlock) void k_load(DevParams p, const double* __restrict__ F, int with_u, S* __restrict__ P,
                                                 double* __restrict__ ref, DevScalars* __restrict__ pend) {
  const int n = blockIdx.x * kBlock + threadIdx.x;
  if (n == 0) {
    pend->lambda_phi = 0.0;
    pend->mubar_psi = 0.0;
    pend->cdef = 0.0;
  }
  if (n >= p.N) return;
  const size_t N = (size_t)p.N;
  const int x = n % p.nx, y = n / p.nx;
  ref[n] = F[n];
  ref[N + n] = p.surf ? F[N + n] : 0.0;
  using Ck = std::conditional_t<std::is_same<S, double>::value, double, float>;
#pragma unroll
  for (int lat = 0; lat < 3; ++lat) {
    const Ck cref = lat == 1 ? (Ck)F[n] : ((lat == 2 && p.surf) ? (Ck)F[N + n] : Ck(0));   // this node writes them
    Ck rest = Ck(0), resid = Ck(0);
#pragma unroll
    for (int j = 0; j < 9; ++j) {
      // receiver node w and direction d whose gather reads stored_j(z)
      int wx = wrap(x + CX(j), p.nx), wy = y + CY(j), d = j;
      if (p.periodic_y) wy = wrap(wy, p.ny);
      else if (wy < 0 || wy >= p.ny) {
        const int bc = wy < 0 ? p.bc_bottom : p.bc_top;
        if (lat == 0 && bc == LBM_BC_FREESLIP) { wy = y; d = MIRY(j); }
        else { wx = x; wy = y; d = OPP(j); }
      }
      const size_t w = (size_t)wy * p.nx + wx;
      const double ph = F[w], ps = p.surf ? F[N + w] : 0.0;
      const double ux = with_u ? F[2 * N + w] : 0.0, uy = with_u ? F[3 * N + w] : 0.0;
      double v;
      if (lat == 0) v = with_u ? feq_flow(d, 0.0, rho_of(p, ph), ux, uy) : 0.0;
      else {
        const double c = lat == 1 ? ph : ps, eta = lat == 1 ? p.eta_phi : p.eta_psi;
        v = d == 0 ? (WQ<double>(0) - 1.0) * eta * c : feq_scalar_moving(d, c, eta, c * ux, c * uy);
        if (lat == 2 && !p.surf) v = 0.0;
      }
      if (kHalf<S> && lat > 0) {   // moving: FP16 with the residual kept for the FP32 rest value
        if (j == 0) {
          rest = (Ck)v;
        } else {
          const S t = encode<S, Ck>(p, lat, j, (Ck)v, cref);
          resid += (Ck)v - decode<S, Ck>(p, lat, j, t, cref);
          P[(size_t)(9 * lat + j) * N + n] = t;
        }
      } else {
        P[(size_t)(9 * lat + j) * N + n] = encode<S, Ck>(p, lat, j, (Ck)v, cref);
      }
    }
    if constexpr (kHalf<S>) {
      if (lat > 0) rest_plane(P, N, lat)[n] = (float)(rest + resid);
    }
  }
}

// Macroscopic fields of the current state: phi psi ux uy p rho mu_phi mu_psi.
template <class S, class C>
__global__ __launch_bounds__(kBlock) void k_fields(DevParams p, const S* __restrict__ P, const double* __restrict__ phipsi,
                                                   const double* __restrict__ mu, double* __restrict__ out) {
  const int n = blockIdx.x * kBlock + threadIdx.x;
  if (n >= p.N) return;
  const size_t N = (size_t)p.N;
  const int x = n % p.nx, y = n / p.nx;
  C f[9];
#pragma unroll
  for (int i = 0; i < 9; ++i) f[i] = pull<S, C>(p, P, 0, i, x, y, nullptr);
  const Macro M = macro_node<C>(p, phipsi, phipsi + N, mu, mu + N, f, x, y);
  out[n] = phipsi[n];
  out[N + n] = phipsi[N + n];
  out[2 * N + n] = M.ux;
  out[3 * N + n] = M.uy;
  out[4 * N + n] = M.pr;
  out[5 * N + n] = M.rho;
  out[6 * N + n] = mu[n];
  out[7 * N + n] = mu[N + n];
}

// Populations of the current state: rest populations of g, h un-shifted and
// the pending multiplier terms added.
template <class S>
__global__ __launch_bounds__(kBlock) void k_pops(DevParams p, const S* __restrict__ P, const double* __restrict__ ref,
                                                 const DevScalars* __restrict__ pend, double* __restrict__ out) {
  const int n = blockIdx.x * kBlock + threadIdx.x;
  if (n >= p.N) return;
  const size_t N = (size_t)p.N;
  const int x = n % p.nx, y = n / p.nx;
  const double lam = pend->cdef * p.M_phi * pend->lambda_phi, mub = pend->cdef * p.M_psi * (pend->mubar_psi - p.mu_ref);
  for (int lat = 0; lat < 3; ++lat)
#pragma unroll
    for (int i = 0; i < 9; ++i) {
      double v = (lat == 2 && !p.surf) ? 0.0 : pull<S, double>(p, P, lat, i, x, y, ref);
      if (lat == 1) v += lam * WQ<double>(i) * hprime(p, ref[emitter(p, i, x, y)]);
      if (lat == 2 && p.surf) v += mub * WQ<double>(i);
      if (i == 0 && lat > 0 && (lat == 1 || p.surf)) v += ref[(size_t)(lat - 1) * N + n];
      out[(size_t)(9 * lat + i) * N + n] = v;
    }
}

// Positive fraction of a linear triangle / segment (two-triangle area, Sec. 4.1).
__device__ double tri_frac(double a, double b, double c) {
  const int np = (a > 0) + (b > 0) + (c > 0);
  if (np == 3) return 1.0;
  if (np == 0) return 0.0;
  if (np == 1) {
    const double pp = a > 0 ? a : (b > 0 ? b : c);
    const double q = a > 0 ? b : (b > 0 ? c : a);
    const double r = a > 0 ? c : (b > 0 ? a : b);
    return pp * pp / ((pp - q) * (pp - r));
  }
  const double m = a <= 0 ? a : (b <= 0 ? b : c);
  const double q = a <= 0 ? b : (b <= 0 ? c : a);
  const double r = a <= 0 ? c : (b <= 0 ? a : b);
  return 1.0 - m * m / ((m - q) * (m - r));
}
__device__ double seg_frac(double a, double b) {
  if (a > 0 && b > 0) return 1.0;
  if (a <= 0 && b <= 0) return 0.0;
  return a > 0 ? a / (a - b) : b / (b - a);
}

constexpr int kInv = kInvValues;

template <class S, class C>
__global__ __launch_bounds__(kBlock) void k_invariants(DevParams p, const S* __restrict__ P, const double* __restrict__ phipsi,
                                                       const double* __restrict__ mu, double* __restrict__ partials) {
  const size_t N = (size_t)p.N;
  const double* phi = phipsi;
  const double* psi = phipsi + N;
  double acc[kInv];
  for (int k = 0; k < kInv; ++k) acc[k] = 0.0;
  for (int n = blockIdx.x * kBlock + threadIdx.x; n < p.N; n += gridDim.x * kBlock) {
    const int x = n % p.nx, y = n / p.nx;
    C f[9];
#pragma unroll
    for (int i = 0; i < 9; ++i) f[i] = pull<S, C>(p, P, 0, i, x, y, nullptr);
    const Macro M = macro_node<C>(p, phi, psi, mu, mu + N, f, x, y);
    const double ph = phi[n], ps = psi[n], ux = M.ux, uy = M.uy, pr = M.pr, rho = M.rho;
    if (!isfinite(ph) || !isfinite(ps) || !isfinite(ux) || !isfinite(uy) || !isfinite(pr)) acc[7] += 1.0;
    if (p.surf && !(ps > 0.0 && ps < 1.0)) acc[8] += 1.0;
    acc[0] += ps;
    acc[1] += 0.5 + gsw(p, ph);
    acc[2] += ph;
    const double u2 = ux * ux + uy * uy;
    acc[4] += 0.5 * rho * u2;
    acc[6] = fmax(acc[6], sqrt(u2));
    // free-energy density with isotropic gradients; wetting ghosts from the BCs
    double gpx = 0, gpy = 0, gsx = 0, gsy = 0;
    for (int i = 1; i < 9; ++i) {
      const Nb b = nbr(p, x, y, CX(i), CY(i));
      double vp = phi[b.idx], vs = psi[b.idx];
      if (b.side && wet_side(p, b.side)) {
        const double pn = vp, sn = vs;
        vp = pn + Jphi(p, pn, sn) / p.kappa;
        if (p.surf && p.lambda_s > 0.0) vs = sn + Jpsi(p, pn, sn) / p.lambda_s;
      }
      const double w3 = 3.0 * WQ<double>(i);
      gpx += w3 * CX(i) * vp; gpy += w3 * CY(i) * vp;
      gsx += w3 * CX(i) * vs; gsy += w3 * CY(i) * vs;
    }
    double e = p.beta * (ph * ph - 1.0) * (ph * ph - 1.0) + 0.5 * p.kappa * (gpx * gpx + gpy * gpy);
    if (p.surf)
      e += p.kBT * (ps * log(ps) + (1.0 - ps) * log(1.0 - ps)) + 0.5 * p.lambda_s * (gsx * gsx + gsy * gsy)
         - p.beta * ps * (1.0 - ph * ph) * (1.0 - ph * ph) + 0.5 * p.W * ps * ph * ph;
    // wall energy and Remark-1 regime on wetting-wall rows
    const bool wall_row_b = !p.periodic_y && y == 0 && p.wet_bottom;
    const bool wall_row_t = !p.periodic_y && y == p.ny - 1 && p.wet_top;
    for (int w = 0; w < 2; ++w) {
      if (!(w == 0 ? wall_row_b : wall_row_t)) continue;
      const double l = p.surf ? log(1.0 - ps) : 0.0;
      const double2 st = wall_surf_terms(p, l);
      e += -(p.sig_cos + st.x) * gsw(p, ph) + 0.5 * st.y + p.fw0;
      if (p.surf) {
        if (p.beta_sg > 0.0 && 1.0 + p.beta_sg * l <= 0.5) acc[9] += 1.0;
        if (p.beta_sl > 0.0 && 1.0 + p.beta_sl * l <= 0.5) acc[9] += 1.0;
      }
    }
    acc[5] += e;
    // area of phi > 0: the cell whose lower-left corner is this node, and the
    // half cells between a wall and the first row
    const int x1 = x + 1 == p.nx ? 0 : x + 1;
    if (p.periodic_y || y + 1 < p.ny) {
      const int y1 = y + 1 == p.ny ? 0 : y + 1;
      const double a = ph, b = phi[(size_t)y * p.nx + x1], c = phi[(size_t)y1 * p.nx + x1], d = phi[(size_t)y1 * p.nx + x];
      acc[3] += 0.5 * tri_frac(a, b, c) + 0.5 * tri_frac(a, c, d);
    }
    if (!p.periodic_y && y == 0) acc[3] += 0.5 * seg_frac(ph, phi[x1]);
    if (!p.periodic_y && y == p.ny - 1) acc[3] += 0.5 * seg_frac(ph, phi[(size_t)y * p.nx + x1]);
  }
  for (int k = 0; k < kInv; ++k) {
    const double r = block_reduce(acc[k], k == 6);
    if (threadIdx.x == 0) partials[(size_t)kInv * blockIdx.x + k] = r;
  }
}

__global__ __launch_bounds__(kBlock) void k_inv_final(int nblk, const double* __restrict__ partials, double* __restrict__ out) {
  for (int k = 0; k < kInv; ++k) {
    double v = 0.0;
    for (int b = threadIdx.x; b < nblk; b += kBlock) {
      const double q = partials[(size_t)kInv * b + k];
      v = k == 6 ? fmax(v, q) : v + q;
    }
    v = block_reduce(v, k == 6);
    if (threadIdx.x == 0) out[k] = v;
  }
}

// Contact diagnostics on the bottom wall (y = -1/2): per column, the height
// above the wall of the first phi = 0 crossing of a liquid column, and the
// positive fractions of the edges to the next column on the first and second
// rows; the width is their sums extrapolated linearly to the wall.
__global__ __launch_bounds__(kBlock) void k_contact_cols(DevParams p, const double* __restrict__ phi, double* __restrict__ cols) {
  const int x = blockIdx.x * kBlock + threadIdx.x;
  if (x >= p.nx) return;
  const int x1 = x + 1 == p.nx ? 0 : x + 1;
  cols[p.nx + x] = seg_frac(phi[x], phi[x1]);
  cols[2 * p.nx + x] = seg_frac(phi[p.nx + x], phi[p.nx + x1]);
  double hx = 0.0;
  if (phi[x] > 0.0) {
    hx = p.ny - 0.5;
    for (int y = 0; y + 1 < p.ny; ++y) {
      const double a = phi[(size_t)y * p.nx + x], b = phi[(size_t)(y + 1) * p.nx + x];
      if (a > 0 && b <= 0) { hx = y + a / (a - b) + 0.5; break; }
    }
  }
  cols[x] = hx;
}
__global__ __launch_bounds__(kBlock) void k_contact_final(int nx, const double* __restrict__ cols, double* __restrict__ out) {
  double L0 = 0.0, L1 = 0.0, H = 0.0;
  for (int x = threadIdx.x; x < nx; x += kBlock) {
    L0 += cols[nx + x];
    L1 += cols[2 * nx + x];
    H = fmax(H, cols[x]);
  }
  L0 = block_reduce(L0, false);
  L1 = block_reduce(L1, false);
  H = block_reduce(H, true);
  if (threadIdx.x == 0) {
    double L = L0 > 0.0 ? L0 + 0.5 * (L0 - L1) : 0.0;
    if (L < 0.0) L = 0.0;
    out[0] = L;
    out[1] = H;
    out[2] = L > 0.0 ? 2.0 * atan(2.0 * H / L) * 180.0 / kPi : 180.0;
  }
}

inline int nblocks(int n) { return (n + kBlock - 1) / kBlock; }
inline int red_blocks(int n) { int b = nblocks(n); return b < kRedBlocks ? b : kRedBlocks; }

// Event pair k of the current timed step (or nothing when not timing).
struct TimedScope {
  StepTimer* t;
  int k;
  hipStream_t st;
  TimedScope(StepTimer* t_, int k_, hipStream_t st_) : t(t_), k(k_), st(st_) {
    if (t) (void)hipEventRecord(t->ev[(t->used * LBM_N_KERNELS + k) * 2 + 0], st);
  }
  ~TimedScope() {
    if (t) (void)hipEventRecord(t->ev[(t->used * LBM_N_KERNELS + k) * 2 + 1], st);
  }
};

// Diagnostics of the current state: phi, psi (pending multiplier terms
// applied), mu, and the multipliers of the current state in the diagnostic
// scalar slot (the pending slot is left untouched).
template <class S, class C>
hipError_t macro_impl(const DevParams& p, DevState& s, hipStream_t st) {
  double* pp = (double*)s.phipsi[s.hcur];
  const double* ref = (const double*)s.phipsi[s.hcur ^ 1];
  const int rb = red_blocks(p.N);
  hipLaunchKernelGGL((k_moments<S, C>), dim3(nblocks(p.N)), dim3(kBlock), 0, st, p, (const S*)s.pops[s.cur], ref,
                     (const DevScalars*)(s.scalars + s.scur), pp);
  hipLaunchKernelGGL(k_mu_partials, dim3(rb), dim3(kBlock), 0, st, p, (const double*)pp, (double*)s.mu, s.partials);
  hipLaunchKernelGGL(k_multipliers, dim3(1), dim3(kBlock), 0, st, p, rb, (const double*)s.partials, s.scalars + 2);
  return hipGetLastError();
}

template <class S, class C>
void launch_step(const DevParams& p, DevState& s, int have_hist, hipStream_t st, StepTimer* t, int fuse,
                 long long step) {
  StepArgs a;
  a.Pin = s.pops[s.cur];
  a.Pout = s.pops[s.cur ^ 1];
  a.ref = (const double*)s.phipsi[s.hcur ^ 1];
  a.out = (double*)s.phipsi[s.hcur];
  a.hin = s.uhist[s.hcur ^ 1];
  a.hout = s.uhist[s.hcur];
  a.pend = s.scalars + s.scur;
  a.next = s.scalars + (s.scur ^ 1);
  a.partials = s.step_partials[s.cur];
  a.have_hist = have_hist;
  a.nstrips = (p.nx + kStripW - 1) / kStripW;
  a.seg_rows = s.tile_rows;
  a.ntiles = (int)step_blocks(p.nx, p.ny, s.tile_rows);
  a.prev_partials = (fuse & kFusePrev) ? s.step_partials[s.cur ^ 1] : nullptr;
  a.prev_have_hist = 1;
  a.split_walls = s.split_walls;
  {
    TimedScope ts(t, LBM_K_STEP, st);
    const DevParams* dp = (const DevParams*)s.dparams;
    if constexpr (std::is_same<S, double>::value) {
      if (p.mms) {   // the accuracy test: periodic, FP64, the row sweep with its sources
        hipLaunchKernelGGL(k_step_mms, dim3(a.ntiles), dim3(kBlock), 0, st, dp, a, (int)step);
        goto finish;
      }
    }
    // the choice depends on the number of workgroups against the device's CUs
    // (256 on an MI355X); every variant gives the same results
    switch (step_variant(p, s)) {
      case kVarSmall:   // small grid: one-shot tiles
        if (p.periodic_y) hipLaunchKernelGGL((k_step_small<S, C, false>), dim3(a.ntiles), dim3(2 * kBlock), 0, st, dp, a);
        else hipLaunchKernelGGL((k_step_small<S, C, true>), dim3(a.ntiles), dim3(2 * kBlock), 0, st, dp, a);
        break;
      case kVarMid:     // mid-size grid
        if (p.periodic_y) hipLaunchKernelGGL((k_step_mid<S, C, false>), dim3(a.ntiles), dim3(kBlock), 0, st, dp, a);
        else hipLaunchKernelGGL((k_step_mid<S, C, true>), dim3(a.ntiles), dim3(kBlock), 0, st, dp, a);
        break;
      case kVarSweepPacked:
        hipLaunchKernelGGL((k_step<S, C, true, kStepMinBlocks<S>>), dim3(a.ntiles), dim3(kBlock), 0, st, dp, a);
        break;
      default:
        if (p.periodic_y) hipLaunchKernelGGL((k_step<S, C, false, 1>), dim3(a.ntiles), dim3(kBlock), 0, st, dp, a);
        else hipLaunchKernelGGL((k_step<S, C, true, 1>), dim3(a.ntiles), dim3(kBlock), 0, st, dp, a);
    }
  }
finish:
  if (!(fuse & kFuseNext)) {
    TimedScope ts(t, LBM_K_FINISH, st);
    hipLaunchKernelGGL(k_step_finish, dim3(1), dim3(kBlock), 0, st, (const DevParams*)s.dparams, (const double*)a.partials,
                       a.ntiles, have_hist, a.next);
  }
}

template <class S, class C>
hipError_t step_impl(const DevParams& p, DevState& s, int have_hist, hipStream_t st, StepTimer* timer, int fuse,
                     long long step) {
  StepTimer* t = (timer && timer->ev && timer->used < timer->max_steps) ? timer : nullptr;
  launch_step<S, C>(p, s, have_hist, st, t, fuse, step);
  if (t) t->used += 1;
  s.cur ^= 1;
  s.hcur ^= 1;
  s.scur ^= 1;
  return hipGetLastError();
}

template <class S, class C>
hipError_t inv_impl(const DevParams& p, DevState& s, hipStream_t st) {
  hipError_t e = macro_impl<S, C>(p, s, st);
  if (e != hipSuccess) return e;
  const int rb = red_blocks(p.N);
  hipLaunchKernelGGL((k_invariants<S, C>), dim3(rb), dim3(kBlock), 0, st, p, (const S*)s.pops[s.cur],
                     (const double*)s.phipsi[s.hcur], (const double*)s.mu, s.inv_partials);
  hipLaunchKernelGGL(k_inv_final, dim3(1), dim3(kBlock), 0, st, rb, (const double*)s.inv_partials, s.inv_out);
  if (!p.periodic_y) {
    hipLaunchKernelGGL(k_contact_cols, dim3(nblocks(p.nx)), dim3(kBlock), 0, st, p, (const double*)s.phipsi[s.hcur], s.contact);
    hipLaunchKernelGGL(k_contact_final, dim3(1), dim3(kBlock), 0, st, p.nx, (const double*)s.contact, s.inv_out + kInv);
  }
  return hipGetLastError();
}

template <class S, class C>
hipError_t fetch_impl(const DevParams& p, DevState& s, hipStream_t st) {
  hipError_t e = macro_impl<S, C>(p, s, st);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL((k_fields<S, C>), dim3(nblocks(p.N)), dim3(kBlock), 0, st, p, (const S*)s.pops[s.cur],
                     (const double*)s.phipsi[s.hcur], (const double*)s.mu, s.field_buf);
  return hipGetLastError();
}

template <class S>
hipError_t load_impl(const DevParams& p, DevState& s, int with_u, hipStream_t st) {
  hipLaunchKernelGGL(k_load<S>, dim3(nblocks(p.N)), dim3(kBlock), 0, st, p, (const double*)s.field_buf, with_u,
                     (S*)s.pops[s.cur], (double*)s.phipsi[s.hcur ^ 1], s.scalars + s.scur);
  return hipGetLastError();
}

template <class S>
hipError_t pops_impl(const DevParams& p, DevState& s, hipStream_t st) {
  hipLaunchKernelGGL(k_pops<S>, dim3(nblocks(p.N)), dim3(kBlock), 0, st, p, (const S*)s.pops[s.cur],
                     (const double*)s.phipsi[s.hcur ^ 1], (const DevScalars*)(s.scalars + s.scur), s.field_buf);
  return hipGetLastError();
}

}  // namespace

size_t storage_bytes(int precision) { return precision == LBM_FP64 ? 8 : (precision == LBM_FP32 ? 4 : 2); }
size_t pops_bytes(int precision, size_t N) {
  return precision == LBM_FP16_SHIFTED ? rest_offset(N) + 2 * N * sizeof(float) : 27 * N * storage_bytes(precision);
}
size_t step_blocks(int nx, int ny, int seg_rows) {
  return (size_t)((nx + kStripW - 1) / kStripW) * (size_t)((ny + seg_rows - 1) / seg_rows);
}
int step_variant(const DevParams& p, const DevState& s) {
  if (p.mms) return kVarSweep;   // the accuracy test runs the row sweep
  const size_t ntiles = step_blocks(p.nx, p.ny, s.tile_rows);
  const size_t cus = (size_t)s.cus;
  const size_t packed = s.precision == LBM_FP64 ? (size_t)kStepMinBlocks<double> : (size_t)kStepMinBlocks<float>;
  if (s.tile_rows == 4 && ntiles <= cus) return kVarSmall;
  if (s.tile_rows == 4 && ntiles <= packed * cus) return kVarMid;
  if (!p.periodic_y && packed > 1 && ntiles > cus) return kVarSweepPacked;
  return kVarSweep;
}
// Rows per workgroup segment: long segments amortise the four extra phi/psi
// rows and two extra mu rows each segment computes, but a grid needs enough
// workgroups to fill the chip.  The tallest segment up to 16 rows (FP32, FP16)
// or 32 rows (FP64, whose step holds two workgroups per CU instead of three)
// that still gives 2048 workgroups; small grids get 4 rows and the one-pass
// tile kernels.  Measured on MI355X (periodic drop, ms per step, rows in
// brackets): FP32 1024^2 0.104 (8) against 0.121 (4), 2048^2 0.403 (16) /
// 0.400 (8) / 0.442 (4), 3072^2 0.924 (16), 4096^2 1.53 (16) against 1.60
// (32); FP64 1024^2 0.173 (8) against 0.192 (4), 2048^2 0.611 (32), 3072^2
// 1.43 (32), 4096^2 2.36 (32) against 2.45 (16) and 2.50 (64).
int step_seg_rows(int nx, int ny, int precision) {
  int seg = precision == LBM_FP64 ? 32 : 16;
  while (seg > 4 && step_blocks(nx, ny, seg) < 2048) seg /= 2;
  return seg;
}
size_t compute_bytes(int precision) { return precision == LBM_FP64 ? 8 : 4; }

#define LBM_DISPATCH(prec, call64, call32, call16)    \
  switch (prec) {                                     \
    case LBM_FP64: return call64;                     \
    case LBM_FP32: return call32;                     \
    case LBM_FP16_SHIFTED: return call16;             \
    default: return hipErrorInvalidValue;             \
  }

hipError_t launch_init(const DevParams& p, DevState& s, hipStream_t st) {
  hipLaunchKernelGGL(k_init_fields, dim3(nblocks(p.N)), dim3(kBlock), 0, st, p, s.field_buf);
  return launch_load(p, s, 0, st);
}
hipError_t launch_load(const DevParams& p, DevState& s, int with_u, hipStream_t st) {
  LBM_DISPATCH(s.precision, (load_impl<double>(p, s, with_u, st)), (load_impl<float>(p, s, with_u, st)),
               (load_impl<_Float16>(p, s, with_u, st)));
}
template <class S, class C>
hipError_t batch_step_impl(bool walls, const BatchCase* d_cases, const int* d_wg_case, int nwg, int count, hipStream_t st,
                           StepTimer* timer) {
  StepTimer* t = (timer && timer->ev && timer->used < timer->max_steps) ? timer : nullptr;
  {
    TimedScope ts(t, LBM_K_STEP, st);
    if (walls) hipLaunchKernelGGL((k_step_batch<S, C, true>), dim3(nwg), dim3(kBlock), 0, st, d_cases, d_wg_case);
    else hipLaunchKernelGGL((k_step_batch<S, C, false>), dim3(nwg), dim3(kBlock), 0, st, d_cases, d_wg_case);
  }
  {
    TimedScope ts(t, LBM_K_FINISH, st);
    hipLaunchKernelGGL(k_step_finish_batch, dim3(count), dim3(kBlock), 0, st, (BatchCase*)d_cases);
  }
  if (t) t->used += 1;
  return hipGetLastError();
}
hipError_t launch_step_batch(int precision, bool walls, const BatchCase* d_cases, const int* d_wg_case, int nwg, int count,
                             hipStream_t st, StepTimer* timer) {
  LBM_DISPATCH(precision, (batch_step_impl<double, double>(walls, d_cases, d_wg_case, nwg, count, st, timer)),
               (batch_step_impl<float, float>(walls, d_cases, d_wg_case, nwg, count, st, timer)),
               (batch_step_impl<_Float16, float>(walls, d_cases, d_wg_case, nwg, count, st, timer)));
}
hipError_t launch_step(const DevParams& p, DevState& s, int have_hist, hipStream_t st, StepTimer* timer, int fuse,
                       int64_t step) {
  LBM_DISPATCH(s.precision, (step_impl<double, double>(p, s, have_hist, st, timer, fuse, step)),
               (step_impl<float, float>(p, s, have_hist, st, timer, fuse, step)),
               (step_impl<_Float16, float>(p, s, have_hist, st, timer, fuse, step)));
}
hipError_t launch_macro(const DevParams& p, DevState& s, hipStream_t st) {
  LBM_DISPATCH(s.precision, (macro_impl<double, double>(p, s, st)), (macro_impl<float, float>(p, s, st)),
               (macro_impl<_Float16, float>(p, s, st)));
}
hipError_t launch_invariants(const DevParams& p, DevState& s, hipStream_t st) {
  LBM_DISPATCH(s.precision, (inv_impl<double, double>(p, s, st)), (inv_impl<float, float>(p, s, st)),
               (inv_impl<_Float16, float>(p, s, st)));
}
hipError_t launch_fetch(const DevParams& p, DevState& s, uint32_t, hipStream_t st) {
  LBM_DISPATCH(s.precision, (fetch_impl<double, double>(p, s, st)), (fetch_impl<float, float>(p, s, st)),
               (fetch_impl<_Float16, float>(p, s, st)));
}
hipError_t launch_fetch_pops(const DevParams& p, DevState& s, hipStream_t st) {
  LBM_DISPATCH(s.precision, (pops_impl<double>(p, s, st)), (pops_impl<float>(p, s, st)),
               (pops_impl<_Float16>(p, s, st)));
}

}  // namespace lbm
