// lbm3d.hip -- gfx950 kernels and C ABI (include/lbm3d.h) of the D3Q19 step of
// the conservative Allen-Cahn / Navier-Stokes surfactant model.
//
// One step is five launches over the nodes (one thread per node, x fastest,
// so every plane access of a wavefront is 64 consecutive elements):
//   k3_mu    chemical potentials (eq_muphi, eq_mupsi) from the FP64 (phi, psi)
//            pairs with the 18-direction isotropic Laplacian, the wall terms
//            of the first fluid layer, and FP64 per-workgroup multiplier sums
//   k3_fin   one wavefront: lambda_phi (eq15) and mubar_psi (AC_psi) from the
//            sums, in a fixed order
//   k3_colf  gradients of rho and of both potentials, the force (eq_Fs0),
//            velocity and pressure, the sources and the advecting velocity
//            (into the history planes), the flow lattice's MRT collision and
//            push streaming into the other population buffer with half-way
//            bounce-back, moving-wall and free-slip walls
//   k3_colgh the phase-field and surfactant lattices: backward differences
//            from the history planes of this step and the previous one, MRT
//            collisions, push streaming
//   (macroscopic fields, stencils and sources in FP64; the collisions in the
//   storage type, FP32 or FP64)
//            (two kernels rather than one: one kernel holding all three
//            lattices needs more than 256 registers a lane, one wave per SIMD)
//   k3_mom   phi, psi of the new state (zeroth moments) into the other FP64
//            pair array
// (phi, psi) and (mu_phi, mu_psi) are stored interleaved, one 16-byte pair a
// node, so a stencil reads a neighbour's pair with one load.
// The rest populations of g and h are stored shifted by the phi, psi of the
// step that wrote them (read back from the FP64 pair array that then holds
// the previous step's values), so FP32 storage rounds only the increments.
// Complex walls: nodes marked solid (lbm3d_set_solid) hold no fluid; a link
// from a fluid node x into a solid node is a half-way bounce-back wall for all
// three lattices, and the stencils see a ghost value there taken at x itself
// (mirror psi, mu; on wetting solids phi(x) + J_phi(x)/kappa, and the wall term
// (2 w_i / c_s^2) J(x) per link), the link-wise form of the flat walls' ghost
// layer.  Sums and the mean potential run over fluid nodes.
// The MRT transform uses the closed form of the D3Q19 raw-moment basis: the
// four edge populations of a coordinate plane (a, b) follow from the moments
// c_a^2 c_b^2, c_a c_b^2, c_a^2 c_b and c_a c_b; the two face populations of
// an axis from c_a^2 and c_a minus their edge parts; the rest population from
// the zeroth moment.
#include <cmath>
#include <cstdlib>
#include <cstring>
#include <string>
#include <vector>

#include <hip/hip_runtime.h>

#include "../../include/lbm.h"
#include "../../include/lbm3d.h"

namespace {

constexpr int Q3 = 19;
constexpr int kT = 256;   // threads per workgroup
constexpr int kRedB = 1024;

// Velocity set: rest; faces +x -x +y -y +z -z; edges of the xy, xz, yz planes
// in the sign order (+,+) (-,+) (+,-) (-,-).
__host__ __device__ constexpr int cx3(int i) {
  constexpr int v[Q3] = {0, 1, -1, 0, 0, 0, 0, 1, -1, 1, -1, 1, -1, 1, -1, 0, 0, 0, 0};
  return v[i];
}
__host__ __device__ constexpr int cy3(int i) {
  constexpr int v[Q3] = {0, 0, 0, 1, -1, 0, 0, 1, 1, -1, -1, 0, 0, 0, 0, 1, -1, 1, -1};
  return v[i];
}
__host__ __device__ constexpr int cz3(int i) {
  constexpr int v[Q3] = {0, 0, 0, 0, 0, 1, -1, 0, 0, 0, 0, 1, 1, -1, -1, 1, 1, -1, -1};
  return v[i];
}
__host__ __device__ constexpr double w3(int i) { return i == 0 ? 1.0 / 3.0 : (i < 7 ? 1.0 / 18.0 : 1.0 / 36.0); }
__host__ __device__ constexpr int opp3(int i) {
  constexpr int v[Q3] = {0, 2, 1, 4, 3, 6, 5, 10, 9, 8, 7, 14, 13, 12, 11, 18, 17, 16, 15};
  return v[i];
}
// direction with c_z negated (specular reflection at a z wall)
__host__ __device__ constexpr int mirz3(int i) {
  constexpr int v[Q3] = {0, 1, 2, 3, 4, 6, 5, 7, 8, 9, 10, 13, 14, 11, 12, 17, 18, 15, 16};
  return v[i];
}
constexpr double kCs2 = 1.0 / 3.0;
// The velocity set as device tables, for loops over directions that are not unrolled.
__constant__ int kC3[Q3][3] = {{0, 0, 0},  {1, 0, 0},  {-1, 0, 0}, {0, 1, 0},  {0, -1, 0}, {0, 0, 1},  {0, 0, -1},
                               {1, 1, 0},  {-1, 1, 0}, {1, -1, 0}, {-1, -1, 0}, {1, 0, 1},  {-1, 0, 1}, {1, 0, -1},
                               {-1, 0, -1}, {0, 1, 1}, {0, -1, 1}, {0, 1, -1}, {0, -1, -1}};
__constant__ double kW3[Q3] = {1.0 / 3.0,  1.0 / 18.0, 1.0 / 18.0, 1.0 / 18.0, 1.0 / 18.0, 1.0 / 18.0, 1.0 / 18.0,
                               1.0 / 36.0, 1.0 / 36.0, 1.0 / 36.0, 1.0 / 36.0, 1.0 / 36.0, 1.0 / 36.0, 1.0 / 36.0,
                               1.0 / 36.0, 1.0 / 36.0, 1.0 / 36.0, 1.0 / 36.0, 1.0 / 36.0};
// w_i / c_s^2, the gradient stencil's coefficients: the same values as the
// unrolled stencil's w3(i) / kCs2, folded at compile time here and there.
#define W3CS(i) (w3(i) / kCs2)
__constant__ double kWC3[Q3] = {W3CS(0),  W3CS(1),  W3CS(2),  W3CS(3),  W3CS(4),  W3CS(5),  W3CS(6),
                                W3CS(7),  W3CS(8),  W3CS(9),  W3CS(10), W3CS(11), W3CS(12), W3CS(13),
                                W3CS(14), W3CS(15), W3CS(16), W3CS(17), W3CS(18)};
#undef W3CS

struct P3 {
  int nx, ny, nz, N, periodic_z, wet_b, wet_t, freeslip_b, freeslip_t, surf, linear, adv_raw, s2_local, phi_hold;
  int has_solid, solid_wet, Nf;   // solid mask present; solids carry the wetting BCs; fluid nodes
  double kappa, beta, W, kBT, phib, inv_phib, lambda_s, M0, M_phi, M_psi, eta_phi, eta_psi;
  double rho_l, rho_g, mu_l, mu_g, gx, gy, gz, uw_b, uw_t;
  double sig_cos, dsb, msb;   // sigma cos(theta0), sigma_sg0 beta_sg -/+ sigma_sl0 beta_sl
  double sf[5], sg[5], sh[5];
  double x0, y0, z0, R0, a, init_scale, psi_b;
  int init_kind;
  double m_ref;
};

struct Scal3 {
  double lambda, mubar;
};

// Device state of one handle.
struct St3 {
  void* pops[2];     // 57 planes each (f 0..18, g 19..37, h 38..56), storage type
  double* pp[2];     // (phi, psi) pairs of a state, interleaved (pp[cur]: current, pp[cur ^ 1]: previous)
  double* mu;        // (mu_phi, mu_psi) pairs, interleaved
  void* uh[2];       // history: ux, uy, uz, vx, vy, vz, R_phi, R_psi of a step, in the storage type
  double* part;      // [kRedB][4] multiplier sums or [kRedB][8] invariant sums
  Scal3* sc;         // multipliers of the current step
  double* stage;     // FP64 staging [9][N]
  double* inv_out;   // [8]
  P3* dp;            // device copy of the parameters
  unsigned char* solid;  // [N] 1 = solid node
};

__device__ __forceinline__ double liquid_frac(const P3& p, double ph) {
  const double w = 0.5 * (1.0 + ph * p.inv_phib);
  return w < 0.0 ? 0.0 : (w > 1.0 ? 1.0 : w);
}
__device__ __forceinline__ double rho_of(const P3& p, double ph) { return p.rho_g + (p.rho_l - p.rho_g) * liquid_frac(p, ph); }
__device__ __forceinline__ double gsw(const P3& p, double ph) {
  const double r = ph * p.inv_phib;
  return 0.75 * r - 0.25 * r * r * r;
}
__device__ __forceinline__ double gsw_d(const P3& p, double ph) {
  const double r = ph * p.inv_phib;
  return 0.75 * p.inv_phib * (1.0 - r * r);
}
__device__ __forceinline__ double hprime(const P3& p, double ph) { return p.linear ? 1.0 : gsw_d(p, ph); }
__device__ __forceinline__ double hval(const P3& p, double ph) { return p.linear ? ph : 0.5 + gsw(p, ph); }
// -df_w/dphi, -df_w/dpsi of the wall energy at a wall-layer node (eq8, boundary)
__device__ __forceinline__ double wall_jphi(const P3& p, double ph, double ps) {
  const double a = p.sig_cos + (p.surf ? log(1.0 - ps) * p.dsb : 0.0);
  return a * gsw_d(p, ph);
}
__device__ __forceinline__ double wall_jpsi(const P3& p, double ph, double ps) {
  return p.surf ? -(p.dsb * gsw(p, ph) - 0.5 * p.msb) / (1.0 - ps) : 0.0;
}

__device__ __forceinline__ int wrap(int a, int n) { return a < 0 ? a + n : (a >= n ? a - n : a); }

// Node index offsets of the layers, rows and columns one step away from (x, y,
// z) along each axis (index 0: -1, 1: 0, 2: +1), periodic wraps included (in z
// as well: where z has walls the caller decides first whether a neighbour
// lies beyond one).  The neighbour along direction i is at3(o, i).
struct Off3 {
  int x[3], y[3], z[3];
};
__device__ __forceinline__ Off3 offsets3(const P3& p, int x, int y, int z) {
  const int nxy = p.nx * p.ny;
  Off3 o;
  o.x[0] = x == 0 ? p.nx - 1 : x - 1;
  o.x[1] = x;
  o.x[2] = x + 1 == p.nx ? 0 : x + 1;
  o.y[0] = (y == 0 ? p.ny - 1 : y - 1) * p.nx;
  o.y[1] = y * p.nx;
  o.y[2] = (y + 1 == p.ny ? 0 : y + 1) * p.nx;
  o.z[0] = (z == 0 ? p.nz - 1 : z - 1) * nxy;
  o.z[1] = z * nxy;
  o.z[2] = (z + 1 == p.nz ? 0 : z + 1) * nxy;
  return o;
}
__device__ __forceinline__ int at3(const Off3& o, int i) { return o.z[cz3(i) + 1] + o.y[cy3(i) + 1] + o.x[cx3(i) + 1]; }

// Neighbour of (x, y, z) along direction i: node index, or -1 / -2 beyond the
// bottom / top wall; *colnode is the node of the same (x, y) column in the
// layer of (x, y, z).
// -3: the neighbour is a solid node (complex walls).
__device__ __forceinline__ int nbr(const P3& p, const unsigned char* __restrict__ solid, int x, int y, int z, int i,
                                   int* colnode) {
  const int xx = wrap(x + cx3(i), p.nx), yy = wrap(y + cy3(i), p.ny);
  int zz = z + cz3(i);
  *colnode = (z * p.ny + yy) * p.nx + xx;
  if (p.periodic_z) zz = wrap(zz, p.nz);
  else if (zz < 0) return -1;
  else if (zz >= p.nz) return -2;
  const int m = (zz * p.ny + yy) * p.nx + xx;
  if (p.has_solid && solid[m]) return -3;
  return m;
}
// The same for a direction given as (cx, cy, cz).
__device__ __forceinline__ int nbr_c(const P3& p, const unsigned char* __restrict__ solid, int x, int y, int z, int cx,
                                     int cy, int cz, int* colnode) {
  const int xx = wrap(x + cx, p.nx), yy = wrap(y + cy, p.ny);
  int zz = z + cz;
  *colnode = (z * p.ny + yy) * p.nx + xx;
  if (p.periodic_z) zz = wrap(zz, p.nz);
  else if (zz < 0) return -1;
  else if (zz >= p.nz) return -2;
  const int m = (zz * p.ny + yy) * p.nx + xx;
  if (p.has_solid && solid[m]) return -3;
  return m;
}
// Nodes whose 18 neighbours are all fluid nodes inside the box: no solid mask,
// and not in the first or last layer of a box walled in z.
__device__ __forceinline__ bool plain_stencil(const P3& p, int z) {
  return !p.has_solid && (p.periodic_z || (z > 0 && z < p.nz - 1));
}


// Element k of plane pl of an array of planes of N values, addressed as a
// wave-uniform plane base plus a 32-bit per-lane byte offset (the node count
// stays below 2^29, so the offset of an FP64 value fits): the base stays in
// scalar registers and no 64-bit address is formed per lane.
template <class T>
__device__ __forceinline__ T& el(T* a, int pl, int N, int k) {
  return *(T*)((char*)(a + (size_t)pl * N) + (unsigned)k * (unsigned)sizeof(T));
}

// (phi, psi) or (mu_phi, mu_psi) of node k: each pair of fields is stored
// interleaved, so a node's pair is one 16-byte access (a wave-uniform base
// plus a 32-bit per-lane offset, as el).
__device__ __forceinline__ double2& pr(double2* a, int k) { return *(double2*)((char*)a + (unsigned)k * 16u); }
__device__ __forceinline__ const double2& pr(const double2* a, int k) {
  return *(const double2*)((const char*)a + (unsigned)k * 16u);
}

// Deterministic FP64 block sum of kT threads (valid in thread 0).
__device__ double block_sum(double v, double* sh) {
  for (int off = 32; off > 0; off >>= 1) v += __shfl_down(v, off, 64);
  __syncthreads();
  if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = v;
  __syncthreads();
  double r = 0.0;
  if (threadIdx.x == 0)
    for (int k = 0; k < kT / 64; ++k) r += sh[k];
  return r;
}

// ---------------------------------------------------------------- k3_mu
// mu_phi = 4 beta (1 - psi)(phi^3 - phi) - kappa L0 phi - T_phi + W psi phi
// mu_psi = kBT ln(psi/(1-psi)) - lambda_s L0 psi - T_psi - beta (1-phi^2)^2 + W phi^2 / 2
// with L0 the Laplacian with mirror ghosts and T the wall term of each
// direction pointing into a wetting wall: (2 w_i / c_s^2) J(column).
__global__ __launch_bounds__(kT) void k3_mu(const P3* __restrict__ pp_, const unsigned char* __restrict__ solid,
                                            const double2* __restrict__ pp, double2* __restrict__ mu,
                                            double* __restrict__ part) {
  const P3& p = *pp_;
  __shared__ double sh[4][kT / 64];
  const int N = p.N;
  double s1 = 0, s2 = 0, s3 = 0, s4 = 0;
  for (int n = blockIdx.x * kT + threadIdx.x; n < N; n += gridDim.x * kT) {
    if (p.has_solid && solid[n]) {
      pr(mu, n) = make_double2(0.0, 0.0);
      continue;
    }
    const int x = n % p.nx, y = (n / p.nx) % p.ny, z = n / (p.nx * p.ny);
    const double ph = pr(pp, n).x, ps = pr(pp, n).y;
    double l0p = 0.0, l0s = 0.0, tp = 0.0, ts = 0.0;
    if (plain_stencil(p, z)) {   // interior: plain stencil, unrolled
      const Off3 o = offsets3(p, x, y, z);
#pragma unroll
      for (int i = 1; i < Q3; ++i) {
        const int m = at3(o, i);
        const double wt = 2.0 * w3(i) / kCs2;
        l0p += wt * (pr(pp, m).x - ph);
        l0s += wt * (pr(pp, m).y - ps);
      }
    } else {   // next to a wall or a solid node: the general stencil, same order, rolled
      const double jp_self = p.solid_wet ? wall_jphi(p, ph, ps) : 0.0;
      const double js_self = p.solid_wet ? wall_jpsi(p, ph, ps) : 0.0;
#pragma unroll 1
      for (int i = 1; i < Q3; ++i) {
        int cn;
        const int m = nbr_c(p, solid, x, y, z, kC3[i][0], kC3[i][1], kC3[i][2], &cn);
        const double wt = 2.0 * kW3[i] / kCs2;
        if (m >= 0) {
          l0p += wt * (pr(pp, m).x - ph);
          l0s += wt * (pr(pp, m).y - ps);
        } else if (m == -3) {   // solid node: link-wise mirror, wall flux of this node
          if (p.solid_wet) {
            tp += wt * jp_self;
            ts += wt * js_self;
          }
        } else {
          l0p += wt * (pr(pp, cn).x - ph);
          l0s += wt * (pr(pp, cn).y - ps);
          if ((m == -1 && p.wet_b) || (m == -2 && p.wet_t)) {
            const double fph = pr(pp, cn).x, fps = pr(pp, cn).y;
            tp += wt * wall_jphi(p, fph, fps);
            ts += wt * wall_jpsi(p, fph, fps);
          }
        }
      }
    }
    const double mphi = 4.0 * p.beta * (1.0 - ps) * (ph * ph * ph - ph) - p.kappa * l0p - tp + p.W * ps * ph;
    const double mpsi = p.surf ? p.kBT * log(ps / (1.0 - ps)) - p.lambda_s * l0s - ts
                                     - p.beta * (1.0 - ph * ph) * (1.0 - ph * ph) + 0.5 * p.W * ph * ph
                               : 0.0;
    pr(mu, n) = make_double2(mphi, mpsi);
    const double hp = hprime(p, ph);
    s1 += hp * mphi;
    s2 += hp * hp;
    s3 += mpsi;
    s4 += hval(p, ph);
  }
  const double r1 = block_sum(s1, sh[0]), r2 = block_sum(s2, sh[1]), r3 = block_sum(s3, sh[2]), r4 = block_sum(s4, sh[3]);
  if (threadIdx.x == 0) {
    part[4 * blockIdx.x + 0] = r1;
    part[4 * blockIdx.x + 1] = r2;
    part[4 * blockIdx.x + 2] = r3;
    part[4 * blockIdx.x + 3] = r4;
  }
}

// One wavefront: lane l sums the partials l, l + 64, ... in order, then a
// fixed shuffle tree combines the lanes (the same order on every call).
__device__ __forceinline__ double wave_sum(double v) {
  for (int off = 32; off > 0; off >>= 1) v += __shfl_down(v, off, 64);
  return v;   // valid in lane 0
}

__global__ __launch_bounds__(64) void k3_fin(const P3* __restrict__ pp_, const double* __restrict__ part, int nb,
                                             Scal3* __restrict__ sc) {
  const P3& p = *pp_;
  double S1 = 0, S2 = 0, S3 = 0, S4 = 0;
  for (int b = threadIdx.x; b < nb; b += 64) {
    S1 += part[4 * b];
    S2 += part[4 * b + 1];
    S3 += part[4 * b + 2];
    S4 += part[4 * b + 3];
  }
  S1 = wave_sum(S1);
  S2 = wave_sum(S2);
  S3 = wave_sum(S3);
  S4 = wave_sum(S4);
  if (threadIdx.x != 0) return;
  double lam = S2 > 0.0 ? S1 / S2 : 0.0;
  if (p.phi_hold && S2 > 0.0 && p.M_phi > 0.0) lam += (p.m_ref - S4) / (p.M_phi * S2);
  sc->lambda = lam;
  sc->mubar = S3 / p.Nf;
}

// ------------------------------------------------------ MRT, closed form
// Raw moments in the order
// 0: 1; 1-3: x y z; 4-9: xx yy zz xy xz yz; 10-15: xxy xxz yyx yyz zzx zzy;
// 16-18: xxyy xxzz yyzz.
// The collision f + M^-1 [-S M (f - feq) + (I - S/2) M v] equals
// M^-1 [(I - S) M f + S M feq + (I - S/2) M v]: with S diagonal by moment
// order o, direction i adds to every moment of order o its raw-moment entry
// times q_o = (1 - s_o) f_i + s_o feq_i + (1 - s_o / 2) v_i.  The post-collision
// moments accumulate in one array while the populations stream in, and no
// population array is kept.
template <class T>
__device__ __forceinline__ void accum3(int i, const T* q, T* m) {
  const int a = cx3(i), b = cy3(i), c = cz3(i);
  m[0] += q[0];
  if (a) m[1] += a * q[1];
  if (b) m[2] += b * q[1];
  if (c) m[3] += c * q[1];
  if (a) m[4] += q[2];
  if (b) m[5] += q[2];
  if (c) m[6] += q[2];
  if (a && b) m[7] += a * b * q[2];
  if (a && c) m[8] += a * c * q[2];
  if (b && c) m[9] += b * c * q[2];
  if (a && b) { m[10] += b * q[3]; m[12] += a * q[3]; m[16] += q[4]; }
  if (a && c) { m[11] += c * q[3]; m[14] += a * q[3]; m[17] += q[4]; }
  if (b && c) { m[13] += c * q[3]; m[15] += b * q[3]; m[18] += q[4]; }
}
template <class T>
__device__ __forceinline__ void accum3(int i, T f, T feq, T v, const T* rate5, T* m) {
  T q[5];
#pragma unroll
  for (int o = 0; o < 5; ++o) q[o] = (T(1) - rate5[o]) * f + rate5[o] * feq + (T(1) - T(0.5) * rate5[o]) * v;
  accum3(i, q, m);
}
// Raw moments of populations as they stream in: direction i adds f to every
// moment its raw-moment entry selects.
template <class T>
__device__ __forceinline__ void raw3(int i, T f, T* m) {
  const T q[5] = {f, f, f, f, f};
  accum3(i, q, m);
}
// Order of raw moment k (the index of its relaxation rate).
__host__ __device__ constexpr int order3(int k) { return k == 0 ? 0 : (k < 4 ? 1 : (k < 10 ? 2 : (k < 16 ? 3 : 4))); }
// Post-collision moments (I - S) m + S meq + (I - S/2) mv, S diagonal by order.
template <class T, class E>
__device__ __forceinline__ void relax3(const T* rate5, const T* mf, const E* meq, const E* mv, T* m) {
#pragma unroll
  for (int k = 0; k < Q3; ++k) {
    const T s = rate5[order3(k)];
    m[k] = (T(1) - s) * mf[k] + s * (T)meq[k] + (T(1) - T(0.5) * s) * (T)mv[k];
  }
}
// Raw moments of D3Q19's weights times the velocity monomials that the
// equilibria below need: sum w = 1, sum w c_a^2 = c_s^2 = 1/3, sum w c_a^2 c_b^2
// = c_s^4 = 1/9 (a != b), sum w c_a^4 = 1/3, sum w c_a^4 c_b^2 = 1/9, and no
// velocity has three nonzero components; odd monomials sum to zero.  From
// these, the moments of the flow equilibrium (Sec. 3, pressure based: p/c_s^2
// (w_i - delta_i0) + rho w_i s_i(u)) and of its forcing vector
// w_i [u.grad rho + c_i.F/c_s^2 + ((c_i.u)(c_i.grad rho) - c_s^2 u.grad rho)/c_s^2]
// follow in closed form: no per-direction equilibrium is formed.
template <class T>
__device__ __forceinline__ void flow_moments3(double pr_, double rho_, const double* u, const double* G_, const double* F_,
                                              T* meq, T* mv) {
  const T pr = (T)pr_, rho = (T)rho_, ux = (T)u[0], uy = (T)u[1], uz = (T)u[2];
  const T G[3] = {(T)G_[0], (T)G_[1], (T)G_[2]}, F[3] = {(T)F_[0], (T)F_[1], (T)F_[2]};
  const T xx = ux * ux, yy = uy * uy, zz = uz * uz;
  meq[0] = T(0);
  meq[1] = rho * ux;
  meq[2] = rho * uy;
  meq[3] = rho * uz;
  meq[4] = pr + rho * xx;
  meq[5] = pr + rho * yy;
  meq[6] = pr + rho * zz;
  meq[7] = rho * ux * uy;
  meq[8] = rho * ux * uz;
  meq[9] = rho * uy * uz;
  const T third = T(1) / T(3), sixth = T(1) / T(6);
  meq[10] = rho * uy * third;   // xxy
  meq[11] = rho * uz * third;   // xxz
  meq[12] = rho * ux * third;   // yyx
  meq[13] = rho * uz * third;   // yyz
  meq[14] = rho * ux * third;   // zzx
  meq[15] = rho * uy * third;   // zzy
  meq[16] = pr * third + rho * ((xx + yy) * third - zz * sixth);
  meq[17] = pr * third + rho * ((xx + zz) * third - yy * sixth);
  meq[18] = pr * third + rho * ((yy + zz) * third - xx * sixth);
  const T gx = ux * G[0], gy = uy * G[1], gz = uz * G[2];
  mv[0] = gx + gy + gz;
  mv[1] = F[0];
  mv[2] = F[1];
  mv[3] = F[2];
  mv[4] = gx + (gy + gz) * third;
  mv[5] = gy + (gx + gz) * third;
  mv[6] = gz + (gx + gy) * third;
  mv[7] = (ux * G[1] + uy * G[0]) * third;
  mv[8] = (ux * G[2] + uz * G[0]) * third;
  mv[9] = (uy * G[2] + uz * G[1]) * third;
  mv[10] = F[1] * third;
  mv[11] = F[2] * third;
  mv[12] = F[0] * third;
  mv[13] = F[2] * third;
  mv[14] = F[0] * third;
  mv[15] = F[1] * third;
  mv[16] = (gx + gy) * third;
  mv[17] = (gx + gz) * third;
  mv[18] = (gy + gz) * third;
}
// The same for a phase-field or surfactant lattice (Sec. 3): equilibrium
// (i = 0: (w_0 - 1) eta c, the rest population taken relative to c; else
// w_i eta c) + w_i c_i.(c v)/c_s^2, forcing w_i c_i.d/c_s^2 with d the backward
// difference of c v.
template <class T>
__device__ __forceinline__ void scalar_moments3(double c_, double eta, const double* v, const double* d_, T* meq, T* mv) {
  const T c = (T)c_, e = (T)(eta * c_), jx = c * (T)v[0], jy = c * (T)v[1], jz = c * (T)v[2];
  const T d[3] = {(T)d_[0], (T)d_[1], (T)d_[2]};
  const T third = T(1) / T(3), ninth = T(1) / T(9);
  meq[0] = T(0);
  meq[1] = jx;
  meq[2] = jy;
  meq[3] = jz;
  meq[4] = meq[5] = meq[6] = e * third;
  meq[7] = meq[8] = meq[9] = T(0);
  meq[10] = jy * third;
  meq[11] = jz * third;
  meq[12] = jx * third;
  meq[13] = jz * third;
  meq[14] = jx * third;
  meq[15] = jy * third;
  meq[16] = meq[17] = meq[18] = e * ninth;
  mv[0] = T(0);
  mv[1] = d[0];
  mv[2] = d[1];
  mv[3] = d[2];
  mv[4] = mv[5] = mv[6] = mv[7] = mv[8] = mv[9] = T(0);
  mv[10] = d[1] * third;
  mv[11] = d[2] * third;
  mv[12] = d[0] * third;
  mv[13] = d[2] * third;
  mv[14] = d[0] * third;
  mv[15] = d[1] * third;
  mv[16] = mv[17] = mv[18] = T(0);
}
// Populations from raw moments (the inverse of moments3).
template <class T>
__device__ __forceinline__ void populations3(const T* m, T* f) {
  // edges of plane (a, b): E0 = m_aabb, Ea = m_abb, Eb = m_aab, Eab = m_ab
  const T E[3][4] = {{m[16], m[12], m[10], m[7]},    // xy: xxyy, yyx, xxy, xy
                          {m[17], m[14], m[11], m[8]},    // xz: xxzz, zzx, xxz, xz
                          {m[18], m[15], m[13], m[9]}};   // yz: yyzz, zzy, yyz, yz
#pragma unroll
  for (int pl = 0; pl < 3; ++pl)
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      const T sa = (k & 1) ? T(-1) : T(1), sb = (k & 2) ? T(-1) : T(1);
      f[7 + 4 * pl + k] = T(0.25) * (E[pl][0] + sa * E[pl][1] + sb * E[pl][2] + sa * sb * E[pl][3]);
    }
  // faces: F0 = m_aa - (edge sums of the two planes through a), F1 = m_a - (their c_a sums)
  const T F0x = m[4] - m[16] - m[17], F1x = m[1] - m[12] - m[14];
  const T F0y = m[5] - m[16] - m[18], F1y = m[2] - m[10] - m[15];
  const T F0z = m[6] - m[17] - m[18], F1z = m[3] - m[11] - m[13];
  f[1] = T(0.5) * (F0x + F1x);
  f[2] = T(0.5) * (F0x - F1x);
  f[3] = T(0.5) * (F0y + F1y);
  f[4] = T(0.5) * (F0y - F1y);
  f[5] = T(0.5) * (F0z + F1z);
  f[6] = T(0.5) * (F0z - F1z);
  f[0] = m[0] - (m[4] + m[5] + m[6]) + (m[16] + m[17] + m[18]);
}
__device__ __forceinline__ double cdot3(int i, double ax, double ay, double az) {
  return cx3(i) * ax + cy3(i) * ay + cz3(i) * az;
}

// Macroscopic state at a node (phi, psi, rho, grad rho, F, u, p, the wall
// terms and the zero-flux Laplacian of psi), from the FP64 pairs and the f
// populations of the current state.
struct Macro3 {
  double ph, ps, rho, gr[3], F[3], u[3], pr, tphi, tpsi, l0s;
};
template <class S>
__device__ Macro3 macro3(const P3& p, const unsigned char* __restrict__ solid, const S* __restrict__ pop,
                         const double2* __restrict__ pp, const double2* __restrict__ mu, int n) {
  Macro3 M;
  const int N = p.N;
  const int x = n % p.nx, y = (n / p.nx) % p.ny, z = n / (p.nx * p.ny);
  M.ph = pr(pp, n).x;
  M.ps = pr(pp, n).y;
  M.rho = rho_of(p, M.ph);
  double gr[3] = {0, 0, 0}, gmp[3] = {0, 0, 0}, gms[3] = {0, 0, 0}, tp = 0.0, ts = 0.0, l0s = 0.0;
  // Interior nodes take the plain stencil, unrolled; nodes next to a wall or a
  // solid node take the general one (the same arithmetic per direction, in the
  // same order), in a loop kept rolled so the kernel's code stays small.
  if (plain_stencil(p, z)) {
    const Off3 o = offsets3(p, x, y, z);
#pragma unroll
    for (int i = 1; i < Q3; ++i) {
      const int m = at3(o, i);
      const double r = rho_of(p, pr(pp, m).x), mp = pr(mu, m).x, ms = pr(mu, m).y, pn = pr(pp, m).y;
      const int c[3] = {cx3(i), cy3(i), cz3(i)};
#pragma unroll
      for (int d = 0; d < 3; ++d) {
        if (c[d] == 0) continue;   // adds zero in the general form
        const double wc = c[d] * (w3(i) / kCs2);
        gr[d] += wc * r;
        gmp[d] += wc * mp;
        gms[d] += wc * ms;
      }
      l0s += 2.0 * w3(i) / kCs2 * (pn - M.ps);
    }
  } else {
    // wall fluxes of this node (for links into solid nodes), evaluated once
    const double jp_self = p.solid_wet ? wall_jphi(p, M.ph, M.ps) : 0.0;
    const double js_self = p.solid_wet ? wall_jpsi(p, M.ph, M.ps) : 0.0;
#pragma unroll 1
    for (int i = 1; i < Q3; ++i) {
      const int cx = kC3[i][0], cy = kC3[i][1], cz = kC3[i][2];
      const double wi = kW3[i];
      int cn;
      const int m = nbr_c(p, solid, x, y, z, cx, cy, cz, &cn);
      double r, mp, ms, pn;
      if (m >= 0) {
        r = rho_of(p, pr(pp, m).x);
        mp = pr(mu, m).x;
        ms = pr(mu, m).y;
        pn = pr(pp, m).y;
      } else if (m == -3) {   // solid node: ghost values of this node
        r = rho_of(p, M.ph + jp_self / p.kappa);
        mp = pr(mu, n).x;
        ms = pr(mu, n).y;
        pn = M.ps;
        if (p.solid_wet) {
          tp += 2.0 * wi / kCs2 * jp_self;
          ts += 2.0 * wi / kCs2 * js_self;
        }
      } else {
        const bool wet = (m == -1 && p.wet_b) || (m == -2 && p.wet_t);
        const double fph = pr(pp, cn).x, fps = pr(pp, cn).y;
        const double jp = wet ? wall_jphi(p, fph, fps) : 0.0;
        r = rho_of(p, fph + jp / p.kappa);
        mp = pr(mu, cn).x;
        ms = pr(mu, cn).y;
        pn = fps;
        if (wet) {
          tp += 2.0 * wi / kCs2 * jp;
          ts += 2.0 * wi / kCs2 * wall_jpsi(p, fph, fps);
        }
      }
      const int c[3] = {cx, cy, cz};
      for (int d = 0; d < 3; ++d) {
        const double wc = c[d] * kWC3[i];
        gr[d] += wc * r;
        gmp[d] += wc * mp;
        gms[d] += wc * ms;
      }
      l0s += 2.0 * wi / kCs2 * (pn - M.ps);
    }
  }
  const double G[3] = {p.gx, p.gy, p.gz}, inv_rho = 1.0 / M.rho;
  double j[3] = {0, 0, 0}, snz = 0.0;
#pragma unroll
  for (int i = 0; i < Q3; ++i) {
    const double fi = (double)el(pop, i, N, n);
    j[0] += cx3(i) * fi;
    j[1] += cy3(i) * fi;
    j[2] += cz3(i) * fi;
    if (i) snz += fi;
  }
#pragma unroll
  for (int d = 0; d < 3; ++d) {
    M.gr[d] = gr[d];
    M.F[d] = -M.ph * gmp[d] - M.ps * gms[d] + M.rho * G[d];
    M.u[d] = (j[d] + 0.5 * M.F[d]) * inv_rho;
  }
  const double ugr = M.u[0] * gr[0] + M.u[1] * gr[1] + M.u[2] * gr[2];
  const double uu = M.u[0] * M.u[0] + M.u[1] * M.u[1] + M.u[2] * M.u[2];
  M.pr = kCs2 / (1.0 - w3(0)) * (snz + 0.5 * ugr - M.rho * w3(0) * uu * 1.5);   // 1 / (2 c_s^2) = 3/2
  M.tphi = tp;
  M.tpsi = ts;
  M.l0s = l0s;
  return M;
}

// ---------------------------------------------------------------- k3_colf
// Macroscopic state, sources and advecting velocity of the step (into the
// history planes hout), then the flow lattice's collision and streaming.
// Launch bound of the flow kernel: four waves per SIMD in FP32 storage, two in
// FP64; both compile without spills to at most 128 registers, so both run at
// four.
template <class S>
constexpr int kColfWaves = sizeof(S) == 8 ? 2 : 4;
template <class S>
__global__ __launch_bounds__(kT, kColfWaves<S>) void k3_colf(
    const P3* __restrict__ pp_, const unsigned char* __restrict__ solid, const S* __restrict__ pin, S* __restrict__ pout,
    const double2* __restrict__ pp, const double2* __restrict__ mu, const S* __restrict__ hin, S* __restrict__ hout,
    const Scal3* __restrict__ sc, int have_hist) {
  const P3& p = *pp_;
  const int N = p.N;
  const int n = blockIdx.x * kT + threadIdx.x;
  if (n >= N) return;
  if (p.has_solid && solid[n]) return;   // no fluid; its population slots stay zero
  const Macro3 M = macro3(p, solid, pin, pp, mu, n);
  const double ph = M.ph, ps = M.ps, rho = M.rho;
  const double lam = sc->lambda, mubar = sc->mubar;
  // sources (Sec. 3): R_phi with the multiplier term and the wall flux, R_psi likewise
  const double Rphi = p.M_phi * (-4.0 * p.beta * (1.0 - ps) * (ph * ph * ph - ph) - p.W * ps * ph + lam * hprime(p, ph))
                    + p.M_phi * M.tphi;
  // The bulk part -kBT ln(psi/(1-psi)) + beta (1-phi^2)^2 - W phi^2 / 2 of
  // R_psi is -(mu_psi + lambda_s L0 psi + T_psi), from mu_psi as k3_mu formed it
  // (the same L0 psi and wall term, summed in the same order): no second
  // logarithm per node.
  const double bulk = -(pr(mu, n).y + p.lambda_s * M.l0s + M.tpsi);
  const double Rpsi = p.surf ? -p.M0 * M.l0s + p.M_psi * (bulk + mubar) + p.M_psi * M.tpsi : 0.0;
  // advecting velocity (the step's own u, or its mean with the previous step's)
  double v[3] = {M.u[0], M.u[1], M.u[2]};
  if (have_hist && !p.adv_raw)
    for (int d = 0; d < 3; ++d) v[d] = 0.5 * (M.u[d] + (double)el(hin, d, N, n));
  for (int d = 0; d < 3; ++d) {
    el(hout, d, N, n) = (S)M.u[d];
    el(hout, (3 + d), N, n) = (S)v[d];
  }
  el(hout, 6, N, n) = (S)Rphi;
  el(hout, 7, N, n) = (S)Rpsi;

  const int x = n % p.nx, y = (n / p.nx) % p.ny, z = n / (p.nx * p.ny);
  using T = S;   // collision arithmetic: the storage type (FP32 or FP64)
  T m[Q3], f[Q3];
  {
    T rates[5];
    for (int k = 0; k < 5; ++k) rates[k] = (T)p.sf[k];
    if (p.s2_local) {
      const double mud = p.mu_g + (p.mu_l - p.mu_g) * liquid_frac(p, ph);
      rates[2] = (T)(1.0 / (3.0 * mud / rho + 0.5));
    }
    T mf[Q3];
#pragma unroll
    for (int k = 0; k < Q3; ++k) mf[k] = T(0);
#pragma unroll
    for (int i = 0; i < Q3; ++i) raw3<T>(i, (T)el(pin, i, N, n), mf);   // pressure-based: of the order of p w_i / c_s^2
    T meq[Q3], mv[Q3];
    flow_moments3<T>(M.pr, rho, M.u, M.gr, M.F, meq, mv);
    relax3(rates, mf, meq, mv, m);
    populations3<T>(m, f);
    // push streaming; walls in z
    const Off3 o = offsets3(p, x, y, z);
    if (!p.has_solid && (p.periodic_z || (z > 0 && z < p.nz - 1))) {   // every target is a fluid node
#pragma unroll
      for (int i = 0; i < Q3; ++i) el(pout, i, N, at3(o, i)) = f[i];
      return;
    }
#pragma unroll
    for (int i = 0; i < Q3; ++i) {
      const double fo = (double)f[i];
      const int zz = z + cz3(i);
      const int t = at3(o, i);
      if ((p.periodic_z || (zz >= 0 && zz < p.nz)) && p.has_solid && solid[t]) {
        el(pout, opp3(i), N, n) = (S)fo;   // half-way bounce-back at a solid node at rest
      } else if (p.periodic_z || (zz >= 0 && zz < p.nz)) {
        el(pout, i, N, t) = (S)fo;
      } else {
        const bool bot = zz < 0;
        if (bot ? p.freeslip_b : p.freeslip_t) {
          el(pout, mirz3(i), N, o.z[1] + o.y[cy3(i) + 1] + o.x[cx3(i) + 1]) = (S)fo;
        } else {
          const double uw = bot ? p.uw_b : p.uw_t;
          el(pout, opp3(i), N, n) = (S)(fo - (2.0 * w3(i) / kCs2) * rho * (cx3(i) * uw));
        }
      }
    }
  }
}

// ---------------------------------------------------------------- k3_colgh
// Phase-field and surfactant lattices: equilibria with phi v, psi v, forcing
// with the backward differences of phi v, psi v and of the sources (from the
// history planes of this step, hcur, and of the previous one, hprev), the
// rest population stored relative to phi, psi of this step.
template <class S>
__global__ __launch_bounds__(kT) void k3_colgh(const P3* __restrict__ pp_, const unsigned char* __restrict__ solid,
                                               const S* __restrict__ pin, S* __restrict__ pout,
                                               const double2* __restrict__ pp, const double2* __restrict__ pprev,
                                               const S* __restrict__ hcur, const S* __restrict__ hprev,
                                               int have_hist) {
  const P3& p = *pp_;
  const int N = p.N;
  const int n = blockIdx.x * kT + threadIdx.x;
  if (n >= N) return;
  if (p.has_solid && solid[n]) return;
  const double2 c2 = pr(pp, n);
  const double ph = c2.x, ps = c2.y;
  const double v[3] = {(double)hcur[(size_t)3 * N + n], (double)hcur[(size_t)4 * N + n], (double)hcur[(size_t)5 * N + n]};
  const double Rphi = (double)hcur[(size_t)6 * N + n], Rpsi = (double)hcur[(size_t)7 * N + n];
  double dph[3] = {0, 0, 0}, dps[3] = {0, 0, 0}, dRp = 0.0, dRs = 0.0;
  if (have_hist) {
    const double2 q2 = pr(pprev, n);
    const double php = q2.x, psp = q2.y;
    for (int d = 0; d < 3; ++d) {
      const double vh = (double)hprev[(size_t)(3 + d) * N + n];
      dph[d] = ph * v[d] - php * vh;
      dps[d] = ps * v[d] - psp * vh;
    }
    dRp = Rphi - (double)hprev[(size_t)6 * N + n];
    dRs = Rpsi - (double)hprev[(size_t)7 * N + n];
  }
  const int x = n % p.nx, y = (n / p.nx) % p.ny, z = n / (p.nx * p.ny);
  using T = S;   // collision arithmetic: the storage type (FP32 or FP64)
  T m[Q3], f[Q3];
  // --- phase-field and surfactant lattices (rest population stored relative to phi, psi of this step)
  for (int lat = 1; lat <= 2; ++lat) {
    if (lat == 2 && !p.surf) {
#pragma unroll
      for (int i = 0; i < Q3; ++i) {   // idle surfactant lattice: keep zeros in the target buffer
        const int zz = z + cz3(i);
        const int xx = wrap(x + cx3(i), p.nx), yy = wrap(y + cy3(i), p.ny);
        const int t = (wrap(zz, p.nz) * p.ny + yy) * p.nx + xx;
        const bool inside = p.periodic_z || (zz >= 0 && zz < p.nz);
        if (inside && !(p.has_solid && solid[t])) pout[(size_t)(38 + i) * N + t] = (S)0.0;
        else pout[(size_t)(38 + opp3(i)) * N + n] = (S)0.0;
      }
      break;
    }
    const double c = lat == 1 ? ph : ps;
    const double eta = lat == 1 ? p.eta_phi : p.eta_psi;
    const double* dj = lat == 1 ? dph : dps;
    T r5[5];
    for (int k = 0; k < 5; ++k) r5[k] = (T)(lat == 1 ? p.sg[k] : p.sh[k]);
    const double extra = lat == 1 ? Rphi + 0.5 * dRp : Rpsi + 0.5 * dRs;
    const int base = 19 * lat;
    const double cref = lat == 1 ? pr(pprev, n).x : pr(pprev, n).y;   // the shift of the stored rest population
    T mf[Q3];
#pragma unroll
    for (int k = 0; k < Q3; ++k) mf[k] = T(0);
#pragma unroll
    for (int i = 0; i < Q3; ++i) {
      // rest population shifted by c (the collision maps g - c e_0 to its image
      // minus c e_0), so the collision sees increments only
      const double fi = (double)pin[(size_t)(base + i) * N + n] + (i == 0 ? cref - c : 0.0);
      raw3<T>(i, (T)fi, mf);
    }
    T meq[Q3], mv[Q3];
    scalar_moments3<T>(c, eta, v, dj, meq, mv);
    relax3(r5, mf, meq, mv, m);
    populations3<T>(m, f);
#pragma unroll
    for (int i = 0; i < Q3; ++i) {
      const double val = (double)f[i] + w3(i) * extra;   // the rest population stays stored relative to c
      const int zz = z + cz3(i);
      const int xx = wrap(x + cx3(i), p.nx), yy = wrap(y + cy3(i), p.ny);
      const int t = (wrap(zz, p.nz) * p.ny + yy) * p.nx + xx;
      const bool inside = p.periodic_z || (zz >= 0 && zz < p.nz);
      if (inside && !(p.has_solid && solid[t])) pout[(size_t)(base + i) * N + t] = (S)val;
      else pout[(size_t)(base + opp3(i)) * N + n] = (S)val;
    }
  }
}

// ---------------------------------------------------------------- k3_mom
// phi, psi of the state just streamed: the moving populations plus the rest
// population and its shift (phi, psi of the step that wrote it).
template <class S>
__global__ __launch_bounds__(kT) void k3_mom(const P3* __restrict__ pp_, const unsigned char* __restrict__ solid,
                                             const S* __restrict__ pop,
                                             const double2* __restrict__ pold, double2* __restrict__ pnew) {
  const P3& p = *pp_;
  const int N = p.N;
  const int n = blockIdx.x * kT + threadIdx.x;
  if (n >= N) return;
  if (p.has_solid && solid[n]) return;   // stays zero
  double a = 0.0, b = 0.0;
#pragma unroll
  for (int i = 1; i < Q3; ++i) {
    a += (double)el(pop, (19 + i), N, n);
    b += (double)el(pop, (38 + i), N, n);
  }
  const double2 o = pr(pold, n);
  pr(pnew, n) = make_double2(o.x + (double)el(pop, 19, N, n) + a, p.surf ? o.y + (double)el(pop, 38, N, n) + b : 0.0);
}

// ------------------------------------------------------- initial state, load
__global__ __launch_bounds__(kT) void k3_profile(const P3* __restrict__ pp_, double* __restrict__ stage) {
  const P3& p = *pp_;
  const int n = blockIdx.x * kT + threadIdx.x;
  if (n >= p.N) return;
  const int x = n % p.nx, y = (n / p.nx) % p.ny, z = n / (p.nx * p.ny);
  double dx = x - p.x0, dy = y - p.y0, dz = z - p.z0;
  dx -= p.nx * floor(dx / p.nx + 0.5);
  dy -= p.ny * floor(dy / p.ny + 0.5);
  if (p.periodic_z) dz -= p.nz * floor(dz / p.nz + 0.5);
  const double r = sqrt(dx * dx + dy * dy + dz * dz);
  const double d = p.init_kind == LBM_INIT_SLAB ? 0.5 * p.a - fabs(dx) : (p.init_kind == LBM_INIT_BUBBLE ? r - p.R0 : p.R0 - r);
  stage[n] = p.phib * tanh(p.init_scale * d);
  stage[p.N + n] = p.surf ? p.psi_b : 0.0;
}

// Equilibrium populations of staged phi, psi (and u) with p = 0; both plane
// pairs take phi, psi (the rest populations are stored relative to them).
template <class S>
__global__ __launch_bounds__(kT) void k3_load(const P3* __restrict__ pp_, const unsigned char* __restrict__ solid,
                                              const double* __restrict__ stage, int with_u, S* __restrict__ pop,
                                              S* __restrict__ pop2, double2* __restrict__ pa, double2* __restrict__ pb) {
  const P3& p = *pp_;
  const int N = p.N;
  const int n = blockIdx.x * kT + threadIdx.x;
  if (n >= N) return;
  if (p.has_solid && solid[n]) {   // no fluid: zero populations in both buffers, zero fields
#pragma unroll
    for (int i = 0; i < 57; ++i) pop[(size_t)i * N + n] = pop2[(size_t)i * N + n] = (S)0.0;
    pr(pa, n) = pr(pb, n) = make_double2(0.0, 0.0);
    return;
  }
  const double ph = stage[n], ps = p.surf ? stage[N + n] : 0.0;
  const double u[3] = {with_u ? stage[2 * (size_t)N + n] : 0.0, with_u ? stage[3 * (size_t)N + n] : 0.0,
                       with_u ? stage[4 * (size_t)N + n] : 0.0};
  const double rho = rho_of(p, ph), uu = u[0] * u[0] + u[1] * u[1] + u[2] * u[2];
#pragma unroll
  for (int i = 0; i < Q3; ++i) {
    const double cu = cdot3(i, u[0], u[1], u[2]);
    const double fe = with_u ? rho * w3(i) * (cu / kCs2 + cu * cu / (2.0 * kCs2 * kCs2) - uu / (2.0 * kCs2)) : 0.0;
    const double ge = (i == 0 ? ph + (w3(0) - 1.0) * p.eta_phi * ph : w3(i) * p.eta_phi * ph) + w3(i) * ph * cu / kCs2;
    const double he = (i == 0 ? ps + (w3(0) - 1.0) * p.eta_psi * ps : w3(i) * p.eta_psi * ps) + w3(i) * ps * cu / kCs2;
    pop[(size_t)i * N + n] = (S)fe;
    pop[(size_t)(19 + i) * N + n] = (S)(i == 0 ? ge - ph : ge);
    pop[(size_t)(38 + i) * N + n] = (S)(p.surf ? (i == 0 ? he - ps : he) : 0.0);
  }
  pr(pa, n) = pr(pb, n) = make_double2(ph, ps);
}

// Fields of the current state into the staging planes:
// phi, psi, ux, uy, uz, p, rho, mu_phi, mu_psi.
template <class S>
__global__ __launch_bounds__(kT) void k3_fields(const P3* __restrict__ pp_, const unsigned char* __restrict__ solid,
                                                const S* __restrict__ pop, const double2* __restrict__ pp,
                                                const double2* __restrict__ mu, double* __restrict__ stage) {
  const P3& p = *pp_;
  const int N = p.N;
  const int n = blockIdx.x * kT + threadIdx.x;
  if (n >= N) return;
  if (p.has_solid && solid[n]) {   // fields of a solid node: zero
#pragma unroll
    for (int k = 0; k < 9; ++k) stage[(size_t)k * N + n] = 0.0;
    return;
  }
  const Macro3 M = macro3(p, solid, pop, pp, mu, n);
  const double v[9] = {M.ph, M.ps, M.u[0], M.u[1], M.u[2], M.pr, M.rho, pr(mu, n).x, pr(mu, n).y};
#pragma unroll
  for (int k = 0; k < 9; ++k) stage[(size_t)k * N + n] = v[k];
}

// Invariant sums from the staged fields: mass_psi, m_phi_h, sum_phi, kinetic,
// umax (max), nonfinite, psi_out_of_range; per workgroup, then k3_inv_fin.
__global__ __launch_bounds__(kT) void k3_inv(const P3* __restrict__ pp_, const unsigned char* __restrict__ solid,
                                             const double* __restrict__ stage, double* __restrict__ part) {
  const P3& p = *pp_;
  __shared__ double sh[6][kT / 64];
  __shared__ double smax[kT];
  const int N = p.N;
  double a[6] = {0, 0, 0, 0, 0, 0}, um = 0.0;
  for (int n = blockIdx.x * kT + threadIdx.x; n < N; n += gridDim.x * kT) {
    if (p.has_solid && solid[n]) continue;
    const double ph = stage[n], ps = stage[N + n], ux = stage[2 * (size_t)N + n], uy = stage[3 * (size_t)N + n],
                 uz = stage[4 * (size_t)N + n], pr = stage[5 * (size_t)N + n], rho = stage[6 * (size_t)N + n];
    const double u2 = ux * ux + uy * uy + uz * uz;
    a[0] += ps;
    a[1] += 0.5 + gsw(p, ph);
    a[2] += ph;
    a[3] += 0.5 * rho * u2;
    if (!(isfinite(ph) && isfinite(ps) && isfinite(u2) && isfinite(pr))) a[4] += 1.0;
    if (p.surf && !(ps > 0.0 && ps < 1.0)) a[5] += 1.0;
    const double s = sqrt(u2);
    um = s > um ? s : um;
  }
  double r[6];
  for (int k = 0; k < 6; ++k) r[k] = block_sum(a[k], sh[k]);
  smax[threadIdx.x] = um;
  __syncthreads();
  for (int off = kT / 2; off > 0; off >>= 1) {
    if ((int)threadIdx.x < off) smax[threadIdx.x] = fmax(smax[threadIdx.x], smax[threadIdx.x + off]);
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    for (int k = 0; k < 6; ++k) part[8 * blockIdx.x + k] = r[k];
    part[8 * blockIdx.x + 6] = smax[0];
  }
}
__global__ __launch_bounds__(64) void k3_inv_fin(const double* __restrict__ part, int nb, double* __restrict__ out) {
  double s[7] = {0, 0, 0, 0, 0, 0, 0};
  for (int b = threadIdx.x; b < nb; b += 64) {
    for (int k = 0; k < 6; ++k) s[k] += part[8 * b + k];
    s[6] = fmax(s[6], part[8 * b + 6]);
  }
  for (int k = 0; k < 6; ++k) s[k] = wave_sum(s[k]);
  for (int off = 32; off > 0; off >>= 1) s[6] = fmax(s[6], __shfl_down(s[6], off, 64));
  if (threadIdx.x == 0)
    for (int k = 0; k < 7; ++k) out[k] = s[k];
}

int nblk(long long n) { return (int)((n + kT - 1) / kT); }
int red_blocks(int N) { const int b = nblk(N); return b < kRedB ? b : kRedB; }
size_t al256(size_t v) { return (v + 255) & ~size_t(255); }

thread_local std::string g_err3 = "no error";
constexpr double kPi = 3.14159265358979323846;

}  // namespace

struct lbm3d_handle {
  lbm3d_params prm;
  P3 p;
  St3 s;
  int cur = 0, have_hist = 0;
  int64_t step = 0;
  bool faulted = false;
  void* buf = nullptr;
  bool own_buf = false;
  hipStream_t stream = nullptr;
  bool own_stream = false;
  std::string err = "no error";
};

namespace {

int fail3(lbm3d_handle* h, int code, const std::string& msg) {
  if (h) h->err = msg;
  else g_err3 = msg;
  return code;
}
#define HIP3(h, expr, where)                                                                          \
  do {                                                                                                \
    hipError_t e_ = (expr);                                                                           \
    if (e_ != hipSuccess) return fail3(h, LBM_E_DEVICE, std::string(where) + ": " + hipGetErrorString(e_)); \
  } while (0)

std::string derive3(const lbm3d_params& q, P3& d) {
  if (q.abi_version != LBM3D_ABI_VERSION) return "abi_version mismatch";
  if (q.nx < 3 || q.ny < 3 || q.nz < 3) return "nx, ny and nz must be >= 3";
  if ((double)q.nx * q.ny * q.nz * 57.0 > 9.0e18 || (double)q.nx * q.ny * q.nz >= 536870912.0) return "grid too large (at most 2^29 nodes)";
  auto bc_ok = [](int b) { return b >= LBM_BC_PERIODIC && b <= LBM_BC_FREESLIP; };
  if (!bc_ok(q.bc_bottom) || !bc_ok(q.bc_top)) return "unknown boundary kind";
  if ((q.bc_bottom == LBM_BC_PERIODIC) != (q.bc_top == LBM_BC_PERIODIC)) return "periodic z needs both walls periodic";
  if (q.precision != LBM_FP64 && q.precision != LBM_FP32) return "precision must be LBM_FP64 or LBM_FP32";
  if (q.constraint_phi != LBM_CONSTRAINT_NONLINEAR && q.constraint_phi != LBM_CONSTRAINT_LINEAR) return "unknown constraint";
  if (q.init_kind < LBM_INIT_DROP || q.init_kind > LBM_INIT_BUBBLE) return "unknown init kind";
  if ((q.adv_raw != 0 && q.adv_raw != 1) || (q.phi_hold != 0 && q.phi_hold != 1) || (q.solid_wet != 0 && q.solid_wet != 1))
    return "adv_raw, phi_hold and solid_wet must be 0 or 1";
  if (q.solid_wet && !(q.theta0_deg > 0.0 && q.theta0_deg < 180.0)) return "theta0 must lie in (0,180) on wetting solids";
  if (!(q.sigma_gl0 > 0.0) || !(q.eps > 0.0)) return "sigma_gl0 and eps must be > 0";
  if (!(q.M_phi >= 0.0) || !(q.M_psi >= 0.0)) return "mobilities must be >= 0";
  if (!(q.psi_b >= 0.0 && q.psi_b < 1.0)) return "psi_b must lie in [0,1)";
  if (!(q.rho_l > 0.0 && q.rho_g > 0.0 && q.mu_l > 0.0 && q.mu_g > 0.0)) return "densities and viscosities must be > 0";
  const bool wet = q.bc_bottom == LBM_BC_WALL_WET || q.bc_top == LBM_BC_WALL_WET || q.solid_wet;
  if (wet && !(q.theta0_deg > 0.0 && q.theta0_deg < 180.0)) return "theta0 must lie in (0,180) on a wetting wall";
  const double* rates[3] = {q.s_f, q.s_g, q.s_h};
  for (int l = 0; l < 3; ++l)
    for (int k = 0; k < 5; ++k)
      if (!(rates[l][k] < 2.0)) return "relaxation rates must lie in (0,2)";
  std::memset(&d, 0, sizeof(d));
  d.nx = q.nx; d.ny = q.ny; d.nz = q.nz; d.N = q.nx * q.ny * q.nz;
  d.periodic_z = q.bc_bottom == LBM_BC_PERIODIC;
  d.wet_b = q.bc_bottom == LBM_BC_WALL_WET;
  d.wet_t = q.bc_top == LBM_BC_WALL_WET;
  d.freeslip_b = q.bc_bottom == LBM_BC_FREESLIP;
  d.freeslip_t = q.bc_top == LBM_BC_FREESLIP;
  d.surf = q.psi_b > 0.0;
  d.linear = q.constraint_phi == LBM_CONSTRAINT_LINEAR;
  d.adv_raw = q.adv_raw;
  d.phi_hold = q.phi_hold;
  d.solid_wet = q.solid_wet;
  d.has_solid = 0;
  d.Nf = d.N;
  const double kappa = 0.375 * q.eps * q.sigma_gl0, beta = 0.75 * q.sigma_gl0 / q.eps;
  const double W = q.W > 0.0 ? q.W : 4.0 * beta / (q.Ex > 0.0 ? q.Ex : 0.5);
  const double kBT = q.kBT > 0.0 ? q.kBT : 4.0 * beta * (q.Pi > 0.0 ? q.Pi : 1.35);
  double phib = 1.0;
  if (q.phi_b > 0.0) phib = q.phi_b;
  else if (d.surf) {
    const double r = 1.0 - W * q.psi_b / (4.0 * beta * (1.0 - q.psi_b));
    if (!(r > 0.0)) return "bulk surfactant too large: phi_b^2 <= 0";
    phib = std::sqrt(r);
  }
  double sg0 = q.sigma_sg0, sl0 = q.sigma_sl0;
  if (!(sg0 >= 0.0 && sl0 >= 0.0)) {
    const double diff = q.sigma_gl0 * std::cos(q.theta0_deg * kPi / 180.0), sum = 16.0 * q.sigma_gl0 / 15.0;
    sg0 = 0.5 * (sum + diff);
    sl0 = 0.5 * (sum - diff);
  }
  const double lambda_s = q.lambda_s >= 0.0 ? q.lambda_s : (wet ? 0.5 * kappa : 0.0);
  if (wet && d.surf && lambda_s == 0.0 && (q.beta_sg != 0.0 || q.beta_sl != 0.0))
    return "lambda_s = 0 cannot carry the solid-adsorption boundary condition";
  const double M0 = q.M0 >= 0.0 ? q.M0 : (lambda_s > 0.0 ? 0.0 : q.M_phi * kappa);
  auto rate = [](double v) { return v > 0.0 ? v : 1.0; };
  const double s1g = rate(q.s_g[1]), s1h = rate(q.s_h[1]);
  d.kappa = kappa; d.beta = beta; d.W = W; d.kBT = kBT; d.phib = phib; d.inv_phib = 1.0 / phib;
  d.lambda_s = lambda_s; d.M0 = M0; d.M_phi = q.M_phi; d.M_psi = q.M_psi;
  d.eta_phi = q.eta_phi > 0.0 ? q.eta_phi : q.M_phi * kappa / ((1.0 / s1g - 0.5) * kCs2);
  d.eta_psi = q.eta_psi > 0.0 ? q.eta_psi : (q.M_psi * lambda_s + M0) / ((1.0 / s1h - 0.5) * kCs2);
  d.rho_l = q.rho_l; d.rho_g = q.rho_g; d.mu_l = q.mu_l; d.mu_g = q.mu_g;
  d.gx = q.gx; d.gy = q.gy; d.gz = q.gz; d.uw_b = q.u_wall_bottom; d.uw_t = q.u_wall_top;
  d.sig_cos = q.sigma_gl0 * std::cos(q.theta0_deg * kPi / 180.0);
  d.dsb = sg0 * q.beta_sg - sl0 * q.beta_sl;
  d.msb = sg0 * q.beta_sg + sl0 * q.beta_sl;
  for (int k = 0; k < 5; ++k) { d.sf[k] = rate(q.s_f[k]); d.sg[k] = rate(q.s_g[k]); d.sh[k] = rate(q.s_h[k]); }
  d.s2_local = !(q.s_f[2] > 0.0);
  d.x0 = q.x0; d.y0 = q.y0; d.z0 = q.z0; d.R0 = q.R0; d.a = q.a;
  d.init_scale = 2.0 * phib * (d.surf ? std::sqrt(1.0 - q.psi_b) : 1.0) / q.eps;
  d.init_kind = q.init_kind;
  d.psi_b = q.psi_b;
  return "";
}

struct Lay3 {
  size_t pops, pp, mu, uh, part, sc, stage, inv, dp, solid, total;
};
Lay3 layout3(const lbm3d_params& q) {
  const size_t N = (size_t)q.nx * q.ny * q.nz, sb = q.precision == LBM_FP64 ? 8 : 4;
  Lay3 L{};
  size_t off = 0;
  auto take = [&](size_t b) { size_t o = off; off += al256(b); return o; };
  L.pops = take(2 * 57 * N * sb);
  L.pp = take(2 * 2 * N * 8);
  L.mu = take(2 * N * 8);
  L.uh = take(2 * 8 * N * sb);
  L.part = take((size_t)kRedB * 8 * 8);
  L.sc = take(sizeof(Scal3));
  L.stage = take(9 * N * 8);
  L.inv = take(8 * 8);
  L.dp = take(sizeof(P3));
  L.solid = take(N);
  L.total = off;
  return L;
}

template <class S>
hipError_t step3(lbm3d_handle* h) {
  const P3& p = h->p;
  St3& s = h->s;
  const int c = h->cur;
  const int rb = red_blocks(p.N);
  hipLaunchKernelGGL(k3_mu, dim3(rb), dim3(kT), 0, h->stream, s.dp, (const unsigned char*)s.solid, (const double2*)s.pp[c],
                     (double2*)s.mu, s.part);
  hipLaunchKernelGGL(k3_fin, dim3(1), dim3(64), 0, h->stream, s.dp, (const double*)s.part, rb, s.sc);
  hipLaunchKernelGGL((k3_colf<S>), dim3(nblk(p.N)), dim3(kT), 0, h->stream, s.dp, (const unsigned char*)s.solid,
                     (const S*)s.pops[c], (S*)s.pops[c ^ 1], (const double2*)s.pp[c], (const double2*)s.mu,
                     (const S*)s.uh[c ^ 1], (S*)s.uh[c], (const Scal3*)s.sc, h->have_hist);
  hipLaunchKernelGGL((k3_colgh<S>), dim3(nblk(p.N)), dim3(kT), 0, h->stream, s.dp, (const unsigned char*)s.solid,
                     (const S*)s.pops[c], (S*)s.pops[c ^ 1], (const double2*)s.pp[c], (const double2*)s.pp[c ^ 1],
                     (const S*)s.uh[c], (const S*)s.uh[c ^ 1], h->have_hist);
  hipLaunchKernelGGL((k3_mom<S>), dim3(nblk(p.N)), dim3(kT), 0, h->stream, s.dp, (const unsigned char*)s.solid,
                     (const S*)s.pops[c ^ 1], (const double2*)s.pp[c], (double2*)s.pp[c ^ 1]);
  return hipGetLastError();
}

// mu and the multipliers of the current state, then the fields into staging
template <class S>
hipError_t fields3(lbm3d_handle* h) {
  const P3& p = h->p;
  St3& s = h->s;
  const int c = h->cur;
  const int rb = red_blocks(p.N);
  hipLaunchKernelGGL(k3_mu, dim3(rb), dim3(kT), 0, h->stream, s.dp, (const unsigned char*)s.solid, (const double2*)s.pp[c],
                     (double2*)s.mu, s.part);
  hipLaunchKernelGGL(k3_fin, dim3(1), dim3(64), 0, h->stream, s.dp, (const double*)s.part, rb, s.sc);
  hipLaunchKernelGGL((k3_fields<S>), dim3(nblk(p.N)), dim3(kT), 0, h->stream, s.dp, (const unsigned char*)s.solid,
                     (const S*)s.pops[c],
                     (const double2*)s.pp[c], (const double2*)s.mu, s.stage);
  return hipGetLastError();
}

hipError_t load3(lbm3d_handle* h, int with_u) {
  St3& s = h->s;
  const int c = h->cur;
  if (h->prm.precision == LBM_FP64)
    hipLaunchKernelGGL((k3_load<double>), dim3(nblk(h->p.N)), dim3(kT), 0, h->stream, s.dp, (const unsigned char*)s.solid,
                       (const double*)s.stage, with_u, (double*)s.pops[c], (double*)s.pops[c ^ 1], (double2*)s.pp[c], (double2*)s.pp[c ^ 1]);
  else
    hipLaunchKernelGGL((k3_load<float>), dim3(nblk(h->p.N)), dim3(kT), 0, h->stream, s.dp, (const unsigned char*)s.solid,
                       (const double*)s.stage, with_u, (float*)s.pops[c], (float*)s.pops[c ^ 1], (double2*)s.pp[c], (double2*)s.pp[c ^ 1]);
  return hipGetLastError();
}

// invariants of the current state into inv_out (synchronises), optionally
// sets phi_hold's reference from them
int invariants3(lbm3d_handle* h, double* v7, Scal3* sc) {
  HIP3(h, h->prm.precision == LBM_FP64 ? fields3<double>(h) : fields3<float>(h), "field kernels");
  const int rb = red_blocks(h->p.N);
  hipLaunchKernelGGL(k3_inv, dim3(rb), dim3(kT), 0, h->stream, h->s.dp, (const unsigned char*)h->s.solid,
                     (const double*)h->s.stage, h->s.part);
  hipLaunchKernelGGL(k3_inv_fin, dim3(1), dim3(64), 0, h->stream, (const double*)h->s.part, rb, h->s.inv_out);
  HIP3(h, hipGetLastError(), "invariant kernels");
  HIP3(h, hipMemcpyAsync(v7, h->s.inv_out, 7 * sizeof(double), hipMemcpyDeviceToHost, h->stream), "copy invariants");
  if (sc) HIP3(h, hipMemcpyAsync(sc, h->s.sc, sizeof(Scal3), hipMemcpyDeviceToHost, h->stream), "copy multipliers");
  HIP3(h, hipStreamSynchronize(h->stream), "synchronise");
  return LBM_OK;
}

int set_ref3(lbm3d_handle* h) {
  if (!h->p.phi_hold) return LBM_OK;
  double v[7];
  const int rc = invariants3(h, v, nullptr);
  if (rc) return rc;
  h->p.m_ref = h->p.linear ? v[2] : v[1];
  HIP3(h, hipMemcpyAsync(h->s.dp, &h->p, sizeof(P3), hipMemcpyHostToDevice, h->stream), "upload parameters");
  HIP3(h, hipStreamSynchronize(h->stream), "synchronise");
  return LBM_OK;
}

}  // namespace

extern "C" {

int lbm3d_required_bytes(const lbm3d_params* q, size_t* bytes) {
  if (!q || !bytes) return fail3(nullptr, LBM_E_ARG, "null argument");
  P3 d;
  const std::string why = derive3(*q, d);
  if (!why.empty()) return fail3(nullptr, LBM_E_ARG, why);
  *bytes = layout3(*q).total;
  return LBM_OK;
}

int lbm3d_init(const lbm3d_params* q, void* dev_buf, size_t buf_bytes, void* hip_stream, lbm3d_handle** out) {
  if (!out) return fail3(nullptr, LBM_E_ARG, "null output handle");
  *out = nullptr;
  if (!q) return fail3(nullptr, LBM_E_ARG, "null parameters");
  lbm3d_handle* h = new lbm3d_handle();
  h->prm = *q;
  const std::string why = derive3(*q, h->p);
  if (!why.empty()) { delete h; return fail3(nullptr, LBM_E_ARG, why); }
  int dev = 0;
  hipDeviceProp_t prop;
  if (hipGetDevice(&dev) != hipSuccess || hipGetDeviceProperties(&prop, dev) != hipSuccess ||
      std::strncmp(prop.gcnArchName, "gfx950", 6) != 0) {
    delete h;
    return fail3(nullptr, LBM_E_DEVICE, "no gfx950 device");
  }
  const Lay3 L = layout3(*q);
  if (dev_buf) {
    if (buf_bytes < L.total || ((uintptr_t)dev_buf & 255)) { delete h; return fail3(nullptr, LBM_E_ARG, "dev_buf too small or not 256-byte aligned"); }
    h->buf = dev_buf;
  } else {
    if (hipMalloc(&h->buf, L.total) != hipSuccess) { delete h; return fail3(nullptr, LBM_E_OOM, "hipMalloc of the state failed"); }
    h->own_buf = true;
  }
  if (hip_stream) h->stream = (hipStream_t)hip_stream;
  else {
    if (hipStreamCreate(&h->stream) != hipSuccess) {
      if (h->own_buf) (void)hipFree(h->buf);
      delete h;
      return fail3(nullptr, LBM_E_DEVICE, "hipStreamCreate failed");
    }
    h->own_stream = true;
  }
  char* b = (char*)h->buf;
  const size_t N = (size_t)h->p.N, sb = q->precision == LBM_FP64 ? 8 : 4;
  h->s.pops[0] = b + L.pops;
  h->s.pops[1] = b + L.pops + 57 * N * sb;
  h->s.pp[0] = (double*)(b + L.pp);
  h->s.pp[1] = h->s.pp[0] + 2 * N;
  h->s.mu = (double*)(b + L.mu);
  h->s.uh[0] = b + L.uh;
  h->s.uh[1] = b + L.uh + 8 * N * sb;
  h->s.part = (double*)(b + L.part);
  h->s.sc = (Scal3*)(b + L.sc);
  h->s.stage = (double*)(b + L.stage);
  h->s.inv_out = (double*)(b + L.inv);
  h->s.dp = (P3*)(b + L.dp);
  h->s.solid = (unsigned char*)(b + L.solid);
  hipError_t e = hipMemsetAsync(h->s.solid, 0, N, h->stream);
  if (e == hipSuccess) e = hipMemcpyAsync(h->s.dp, &h->p, sizeof(P3), hipMemcpyHostToDevice, h->stream);
  if (e == hipSuccess) {
    hipLaunchKernelGGL(k3_profile, dim3(nblk(h->p.N)), dim3(kT), 0, h->stream, h->s.dp, h->s.stage);
    e = load3(h, 0);
  }
  if (e == hipSuccess) e = hipStreamSynchronize(h->stream);
  int rc = e == hipSuccess ? set_ref3(h) : LBM_E_DEVICE;
  if (rc != LBM_OK) {
    const std::string msg = e != hipSuccess ? std::string("initialisation: ") + hipGetErrorString(e) : h->err;
    lbm3d_destroy(h);
    return fail3(nullptr, LBM_E_DEVICE, msg);
  }
  *out = h;
  return LBM_OK;
}

int lbm3d_step(lbm3d_handle* h, int64_t n) {
  if (!h) return fail3(nullptr, LBM_E_ARG, "null handle");
  if (n < 0) return fail3(h, LBM_E_ARG, "negative step count");
  if (h->faulted) return fail3(h, LBM_E_STATE, "state holds non-finite or out-of-range values; load fields first");
  for (int64_t k = 0; k < n; ++k) {
    HIP3(h, h->prm.precision == LBM_FP64 ? step3<double>(h) : step3<float>(h), "step kernels");
    h->cur ^= 1;
    h->have_hist = 1;
    h->step += 1;
  }
  return LBM_OK;
}

int lbm3d_reduce_invariants(lbm3d_handle* h, lbm3d_invariants* out) {
  if (!h || !out) return fail3(h, LBM_E_ARG, "null argument");
  double v[7];
  Scal3 sc;
  int rc = invariants3(h, v, &sc);
  if (rc) return rc;
  std::memset(out, 0, sizeof(*out));
  out->step = h->step;
  out->mass_psi = v[0];
  out->m_phi_h = v[1];
  out->sum_phi = v[2];
  out->kinetic = v[3];
  out->nonfinite = (int64_t)v[4];
  out->psi_out_of_range = (int64_t)v[5];
  out->umax = v[6];
  out->lambda_phi = sc.lambda;
  out->mubar_psi = sc.mubar;
  if (out->psi_out_of_range > 0) { h->faulted = true; return fail3(h, LBM_E_RANGE, "psi left (0,1)"); }
  if (out->nonfinite > 0) { h->faulted = true; return fail3(h, LBM_E_NONFINITE, "non-finite values in the fields"); }
  return LBM_OK;
}

int lbm3d_fetch_fields(lbm3d_handle* h, uint32_t mask, double* host, size_t n_doubles) {
  if (!h || !host) return fail3(h, LBM_E_ARG, "null argument");
  if (mask == 0 || (mask & ~0x1FFu)) return fail3(h, LBM_E_ARG, "bad field mask");
  const size_t N = (size_t)h->p.N;
  if (n_doubles < (size_t)__builtin_popcount(mask) * N) return fail3(h, LBM_E_ARG, "host buffer too small");
  HIP3(h, h->prm.precision == LBM_FP64 ? fields3<double>(h) : fields3<float>(h), "field kernels");
  size_t k = 0;
  for (int bit = 0; bit < 9; ++bit)
    if (mask & (1u << bit))
      HIP3(h, hipMemcpyAsync(host + (k++) * N, h->s.stage + (size_t)bit * N, N * sizeof(double), hipMemcpyDeviceToHost,
                             h->stream), "copy fields");
  HIP3(h, hipStreamSynchronize(h->stream), "synchronise");
  return LBM_OK;
}

int lbm3d_load_fields(lbm3d_handle* h, int32_t with_u, const double* host, size_t n_doubles) {
  if (!h || !host) return fail3(h, LBM_E_ARG, "null argument");
  const size_t N = (size_t)h->p.N, planes = with_u ? 5 : 2;
  if (n_doubles < planes * N) return fail3(h, LBM_E_ARG, "host buffer too small");
  HIP3(h, hipMemcpyAsync(h->s.stage, host, planes * N * sizeof(double), hipMemcpyHostToDevice, h->stream), "copy fields");
  HIP3(h, load3(h, with_u ? 1 : 0), "load kernel");
  HIP3(h, hipStreamSynchronize(h->stream), "synchronise");
  h->have_hist = 0;
  h->faulted = false;
  return set_ref3(h);
}

int lbm3d_set_solid(lbm3d_handle* h, const uint8_t* mask, size_t n) {
  if (!h || !mask) return fail3(h, LBM_E_ARG, "null argument");
  const size_t N = (size_t)h->p.N;
  if (n < N) return fail3(h, LBM_E_ARG, "mask smaller than nx ny nz");
  int nf = 0, any = 0;
  for (size_t k = 0; k < N; ++k) {
    nf += mask[k] ? 0 : 1;
    any |= mask[k] ? 1 : 0;
  }
  if (nf == 0) return fail3(h, LBM_E_ARG, "no fluid node left");
  // the current phi, psi (fluid nodes) are rebuilt into equilibrium populations under the new mask
  HIP3(h, h->prm.precision == LBM_FP64 ? fields3<double>(h) : fields3<float>(h), "field kernels");
  std::vector<unsigned char> m(N);
  for (size_t k = 0; k < N; ++k) m[k] = mask[k] ? 1 : 0;
  HIP3(h, hipMemcpyAsync(h->s.solid, m.data(), N, hipMemcpyHostToDevice, h->stream), "copy mask");
  h->p.has_solid = any;
  h->p.Nf = nf;
  HIP3(h, hipMemcpyAsync(h->s.dp, &h->p, sizeof(P3), hipMemcpyHostToDevice, h->stream), "upload parameters");
  HIP3(h, load3(h, 0), "load kernel");
  HIP3(h, hipStreamSynchronize(h->stream), "synchronise");
  h->have_hist = 0;
  h->faulted = false;
  return set_ref3(h);
}

int lbm3d_bytes_per_node_step(lbm3d_handle* h, double* bytes) {
  if (!h || !bytes) return fail3(h, LBM_E_ARG, "null argument");
  const double sb = h->prm.precision == LBM_FP64 ? 8.0 : 4.0;
  // k3_mu: phi/psi read, mu written; k3_colf: 19 populations, phi/psi, mu and the previous u read, 19
  // populations and 8 history planes written; k3_colgh: 38 populations, phi/psi of two steps and 5 history
  // planes of two steps read, 38 populations written; k3_mom: 38 populations and phi/psi read, phi/psi written
  *bytes = (2 * 8 + 2 * 8) + (19 * sb + 2 * 8 + 2 * 8 + 3 * sb + 19 * sb + 8 * sb) +
           (38 * sb + 4 * 8 + 10 * sb + 38 * sb) + (38 * sb + 2 * 8 + 2 * 8);
  return LBM_OK;
}

int lbm3d_destroy(lbm3d_handle* h) {
  if (!h) return LBM_OK;
  if (h->stream) (void)hipStreamSynchronize(h->stream);
  if (h->own_buf && h->buf) (void)hipFree(h->buf);
  if (h->own_stream && h->stream) (void)hipStreamDestroy(h->stream);
  delete h;
  return LBM_OK;
}

const char* lbm3d_last_error(const lbm3d_handle* h) { return h ? h->err.c_str() : g_err3.c_str(); }

}  // extern "C"
