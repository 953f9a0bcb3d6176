// lbm_internal.h -- device-side parameter block and launcher interface shared
// by the C-ABI host code (lbm_capi.cpp) and the gfx950 kernels (lbm_kernels.hip).
#pragma once

#include <hip/hip_runtime.h>
#include <cstddef>
#include <cstdint>
#include <string>

struct lbm_handle;   // the C ABI's opaque handle (lbm_capi.cpp)

namespace lbm {

// Everything a kernel needs, derived once on the host (lattice units, FP64).
struct DevParams {
  int nx, ny, N;
  int periodic_y, bc_bottom, bc_top;
  int surf;        // surfactant lattice active
  int linear;      // linear constraint h = phi
  int adv_raw;     // advect phi/psi with u(n) instead of (u(n) + u(n-1))/2
  int s2_local;    // f viscosity rate from the local dynamic viscosity
  int wet_bottom, wet_top;
  double kappa, beta, W, kBT, phib, inv_phib, lambda_s, M0, M_phi, M_psi, eta_phi, eta_psi;
  double rho_l, rho_g, mu_l, mu_g, gx, gy, uw_bottom, uw_top;
  double sig_cos;  // sigma_gl0 cos(theta0)
  double dsb;      // sigma_sg0 beta_sg - sigma_sl0 beta_sl
  double msb;      // sigma_sg0 beta_sg + sigma_sl0 beta_sl
  double fw0;      // (sigma_sg0 + sigma_sl0) / 2
  double beta_sg, beta_sl;
  // Remark 1: with sat_cap each solid-fluid tension sigma_sa0 (1 + beta_sa
  // ln(1 - psi)) is held at sigma_sa0 / 2 or more.
  int sat_cap;
  double sg0, sl0;
  double sf[5], sg[5], sh[5];
  double x0, y0, R0, a;
  double psi_b, init_scale;  // init_scale = 2 phi_b sqrt(1 - psi_b) / eps
  // Reference surfactant potential: mu_psi of the bulk of the initial state.
  // Each step's collision carries M_psi mu_ref in its psi source, so that the
  // deferred multiplier term is only M_psi (mubar - mu_ref): the same total in
  // exact arithmetic (a uniform source c adds w_i c to every population,
  // before or after the next gather), but populations of the size of the
  // sources' departure from equilibrium instead of M_psi mu_psi itself.
  double mu_ref;
  // With phi_hold the phi multiplier also returns sum h_phi(phi) to m_ref, its
  // value in the initial (or last loaded) state: lambda = S1/S2 + (m_ref - S4) /
  // (M_phi S2).  Off, lambda is eq15's S1/S2.
  int phi_hold;
  double m_ref;
  int init_kind;
  // Accuracy test of Sec. 4.1 (mms != 0): grid spacing and time step of the
  // unit square, the prescribed velocity in lattice units.
  int mms;
  double mms_dx, mms_dt, mms_ux, mms_uy;
};

// FP64 multiplier state kept on the device.  The fused step leaves the
// multiplier terms of its own sources (for psi: their part beyond M_psi mu_ref)
// out of the stored populations and applies them when the next step gathers
// them: cdef is the weight of that pending term (1.5 from R + dR/2, or 1 on a first step; 0 when nothing is
// pending, e.g. right after loading fields).
// Per-workgroup sums of a step: S1 = sum h'(phi) mu_phi, S2 = sum h'(phi)^2,
// S3 = sum mu_psi, S4 = sum h_phi(phi).
constexpr int kSums = 4;

struct DevScalars {
  double lambda_phi, mubar_psi, cdef;
};

// FP64 invariant accumulators per block: mass_psi, m_phi_h, sum_phi, area,
// kinetic, free_energy, umax (max), nonfinite, psi_out_of_range, cap_violations;
// the final vector adds contact width, cap height and apparent angle.
constexpr int kInvValues = 10;
constexpr int kInvOut = kInvValues + 3;

// Device buffers of one simulation (all planes N elements, x fastest).
struct DevState {
  int precision;           // LBM_FP64 / LBM_FP32 / LBM_FP16_SHIFTED
  void* pops[2];           // 27 planes each, storage type
  void* phipsi[2];         // 2 planes each (phi, psi), FP64; also the shift reference of g_0, h_0
  void* mu;                // 2 planes (mu_phi, mu_psi), FP64
  void* uhist[2];          // 6 planes each: ux, uy, vx, vy (velocity and advecting velocity) and the
                           // stored sources R_phi, R_psi (without their multiplier terms), compute type
  double* partials;        // reduction partials [kRedBlocks][3] (diagnostics; the batched step)
  double* step_partials[2];  // the single-handle step's sums [ntiles][3], by population parity cur
  double* inv_partials;    // invariant partials [kRedBlocks][kInvValues]
  double* inv_out;         // final invariants [kInvOut]
  double* contact;         // [nx] column heights + 2 x [nx] edge fractions (rows 0 and 1)
  DevScalars* scalars;     // [3]: pending multipliers (ping-pong by scur) and the diagnostic slot [2]
  double* field_buf;       // FP64 staging for fetch/load, [27][N]
  DevParams* dparams;      // device copy of the parameter block (read by the step kernel)
  int scur;                // scalars[scur] holds the multipliers pending on the stored populations
  int tile_rows;           // rows per workgroup segment of the step kernel (a multiple of 4)
  int cus = 256;           // compute units of the device (the step kernel's variant choice)
  int split_walls = 1;     // walled sweep: wall-free segments take the periodic form (same results)
  int cur;                 // index of the current population buffer
  int hcur;                // phi/psi and history buffer written by the next step
};

// One case of a batch, as the batched step kernels see it (device memory).
// The buffer parity selects, as cur = hcur = scur does for a single handle,
// which population, phi/psi, history and multiplier buffers are current.
struct BatchCase {
  DevParams p;
  void* pops[2];
  double* phipsi[2];
  void* uhist[2];
  DevScalars* scalars;     // [3], as DevState::scalars
  double* partials;
  int nstrips, seg_rows, ntiles, tile_begin;   // workgroups tile_begin .. tile_begin + ntiles of the launch
  int active;              // 0: retired, not stepped
  int parity;
  int have_hist;
  int pad;
  long long step;
};

constexpr int kBlock = 256;
constexpr int kRedBlocks = 1024;
constexpr int kStripW = 60;   // interior columns of a step workgroup (its 64 lanes add 2 halo columns a side)
constexpr int NWAVE = kBlock / 64;
constexpr int kMaxTiles = 1 << 22;   // partials of the fused step: [kMaxTiles][3] at most (grid <= 2^28 nodes at 64x16)

size_t storage_bytes(int precision);
size_t pops_bytes(int precision, size_t N);   // one population buffer (FP16: 27 FP16 planes + 2 FP32 rest planes)
int step_seg_rows(int nx, int ny, int precision);                 // rows per workgroup segment of the step kernel
// Kernel of a single handle's step (the values of LBM_KV_* in lbm.h): one-pass
// 4-row tiles with eight waves (grids of at most one such workgroup per CU),
// with four waves (up to kStepMinBlocks per CU), or the row sweep, built for
// one workgroup per CU or, on walled grids of more workgroups than CUs, for
// kStepMinBlocks.  Chosen from the workgroup count against DevState::cus.
enum { kVarSmall = 0, kVarMid = 1, kVarSweep = 2, kVarSweepPacked = 3 };
int step_variant(const DevParams& p, const DevState& s);
size_t step_blocks(int nx, int ny, int seg_rows);  // workgroups of the step kernel
size_t compute_bytes(int precision);
int set_init_error(int code, const std::string& msg);   // message for lbm_last_error(NULL); returns code

// Launchers (lbm_kernels.hip).  All enqueue on `stream` and return the HIP status.
hipError_t launch_init(const DevParams& p, DevState& s, hipStream_t stream);
hipError_t launch_load(const DevParams& p, DevState& s, int with_u, hipStream_t stream);
// Optional event pairs bracketing each kernel of a step (index by LBM_K_*).
struct StepTimer {
  hipEvent_t* ev = nullptr;  // [max_steps][LBM_N_KERNELS][2]
  int64_t max_steps = 0, used = 0;
};
// fuse: kFusePrev -- the step reduces the previous step's sums itself (that
// step ran with kFuseNext, i.e. without k_step_finish); only for consecutive
// steps with a history and at most kFuseTiles workgroups.
enum { kFusePrev = 1, kFuseNext = 2 };
constexpr int kFuseTiles = 1024;
// step: index of the step being taken (the accuracy test's source time).
hipError_t launch_step(const DevParams& p, DevState& s, int have_hist, hipStream_t stream, StepTimer* timer = nullptr,
                       int fuse = 0, int64_t step = 0);
hipError_t launch_step_batch(int precision, bool walls, const BatchCase* d_cases, const int* d_wg_case, int nwg, int count,
                             hipStream_t stream, StepTimer* timer = nullptr);
hipError_t launch_macro(const DevParams& p, DevState& s, hipStream_t stream);  // phi/psi, mu, multipliers of the current state
hipError_t launch_invariants(const DevParams& p, DevState& s, hipStream_t stream);
hipError_t launch_fetch(const DevParams& p, DevState& s, uint32_t mask, hipStream_t stream);
hipError_t launch_fetch_pops(const DevParams& p, DevState& s, hipStream_t stream);

// Access of the batch layer to the handles it is built from (lbm_capi.cpp).
struct HandleView {
  const DevParams* dp;
  DevState* ds;
  int* have_hist;
  int64_t* step;
  bool* faulted;
};
HandleView handle_view(lbm_handle* h);
int handle_reinit(lbm_handle* h);   // back to the initial fields of its parameters, step 0

}  // namespace lbm
