// lbm_capi.cpp -- C ABI of the gfx950 lattice Boltzmann library (declared in
// include/lbm.h): parameter validation and derivation, device memory layout,
// stream ordering, error state, checkpoint blobs.
#include "../../include/lbm.h"
#include "lbm_internal.h"

#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <string>

namespace {

constexpr double kPi = 3.14159265358979323846;
constexpr uint64_t kStateMagic = 0x4c424d5354415432ull;  // "LBMSTAT2"

thread_local std::string g_init_error = "no error";

struct StateHeader {
  uint64_t magic;
  int32_t precision, nx, ny, have_hist;
  int64_t step;
  uint64_t params_hash;
  double pending[3];  // multipliers pending on the stored populations (lambda, mubar, weight)
  double m_ref;       // phi_hold's reference sum h_phi (of the initial or last loaded fields)
};

uint64_t hash_bytes(const void* data, size_t n) {  // FNV-1a
  const unsigned char* b = (const unsigned char*)data;
  uint64_t h = 1469598103934665603ull;
  for (size_t k = 0; k < n; ++k) { h ^= b[k]; h *= 1099511628211ull; }
  return h;
}

size_t align_up(size_t v) { return (v + 255) & ~size_t(255); }

struct Layout {
  size_t pops, phipsi, mu, uhist, partials, step_partials, inv_partials, inv_out, contact, scalars, dparams, field_buf, total;
};

Layout make_layout(const lbm_params& p) {
  const size_t N = (size_t)p.nx * (size_t)p.ny;
  const size_t cb = lbm::compute_bytes(p.precision);
  Layout L{};
  size_t off = 0;
  auto take = [&](size_t bytes) { size_t o = off; off += align_up(bytes); return o; };
  L.pops = take(2 * lbm::pops_bytes(p.precision, N));
  L.phipsi = take(2 * 2 * N * sizeof(double));  // phi, psi: FP64 in every precision
  L.mu = take(2 * N * sizeof(double));
  L.uhist = take(2 * 6 * N * cb);  // u, v (advecting), R_phi, R_psi history, ping-pong
  const size_t ntile = lbm::step_blocks(p.nx, p.ny, 4);  // the most workgroups any segment height gives
  L.partials = take((ntile > (size_t)lbm::kRedBlocks ? ntile : (size_t)lbm::kRedBlocks) * lbm::kSums * sizeof(double));
  L.step_partials = take(2 * ntile * lbm::kSums * sizeof(double));
  L.inv_partials = take(lbm::kRedBlocks * lbm::kInvValues * sizeof(double));
  L.inv_out = take(lbm::kInvOut * sizeof(double));
  L.contact = take(3 * (size_t)p.nx * sizeof(double));
  L.scalars = take(3 * sizeof(lbm::DevScalars));
  L.dparams = take(sizeof(lbm::DevParams));
  L.field_buf = take(27 * N * sizeof(double));
  L.total = off;
  return L;
}

bool in_open(double v, double lo, double hi) { return v > lo && v < hi; }

// Validation and derivation of the lattice constants (Sec. 2 and Sec. 3).
// Returns an empty string on success, else the reason.
std::string derive(const lbm_params& p, lbm::DevParams& d, double* derived) {
  if (p.abi_version != LBM_ABI_VERSION) return "abi_version mismatch";
  if (p.nx < 3 || p.ny < 3) return "nx and ny must be >= 3";
  if ((double)p.nx * (double)p.ny > 2.0e9) return "grid too large for 32-bit node indices";
  auto bc_ok = [](int b) { return b >= LBM_BC_PERIODIC && b <= LBM_BC_FREESLIP; };
  if (!bc_ok(p.bc_bottom) || !bc_ok(p.bc_top)) return "unknown boundary kind";
  if ((p.bc_bottom == LBM_BC_PERIODIC) != (p.bc_top == LBM_BC_PERIODIC)) return "periodic y needs both walls periodic";
  if (p.precision != LBM_FP64 && p.precision != LBM_FP32 && p.precision != LBM_FP16_SHIFTED) return "unknown precision";
  if (p.constraint_phi != LBM_CONSTRAINT_NONLINEAR && p.constraint_phi != LBM_CONSTRAINT_LINEAR) return "unknown constraint";
  if (p.init_kind < LBM_INIT_DROP || p.init_kind > LBM_INIT_BUBBLE) return "unknown init kind";
  if (p.adv_raw != 0 && p.adv_raw != 1) return "adv_raw must be 0 or 1";
  if (p.phi_hold != 0 && p.phi_hold != 1) return "phi_hold must be 0 or 1";
  if (p.sat_cap != 0 && p.sat_cap != 1) return "sat_cap must be 0 or 1";
  if (p.tile_rows < 0 || p.tile_rows % 4 != 0 || p.tile_rows > 4096) return "tile_rows must be 0 or a multiple of 4 up to 4096";
  if (!(p.sigma_gl0 > 0.0) || !(p.eps > 0.0)) return "sigma_gl0 and eps must be > 0";
  if (!(p.M_phi >= 0.0) || !(p.M_psi >= 0.0)) return "mobilities must be >= 0";
  if (!(p.psi_b >= 0.0 && p.psi_b < 1.0)) return "psi_b must lie in [0,1)";
  if (!(p.rho_l > 0.0 && p.rho_g > 0.0 && p.mu_l > 0.0 && p.mu_g > 0.0)) return "densities and viscosities must be > 0";
  const bool wet_b = p.bc_bottom == LBM_BC_WALL_WET, wet_t = p.bc_top == LBM_BC_WALL_WET;
  if ((wet_b || wet_t) && !in_open(p.theta0_deg, 0.0, 180.0)) return "theta0 must lie in (0,180) on a wetting wall";
  const double* rates[3] = {p.s_f, p.s_g, p.s_h};
  for (int l = 0; l < 3; ++l)
    for (int k = 0; k < 5; ++k)
      if (!(rates[l][k] < 2.0) || std::isnan(rates[l][k])) return "relaxation rates must lie in (0,2)";

  if (!(p.mms_dx >= 0.0)) return "mms_dx must be >= 0";
  if (p.mms_dx > 0.0) {
    if (p.bc_bottom != LBM_BC_PERIODIC) return "the accuracy test needs periodic boundaries";
    if (std::fabs(p.nx * p.mms_dx - 1.0) > 1e-9 || std::fabs(p.ny * p.mms_dx - 1.0) > 1e-9)
      return "the accuracy test runs on the unit square: nx mms_dx = ny mms_dx = 1";
    if (p.precision != LBM_FP64) return "the accuracy test runs in FP64 storage";
    if (p.constraint_phi != LBM_CONSTRAINT_LINEAR) return "the accuracy test uses the linear constraint";
    if (!(p.psi_b > 0.0)) return "the accuracy test needs the surfactant (psi_b > 0)";
  }

  std::memset(&d, 0, sizeof(d));
  d.nx = p.nx; d.ny = p.ny; d.N = p.nx * p.ny;
  if (p.mms_dx > 0.0) {
    d.mms = 1;
    d.mms_dx = p.mms_dx;
    d.mms_dt = p.mms_dx * p.mms_dx / 0.15;
    d.mms_ux = 0.05 * d.mms_dt / p.mms_dx;
    d.mms_uy = -0.03 * d.mms_dt / p.mms_dx;
  }
  d.periodic_y = p.bc_bottom == LBM_BC_PERIODIC;
  d.bc_bottom = p.bc_bottom; d.bc_top = p.bc_top;
  d.wet_bottom = wet_b; d.wet_top = wet_t;
  d.surf = p.psi_b > 0.0;
  d.linear = p.constraint_phi == LBM_CONSTRAINT_LINEAR;
  d.adv_raw = p.adv_raw;
  d.phi_hold = p.phi_hold;
  // interface coefficients of the Ginzburg-Landau energy
  const double kappa = 0.375 * p.eps * p.sigma_gl0, beta = 0.75 * p.sigma_gl0 / p.eps;
  const double W = p.W > 0.0 ? p.W : 4.0 * beta / (p.Ex > 0.0 ? p.Ex : 0.5);
  const double kBT = p.kBT > 0.0 ? p.kBT : 4.0 * beta * (p.Pi > 0.0 ? p.Pi : 1.35);
  double phib = 1.0;
  if (p.phi_b > 0.0) phib = p.phi_b;
  else if (d.surf) {
    const double q = 1.0 - W * p.psi_b / (4.0 * beta * (1.0 - p.psi_b));
    if (!(q > 0.0)) return "bulk surfactant too large: phi_b^2 <= 0";
    phib = std::sqrt(q);
  }
  double sg0 = p.sigma_sg0, sl0 = p.sigma_sl0;
  if (!(sg0 >= 0.0 && sl0 >= 0.0)) {
    const double diff = p.sigma_gl0 * std::cos(p.theta0_deg * kPi / 180.0), sum = 16.0 * p.sigma_gl0 / 15.0;
    sg0 = 0.5 * (sum + diff);
    sl0 = 0.5 * (sum - diff);
  }
  const double lambda_s = p.lambda_s >= 0.0 ? p.lambda_s : ((wet_b || wet_t) ? 0.5 * kappa : 0.0);
  if ((wet_b || wet_t) && d.surf && lambda_s == 0.0 && (p.beta_sg != 0.0 || p.beta_sl != 0.0))
    return "lambda_s = 0 cannot carry the solid-adsorption boundary condition";
  const double M0 = p.M0 >= 0.0 ? p.M0 : (lambda_s > 0.0 ? 0.0 : p.M_phi * kappa);
  auto rate = [](double v) { return v > 0.0 ? v : 1.0; };
  const double s1g = rate(p.s_g[1]), s1h = rate(p.s_h[1]);
  const double eta_phi = p.eta_phi > 0.0 ? p.eta_phi : p.M_phi * kappa / ((1.0 / s1g - 0.5) / 3.0);
  const double eta_psi = p.eta_psi > 0.0 ? p.eta_psi : (p.M_psi * lambda_s + M0) / ((1.0 / s1h - 0.5) / 3.0);
  d.kappa = kappa; d.beta = beta; d.W = W; d.kBT = kBT; d.phib = phib; d.inv_phib = 1.0 / phib;
  d.lambda_s = lambda_s; d.M0 = M0; d.M_phi = p.M_phi; d.M_psi = p.M_psi; d.eta_phi = eta_phi; d.eta_psi = eta_psi;
  d.rho_l = p.rho_l; d.rho_g = p.rho_g; d.mu_l = p.mu_l; d.mu_g = p.mu_g; d.gx = p.gx; d.gy = p.gy;
  d.uw_bottom = p.u_wall_bottom; d.uw_top = p.u_wall_top;
  d.sig_cos = p.sigma_gl0 * std::cos(p.theta0_deg * kPi / 180.0);
  d.dsb = sg0 * p.beta_sg - sl0 * p.beta_sl;
  d.msb = sg0 * p.beta_sg + sl0 * p.beta_sl;
  d.fw0 = 0.5 * (sg0 + sl0);
  d.beta_sg = p.beta_sg; d.beta_sl = p.beta_sl;
  d.sat_cap = p.sat_cap; d.sg0 = sg0; d.sl0 = sl0;
  for (int k = 0; k < 5; ++k) { d.sf[k] = rate(p.s_f[k]); d.sg[k] = rate(p.s_g[k]); d.sh[k] = rate(p.s_h[k]); }
  d.s2_local = !(p.s_f[2] > 0.0);
  d.x0 = p.x0; d.y0 = p.y0; d.R0 = p.R0; d.a = p.a;
  d.psi_b = p.psi_b;
  d.mu_ref = d.surf ? kBT * std::log(p.psi_b / (1.0 - p.psi_b)) - beta * (1.0 - phib * phib) * (1.0 - phib * phib) + 0.5 * W * phib * phib : 0.0;
  d.init_scale = 2.0 * phib * (d.surf ? std::sqrt(1.0 - p.psi_b) : 1.0) / p.eps;
  d.init_kind = p.init_kind;
  const double psi_c = std::exp(-(beta + 0.5 * W) / kBT);
  const double out[LBM_N_DERIVED] = {kappa, beta, W, kBT, phib, sg0, sl0, lambda_s, M0, eta_phi, eta_psi, psi_c};
  std::memcpy(derived, out, sizeof(out));
  return "";
}

}  // namespace

struct lbm_handle {
  lbm_params prm;
  lbm::DevParams dp;
  lbm::DevState ds;
  Layout lay;
  hipStream_t stream = nullptr;
  bool own_stream = false;
  void* buf = nullptr;
  bool own_buf = false;
  int64_t step = 0;
  int have_hist = 0;
  bool faulted = false;
  double derived[LBM_N_DERIVED];
  lbm::StepTimer timer;
  // graph[k]: 2^(k+1) steps captured from buffer parity graph_parity[k] (k < kGraphKinds)
  hipGraphExec_t graph[5] = {nullptr, nullptr, nullptr, nullptr, nullptr};
  int graph_parity[5] = {0, 0, 0, 0, 0};
  std::string err = "no error";
};

namespace {

int fail(lbm_handle* h, int code, const std::string& msg) {
  if (h) h->err = msg;
  else g_init_error = msg;
  return code;
}
int hip_fail(lbm_handle* h, hipError_t e, const char* where) {
  return fail(h, LBM_E_DEVICE, std::string(where) + ": " + hipGetErrorString(e));
}
#define HIP_OR_FAIL(h, expr, where)               \
  do {                                            \
    hipError_t e_ = (expr);                       \
    if (e_ != hipSuccess) return hip_fail(h, e_, where); \
  } while (0)

void carve(lbm_handle* h) {
  char* b = (char*)h->buf;
  const Layout& L = h->lay;
  const size_t N = (size_t)h->dp.N;
  const size_t cb = lbm::compute_bytes(h->prm.precision);
  lbm::DevState& s = h->ds;
  s.precision = h->prm.precision;
  s.pops[0] = b + L.pops;
  s.pops[1] = b + L.pops + lbm::pops_bytes(h->prm.precision, N);
  s.phipsi[0] = b + L.phipsi;
  s.phipsi[1] = b + L.phipsi + 2 * N * sizeof(double);
  s.mu = b + L.mu;
  s.uhist[0] = b + L.uhist;
  s.uhist[1] = b + L.uhist + 6 * N * cb;
  s.partials = (double*)(b + L.partials);
  {
    const size_t ntile = lbm::step_blocks(h->dp.nx, h->dp.ny, 4);
    s.step_partials[0] = (double*)(b + L.step_partials);
    s.step_partials[1] = s.step_partials[0] + lbm::kSums * ntile;
  }
  s.inv_partials = (double*)(b + L.inv_partials);
  s.inv_out = (double*)(b + L.inv_out);
  s.contact = (double*)(b + L.contact);
  s.scalars = (lbm::DevScalars*)(b + L.scalars);
  s.dparams = (lbm::DevParams*)(b + L.dparams);
  s.scur = 0;
  s.tile_rows = h->prm.tile_rows ? h->prm.tile_rows : lbm::step_seg_rows(h->dp.nx, h->dp.ny, h->prm.precision);
  s.field_buf = (double*)(b + L.field_buf);
  s.cur = 0;
  s.hcur = 0;
}

int check_device(std::string& why, int* cus = nullptr) {
  int count = 0;
  if (hipGetDeviceCount(&count) != hipSuccess || count <= 0) { why = "no HIP device"; return LBM_E_DEVICE; }
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) { why = "hipGetDevice failed"; return LBM_E_DEVICE; }
  hipDeviceProp_t prop;
  if (hipGetDeviceProperties(&prop, dev) != hipSuccess) { why = "hipGetDeviceProperties failed"; return LBM_E_DEVICE; }
  if (std::strncmp(prop.gcnArchName, "gfx950", 6) != 0) { why = std::string("device is ") + prop.gcnArchName + ", not gfx950"; return LBM_E_DEVICE; }
  if (cus) *cus = prop.multiProcessorCount > 0 ? prop.multiProcessorCount : 256;
  return LBM_OK;
}

}  // namespace

extern "C" {

int lbm_required_bytes(const lbm_params* p, size_t* bytes) {
  if (!p || !bytes) return fail(nullptr, LBM_E_ARG, "null argument");
  lbm::DevParams d;
  double derived[LBM_N_DERIVED];
  std::string why = derive(*p, d, derived);
  if (!why.empty()) return fail(nullptr, LBM_E_ARG, why);
  *bytes = make_layout(*p).total;
  return LBM_OK;
}

// With phi_hold: m_ref := sum h_phi(phi) of the state the handle holds now (the
// initial or a loaded one), from the invariant sums, written to the device copy
// of the parameters.  Synchronises the handle's stream.
static hipError_t set_m_ref(lbm_handle* h) {
  if (!h->dp.phi_hold) return hipSuccess;
  hipError_t e = lbm::launch_invariants(h->dp, h->ds, h->stream);
  double v[lbm::kInvOut] = {0};
  if (e == hipSuccess) e = hipMemcpyAsync(v, h->ds.inv_out, sizeof(v), hipMemcpyDeviceToHost, h->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(h->stream);
  if (e != hipSuccess) return e;
  h->dp.m_ref = h->dp.linear ? v[2] : v[1];   // sum phi, or sum of 1/2 + g(phi)
  e = hipMemcpyAsync(h->ds.dparams, &h->dp, sizeof(h->dp), hipMemcpyHostToDevice, h->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(h->stream);
  return e;
}

int lbm_init(const lbm_params* p, void* dev_buf, size_t buf_bytes, void* hip_stream, lbm_handle** out) {
  if (!out) return fail(nullptr, LBM_E_ARG, "null output handle");
  *out = nullptr;
  if (!p) return fail(nullptr, LBM_E_ARG, "null parameters");
  lbm_handle* h = new lbm_handle();
  h->prm = *p;
  std::string why = derive(*p, h->dp, h->derived);
  if (!why.empty()) { delete h; return fail(nullptr, LBM_E_ARG, why); }
  int cus = 256;
  int dc = check_device(why, &cus);
  if (dc != LBM_OK) { delete h; return fail(nullptr, dc, why); }
  h->lay = make_layout(*p);
  if (dev_buf) {
    if (buf_bytes < h->lay.total) { delete h; return fail(nullptr, LBM_E_ARG, "dev_buf smaller than lbm_required_bytes"); }
    if (((uintptr_t)dev_buf & 255) != 0) { delete h; return fail(nullptr, LBM_E_ARG, "dev_buf must be 256-byte aligned"); }
    h->buf = dev_buf;
  } else {
    if (hipMalloc(&h->buf, h->lay.total) != hipSuccess) { delete h; return fail(nullptr, LBM_E_OOM, "hipMalloc of the state failed"); }
    h->own_buf = true;
  }
  if (hip_stream) h->stream = (hipStream_t)hip_stream;
  else {
    if (hipStreamCreate(&h->stream) != hipSuccess) {
      if (h->own_buf) (void)hipFree(h->buf);
      delete h;
      return fail(nullptr, LBM_E_DEVICE, "hipStreamCreate failed");
    }
    h->own_stream = true;
  }
  carve(h);
  h->ds.cus = cus;
  // Override of the CU count the step kernel's variant is chosen against (a
  // test aid: every variant then runs on one device); results do not change.
  if (const char* ov = std::getenv("LBM_KERNEL_CUS")) {
    const long v = std::strtol(ov, nullptr, 10);
    if (v >= 1 && v <= 65536) h->ds.cus = (int)v;
  }
  // LBM_STEP_SPLIT_WALLS=0 runs every segment of a walled grid in the walled
  // form of the sweep (a test aid: the split gives the same results).
  if (const char* ov = std::getenv("LBM_STEP_SPLIT_WALLS")) h->ds.split_walls = std::strcmp(ov, "0") != 0;
  hipError_t e = hipMemcpyAsync(h->ds.dparams, &h->dp, sizeof(h->dp), hipMemcpyHostToDevice, h->stream);
  if (e == hipSuccess) e = lbm::launch_init(h->dp, h->ds, h->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(h->stream);
  if (e == hipSuccess) e = set_m_ref(h);
  if (e != hipSuccess) {
    std::string msg = std::string("initialisation kernels: ") + hipGetErrorString(e);
    lbm_destroy(h);
    return fail(nullptr, LBM_E_DEVICE, msg);
  }
  *out = h;
  return LBM_OK;
}

// Runs of steps are replayed from captured HIP graphs of 2, 4, 8, 16 or 32
// steps (even counts, so the ping-pong buffers end where they started): one
// graph launch instead of two kernel launches per step.  A run is split into
// the longest such pieces; steps while kernel timing is on, the first step
// (no history yet) and an odd last step run eagerly.
constexpr int kGraphKinds = 5;

int capture_graph(lbm_handle* h, int kind) {
  const int64_t kGraphSteps = int64_t(2) << kind;
  lbm::DevState s = h->ds;  // the capture advances a copy's buffer parity
  hipGraph_t g = nullptr;
  HIP_OR_FAIL(h, hipStreamBeginCapture(h->stream, hipStreamCaptureModeThreadLocal), "begin graph capture");
  hipError_t e = hipSuccess;
  // On grids of few workgroups the captured steps after the first reduce the
  // previous step's multiplier sums themselves: one k_step_finish per graph
  // (after the last step) instead of one per step.
  const bool fuse = lbm::step_blocks(h->dp.nx, h->dp.ny, s.tile_rows) <= (size_t)lbm::kFuseTiles;
  for (int64_t k = 0; k < kGraphSteps && e == hipSuccess; ++k) {
    const int f = fuse ? ((k > 0 ? lbm::kFusePrev : 0) | (k + 1 < kGraphSteps ? lbm::kFuseNext : 0)) : 0;
    e = lbm::launch_step(h->dp, s, 1, h->stream, nullptr, f);
  }
  const hipError_t e_end = hipStreamEndCapture(h->stream, &g);
  if (e == hipSuccess) e = e_end;
  if (e == hipSuccess) e = hipGraphInstantiate(&h->graph[kind], g, nullptr, nullptr, 0);
  if (g) (void)hipGraphDestroy(g);
  if (e != hipSuccess) {
    h->graph[kind] = nullptr;
    return hip_fail(h, e, "graph capture of the step kernels");
  }
  h->graph_parity[kind] = h->ds.cur;
  return LBM_OK;
}

int lbm_step(lbm_handle* h, int64_t n) {
  if (!h) return fail(nullptr, LBM_E_ARG, "null handle");
  if (n < 0) return fail(h, LBM_E_ARG, "negative step count");
  if (h->faulted) return fail(h, LBM_E_STATE, "state holds non-finite or out-of-range values; load a state or fields first");
  int64_t k = 0;
  while (k < n) {
    const bool timing = h->timer.ev && h->timer.used < h->timer.max_steps;
    int kind = kGraphKinds - 1;
    while (kind >= 0 && n - k < (int64_t(2) << kind)) --kind;
    if (!timing && !h->dp.mms && kind >= 0 && h->have_hist && h->ds.cur == h->ds.hcur && h->ds.cur == h->ds.scur &&
        (!h->graph[kind] || h->ds.cur == h->graph_parity[kind])) {
      if (!h->graph[kind]) {
        const int rc = capture_graph(h, kind);
        if (rc) return rc;
      }
      HIP_OR_FAIL(h, hipGraphLaunch(h->graph[kind], h->stream), "graph launch");
      h->step += int64_t(2) << kind;
      k += int64_t(2) << kind;
      continue;
    }
    HIP_OR_FAIL(h, lbm::launch_step(h->dp, h->ds, h->have_hist, h->stream, &h->timer, 0, h->step), "step kernels");
    h->have_hist = 1;
    h->step += 1;
    k += 1;
  }
  return LBM_OK;
}

int lbm_reduce_invariants(lbm_handle* h, lbm_invariants* out) {
  if (!h || !out) return fail(h, LBM_E_ARG, "null argument");
  HIP_OR_FAIL(h, lbm::launch_invariants(h->dp, h->ds, h->stream), "invariant kernels");
  double v[lbm::kInvOut] = {0};
  lbm::DevScalars sc;
  HIP_OR_FAIL(h, hipMemcpyAsync(v, h->ds.inv_out, sizeof(v), hipMemcpyDeviceToHost, h->stream), "copy invariants");
  HIP_OR_FAIL(h, hipMemcpyAsync(&sc, h->ds.scalars + 2, sizeof(sc), hipMemcpyDeviceToHost, h->stream), "copy multipliers");
  HIP_OR_FAIL(h, hipStreamSynchronize(h->stream), "synchronise");
  std::memset(out, 0, sizeof(*out));
  out->step = h->step;
  out->mass_psi = v[0];
  out->m_phi_h = v[1];
  out->sum_phi = v[2];
  out->area_phi_pos = v[3];
  out->kinetic = v[4];
  out->free_energy = v[5];
  out->umax = v[6];
  out->nonfinite = (int64_t)v[7];
  out->psi_out_of_range = (int64_t)v[8];
  out->cap_violations = (int64_t)v[9];
  out->lambda_phi = sc.lambda_phi;
  out->mubar_psi = sc.mubar_psi;
  if (!h->dp.periodic_y) {
    out->contact_width = v[10];
    out->cap_height = v[11];
    out->theta_app_deg = v[12];
  }
  // psi outside (0,1) is the cause when both are present (ln(psi/(1-psi)) is then not finite)
  if (out->psi_out_of_range > 0) {
    h->faulted = true;
    return fail(h, LBM_E_RANGE, "psi left (0,1)");
  }
  if (out->nonfinite > 0) {
    h->faulted = true;
    return fail(h, LBM_E_NONFINITE, "non-finite values in the fields");
  }
  return LBM_OK;
}

int lbm_fetch_fields(lbm_handle* h, uint32_t mask, double* host, size_t n_doubles) {
  if (!h || !host) return fail(h, LBM_E_ARG, "null argument");
  if (mask == 0 || (mask & ~0xFFu)) return fail(h, LBM_E_ARG, "bad field mask");
  const size_t N = (size_t)h->dp.N;
  size_t planes = (size_t)__builtin_popcount(mask);
  if (n_doubles < planes * N) return fail(h, LBM_E_ARG, "host buffer too small");
  HIP_OR_FAIL(h, lbm::launch_fetch(h->dp, h->ds, mask, h->stream), "field kernels");
  size_t k = 0;
  for (int b = 0; b < 8; ++b) {
    if (!(mask & (1u << b))) continue;
    HIP_OR_FAIL(h, hipMemcpyAsync(host + k * N, h->ds.field_buf + (size_t)b * N, N * sizeof(double), hipMemcpyDeviceToHost, h->stream), "copy fields");
    ++k;
  }
  HIP_OR_FAIL(h, hipStreamSynchronize(h->stream), "synchronise");
  return LBM_OK;
}

int lbm_load_fields(lbm_handle* h, uint32_t mask, const double* host, size_t n_doubles) {
  if (!h || !host) return fail(h, LBM_E_ARG, "null argument");
  const uint32_t need = LBM_F_PHI | LBM_F_PSI, vel = LBM_F_UX | LBM_F_UY;
  if ((mask & need) != need || (mask & ~(need | vel)) || ((mask & vel) && (mask & vel) != vel))
    return fail(h, LBM_E_ARG, "mask must be PHI|PSI, optionally with UX|UY");
  const size_t N = (size_t)h->dp.N;
  const size_t planes = (size_t)__builtin_popcount(mask);
  if (n_doubles < planes * N) return fail(h, LBM_E_ARG, "host buffer too small");
  for (size_t k = 0; k < planes; ++k)
    HIP_OR_FAIL(h, hipMemcpyAsync(h->ds.field_buf + k * N, host + k * N, N * sizeof(double), hipMemcpyHostToDevice, h->stream), "copy fields");
  HIP_OR_FAIL(h, lbm::launch_load(h->dp, h->ds, (mask & vel) ? 1 : 0, h->stream), "load kernel");
  HIP_OR_FAIL(h, hipStreamSynchronize(h->stream), "synchronise");
  HIP_OR_FAIL(h, set_m_ref(h), "constraint reference");
  h->have_hist = 0;
  h->faulted = false;
  return LBM_OK;
}

int lbm_state_bytes(lbm_handle* h, size_t* bytes) {
  if (!h || !bytes) return fail(h, LBM_E_ARG, "null argument");
  const size_t N = (size_t)h->dp.N;
  const size_t cb = lbm::compute_bytes(h->prm.precision);
  *bytes = sizeof(StateHeader) + lbm::pops_bytes(h->prm.precision, N) + 2 * N * sizeof(double) + 6 * N * cb;
  return LBM_OK;
}

int lbm_save_state(lbm_handle* h, void* host, size_t bytes) {
  size_t need = 0;
  int rc = lbm_state_bytes(h, &need);
  if (rc) return rc;
  if (!host || bytes < need) return fail(h, LBM_E_ARG, "state buffer too small");
  const size_t N = (size_t)h->dp.N;
  const size_t cb = lbm::compute_bytes(h->prm.precision);
  StateHeader hd{kStateMagic, h->prm.precision, h->prm.nx, h->prm.ny, h->have_hist, h->step,
                 hash_bytes(&h->prm, sizeof(h->prm)), {0, 0, 0}, h->dp.m_ref};
  HIP_OR_FAIL(h, hipMemcpyAsync(hd.pending, h->ds.scalars + h->ds.scur, sizeof(hd.pending), hipMemcpyDeviceToHost, h->stream), "save");
  HIP_OR_FAIL(h, hipStreamSynchronize(h->stream), "synchronise");
  char* o = (char*)host;
  std::memcpy(o, &hd, sizeof(hd));
  o += sizeof(hd);
  const int hp = h->ds.hcur ^ 1;  // history written by the last step
  HIP_OR_FAIL(h, hipMemcpyAsync(o, h->ds.pops[h->ds.cur], lbm::pops_bytes(h->prm.precision, N), hipMemcpyDeviceToHost, h->stream), "save");
  o += lbm::pops_bytes(h->prm.precision, N);
  HIP_OR_FAIL(h, hipMemcpyAsync(o, h->ds.phipsi[hp], 2 * N * sizeof(double), hipMemcpyDeviceToHost, h->stream), "save");
  o += 2 * N * sizeof(double);
  HIP_OR_FAIL(h, hipMemcpyAsync(o, h->ds.uhist[hp], 6 * N * cb, hipMemcpyDeviceToHost, h->stream), "save");
  HIP_OR_FAIL(h, hipStreamSynchronize(h->stream), "synchronise");
  return LBM_OK;
}

int lbm_load_state(lbm_handle* h, const void* host, size_t bytes) {
  size_t need = 0;
  int rc = lbm_state_bytes(h, &need);
  if (rc) return rc;
  if (!host || bytes < need) return fail(h, LBM_E_ARG, "state buffer too small");
  StateHeader hd;
  std::memcpy(&hd, host, sizeof(hd));
  if (hd.magic != kStateMagic || hd.precision != h->prm.precision || hd.nx != h->prm.nx || hd.ny != h->prm.ny ||
      hd.params_hash != hash_bytes(&h->prm, sizeof(h->prm)))
    return fail(h, LBM_E_ARG, "state blob does not match this handle's parameters");
  const size_t N = (size_t)h->dp.N;
  const size_t cb = lbm::compute_bytes(h->prm.precision);
  const char* o = (const char*)host + sizeof(hd);
  const int hp = h->ds.hcur ^ 1;
  HIP_OR_FAIL(h, hipMemcpyAsync(h->ds.pops[h->ds.cur], o, lbm::pops_bytes(h->prm.precision, N), hipMemcpyHostToDevice, h->stream), "load");
  o += lbm::pops_bytes(h->prm.precision, N);
  HIP_OR_FAIL(h, hipMemcpyAsync(h->ds.phipsi[hp], o, 2 * N * sizeof(double), hipMemcpyHostToDevice, h->stream), "load");
  o += 2 * N * sizeof(double);
  HIP_OR_FAIL(h, hipMemcpyAsync(h->ds.uhist[hp], o, 6 * N * cb, hipMemcpyHostToDevice, h->stream), "load");
  HIP_OR_FAIL(h, hipMemcpyAsync(h->ds.scalars + h->ds.scur, hd.pending, sizeof(hd.pending), hipMemcpyHostToDevice, h->stream), "load");
  h->dp.m_ref = hd.m_ref;
  HIP_OR_FAIL(h, hipMemcpyAsync(h->ds.dparams, &h->dp, sizeof(h->dp), hipMemcpyHostToDevice, h->stream), "load");
  HIP_OR_FAIL(h, hipStreamSynchronize(h->stream), "synchronise");
  h->have_hist = hd.have_hist;
  h->step = hd.step;
  h->faulted = false;
  return LBM_OK;
}

int lbm_derived(lbm_handle* h, double* out) {
  if (!h || !out) return fail(h, LBM_E_ARG, "null argument");
  std::memcpy(out, h->derived, sizeof(h->derived));
  return LBM_OK;
}

int lbm_fetch_populations(lbm_handle* h, double* host, size_t n_doubles) {
  if (!h || !host) return fail(h, LBM_E_ARG, "null argument");
  const size_t N = (size_t)h->dp.N;
  if (n_doubles < 27 * N) return fail(h, LBM_E_ARG, "host buffer too small");
  HIP_OR_FAIL(h, lbm::launch_fetch_pops(h->dp, h->ds, h->stream), "population kernel");
  HIP_OR_FAIL(h, hipMemcpyAsync(host, h->ds.field_buf, 27 * N * sizeof(double), hipMemcpyDeviceToHost, h->stream), "copy");
  HIP_OR_FAIL(h, hipStreamSynchronize(h->stream), "synchronise");
  return LBM_OK;
}

namespace {
void release_timer(lbm_handle* h) {
  if (!h->timer.ev) return;
  for (int64_t k = 0; k < h->timer.max_steps * 2 * LBM_N_KERNELS; ++k) (void)hipEventDestroy(h->timer.ev[k]);
  delete[] h->timer.ev;
  h->timer = lbm::StepTimer();
}
}  // namespace

int lbm_timing_begin(lbm_handle* h, int64_t max_steps) {
  if (!h) return fail(nullptr, LBM_E_ARG, "null handle");
  if (max_steps <= 0 || max_steps > 1000000) return fail(h, LBM_E_ARG, "max_steps must lie in [1, 1e6]");
  release_timer(h);
  const int64_t per_step = 2 * LBM_N_KERNELS;
  h->timer.ev = new hipEvent_t[max_steps * per_step];
  for (int64_t k = 0; k < max_steps * per_step; ++k) {
    hipError_t e = hipEventCreate(&h->timer.ev[k]);
    if (e != hipSuccess) {
      for (int64_t j = 0; j < k; ++j) (void)hipEventDestroy(h->timer.ev[j]);
      delete[] h->timer.ev;
      h->timer = lbm::StepTimer();
      return hip_fail(h, e, "hipEventCreate");
    }
  }
  h->timer.max_steps = max_steps;
  h->timer.used = 0;
  return LBM_OK;
}

int lbm_timing_end(lbm_handle* h, double* ms, int64_t* launches) {
  if (!h || !ms || !launches) return fail(h, LBM_E_ARG, "null argument");
  if (!h->timer.ev) return fail(h, LBM_E_STATE, "lbm_timing_begin was not called");
  HIP_OR_FAIL(h, hipStreamSynchronize(h->stream), "synchronise");
  for (int k = 0; k < LBM_N_KERNELS; ++k) { ms[k] = 0.0; launches[k] = 0; }
  for (int64_t s = 0; s < h->timer.used; ++s)
    for (int k = 0; k < LBM_N_KERNELS; ++k) {
      float t = 0.f;
      hipError_t e = hipEventElapsedTime(&t, h->timer.ev[(s * LBM_N_KERNELS + k) * 2], h->timer.ev[(s * LBM_N_KERNELS + k) * 2 + 1]);
      if (e != hipSuccess) { release_timer(h); return hip_fail(h, e, "hipEventElapsedTime"); }
      ms[k] += t;
      launches[k] += 1;
    }
  release_timer(h);
  return LBM_OK;
}

int lbm_bytes_per_node_step(lbm_handle* h, double* bytes) {
  if (!h || !bytes) return fail(h, LBM_E_ARG, "null argument");
  const double sb = (double)lbm::storage_bytes(h->prm.precision), cb = (double)lbm::compute_bytes(h->prm.precision);
  const double planes_s = h->dp.surf ? 27.0 : 18.0;     // h lattice idle without surfactant
  const double fp64_planes = h->dp.surf ? 2.0 : 1.0;    // phi (and psi) reference planes
  // FP16 storage keeps the rest populations of g and h in FP32 planes
  const double pops = h->prm.precision == LBM_FP16_SHIFTED ? (planes_s - fp64_planes) * sb + fp64_planes * 4.0 : planes_s * sb;
  // read + write of: populations, FP64 phi/psi, velocity/advecting-velocity history (4), source history (2)
  *bytes = 2.0 * (pops + fp64_planes * 8.0 + 4.0 * cb + 2.0 * cb);
  return LBM_OK;
}

int lbm_step_kernel(lbm_handle* h, int32_t* variant, int32_t* workgroups, int32_t* cus) {
  if (!h || !variant || !workgroups || !cus) return fail(h, LBM_E_ARG, "null argument");
  *variant = lbm::step_variant(h->dp, h->ds);
  *workgroups = (int32_t)lbm::step_blocks(h->dp.nx, h->dp.ny, h->ds.tile_rows);
  *cus = h->ds.cus;
  return LBM_OK;
}

int lbm_destroy(lbm_handle* h) {
  if (!h) return LBM_OK;
  release_timer(h);
  if (h->stream) (void)hipStreamSynchronize(h->stream);
  for (int k = 0; k < kGraphKinds; ++k)
    if (h->graph[k]) (void)hipGraphExecDestroy(h->graph[k]);
  if (h->own_buf && h->buf) (void)hipFree(h->buf);
  if (h->own_stream && h->stream) (void)hipStreamDestroy(h->stream);
  delete h;
  return LBM_OK;
}

const char* lbm_last_error(const lbm_handle* h) { return h ? h->err.c_str() : g_init_error.c_str(); }

}  // extern "C"

namespace lbm {

int set_init_error(int code, const std::string& msg) { return fail(nullptr, code, msg); }

HandleView handle_view(lbm_handle* h) { return HandleView{&h->dp, &h->ds, &h->have_hist, &h->step, &h->faulted}; }

int handle_reinit(lbm_handle* h) {
  h->ds.cur = h->ds.hcur = h->ds.scur = 0;
  hipError_t e = lbm::launch_init(h->dp, h->ds, h->stream);
  if (e == hipSuccess) e = set_m_ref(h);
  if (e != hipSuccess) return hip_fail(h, e, "initialisation kernels");
  h->have_hist = 0;
  h->step = 0;
  h->faulted = false;
  return LBM_OK;
}

}  // namespace lbm
