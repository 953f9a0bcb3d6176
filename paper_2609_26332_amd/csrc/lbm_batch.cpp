// lbm_batch.cpp -- C ABI of the batched sweep: many independent cases (their
// own grids, parameters and buffers) advanced by one kernel launch per step.
//
// A batch is built from ordinary handles, one per case, whose states sit in
// sub-ranges of one device buffer; initialisation and diagnostics go through
// those handles.  Stepping goes through a device table of the cases
// (BatchCase): k_step_batch maps each of its workgroups to a case and runs the
// same step body as the single-case kernel, k_step_finish_batch forms each
// case's multipliers and flips its buffer parity.  Parity, history flag, step
// count and activity live in the table on the device, so runs of steps replay
// from one captured HIP graph whatever the cases' states, and cases retire
// (activity 0) without rebuilding anything.
#include <cmath>
#include <cstring>
#include <string>
#include <vector>

#include "lbm_internal.h"
#include "../../include/lbm.h"

struct lbm_batch {
  std::vector<lbm_handle*> h;
  std::vector<size_t> off;  // byte offset of each case's state in buf
  std::vector<size_t> slot_bytes;  // bytes of buf each case's slot holds (a refill must fit)
  std::vector<int> active;         // activity of each slot, as the device table holds it
  bool table_dirty = false;        // a refill changed the tiling: table and workgroup map are rebuilt before use
  int count = 0;
  int precision = 0;
  bool walls = false;
  void* buf = nullptr;
  bool own_buf = false;
  hipStream_t stream = nullptr;
  bool own_stream = false;
  lbm::BatchCase* d_cases = nullptr;  // [count], in buf
  int* d_wg = nullptr;                // [max workgroups], in buf
  int nwg = 0;
  int seg_rows = 4;
  std::vector<lbm::BatchCase> hc;  // host mirror of the table
  bool device_ahead = false;       // the table holds positions newer than the handles
  hipGraphExec_t graph[6] = {nullptr, nullptr, nullptr, nullptr, nullptr, nullptr};  // 2^k steps
  int64_t step = 0;
  lbm::StepTimer timer;
  // the last autotune: per candidate segment height, time of its trial steps,
  // largest relative deviation of its checked sums from the first candidate's,
  // and whether it passed that check
  struct TuneRow { int seg; double ms; double dev; int ok; };
  std::vector<TuneRow> tune;
  std::string err = "no error";
};

namespace {

std::string g_batch_error = "no error";
// Runs of steps replay from captured graphs of 1, 2, 4, 8, 16 or 32 steps (the
// cases' buffer parities live in the device table, so any length replays from
// any state); a run is split into the longest such pieces.
constexpr int kBatchGraphKinds = 6;

int bfail(lbm_batch* b, int code, const std::string& msg) {
  if (b) b->err = msg;
  else g_batch_error = msg;
  return code;
}
#define BHIP(b, expr, where)                                                                              \
  do {                                                                                                    \
    hipError_t e_ = (expr);                                                                               \
    if (e_ != hipSuccess) return bfail(b, LBM_E_DEVICE, std::string(where) + ": " + hipGetErrorString(e_)); \
  } while (0)

size_t align256(size_t v) { return (v + 255) & ~size_t(255); }
void drop_graph(lbm_batch* b);

struct Plan {
  std::vector<size_t> case_bytes, off;
  size_t table = 0, wg = 0, total = 0;
  int max_wg = 0;
};

// Validates the cases (each on its own, then as a batch: one storage
// precision, one kind of y boundary) and lays out the buffer.
int plan(const lbm_params* cases, int32_t count, Plan& P, std::string& why) {
  if (!cases || count <= 0 || count > (1 << 20)) { why = "count must lie in [1, 2^20] with a case array"; return LBM_E_ARG; }
  P.case_bytes.resize(count);
  P.off.resize(count);
  const bool walls0 = cases[0].bc_bottom != LBM_BC_PERIODIC;
  size_t wg = 0;
  for (int c = 0; c < count; ++c) {
    size_t bytes = 0;
    if (lbm_required_bytes(&cases[c], &bytes) != LBM_OK) {
      why = "case " + std::to_string(c) + ": " + lbm_last_error(nullptr);
      return LBM_E_ARG;
    }
    if (cases[c].precision != cases[0].precision) { why = "all cases of a batch share one storage precision"; return LBM_E_ARG; }
    if (cases[c].mms_dx > 0.0) { why = "the accuracy test (mms_dx) runs on single handles, not in a batch"; return LBM_E_ARG; }
    if ((cases[c].bc_bottom != LBM_BC_PERIODIC) != walls0) { why = "all cases of a batch are walled in y, or all periodic"; return LBM_E_ARG; }
    P.case_bytes[c] = align256(bytes);
    wg += lbm::step_blocks(cases[c].nx, cases[c].ny, 4);
  }
  if (wg > (size_t)1 << 30) { why = "too many workgroups in one batch"; return LBM_E_ARG; }
  P.max_wg = (int)wg;
  P.table = 0;
  P.wg = align256(sizeof(lbm::BatchCase) * count);
  size_t off = P.wg + align256(sizeof(int) * wg);
  for (int c = 0; c < count; ++c) {
    P.off[c] = off;
    off += P.case_bytes[c];
  }
  P.total = off;
  return LBM_OK;
}

// Device table for the current segment height, positions taken from the handles
// (which must be current), activity from b->active.  Graphs captured on an
// earlier table keep its workgroup count and are dropped.
int build_table(lbm_batch* b) {
  drop_graph(b);
  b->hc.assign(b->count, lbm::BatchCase());
  std::vector<int> wg;
  for (int c = 0; c < b->count; ++c) {
    lbm::HandleView v = lbm::handle_view(b->h[c]);
    v.ds->tile_rows = b->seg_rows;
    lbm::BatchCase& e = b->hc[c];
    std::memset(&e, 0, sizeof(e));
    e.p = *v.dp;
    for (int k = 0; k < 2; ++k) {
      e.pops[k] = v.ds->pops[k];
      e.phipsi[k] = (double*)v.ds->phipsi[k];
      e.uhist[k] = v.ds->uhist[k];
    }
    e.scalars = v.ds->scalars;
    e.partials = v.ds->partials;
    e.nstrips = (v.dp->nx + lbm::kStripW - 1) / lbm::kStripW;
    e.seg_rows = b->seg_rows;
    e.ntiles = (int)lbm::step_blocks(v.dp->nx, v.dp->ny, b->seg_rows);
    e.tile_begin = (int)wg.size();
    e.active = b->active[c];
    e.parity = v.ds->cur;
    e.have_hist = *v.have_hist;
    e.step = *v.step;
    wg.insert(wg.end(), (size_t)e.ntiles, c);
  }
  b->nwg = (int)wg.size();
  BHIP(b, hipMemcpyAsync(b->d_cases, b->hc.data(), sizeof(lbm::BatchCase) * b->count, hipMemcpyHostToDevice, b->stream), "upload batch table");
  BHIP(b, hipMemcpyAsync(b->d_wg, wg.data(), sizeof(int) * wg.size(), hipMemcpyHostToDevice, b->stream), "upload workgroup map");
  BHIP(b, hipStreamSynchronize(b->stream), "synchronise");
  b->device_ahead = false;
  b->table_dirty = false;
  return LBM_OK;
}

// Bring the handles up to the positions the device table holds.
int sync_handles(lbm_batch* b) {
  if (!b->device_ahead) return LBM_OK;
  BHIP(b, hipMemcpyAsync(b->hc.data(), b->d_cases, sizeof(lbm::BatchCase) * b->count, hipMemcpyDeviceToHost, b->stream), "download batch table");
  BHIP(b, hipStreamSynchronize(b->stream), "synchronise");
  for (int c = 0; c < b->count; ++c) {
    lbm::HandleView v = lbm::handle_view(b->h[c]);
    v.ds->cur = v.ds->hcur = v.ds->scur = b->hc[c].parity;
    *v.have_hist = b->hc[c].have_hist;
    *v.step = b->hc[c].step;
  }
  b->device_ahead = false;
  return LBM_OK;
}

// A refill that changed a slot's tiling leaves the table to be rebuilt here,
// before the next use of the table on the device.
int ensure_table(lbm_batch* b) {
  if (!b->table_dirty) return LBM_OK;
  const int rc = sync_handles(b);
  return rc ? rc : build_table(b);
}

// After a host-side change to case c (its handle is current): its table entry again.
int push_case(lbm_batch* b, int c) {
  lbm::HandleView v = lbm::handle_view(b->h[c]);
  lbm::BatchCase& e = b->hc[c];
  e.p = *v.dp;
  e.parity = v.ds->cur;
  e.have_hist = *v.have_hist;
  e.step = *v.step;
  BHIP(b, hipMemcpyAsync(b->d_cases + c, &e, sizeof(e), hipMemcpyHostToDevice, b->stream), "upload batch case");
  BHIP(b, hipStreamSynchronize(b->stream), "synchronise");
  return LBM_OK;
}

void drop_graph(lbm_batch* b) {
  for (int k = 0; k < kBatchGraphKinds; ++k) {
    if (b->graph[k]) (void)hipGraphExecDestroy(b->graph[k]);
    b->graph[k] = nullptr;
  }
}

void release_batch_timer(lbm_batch* b) {
  if (!b->timer.ev) return;
  for (int64_t k = 0; k < b->timer.max_steps * 2 * LBM_N_KERNELS; ++k) (void)hipEventDestroy(b->timer.ev[k]);
  delete[] b->timer.ev;
  b->timer = lbm::StepTimer();
}

int capture_batch_graph(lbm_batch* b, int kind) {
  const int64_t kBatchGraphSteps = int64_t(1) << kind;
  hipGraph_t g = nullptr;
  BHIP(b, hipStreamBeginCapture(b->stream, hipStreamCaptureModeThreadLocal), "begin graph capture");
  hipError_t e = hipSuccess;
  for (int64_t k = 0; k < kBatchGraphSteps && e == hipSuccess; ++k)
    e = lbm::launch_step_batch(b->precision, b->walls, b->d_cases, b->d_wg, b->nwg, b->count, b->stream, nullptr);
  const hipError_t e_end = hipStreamEndCapture(b->stream, &g);
  if (e == hipSuccess) e = e_end;
  if (e == hipSuccess) e = hipGraphInstantiate(&b->graph[kind], g, nullptr, nullptr, 0);
  if (g) (void)hipGraphDestroy(g);
  if (e != hipSuccess) {
    b->graph[kind] = nullptr;
    return bfail(b, LBM_E_DEVICE, std::string("graph capture of the batch step: ") + hipGetErrorString(e));
  }
  return LBM_OK;
}

int check_index(lbm_batch* b, int32_t index) {
  if (index < 0 || index >= b->count) return bfail(b, LBM_E_ARG, "case index out of range");
  return LBM_OK;
}

}  // namespace

extern "C" {

int lbm_batch_required_bytes(const lbm_params* cases, int32_t count, size_t* bytes) {
  if (!bytes) return bfail(nullptr, LBM_E_ARG, "null argument");
  Plan P;
  std::string why;
  const int rc = plan(cases, count, P, why);
  if (rc) return bfail(nullptr, rc, why);
  *bytes = P.total;
  return LBM_OK;
}

int lbm_batch_init(const lbm_params* cases, int32_t count, int32_t seg_rows, void* dev_buf, size_t buf_bytes,
                   void* hip_stream, lbm_batch** out) {
  if (!out) return bfail(nullptr, LBM_E_ARG, "null output batch");
  *out = nullptr;
  if (seg_rows < 0 || seg_rows % 4 != 0 || seg_rows > 4096) return bfail(nullptr, LBM_E_ARG, "seg_rows must be 0 or a multiple of 4 up to 4096");
  Plan P;
  std::string why;
  int rc = plan(cases, count, P, why);
  if (rc) return bfail(nullptr, rc, why);
  lbm_batch* b = new lbm_batch();
  b->count = count;
  b->precision = cases[0].precision;
  b->walls = cases[0].bc_bottom != LBM_BC_PERIODIC;
  if (dev_buf) {
    if (buf_bytes < P.total) { delete b; return bfail(nullptr, LBM_E_ARG, "dev_buf smaller than lbm_batch_required_bytes"); }
    if (((uintptr_t)dev_buf & 255) != 0) { delete b; return bfail(nullptr, LBM_E_ARG, "dev_buf must be 256-byte aligned"); }
    b->buf = dev_buf;
  } else {
    if (hipMalloc(&b->buf, P.total) != hipSuccess) { delete b; return bfail(nullptr, LBM_E_OOM, "hipMalloc of the batch state failed"); }
    b->own_buf = true;
  }
  if (hip_stream) b->stream = (hipStream_t)hip_stream;
  else {
    if (hipStreamCreate(&b->stream) != hipSuccess) {
      if (b->own_buf) (void)hipFree(b->buf);
      delete b;
      return bfail(nullptr, LBM_E_DEVICE, "hipStreamCreate failed");
    }
    b->own_stream = true;
  }
  char* base = (char*)b->buf;
  b->d_cases = (lbm::BatchCase*)(base + P.table);
  b->d_wg = (int*)(base + P.wg);
  b->off = P.off;
  b->slot_bytes = P.case_bytes;
  b->active.assign(count, 1);
  b->h.assign(count, nullptr);
  for (int c = 0; c < count; ++c) {
    rc = lbm_init(&cases[c], base + P.off[c], P.case_bytes[c], b->stream, &b->h[c]);
    if (rc) {
      const std::string msg = "case " + std::to_string(c) + ": " + lbm_last_error(nullptr);
      lbm_batch_destroy(b);
      return bfail(nullptr, rc, msg);
    }
  }
  if (seg_rows == 0) {  // as for one grid: enough workgroups to fill the chip
    seg_rows = 32;
    for (;;) {
      size_t wg = 0;
      for (int c = 0; c < count; ++c) wg += lbm::step_blocks(cases[c].nx, cases[c].ny, seg_rows);
      if (seg_rows == 4 || wg >= 8192) break;
      seg_rows /= 2;
    }
  }
  b->seg_rows = seg_rows;
  rc = build_table(b);
  if (rc) {
    const std::string msg = b->err;
    lbm_batch_destroy(b);
    return bfail(nullptr, rc, msg);
  }
  *out = b;
  return LBM_OK;
}

int lbm_batch_step(lbm_batch* b, int64_t n) {
  if (!b) return bfail(nullptr, LBM_E_ARG, "null batch");
  if (n < 0) return bfail(b, LBM_E_ARG, "negative step count");
  for (int c = 0; c < b->count; ++c)
    if (*lbm::handle_view(b->h[c]).faulted && b->hc[c].active)
      return bfail(b, LBM_E_STATE, "case " + std::to_string(c) + " holds non-finite or out-of-range values; retire or reload it");
  const int rt = ensure_table(b);
  if (rt) return rt;
  int64_t k = 0;
  while (k < n) {
    const bool timing = b->timer.ev && b->timer.used < b->timer.max_steps;
    int kind = kBatchGraphKinds - 1;
    while (kind > 0 && n - k < (int64_t(1) << kind)) --kind;
    if (!timing) {
      if (!b->graph[kind]) {
        const int rc = capture_batch_graph(b, kind);
        if (rc) return rc;
      }
      BHIP(b, hipGraphLaunch(b->graph[kind], b->stream), "graph launch");
      k += int64_t(1) << kind;
    } else {
      BHIP(b, lbm::launch_step_batch(b->precision, b->walls, b->d_cases, b->d_wg, b->nwg, b->count, b->stream, &b->timer),
           "batch step kernels");
      k += 1;
    }
  }
  b->step += n;
  if (n) b->device_ahead = true;
  return LBM_OK;
}

int lbm_batch_set_active(lbm_batch* b, const int32_t* active) {
  if (!b || !active) return bfail(b, LBM_E_ARG, "null argument");
  int rc = sync_handles(b);
  if (!rc) rc = ensure_table(b);
  if (rc) return rc;
  for (int c = 0; c < b->count; ++c) b->hc[c].active = b->active[c] = active[c] ? 1 : 0;
  BHIP(b, hipMemcpyAsync(b->d_cases, b->hc.data(), sizeof(lbm::BatchCase) * b->count, hipMemcpyHostToDevice, b->stream), "upload batch table");
  BHIP(b, hipStreamSynchronize(b->stream), "synchronise");
  return LBM_OK;
}

int lbm_batch_reduce_invariants(lbm_batch* b, lbm_invariants* out) {
  if (!b || !out) return bfail(b, LBM_E_ARG, "null argument");
  int rc = sync_handles(b);
  if (rc) return rc;
  int first = LBM_OK;
  for (int c = 0; c < b->count; ++c) {
    rc = lbm_reduce_invariants(b->h[c], &out[c]);
    if (rc && first == LBM_OK) {
      first = rc;
      bfail(b, rc, "case " + std::to_string(c) + ": " + lbm_last_error(b->h[c]));
    }
  }
  return first;
}

int lbm_batch_fetch_fields(lbm_batch* b, int32_t index, uint32_t mask, double* host, size_t n_doubles) {
  if (!b) return bfail(nullptr, LBM_E_ARG, "null batch");
  int rc = check_index(b, index);
  if (!rc) rc = sync_handles(b);
  if (rc) return rc;
  rc = lbm_fetch_fields(b->h[index], mask, host, n_doubles);
  if (rc) return bfail(b, rc, lbm_last_error(b->h[index]));
  return LBM_OK;
}

int lbm_batch_replace_case(lbm_batch* b, int32_t index, const lbm_params* p) {
  if (!b || !p) return bfail(b, LBM_E_ARG, "null argument");
  int rc = check_index(b, index);
  if (!rc) rc = sync_handles(b);
  if (rc) return rc;
  if (p->precision != b->precision || (p->bc_bottom != LBM_BC_PERIODIC) != b->walls)
    return bfail(b, LBM_E_ARG, "a replacement case needs the precision and y-boundary kind of the batch");
  size_t bytes = 0;
  if (lbm_required_bytes(p, &bytes) != LBM_OK) return bfail(b, LBM_E_ARG, lbm_last_error(nullptr));
  if (bytes > b->slot_bytes[index])
    return bfail(b, LBM_E_ARG, "the replacement case needs " + std::to_string(bytes) + " bytes; slot " +
                                   std::to_string(index) + " holds " + std::to_string(b->slot_bytes[index]));
  lbm_handle* nh = nullptr;
  rc = lbm_init(p, (char*)b->buf + b->off[index], b->slot_bytes[index], b->stream, &nh);
  if (rc) {   // the slot's memory may be partly overwritten: retire the slot
    const std::string msg = lbm_last_error(nullptr);
    b->active[index] = 0;
    b->hc[index].active = 0;
    if (!b->table_dirty) (void)push_case(b, index);
    return bfail(b, rc, msg);
  }
  lbm::HandleView old = lbm::handle_view(b->h[index]);
  const bool same_tiling = old.dp->nx == p->nx && old.dp->ny == p->ny;
  lbm_destroy(b->h[index]);   // does not own the buffer or the stream
  b->h[index] = nh;
  lbm::handle_view(nh).ds->tile_rows = b->seg_rows;
  b->active[index] = 1;
  b->hc[index].active = 1;
  if (!same_tiling || b->table_dirty) {   // another grid: new workgroup map at the next use
    b->table_dirty = true;
    return LBM_OK;
  }
  return push_case(b, index);
}

int lbm_batch_slot_bytes(lbm_batch* b, int32_t index, size_t* bytes) {
  if (!b || !bytes) return bfail(b, LBM_E_ARG, "null argument");
  const int rc = check_index(b, index);
  if (rc) return rc;
  *bytes = b->slot_bytes[index];
  return LBM_OK;
}

// Relative tolerance of the autotuner's check: candidates differ only in how
// the FP64 multiplier sums are grouped (their last bits), which the storage
// rounding then carries into the fields.
static double tune_tol(int precision) {
  return precision == LBM_FP64 ? 1e-10 : (precision == LBM_FP32 ? 1e-6 : 1e-4);
}

int lbm_batch_autotune(lbm_batch* b, int32_t trial_steps, int32_t* seg_rows_out) {
  if (!b || !seg_rows_out) return bfail(b, LBM_E_ARG, "null argument");
  if (trial_steps < 2 || trial_steps > 10000) return bfail(b, LBM_E_ARG, "trial_steps must lie in [2, 10000]");
  if (b->step != 0) return bfail(b, LBM_E_STATE, "autotune before the first step of a batch");
  int rc = ensure_table(b);
  if (rc) return rc;
  const int cand[] = {4, 8, 16, 32, 64};
  double best = 1e300;
  int best_seg = b->seg_rows;
  // Every candidate steps the batch from its initial state; the conserved sums
  // and the multiplier of each active case after the trial are compared with
  // the first candidate's, and a candidate that departs is not chosen.
  std::vector<lbm_invariants> ref(b->count), cur(b->count);
  b->tune.clear();
  const double tol = tune_tol(b->precision);
  for (int seg : cand) {
    b->seg_rows = seg;
    drop_graph(b);
    rc = build_table(b);
    if (rc) return rc;
    BHIP(b, lbm::launch_step_batch(b->precision, b->walls, b->d_cases, b->d_wg, b->nwg, b->count, b->stream, nullptr), "warm-up step");
    hipEvent_t e0, e1;
    BHIP(b, hipEventCreate(&e0), "hipEventCreate");
    BHIP(b, hipEventCreate(&e1), "hipEventCreate");
    (void)hipEventRecord(e0, b->stream);
    for (int k = 0; k < trial_steps; ++k)
      (void)lbm::launch_step_batch(b->precision, b->walls, b->d_cases, b->d_wg, b->nwg, b->count, b->stream, nullptr);
    (void)hipEventRecord(e1, b->stream);
    hipError_t e = hipEventSynchronize(e1);
    float ms = 0.f;
    if (e == hipSuccess) e = hipEventElapsedTime(&ms, e0, e1);
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (e != hipSuccess) return bfail(b, LBM_E_DEVICE, std::string("autotune timing: ") + hipGetErrorString(e));
    b->device_ahead = true;
    rc = sync_handles(b);
    if (rc) return rc;
    std::vector<lbm_invariants>& out = b->tune.empty() ? ref : cur;
    double dev = 0.0;
    int ok = 1;
    for (int c = 0; c < b->count; ++c) {
      if (!b->active[c]) continue;
      const int r = lbm_reduce_invariants(b->h[c], &out[c]);   // a non-finite or out-of-range field fails the candidate
      if (r != LBM_OK && r != LBM_E_NONFINITE && r != LBM_E_RANGE) return bfail(b, r, lbm_last_error(b->h[c]));
      if (r != LBM_OK || out[c].nonfinite) ok = 0;
      if (&out == &cur) {
        const double a[4] = {ref[c].mass_psi, ref[c].sum_phi, ref[c].m_phi_h, ref[c].lambda_phi};
        const double q[4] = {cur[c].mass_psi, cur[c].sum_phi, cur[c].m_phi_h, cur[c].lambda_phi};
        for (int k = 0; k < 4; ++k) {
          const double d = std::fabs(q[k] - a[k]) / std::fmax(std::fabs(a[k]), 1e-300);
          dev = std::isnan(d) ? 1e300 : std::fmax(dev, d);
        }
      }
    }
    if (dev > tol) ok = 0;
    b->tune.push_back({seg, (double)ms, dev, ok});
    if (ok && ms < best) { best = ms; best_seg = seg; }
    for (int c = 0; c < b->count; ++c) {  // back to the initial state
      rc = lbm::handle_reinit(b->h[c]);
      if (rc) return bfail(b, rc, lbm_last_error(b->h[c]));
    }
  }
  if (best == 1e300) return bfail(b, LBM_E_NONFINITE, "autotune: every candidate's trial left a non-finite field");
  b->seg_rows = best_seg;
  drop_graph(b);
  rc = build_table(b);
  if (rc) return rc;
  *seg_rows_out = best_seg;
  return LBM_OK;
}

int lbm_batch_autotune_report(lbm_batch* b, int32_t max_rows, int32_t* seg_rows, double* ms, double* max_rel_dev,
                              int32_t* passed, int32_t* rows) {
  if (!b || !rows || (max_rows > 0 && (!seg_rows || !ms || !max_rel_dev || !passed)))
    return bfail(b, LBM_E_ARG, "null argument");
  if (max_rows < (int32_t)b->tune.size()) {
    *rows = (int32_t)b->tune.size();
    return bfail(b, LBM_E_ARG, "max_rows is smaller than the number of candidates");
  }
  for (size_t k = 0; k < b->tune.size(); ++k) {
    seg_rows[k] = b->tune[k].seg;
    ms[k] = b->tune[k].ms;
    max_rel_dev[k] = b->tune[k].dev;
    passed[k] = b->tune[k].ok;
  }
  *rows = (int32_t)b->tune.size();
  return LBM_OK;
}

int lbm_batch_info(lbm_batch* b, int32_t* count, int32_t* seg_rows, int32_t* workgroups, int64_t* nodes) {
  if (!b || !count || !seg_rows || !workgroups || !nodes) return bfail(b, LBM_E_ARG, "null argument");
  *count = b->count;
  *seg_rows = b->seg_rows;
  *workgroups = b->nwg;
  int64_t n = 0;
  for (int c = 0; c < b->count; ++c) n += lbm::handle_view(b->h[c]).dp->N;
  *nodes = n;
  return LBM_OK;
}

int lbm_batch_timing_begin(lbm_batch* b, int64_t max_steps) {
  if (!b) return bfail(nullptr, LBM_E_ARG, "null batch");
  if (max_steps <= 0 || max_steps > 1000000) return bfail(b, LBM_E_ARG, "max_steps must lie in [1, 1e6]");
  release_batch_timer(b);
  const int64_t nev = max_steps * 2 * LBM_N_KERNELS;
  b->timer.ev = new hipEvent_t[nev];
  for (int64_t k = 0; k < nev; ++k) {
    hipError_t e = hipEventCreate(&b->timer.ev[k]);
    if (e != hipSuccess) {
      for (int64_t j = 0; j < k; ++j) (void)hipEventDestroy(b->timer.ev[j]);
      delete[] b->timer.ev;
      b->timer = lbm::StepTimer();
      return bfail(b, LBM_E_DEVICE, std::string("hipEventCreate: ") + hipGetErrorString(e));
    }
  }
  b->timer.max_steps = max_steps;
  b->timer.used = 0;
  return LBM_OK;
}

int lbm_batch_timing_end(lbm_batch* b, double* ms, int64_t* launches) {
  if (!b || !ms || !launches) return bfail(b, LBM_E_ARG, "null argument");
  if (!b->timer.ev) return bfail(b, LBM_E_STATE, "lbm_batch_timing_begin was not called");
  BHIP(b, hipStreamSynchronize(b->stream), "synchronise");
  for (int k = 0; k < LBM_N_KERNELS; ++k) { ms[k] = 0.0; launches[k] = 0; }
  for (int64_t s = 0; s < b->timer.used; ++s)
    for (int k = 0; k < LBM_N_KERNELS; ++k) {
      float t = 0.f;
      hipError_t e = hipEventElapsedTime(&t, b->timer.ev[(s * LBM_N_KERNELS + k) * 2], b->timer.ev[(s * LBM_N_KERNELS + k) * 2 + 1]);
      if (e != hipSuccess) { release_batch_timer(b); return bfail(b, LBM_E_DEVICE, std::string("hipEventElapsedTime: ") + hipGetErrorString(e)); }
      ms[k] += t;
      launches[k] += 1;
    }
  release_batch_timer(b);
  return LBM_OK;
}

int lbm_batch_destroy(lbm_batch* b) {
  if (!b) return LBM_OK;
  if (b->stream) (void)hipStreamSynchronize(b->stream);
  release_batch_timer(b);
  drop_graph(b);
  for (lbm_handle* h : b->h)
    if (h) lbm_destroy(h);
  if (b->own_buf && b->buf) (void)hipFree(b->buf);
  if (b->own_stream && b->stream) (void)hipStreamDestroy(b->stream);
  delete b;
  return LBM_OK;
}

const char* lbm_batch_last_error(const lbm_batch* b) { return b ? b->err.c_str() : g_batch_error.c_str(); }

}  // extern "C"
