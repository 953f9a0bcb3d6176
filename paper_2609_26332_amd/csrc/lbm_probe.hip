// lbm_probe.hip -- achievable-bandwidth probe for the step's memory traffic
// (a measurement aid beside the roofline, not part of the method).
//
// One kernel moves per node exactly the bytes lbm_bytes_per_node_step counts
// for a step with surfactant, in the step's access pattern and none of its
// arithmetic: the 27 populations pulled from the neighbours streaming reads
// (x - c_i, y - c_i on a periodic grid; FP16 storage: the two rest
// populations of g and h from FP32 planes), six history planes in the
// collision type and two FP64 planes, each read once and written once, with
// the hints of the row sweep (non-temporal loads of f, plain loads and stores
// otherwise).  Thread (x, y) owns node (x, y); blocks of 64 x 4 nodes.
// A plain streaming copy (16-byte non-temporal loads and stores) gives the
// device's copy ceiling beside it.
#include <hip/hip_runtime.h>

#include <string>

#include "lbm.h"
#include "lbm_internal.h"

namespace lbm {
namespace {

__device__ __forceinline__ int pcx(int d) { return (d == 1 || d == 5 || d == 8) ? 1 : ((d == 3 || d == 6 || d == 7) ? -1 : 0); }
__device__ __forceinline__ int pcy(int d) { return (d == 2 || d == 5 || d == 6) ? 1 : ((d == 4 || d == 7 || d == 8) ? -1 : 0); }

struct ProbeLayout {
  size_t pops, rest, hist, f64, total;   // bytes of one copy of each region
};

ProbeLayout probe_layout(int nx, int ny, int precision) {
  auto up = [](size_t b) { return (b + 255) / 256 * 256; };
  const size_t N = (size_t)nx * ny;
  ProbeLayout L;
  L.pops = up(27 * N * storage_bytes(precision));
  L.rest = precision == LBM_FP16_SHIFTED ? up(2 * N * 4) : 0;
  L.hist = up(6 * N * compute_bytes(precision));
  L.f64 = up(2 * N * 8);
  L.total = 2 * (L.pops + L.rest + L.hist + L.f64);
  return L;
}

template <class S, class C>
__global__ __launch_bounds__(256) void k_probe(int nx, int ny, const S* __restrict__ Pin, S* __restrict__ Pout,
                                               const float* __restrict__ Rin, float* __restrict__ Rout,
                                               const C* __restrict__ hin, C* __restrict__ hout,
                                               const double* __restrict__ fin, double* __restrict__ fout) {
  const int x = blockIdx.x * 64 + (threadIdx.x & 63);
  const int y = blockIdx.y * 4 + (threadIdx.x >> 6);
  if (x >= nx || y >= ny) return;
  const size_t N = (size_t)nx * ny, n = (size_t)y * nx + x;
  constexpr bool half = sizeof(S) == 2;
  float acc = 0.f;
#pragma unroll
  for (int i = 0; i < 27; ++i) {
    const int d = i % 9;
    if (half && (i == 9 || i == 18)) {   // rest populations of g, h: FP32 planes, not streamed
      const int r = i / 9 - 1;
      acc += Rin[r * N + n];
      Rout[r * N + n] = acc;
      continue;
    }
    int sx = x - pcx(d), sy = y - pcy(d);
    sx = sx < 0 ? sx + nx : (sx >= nx ? sx - nx : sx);
    sy = sy < 0 ? sy + ny : (sy >= ny ? sy - ny : sy);
    const S* q = Pin + (size_t)i * N + (size_t)sy * nx + sx;
    acc += (float)(i < 9 ? __builtin_nontemporal_load(q) : *q);   // f streams past the L2, as in the step
    Pout[(size_t)i * N + n] = (S)(0.5f * acc);
  }
#pragma unroll
  for (int k = 0; k < 6; ++k) {
    acc += (float)hin[k * N + n];
    hout[k * N + n] = (C)acc;
  }
  const double a = fin[n] + fin[N + n] + (double)acc;
  fout[n] = a;
  fout[N + n] = 0.5 * a;
}

template <class S, class C>
hipError_t run_probe(int nx, int ny, int precision, int reps, char* buf, hipStream_t st, float* ms) {
  const ProbeLayout L = probe_layout(nx, ny, precision);
  char* half[2] = {buf, buf + L.total / 2};
  dim3 grid((unsigned)((nx + 63) / 64), (unsigned)((ny + 3) / 4));
  auto launch = [&](int r) {
    char* a = half[r & 1];
    char* b = half[(r + 1) & 1];
    const size_t r0 = L.pops, h0 = r0 + L.rest, f0 = h0 + L.hist;   // region offsets in each half
    k_probe<S, C><<<grid, 256, 0, st>>>(nx, ny, (const S*)a, (S*)b, (const float*)(a + r0), (float*)(b + r0),
                                        (const C*)(a + h0), (C*)(b + h0), (const double*)(a + f0), (double*)(b + f0));
    return hipGetLastError();
  };
  hipError_t e;
  for (int w = 0; w < 2; ++w)
    if ((e = launch(w)) != hipSuccess) return e;
  hipEvent_t e0, e1;
  if ((e = hipEventCreate(&e0)) != hipSuccess) return e;
  if ((e = hipEventCreate(&e1)) != hipSuccess) { (void)hipEventDestroy(e0); return e; }
  e = hipEventRecord(e0, st);
  for (int r = 0; r < reps && e == hipSuccess; ++r) e = launch(r);
  if (e == hipSuccess) e = hipEventRecord(e1, st);
  if (e == hipSuccess) e = hipEventSynchronize(e1);
  float t = 0.f;
  if (e == hipSuccess) e = hipEventElapsedTime(&t, e0, e1);
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  *ms = t / (float)reps;
  return e;
}

// Plain streaming copy: each thread moves four 16-byte vectors 256 apart
// (one 16 KiB block per workgroup), non-temporal loads and stores.
typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));
__global__ __launch_bounds__(256) void k_copy16(const u32x4* __restrict__ src, u32x4* __restrict__ dst, size_t n16) {
  const size_t base = (size_t)blockIdx.x * 1024 + threadIdx.x;
  u32x4 v[4];
#pragma unroll
  for (int u = 0; u < 4; ++u) {
    const size_t j = base + (size_t)u * 256;
    if (j < n16) v[u] = __builtin_nontemporal_load(src + j);
  }
#pragma unroll
  for (int u = 0; u < 4; ++u) {
    const size_t j = base + (size_t)u * 256;
    if (j < n16) __builtin_nontemporal_store(v[u], dst + j);
  }
}

}  // namespace
}  // namespace lbm

extern "C" {

int lbm_probe_copy(const void* src, void* dst, size_t bytes, int32_t reps, void* hip_stream, float* ms_out) {
  if (!src || !dst || !ms_out) return lbm::set_init_error(LBM_E_ARG, "null argument");
  if ((((uintptr_t)src | (uintptr_t)dst) & 15) != 0 || bytes % 16 != 0 || bytes == 0)
    return lbm::set_init_error(LBM_E_ARG, "src, dst and bytes must be multiples of 16 (bytes > 0)");
  if (reps < 1 || reps > 10000) return lbm::set_init_error(LBM_E_ARG, "reps out of range");
  const size_t n16 = bytes / 16, blocks = (n16 + 1023) / 1024;
  if (blocks > 0x7fffffffull) return lbm::set_init_error(LBM_E_ARG, "copy too large");
  hipStream_t st = (hipStream_t)hip_stream;
  auto launch = [&]() {
    hipLaunchKernelGGL(lbm::k_copy16, dim3((unsigned)blocks), dim3(256), 0, st, (const lbm::u32x4*)src, (lbm::u32x4*)dst,
                       n16);
    return hipGetLastError();
  };
  hipError_t e = launch();
  if (e == hipSuccess) e = launch();
  hipEvent_t e0 = nullptr, e1 = nullptr;
  if (e == hipSuccess) e = hipEventCreate(&e0);
  if (e == hipSuccess) e = hipEventCreate(&e1);
  if (e == hipSuccess) e = hipEventRecord(e0, st);
  for (int r = 0; r < reps && e == hipSuccess; ++r) e = launch();
  if (e == hipSuccess) e = hipEventRecord(e1, st);
  if (e == hipSuccess) e = hipEventSynchronize(e1);
  float t = 0.f;
  if (e == hipSuccess) e = hipEventElapsedTime(&t, e0, e1);
  if (e0) (void)hipEventDestroy(e0);
  if (e1) (void)hipEventDestroy(e1);
  if (e != hipSuccess) return lbm::set_init_error(LBM_E_DEVICE, std::string("copy kernel: ") + hipGetErrorString(e));
  *ms_out = t / (float)reps;
  return LBM_OK;
}

int lbm_probe_bytes(int32_t nx, int32_t ny, int32_t precision, size_t* bytes) {
  if (!bytes) return lbm::set_init_error(LBM_E_ARG, "null argument");
  if (nx < 1 || ny < 1 || (int64_t)nx * ny > (1ll << 28) || (ny + 3) / 4 > 65535)
    return lbm::set_init_error(LBM_E_ARG, "grid out of range");
  if (precision < LBM_FP64 || precision > LBM_FP16_SHIFTED) return lbm::set_init_error(LBM_E_ARG, "unknown precision");
  *bytes = lbm::probe_layout(nx, ny, precision).total;
  return LBM_OK;
}

int lbm_probe_stream(int32_t nx, int32_t ny, int32_t precision, int32_t reps, void* dev_buf, size_t buf_bytes,
                     void* hip_stream, float* ms_out) {
  size_t need = 0;
  const int rc = lbm_probe_bytes(nx, ny, precision, &need);
  if (rc != LBM_OK) return rc;
  if (!dev_buf || !ms_out) return lbm::set_init_error(LBM_E_ARG, "null argument");
  if (((uintptr_t)dev_buf & 255) != 0) return lbm::set_init_error(LBM_E_ARG, "dev_buf must be 256-byte aligned");
  if (buf_bytes < need) return lbm::set_init_error(LBM_E_ARG, "dev_buf smaller than lbm_probe_bytes");
  if (reps < 1 || reps > 10000) return lbm::set_init_error(LBM_E_ARG, "reps out of range");
  hipStream_t st = (hipStream_t)hip_stream;
  char* buf = (char*)dev_buf;
  hipError_t e;
  switch (precision) {
    case LBM_FP64: e = lbm::run_probe<double, double>(nx, ny, precision, reps, buf, st, ms_out); break;
    case LBM_FP32: e = lbm::run_probe<float, float>(nx, ny, precision, reps, buf, st, ms_out); break;
    default: e = lbm::run_probe<_Float16, float>(nx, ny, precision, reps, buf, st, ms_out); break;
  }
  if (e != hipSuccess) return lbm::set_init_error(LBM_E_DEVICE, std::string("probe kernel: ") + hipGetErrorString(e));
  return LBM_OK;
}

}  // extern "C"
