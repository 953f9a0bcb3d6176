// mlp.hip -- gfx950 kernels and C ABI (include/mlp.h) of the surrogate MLP:
// 5 -> 256 -> 256 -> 256 -> 2, exact GELU, ensemble of members.
//
// Every matrix product is one kernel, k_gemm: a 64 x 64 output tile per
// workgroup of four waves (grid z: ensemble members, each with its own
// operand offsets, so the members train or predict in the same launches), each wave a 32 x 32 block of 2 x 2 matrix-core
// tiles (v_mfma_f32_16x16x32_bf16: bfloat16 operands, FP32 accumulation),
// operands staged through LDS with zero padding at the edges, strided so the
// same kernel forms X W, dZ W^T and A^T dZ; epilogues add the bias and apply
// GELU (storing the FP32 pre-activation for the backward pass and the
// bfloat16 activation for the next product) or its derivative.  The biases,
// the loss, the column sums of the bias gradients and Adam run in FP32.
#include <cmath>
#include <cstring>
#include <string>
#include <vector>

#include <hip/hip_runtime.h>

#include "../../include/mlp.h"

namespace {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

constexpr int kIn = 5, kHid = 256, kOut = 2, kLayers = 4;
constexpr int kDims[kLayers + 1] = {kIn, kHid, kHid, kHid, kOut};
constexpr int kParams = kIn * kHid + kHid + 2 * (kHid * kHid + kHid) + kHid * kOut + kOut;   // 133634
constexpr int kThreads = 256;
constexpr int kRed = 256;   // partial sums of the loss

__host__ __device__ constexpr int w_off(int l) {   // offset of W_l (l = 0..3) in a parameter vector
  int o = 0;
  for (int k = 0; k < l; ++k) o += kDims[k] * kDims[k + 1] + kDims[k + 1];
  return o;
}
__host__ __device__ constexpr int b_off(int l) { return w_off(l) + kDims[l] * kDims[l + 1]; }
static_assert(w_off(kLayers) == kParams, "layout");
// Members' parameter vectors inside the library sit kPStride apart (a whole
// number of 8-element groups, so every member's weight matrices start on a
// 16-byte boundary for the matrix-core staging loads).
constexpr int kPStride = (kParams + 7) / 8 * 8;

__device__ __forceinline__ float gelu(float z) { return 0.5f * z * (1.0f + erff(z * 0.70710678118654752f)); }
__device__ __forceinline__ float gelu_d(float z) {
  return 0.5f * (1.0f + erff(z * 0.70710678118654752f)) + z * expf(-0.5f * z * z) * 0.39894228040143268f;
}

enum { EPI_STORE = 0, EPI_BIAS_GELU = 1, EPI_BIAS = 2, EPI_DGELU = 3 };

// C(m, n) = sum_k A(m, k) B(k, n) with A(m, k) = A[m sam + k sak], B(k, n) = B[k sbk + n sbn].
struct Gemm {
  const __bf16* A;
  long long sam, sak;
  const __bf16* B;
  long long sbk, sbn;
  int M, N, K, epi;
  float* C;          // FP32 result (after the epilogue), row stride scm
  long long scm;
  __bf16* Cb;        // bfloat16 copy: GELU(z) (EPI_BIAS_GELU) or the scaled result (EPI_DGELU)
  const float* bias; // [N]
  const float* Zp;   // EPI_DGELU: pre-activation multiplied in through GELU', same layout as C
  // element offsets between consecutive members (blockIdx.z) of A, B, C / Cb / Zp and bias
  long long zA, zB, zC, zbias;
  // how each operand is staged: STAGE_K (8 consecutive k in one 16-byte load),
  // STAGE_MN (8 consecutive m or n in one load, scattered into LDS) or
  // STAGE_ELEM (element by element); chosen on the host from strides and alignment
  int a_stage, b_stage;
};
enum { STAGE_ELEM = 0, STAGE_K = 1, STAGE_MN = 2 };

constexpr int TM = 64, TN = 64, TK = 32, LDK = TK + 8;   // LDS rows padded to 80 bytes (16-byte aligned fragments)

// Stage the 64 x 32 operand tile X(row, k), rows r0 .. r0+63 and k0 .. k0+31,
// into LDS as T[row][k] (zero beyond the matrix), with X(row, k) =
// X[row * srow + k * sk].  STAGE_K: thread t loads 8 consecutive k of row
// t / 4 in one 16-byte load (sk = 1); STAGE_MN: thread t loads 8 consecutive
// rows at k0 + t / 8 (srow = 1; eight lanes cover 64 rows of one k) and
// scatters them; both fall back to single elements at the matrix's edges.
__device__ __forceinline__ void stage_tile(const __bf16* __restrict__ X, long long srow, long long sk, int R, int K,
                                           int r0, int k0, int mode, __bf16 (*T)[LDK], int t) {
  if (mode == STAGE_K) {
    const int r = t >> 2, kq = (t & 3) * 8;
    const int row = r0 + r, k = k0 + kq;
    bf16x8 v;
    if (row < R && k + 7 < K) {
      v = *(const bf16x8*)(X + row * srow + k);
    } else {
#pragma unroll
      for (int j = 0; j < 8; ++j) v[j] = (row < R && k + j < K) ? X[row * srow + k + j] : (__bf16)0.0f;
    }
    *(bf16x8*)&T[r][kq] = v;
  } else if (mode == STAGE_MN) {
    const int kk = t >> 3, rq = (t & 7) * 8;
    const int k = k0 + kk, row = r0 + rq;
    bf16x8 v;
    if (k < K && row + 7 < R) {
      v = *(const bf16x8*)(X + k * sk + row);
    } else {
#pragma unroll
      for (int j = 0; j < 8; ++j) v[j] = (k < K && row + j < R) ? X[k * sk + row + j] : (__bf16)0.0f;
    }
#pragma unroll
    for (int j = 0; j < 8; ++j) T[rq + j][kk] = v[j];
  } else {
    const int r = t >> 2, kq = (t & 3) * 8;
    const int row = r0 + r;
#pragma unroll
    for (int j = 0; j < 8; ++j) {
      const int k = k0 + kq + j;
      T[r][kq + j] = (row < R && k < K) ? X[row * srow + k * sk] : (__bf16)0.0f;
    }
  }
}

__global__ __launch_bounds__(kThreads) void k_gemm(Gemm g) {
  __shared__ __attribute__((aligned(16))) __bf16 As[TM][LDK];   // [m][k]
  __shared__ __attribute__((aligned(16))) __bf16 Bs[TN][LDK];   // [n][k]: a lane's 8 k values are contiguous
  const int t = threadIdx.x, lane = t & 63, w = t >> 6;
  const int m0 = blockIdx.y * TM, n0 = blockIdx.x * TN;
  const long long z = blockIdx.z;
  const __bf16* __restrict__ gA = g.A + z * g.zA;
  const __bf16* __restrict__ gB = g.B + z * g.zB;
  const int wm = (w >> 1) * 32, wn = (w & 1) * 32;
  f32x4 acc[2][2];
  for (int i = 0; i < 2; ++i)
    for (int j = 0; j < 2; ++j) acc[i][j] = f32x4{0.f, 0.f, 0.f, 0.f};
  for (int k0 = 0; k0 < g.K; k0 += TK) {
    stage_tile(gA, g.sam, g.sak, g.M, g.K, m0, k0, g.a_stage, As, t);
    stage_tile(gB, g.sbn, g.sbk, g.N, g.K, n0, k0, g.b_stage, Bs, t);
    __syncthreads();
    // matrix-core fragments: lane l holds row (l mod 16) and k = 8 (l / 16) .. +7
#pragma unroll
    for (int bm = 0; bm < 2; ++bm)
#pragma unroll
      for (int bn = 0; bn < 2; ++bn) {
        const bf16x8 a = *(const bf16x8*)&As[wm + bm * 16 + (lane & 15)][(lane >> 4) * 8];
        const bf16x8 b = *(const bf16x8*)&Bs[wn + bn * 16 + (lane & 15)][(lane >> 4) * 8];
        acc[bm][bn] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, acc[bm][bn], 0, 0, 0);
      }
    __syncthreads();
  }
  // result tile: lane l holds column (l mod 16), rows 4 (l / 16) .. +3
  float* __restrict__ gC = g.C + z * g.zC;
  __bf16* __restrict__ gCb = g.Cb ? g.Cb + z * g.zC : nullptr;
  const float* __restrict__ gbias = g.bias ? g.bias + z * g.zbias : nullptr;
  const float* __restrict__ gZp = g.Zp ? g.Zp + z * g.zC : nullptr;
#pragma unroll
  for (int bm = 0; bm < 2; ++bm)
#pragma unroll
    for (int bn = 0; bn < 2; ++bn)
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        const int m = m0 + wm + bm * 16 + (lane >> 4) * 4 + j, n = n0 + wn + bn * 16 + (lane & 15);
        if (m >= g.M || n >= g.N) continue;
        const long long at = m * g.scm + n;
        float v = acc[bm][bn][j];
        if (g.epi == EPI_BIAS_GELU) {
          v += gbias[n];
          gC[at] = v;
          gCb[at] = (__bf16)gelu(v);
        } else if (g.epi == EPI_BIAS) {
          gC[at] = v + gbias[n];
        } else if (g.epi == EPI_DGELU) {
          v *= gelu_d(gZp[at]);
          gC[at] = v;
          gCb[at] = (__bf16)v;
        } else {
          gC[at] = v;
        }
      }
}

__global__ __launch_bounds__(kThreads) void k_cast_bf16(const float* __restrict__ src, __bf16* __restrict__ dst, int n) {
  const int i = blockIdx.x * kThreads + threadIdx.x;
  if (i < n) dst[i] = (__bf16)src[i];
}

__device__ float block_sum(float v) {
  __shared__ float sh[kThreads / 64];
  for (int off = 32; off > 0; off >>= 1) v += __shfl_down(v, off, 64);
  if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = v;
  __syncthreads();
  float r = 0.f;
  if (threadIdx.x == 0)
    for (int k = 0; k < kThreads / 64; ++k) r += sh[k];
  __syncthreads();
  return r;   // valid in thread 0
}

// 1 / max(sum of the mask, 1), one workgroup per member (blockIdx.x)
__global__ __launch_bounds__(kThreads) void k_mask_norm(const float* __restrict__ m, int n2, float* __restrict__ inv) {
  m += (long long)blockIdx.x * n2;
  inv += blockIdx.x;
  float s = 0.f;
  for (int i = threadIdx.x; i < n2; i += kThreads) s += m[i];
  s = block_sum(s);
  if (threadIdx.x == 0) *inv = 1.0f / fmaxf(s, 1.0f);
}

// dY = 2 m (y - t) / sum(m) in FP32 and bfloat16; per-workgroup partial sums
// of m (y - t)^2 (member blockIdx.y; its arrays n2 apart, its partials kRed apart)
__global__ __launch_bounds__(kThreads) void k_dy(const float* __restrict__ y, const float* __restrict__ t,
                                                 const float* __restrict__ m, int n2, const float* __restrict__ inv,
                                                 float* __restrict__ dy, __bf16* __restrict__ dyb, float* __restrict__ part) {
  const long long zo = (long long)blockIdx.y * n2;
  y += zo;
  t += zo;
  m += zo;
  dy += zo;
  dyb += zo;
  inv += blockIdx.y;
  part += (long long)blockIdx.y * kRed;
  float s = 0.f;
  const float sc = 2.0f * *inv;
  for (int i = blockIdx.x * kThreads + threadIdx.x; i < n2; i += gridDim.x * kThreads) {
    const float r = y[i] - t[i];
    s += m[i] * r * r;
    const float d = sc * m[i] * r;
    dy[i] = d;
    dyb[i] = (__bf16)d;
  }
  s = block_sum(s);
  if (threadIdx.x == 0) part[blockIdx.x] = s;
}

__global__ __launch_bounds__(kThreads) void k_loss_final(const float* __restrict__ part, int nb, const float* __restrict__ inv,
                                                         float* __restrict__ loss) {
  part += (long long)blockIdx.x * nb;
  inv += blockIdx.x;
  loss += blockIdx.x;
  float s = 0.f;
  for (int i = threadIdx.x; i < nb; i += kThreads) s += part[i];
  s = block_sum(s);
  if (threadIdx.x == 0) *loss = s * *inv;
}

// db[j] = sum over rows of dz[row][j] (member blockIdx.y: dz rows * cols apart,
// db kPStride apart).  A workgroup takes 64 columns; its four waves sum every
// fourth row each (eight loads in flight per lane), then wave 0 adds the four
// partial sums in wave order: the same order on every call.
constexpr int kColW = 64, kColRowGroups = kThreads / kColW;
__global__ __launch_bounds__(kThreads) void k_colsum(const float* __restrict__ dz, int rows, int cols, float* __restrict__ db) {
  __shared__ float part[kColRowGroups][kColW];
  const int tx = threadIdx.x % kColW, ty = threadIdx.x / kColW;
  const int j = blockIdx.x * kColW + tx;
  dz += (long long)blockIdx.y * rows * cols;
  db += (long long)blockIdx.y * kPStride;
  float s = 0.f;
  if (j < cols) {
    int r = ty;
    for (; r + 7 * kColRowGroups < rows; r += 8 * kColRowGroups) {
      float v[8];
#pragma unroll
      for (int u = 0; u < 8; ++u) v[u] = dz[(long long)(r + u * kColRowGroups) * cols + j];
#pragma unroll
      for (int u = 0; u < 8; ++u) s += v[u];
    }
    for (; r < rows; r += kColRowGroups) s += dz[(long long)r * cols + j];
  }
  part[ty][tx] = s;
  __syncthreads();
  if (ty == 0 && j < cols) {
    float t = part[0][tx];
#pragma unroll
    for (int g = 1; g < kColRowGroups; ++g) t += part[g][tx];
    db[j] = t;
  }
}

// Bias corrections 1 - beta^t of Adam, per member.
constexpr int kMaxMembers = 64;
struct AdamCorr {
  float c1[kMaxMembers], c2[kMaxMembers];
};

// Adam on the FP32 master parameters, then their bfloat16 copy (member
// blockIdx.y: its arrays kPStride apart, n of them used)
__global__ __launch_bounds__(kThreads) void k_adam(float* __restrict__ th, float* __restrict__ mo, float* __restrict__ ve,
                                                   const float* __restrict__ g, __bf16* __restrict__ thb, int n, float lr,
                                                   AdamCorr corr) {
  const int i = blockIdx.x * kThreads + threadIdx.x;
  if (i >= n) return;
  const int z = blockIdx.y;
  const long long zo = (long long)z * kPStride;
  th += zo;
  mo += zo;
  ve += zo;
  g += zo;
  thb += zo;
  const float c1 = corr.c1[z], c2 = corr.c2[z];
  const float gi = g[i];
  const float m = 0.9f * mo[i] + 0.1f * gi;
  const float v = 0.999f * ve[i] + 0.001f * gi * gi;
  mo[i] = m;
  ve[i] = v;
  const float x = th[i] - lr * (m / c1) / (sqrtf(v / c2) + 1e-8f);
  th[i] = x;
  thb[i] = (__bf16)x;
}

// ensemble mean and population standard deviation over members
__global__ __launch_bounds__(kThreads) void k_ens(const float* __restrict__ ys, int members, int n2, float* __restrict__ mean,
                                                  float* __restrict__ sd) {
  const int i = blockIdx.x * kThreads + threadIdx.x;
  if (i >= n2) return;
  float s = 0.f;
  for (int k = 0; k < members; ++k) s += ys[(long long)k * n2 + i];
  const float mu = s / members;
  float q = 0.f;
  for (int k = 0; k < members; ++k) {
    const float d = ys[(long long)k * n2 + i] - mu;
    q += d * d;
  }
  mean[i] = mu;
  sd[i] = sqrtf(q / members);
}

size_t al256(size_t v) { return (v + 255) & ~size_t(255); }
int nblk(long long n) { return (int)((n + kThreads - 1) / kThreads); }

std::string g_mlp_error = "no error";

}  // namespace

struct mlp_handle {
  int members = 0, max_batch = 0;
  void* buf = nullptr;
  bool own_buf = false;
  hipStream_t stream = nullptr;
  bool own_stream = false;
  // per member [members][kPStride] (the first kParams of each used)
  float *master = nullptr, *mom = nullptr, *vel = nullptr, *grad = nullptr;
  __bf16* wbf = nullptr;
  std::vector<int> adam_t;
  // Work arrays, one slot of max_batch samples per member; a call on n
  // samples packs the members' slots n samples apart.
  __bf16* xb = nullptr;                        // bfloat16 inputs [members][n][5]
  float* Z[3] = {nullptr, nullptr, nullptr};   // pre-activations of the hidden layers [members][n][256]
  __bf16* A[3] = {nullptr, nullptr, nullptr};  // their bfloat16 GELU outputs
  float* y = nullptr;                          // outputs [members][n][2]
  float *dy = nullptr, *dzf[2] = {nullptr, nullptr};
  __bf16 *dyb = nullptr, *dzb[2] = {nullptr, nullptr};
  float *part = nullptr, *inv = nullptr, *loss = nullptr;   // [members][kRed], [members], [members]
  std::string err = "no error";
};

namespace {

struct MlpLayout {
  size_t master, mom, vel, grad, wbf, xb, Z, A, y, dy, dyb, dzf, dzb, part, inv, loss, total;
};

MlpLayout mlp_layout(int members, int B) {
  MlpLayout L{};
  size_t off = 0;
  auto take = [&](size_t bytes) { size_t o = off; off += al256(bytes); return o; };
  const size_t P = (size_t)members * kPStride, MB = (size_t)members * B;
  L.master = take(P * 4);
  L.mom = take(P * 4);
  L.vel = take(P * 4);
  L.grad = take(P * 4);
  L.wbf = take(P * 2);
  L.xb = take(MB * kIn * 2);
  L.Z = take(3 * MB * kHid * 4);
  L.A = take(3 * MB * kHid * 2);
  L.y = take(MB * kOut * 4);
  L.dy = take(MB * kOut * 4);
  L.dyb = take(MB * kOut * 2);
  L.dzf = take(2 * MB * kHid * 4);
  L.dzb = take(2 * MB * kHid * 2);
  L.part = take((size_t)members * kRed * 4);
  L.inv = take((size_t)members * 4);
  L.loss = take((size_t)members * 4);
  L.total = off;
  return L;
}

int mfail(mlp_handle* h, int code, const std::string& msg) {
  if (h) h->err = msg;
  else g_mlp_error = msg;
  return code;
}
#define MHIP(h, expr, where)                                                                             \
  do {                                                                                                   \
    hipError_t e_ = (expr);                                                                              \
    if (e_ != hipSuccess) return mfail(h, -4, std::string(where) + ": " + hipGetErrorString(e_));        \
  } while (0)

// Staging of an operand X(row, k) = X[row * srow + k * sk] (member offsets
// zoff): 16-byte loads need a unit stride along k or along the rows, the other
// stride and the member offset in whole 8-element groups, and an aligned base.
int stage_mode(const __bf16* X, long long srow, long long sk, long long zoff) {
  const bool aligned = ((uintptr_t)X % 16) == 0 && zoff % 8 == 0;
  if (aligned && sk == 1 && srow % 8 == 0) return STAGE_K;
  if (aligned && srow == 1 && sk % 8 == 0) return STAGE_MN;
  return STAGE_ELEM;
}

// Member offsets of one product (elements): A, B, C (and Cb, Zp), bias.
struct ZStride {
  long long A = 0, B = 0, C = 0, bias = 0;
};

void gemm(hipStream_t st, const __bf16* A, long long sam, long long sak, const __bf16* B, long long sbk, long long sbn,
          int M, int N, int K, int epi, float* C, long long scm, __bf16* Cb, const float* bias, const float* Zp,
          int count = 1, ZStride zs = ZStride()) {
  Gemm g{A, sam, sak, B, sbk, sbn, M, N, K, epi, C, scm, Cb, bias, Zp, zs.A, zs.B, zs.C, zs.bias,
         stage_mode(A, sam, sak, zs.A), stage_mode(B, sbn, sbk, zs.B)};
  hipLaunchKernelGGL(k_gemm, dim3((N + TN - 1) / TN, (M + TM - 1) / TM, count), dim3(kThreads), 0, st, g);
}

// Forward of members k0 .. k0 + count - 1 on n inputs in h->xb (x_stride
// elements between the members' inputs: 0 when they share one input batch);
// outputs to y[count][n][2].
void forward(mlp_handle* h, int k0, int count, int n, long long x_stride, float* y) {
  const __bf16* W = h->wbf + (size_t)k0 * kPStride;
  const float* P = h->master + (size_t)k0 * kPStride;
  const long long act = (long long)n * kHid;
  const __bf16* a = h->xb;
  long long az = x_stride;
  int in = kIn;
  for (int l = 0; l < 3; ++l) {
    ZStride zs;
    zs.A = az;
    zs.B = kPStride;
    zs.C = act;
    zs.bias = kPStride;
    gemm(h->stream, a, in, 1, W + w_off(l), kHid, 1, n, kHid, in, EPI_BIAS_GELU, h->Z[l], kHid, h->A[l], P + b_off(l),
         nullptr, count, zs);
    a = h->A[l];
    az = act;
    in = kHid;
  }
  ZStride zs;
  zs.A = act;
  zs.B = kPStride;
  zs.C = (long long)n * kOut;
  zs.bias = kPStride;
  gemm(h->stream, a, kHid, 1, W + w_off(3), kOut, 1, n, kOut, kHid, EPI_BIAS, y, kOut, nullptr, P + b_off(3), nullptr,
       count, zs);
}

// Loss and gradient of members k0 .. k0 + count - 1 after forward() on their
// own inputs (h->xb, n apart), targets t and masks m [count][n][2]; gradients
// into h->grad of those members, losses into h->loss[0 .. count).
void backward(mlp_handle* h, int k0, int count, const float* t, const float* m, int n) {
  const __bf16* W = h->wbf + (size_t)k0 * kPStride;
  float* G = h->grad + (size_t)k0 * kPStride;
  const long long act = (long long)n * kHid;
  hipLaunchKernelGGL(k_mask_norm, dim3(count), dim3(kThreads), 0, h->stream, m, n * kOut, h->inv);
  hipLaunchKernelGGL(k_dy, dim3(kRed, count), dim3(kThreads), 0, h->stream, h->y, t, m, n * kOut, h->inv, h->dy, h->dyb,
                     h->part);
  hipLaunchKernelGGL(k_loss_final, dim3(count), dim3(kThreads), 0, h->stream, h->part, kRed, h->inv, h->loss);
  // layer l: dW = A_{l-1}^T dZ, db = column sums of dZ, dZ_{l-1} = (dZ W^T) . GELU'(Z_{l-1})
  const float* dzf = h->dy;
  const __bf16* dzb = h->dyb;
  int out = kOut;
  for (int l = 3; l >= 0; --l) {
    const int in = kDims[l];
    const __bf16* ain = l ? h->A[l - 1] : h->xb;
    ZStride zw;
    zw.A = (long long)n * in;
    zw.B = (long long)n * out;
    zw.C = kPStride;
    gemm(h->stream, ain, 1, in, dzb, out, 1, in, out, n, EPI_STORE, G + w_off(l), out, nullptr, nullptr, nullptr, count, zw);
    hipLaunchKernelGGL(k_colsum, dim3((out + kColW - 1) / kColW, count), dim3(kThreads), 0, h->stream, dzf, n, out, G + b_off(l));
    if (l > 0) {
      float* nf = h->dzf[l & 1];
      __bf16* nb = h->dzb[l & 1];
      ZStride zd;
      zd.A = (long long)n * out;
      zd.B = kPStride;
      zd.C = act;
      gemm(h->stream, dzb, out, 1, W + w_off(l), 1, out, n, in, out, EPI_DGELU, nf, in, nb, nullptr, h->Z[l - 1], count, zd);
      dzf = nf;
      dzb = nb;
      out = in;
    }
  }
}

// Adam step of members k0 .. k0 + count - 1 (their step counters advance).
void adam(mlp_handle* h, int k0, int count, float lr) {
  AdamCorr corr{};
  for (int k = 0; k < count; ++k) {
    const int t = ++h->adam_t[k0 + k];
    corr.c1[k] = 1.0f - std::pow(0.9f, (float)t);
    corr.c2[k] = 1.0f - std::pow(0.999f, (float)t);
  }
  const size_t o = (size_t)k0 * kPStride;
  hipLaunchKernelGGL(k_adam, dim3(nblk(kParams), count), dim3(kThreads), 0, h->stream, h->master + o, h->mom + o,
                     h->vel + o, (const float*)(h->grad + o), h->wbf + o, kParams, lr, corr);
}

// ------------------------------------------------------------------------
// Scratch of mlp_predict_ensemble_noalloc: the bfloat16 weights of every
// member, the bfloat16 inputs, one FP32 pre-activation buffer and two
// bfloat16 activation buffers (ping-pong between layers), and the members'
// outputs, for batches of up to kNoAllocMaxBatch samples and up to
// kNoAllocMaxMembers members.  One copy per device, held until the process
// ends; host code reaches it only through the address hipGetSymbolAddress
// returns on that device.
constexpr int kNoAllocMaxBatch = 1024, kNoAllocMaxMembers = 8, kMaxDevices = 64;
struct NoAllocLayout {
  static constexpr size_t wbf = 0;
  static constexpr size_t xb = wbf + ((size_t)kNoAllocMaxMembers * kPStride * 2 + 255) / 256 * 256;
  static constexpr size_t Z = xb + ((size_t)kNoAllocMaxBatch * kIn * 2 + 255) / 256 * 256;
  static constexpr size_t A = Z + (size_t)kNoAllocMaxBatch * kHid * 4;
  static constexpr size_t ys = A + 2 * (size_t)kNoAllocMaxBatch * kHid * 2;
  static constexpr size_t total = ys + (size_t)kNoAllocMaxMembers * kNoAllocMaxBatch * kOut * 4;
};
__device__ __attribute__((aligned(256))) unsigned char scratch[NoAllocLayout::total];

unsigned char* g_scratch_ptr[kMaxDevices] = {nullptr};

// Address of this device's scratch (looked up once per device, with that
// device current); nullptr with a message on failure.
unsigned char* scratch_on_device(int dev, std::string& why) {
  if (dev < 0 || dev >= kMaxDevices) { why = "device index beyond the supported range"; return nullptr; }
  unsigned char* p = __atomic_load_n(&g_scratch_ptr[dev], __ATOMIC_ACQUIRE);
  if (p) return p;
  void* q = nullptr;
  const hipError_t e = hipGetSymbolAddress(&q, HIP_SYMBOL(scratch));
  if (e != hipSuccess || !q) { why = std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e); return nullptr; }
  __atomic_store_n(&g_scratch_ptr[dev], (unsigned char*)q, __ATOMIC_RELEASE);
  return (unsigned char*)q;
}

int check(mlp_handle* h, int member, int n) {
  if (!h) return mfail(nullptr, -1, "null handle");
  if (member < 0 || member >= h->members) return mfail(h, -1, "member out of range");
  if (n <= 0 || n > h->max_batch) return mfail(h, -1, "n must lie in [1, max_batch]");
  return 0;
}

}  // namespace

extern "C" {

int32_t mlp_param_count(void) { return kParams; }

int mlp_required_bytes(int32_t members, int32_t max_batch, size_t* bytes) {
  if (!bytes || members <= 0 || members > 64 || max_batch <= 0 || max_batch > (1 << 22))
    return mfail(nullptr, -1, "members must lie in [1, 64] and max_batch in [1, 2^22]");
  *bytes = mlp_layout(members, max_batch).total;
  return 0;
}

int mlp_init(int32_t members, int32_t max_batch, void* dev_buf, size_t buf_bytes, void* hip_stream, mlp_handle** out) {
  if (!out) return mfail(nullptr, -1, "null output handle");
  *out = nullptr;
  size_t need = 0;
  int rc = mlp_required_bytes(members, max_batch, &need);
  if (rc) return rc;
  int dev = 0;
  hipDeviceProp_t prop;
  if (hipGetDevice(&dev) != hipSuccess || hipGetDeviceProperties(&prop, dev) != hipSuccess ||
      std::strncmp(prop.gcnArchName, "gfx950", 6) != 0)
    return mfail(nullptr, -4, "no gfx950 device");
  mlp_handle* h = new mlp_handle();
  h->members = members;
  h->max_batch = max_batch;
  if (dev_buf) {
    if (buf_bytes < need || ((uintptr_t)dev_buf & 255)) { delete h; return mfail(nullptr, -1, "dev_buf too small or not 256-byte aligned"); }
    h->buf = dev_buf;
  } else {
    if (hipMalloc(&h->buf, need) != hipSuccess) { delete h; return mfail(nullptr, -3, "hipMalloc failed"); }
    h->own_buf = true;
  }
  if (hip_stream) h->stream = (hipStream_t)hip_stream;
  else {
    if (hipStreamCreate(&h->stream) != hipSuccess) {
      if (h->own_buf) (void)hipFree(h->buf);
      delete h;
      return mfail(nullptr, -4, "hipStreamCreate failed");
    }
    h->own_stream = true;
  }
  const MlpLayout L = mlp_layout(members, max_batch);
  char* b = (char*)h->buf;
  const size_t MB = (size_t)members * max_batch;
  h->master = (float*)(b + L.master);
  h->mom = (float*)(b + L.mom);
  h->vel = (float*)(b + L.vel);
  h->grad = (float*)(b + L.grad);
  h->wbf = (__bf16*)(b + L.wbf);
  h->xb = (__bf16*)(b + L.xb);
  for (int l = 0; l < 3; ++l) {
    h->Z[l] = (float*)(b + L.Z) + l * MB * kHid;
    h->A[l] = (__bf16*)(b + L.A) + l * MB * kHid;
  }
  h->y = (float*)(b + L.y);
  h->dy = (float*)(b + L.dy);
  h->dyb = (__bf16*)(b + L.dyb);
  for (int k = 0; k < 2; ++k) {
    h->dzf[k] = (float*)(b + L.dzf) + k * MB * kHid;
    h->dzb[k] = (__bf16*)(b + L.dzb) + k * MB * kHid;
  }
  h->part = (float*)(b + L.part);
  h->inv = (float*)(b + L.inv);
  h->loss = (float*)(b + L.loss);
  h->adam_t.assign(members, 0);
  hipError_t e = hipMemsetAsync(h->buf, 0, L.xb, h->stream);   // parameters, moments, gradients, bf16 copies
  if (e == hipSuccess) e = hipStreamSynchronize(h->stream);
  if (e != hipSuccess) {
    mlp_destroy(h);
    return mfail(nullptr, -4, std::string("initialisation: ") + hipGetErrorString(e));
  }
  *out = h;
  return 0;
}

int mlp_set_params(mlp_handle* h, int32_t member, const float* params_host) {
  int rc = check(h, member, 1);
  if (rc) return rc;
  if (!params_host) return mfail(h, -1, "null parameters");
  const size_t o = (size_t)member * kPStride;
  MHIP(h, hipMemcpyAsync(h->master + o, params_host, kParams * 4, hipMemcpyHostToDevice, h->stream), "copy parameters");
  MHIP(h, hipMemsetAsync(h->mom + o, 0, kParams * 4, h->stream), "reset moments");
  MHIP(h, hipMemsetAsync(h->vel + o, 0, kParams * 4, h->stream), "reset moments");
  hipLaunchKernelGGL(k_cast_bf16, dim3(nblk(kParams)), dim3(kThreads), 0, h->stream, h->master + o, h->wbf + o, kParams);
  MHIP(h, hipGetLastError(), "cast kernel");
  MHIP(h, hipStreamSynchronize(h->stream), "synchronise");
  h->adam_t[member] = 0;
  return 0;
}

int mlp_get_params(mlp_handle* h, int32_t member, float* params_host) {
  int rc = check(h, member, 1);
  if (rc) return rc;
  if (!params_host) return mfail(h, -1, "null parameters");
  MHIP(h, hipMemcpyAsync(params_host, h->master + (size_t)member * kPStride, kParams * 4, hipMemcpyDeviceToHost, h->stream), "copy parameters");
  MHIP(h, hipStreamSynchronize(h->stream), "synchronise");
  return 0;
}

int mlp_forward(mlp_handle* h, int32_t member, const float* x_dev, int32_t n, float* y_dev) {
  int rc = check(h, member, n);
  if (rc) return rc;
  if (!x_dev || !y_dev) return mfail(h, -1, "null argument");
  hipLaunchKernelGGL(k_cast_bf16, dim3(nblk((long long)n * kIn)), dim3(kThreads), 0, h->stream, x_dev, h->xb, n * kIn);
  forward(h, member, 1, n, 0, y_dev);
  MHIP(h, hipGetLastError(), "forward kernels");
  return 0;
}

int mlp_loss_grad(mlp_handle* h, int32_t member, const float* x_dev, const float* t_dev, const float* m_dev, int32_t n,
                  float* loss_host, float* grad_host) {
  int rc = check(h, member, n);
  if (rc) return rc;
  if (!x_dev || !t_dev || !m_dev) return mfail(h, -1, "null argument");
  hipLaunchKernelGGL(k_cast_bf16, dim3(nblk((long long)n * kIn)), dim3(kThreads), 0, h->stream, x_dev, h->xb, n * kIn);
  forward(h, member, 1, n, 0, h->y);
  backward(h, member, 1, t_dev, m_dev, n);
  MHIP(h, hipGetLastError(), "training kernels");
  if (loss_host) MHIP(h, hipMemcpyAsync(loss_host, h->loss, 4, hipMemcpyDeviceToHost, h->stream), "copy loss");
  if (grad_host)
    MHIP(h, hipMemcpyAsync(grad_host, h->grad + (size_t)member * kPStride, kParams * 4, hipMemcpyDeviceToHost, h->stream), "copy gradient");
  MHIP(h, hipStreamSynchronize(h->stream), "synchronise");
  return 0;
}

int mlp_train_step(mlp_handle* h, int32_t member, const float* x_dev, const float* t_dev, const float* m_dev, int32_t n,
                   float lr, float* loss_host) {
  int rc = check(h, member, n);
  if (rc) return rc;
  if (!x_dev || !t_dev || !m_dev || !(lr > 0.f)) return mfail(h, -1, "null argument or non-positive rate");
  hipLaunchKernelGGL(k_cast_bf16, dim3(nblk((long long)n * kIn)), dim3(kThreads), 0, h->stream, x_dev, h->xb, n * kIn);
  forward(h, member, 1, n, 0, h->y);
  backward(h, member, 1, t_dev, m_dev, n);
  adam(h, member, 1, lr);
  MHIP(h, hipGetLastError(), "training kernels");
  if (loss_host) {
    MHIP(h, hipMemcpyAsync(loss_host, h->loss, 4, hipMemcpyDeviceToHost, h->stream), "copy loss");
    MHIP(h, hipStreamSynchronize(h->stream), "synchronise");
  }
  return 0;
}

int mlp_train_step_ensemble(mlp_handle* h, const float* x_dev, const float* t_dev, const float* m_dev, int32_t n, float lr,
                            float* loss_host) {
  int rc = check(h, 0, n);
  if (rc) return rc;
  if (!x_dev || !t_dev || !m_dev || !(lr > 0.f)) return mfail(h, -1, "null argument or non-positive rate");
  const int M = h->members;
  hipLaunchKernelGGL(k_cast_bf16, dim3(nblk((long long)M * n * kIn)), dim3(kThreads), 0, h->stream, x_dev, h->xb,
                     M * n * kIn);
  forward(h, 0, M, n, (long long)n * kIn, h->y);
  backward(h, 0, M, t_dev, m_dev, n);
  adam(h, 0, M, lr);
  MHIP(h, hipGetLastError(), "training kernels");
  if (loss_host) {
    MHIP(h, hipMemcpyAsync(loss_host, h->loss, 4 * (size_t)M, hipMemcpyDeviceToHost, h->stream), "copy losses");
    MHIP(h, hipStreamSynchronize(h->stream), "synchronise");
  }
  return 0;
}

int mlp_predict_ensemble(mlp_handle* h, const float* x_dev, int32_t n, float* mean_dev, float* std_dev) {
  int rc = check(h, 0, n);
  if (rc) return rc;
  if (!x_dev || !mean_dev || !std_dev) return mfail(h, -1, "null argument");
  hipLaunchKernelGGL(k_cast_bf16, dim3(nblk((long long)n * kIn)), dim3(kThreads), 0, h->stream, x_dev, h->xb, n * kIn);
  forward(h, 0, h->members, n, 0, h->y);
  hipLaunchKernelGGL(k_ens, dim3(nblk((long long)n * kOut)), dim3(kThreads), 0, h->stream, (const float*)h->y, h->members,
                     n * kOut, mean_dev, std_dev);
  MHIP(h, hipGetLastError(), "ensemble kernels");
  return 0;
}

int mlp_predict_ensemble_noalloc(const float* params_dev, int32_t members, const float* x_dev, int32_t n,
                                 float* mean_dev, float* std_dev, void* hip_stream) {
  if (!params_dev || !x_dev || !mean_dev || !std_dev) return mfail(nullptr, -1, "null argument");
  if (members < 1 || members > kNoAllocMaxMembers)
    return mfail(nullptr, -1, "members must lie in [1, " + std::to_string(kNoAllocMaxMembers) + "] without allocation");
  if (n < 1 || n > kNoAllocMaxBatch)
    return mfail(nullptr, -1, "n must lie in [1, " + std::to_string(kNoAllocMaxBatch) + "] without allocation");
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) return mfail(nullptr, -4, "hipGetDevice failed");
  std::string why;
  unsigned char* sp = scratch_on_device(dev, why);
  if (!sp) return mfail(nullptr, -4, why);
  const hipStream_t st = (hipStream_t)hip_stream;
  __bf16* wbf = (__bf16*)(sp + NoAllocLayout::wbf);
  __bf16* xb = (__bf16*)(sp + NoAllocLayout::xb);
  float* Z = (float*)(sp + NoAllocLayout::Z);
  __bf16* A[2] = {(__bf16*)(sp + NoAllocLayout::A), (__bf16*)(sp + NoAllocLayout::A) + (size_t)kNoAllocMaxBatch * kHid};
  float* ys = (float*)(sp + NoAllocLayout::ys);
  // every scratch element read below is written first in the same call
  for (int k = 0; k < members; ++k)   // the caller's parameters are kParams apart, the bfloat16 copies kPStride
    hipLaunchKernelGGL(k_cast_bf16, dim3(nblk(kParams)), dim3(kThreads), 0, st, params_dev + (size_t)k * kParams,
                       wbf + (size_t)k * kPStride, kParams);
  hipLaunchKernelGGL(k_cast_bf16, dim3(nblk((long long)n * kIn)), dim3(kThreads), 0, st, x_dev, xb, n * kIn);
  for (int k = 0; k < members; ++k) {
    const __bf16* W = wbf + (size_t)k * kPStride;
    const float* P = params_dev + (size_t)k * kParams;
    const __bf16* a = xb;
    int in = kIn;
    for (int l = 0; l < 3; ++l) {
      gemm(st, a, in, 1, W + w_off(l), kHid, 1, n, kHid, in, EPI_BIAS_GELU, Z, kHid, A[l & 1], P + b_off(l), nullptr);
      a = A[l & 1];
      in = kHid;
    }
    gemm(st, a, kHid, 1, W + w_off(3), kOut, 1, n, kOut, kHid, EPI_BIAS, ys + (size_t)k * n * kOut, kOut, nullptr,
         P + b_off(3), nullptr);
  }
  hipLaunchKernelGGL(k_ens, dim3(nblk((long long)n * kOut)), dim3(kThreads), 0, st, (const float*)ys, members, n * kOut,
                     mean_dev, std_dev);
  const hipError_t e = hipGetLastError();
  if (e != hipSuccess) return mfail(nullptr, -4, std::string("ensemble kernels: ") + hipGetErrorString(e));
  return 0;
}

int mlp_destroy(mlp_handle* h) {
  if (!h) return 0;
  if (h->stream) (void)hipStreamSynchronize(h->stream);
  if (h->own_buf && h->buf) (void)hipFree(h->buf);
  if (h->own_stream && h->stream) (void)hipStreamDestroy(h->stream);
  delete h;
  return 0;
}

const char* mlp_last_error(const mlp_handle* h) { return h ? h->err.c_str() : g_mlp_error.c_str(); }

}  // extern "C"
