// Learned initial guess for the Landau-frame solve (not part of the paper's
// method): a 9 -> 64 -> 64 -> 64 -> 3 SiLU perceptron from the nine moments
// of a site divided by N^0 to (eps/N^0, u_x, u_y).  float32 master weights,
// bfloat16 roundings of them in every product, float32 accumulation.
//
// Training kernels (this file) work on float32 activations; the in-step
// inference (rlbm_lib.hip) uses matrix-core products on bfloat16 operands,
// with the weights re-packed here into the per-lane fragment order of the
// 32x32x16 bf16 matrix instruction.
#include <hip/hip_runtime.h>
#include <stdio.h>
#include <string.h>

#include <cmath>
#include <vector>

#include "../../include/rlbm.h"
#include "rlbm_mlp.h"
#include "rlbm_stencil.h"

namespace rlbm_mlp_k {

constexpr int kT = 256;

__device__ __forceinline__ float bf16_round(float x) {
  unsigned u = __float_as_uint(x);
  u = (u + 0x7FFFu + ((u >> 16) & 1u)) & 0xFFFF0000u;
  return __uint_as_float(u);
}

__device__ __forceinline__ float silu(float z) { return z / (1.0f + expf(-z)); }
__device__ __forceinline__ float dsilu(float z) {
  const float s = 1.0f / (1.0f + expf(-z));
  return s * (1.0f + z * (1.0f - s));
}

// bf[i] = bf16(master[i])
__global__ void k_round(const float* __restrict__ master, float* __restrict__ bf, int n) {
  const int i = blockIdx.x * kT + threadIdx.x;
  if (i < n) bf[i] = bf16_round(master[i]);
}

// standardised inputs and targets: x = (raw/raw0 - mx)/sx, y = ((eps/N0, ux, uy) - my)/sy
__global__ void k_standardise(const float* __restrict__ raw9, const float* __restrict__ target, int B,
                              const float* __restrict__ norm, float* __restrict__ X, float* __restrict__ Y) {
  const int b = blockIdx.x * kT + threadIdx.x;
  if (b >= B) return;
  const float n0 = raw9[b * 9];
  for (int i = 0; i < 9; ++i) X[b * 9 + i] = (raw9[b * 9 + i] / n0 - norm[i]) / norm[9 + i];
  if (target) {
    const float y[3] = {target[b * 3] / n0, target[b * 3 + 1], target[b * 3 + 2]};
    for (int o = 0; o < 3; ++o) Y[b * 3 + o] = (y[o] - norm[18 + o]) / norm[21 + o];
  }
}

// z = A W^T + b, a = silu(z) (or a = z on the output layer); one thread per (b, o)
__global__ void k_fwd(const float* __restrict__ A, int nin, const float* __restrict__ W, const float* __restrict__ bias,
                      int nout, int B, int act, float* __restrict__ Z, float* __restrict__ Aout) {
  const int t = blockIdx.x * kT + threadIdx.x;
  if (t >= B * nout) return;
  const int b = t / nout, o = t - b * nout;
  float s = bias[o];
  for (int i = 0; i < nin; ++i) s = fmaf(A[b * nin + i], W[o * nin + i], s);
  Z[t] = s;
  Aout[t] = act ? silu(s) : s;
}

// output-layer error d = 2 (out - y)/(3B) and the loss sum
__global__ void k_loss(const float* __restrict__ out, const float* __restrict__ Y, int B, float* __restrict__ d,
                       float* __restrict__ loss) {
  const int t = blockIdx.x * kT + threadIdx.x;
  float e = 0.0f;
  if (t < B * 3) {
    const float r = out[t] - Y[t];
    d[t] = 2.0f * r / (3.0f * B);
    e = r * r;
  }
  for (int off = 32; off > 0; off >>= 1) e += __shfl_xor(e, off);
  if ((threadIdx.x & 63) == 0 && e != 0.0f) atomicAdd(loss, e / (3.0f * B));
}

// dprev[b][i] = (sum_o d[b][o] W[o][i]) silu'(zprev[b][i])
__global__ void k_bwd_act(const float* __restrict__ d, int nout, const float* __restrict__ W, int nin,
                          const float* __restrict__ zprev, int B, float* __restrict__ dprev) {
  const int t = blockIdx.x * kT + threadIdx.x;
  if (t >= B * nin) return;
  const int b = t / nin, i = t - b * nin;
  float s = 0.0f;
  for (int o = 0; o < nout; ++o) s = fmaf(d[b * nout + o], W[o * nin + i], s);
  dprev[t] = s * dsilu(zprev[t]);
}

// Weight gradients gW[o][i] = sum_b d[b][o] a[b][i], gb[o] = sum_b d[b][o],
// in two deterministic passes: each workgroup stages a chunk of kChunk batch
// rows of d and a in LDS and writes the chunk's partial sums for every
// (o, i) (i = nin: the bias); a second pass adds the chunks in order.
constexpr int kChunk = 64;
constexpr int kMaxUnits = 64;

__global__ void __launch_bounds__(kT) k_bwd_w_part(const float* __restrict__ d, int nout, const float* __restrict__ A,
                                                   int nin, int B, float* __restrict__ part) {
  __shared__ float ds[kChunk][kMaxUnits];
  __shared__ float as[kChunk][kMaxUnits + 1];
  const int b0 = blockIdx.x * kChunk;
  const int rows = min(kChunk, B - b0);
  for (int e = threadIdx.x; e < kChunk * kMaxUnits; e += kT) {
    const int r = e / kMaxUnits, c = e - r * kMaxUnits;
    ds[r][c] = (r < rows && c < nout) ? d[(long long)(b0 + r) * nout + c] : 0.0f;
    as[r][c] = (r < rows && c < nin) ? A[(long long)(b0 + r) * nin + c] : 0.0f;
  }
  for (int r = threadIdx.x; r < kChunk; r += kT) as[r][kMaxUnits] = r < rows ? 1.0f : 0.0f;
  __syncthreads();
  const int nel = nout * (nin + 1);
  float* out = part + (long long)blockIdx.x * kMaxUnits * (kMaxUnits + 1);
  for (int t = threadIdx.x; t < nel; t += kT) {
    const int o = t / (nin + 1), i = t - o * (nin + 1);
    const int col = i < nin ? i : kMaxUnits;  // the bias column holds ones
    float s = 0.0f;
#pragma unroll 16
    for (int r = 0; r < kChunk; ++r) s = fmaf(ds[r][o], as[r][col], s);
    out[t] = s;
  }
}

__global__ void __launch_bounds__(kT) k_bwd_w_sum(const float* __restrict__ part, int chunks, int nout, int nin,
                                                  float* __restrict__ gW, float* __restrict__ gb) {
  const int t = blockIdx.x * kT + threadIdx.x;
  if (t >= nout * (nin + 1)) return;
  float s = 0.0f;
  for (int c = 0; c < chunks; ++c) s += part[(long long)c * kMaxUnits * (kMaxUnits + 1) + t];
  const int o = t / (nin + 1), i = t - o * (nin + 1);
  if (i < nin)
    gW[o * nin + i] = s;
  else
    gb[o] = s;
}

__global__ void k_adam(float* __restrict__ p, const float* __restrict__ g, float* __restrict__ m, float* __restrict__ v,
                       int n, float lr, float c1, float c2) {
  const int i = blockIdx.x * kT + threadIdx.x;
  if (i >= n) return;
  const float gi = g[i];
  const float mi = 0.9f * m[i] + 0.1f * gi;
  const float vi = 0.999f * v[i] + 0.001f * gi * gi;
  m[i] = mi;
  v[i] = vi;
  p[i] -= lr * (mi / c1) / (sqrtf(vi / c2) + 1e-8f);
}

// de-standardised prediction (eps, ux, uy) with eps = (eps/N0) N0
__global__ void k_output(const float* __restrict__ out, const float* __restrict__ raw9, int B,
                         const float* __restrict__ norm, float* __restrict__ pred) {
  const int b = blockIdx.x * kT + threadIdx.x;
  if (b >= B) return;
  const float n0 = raw9[b * 9];
  pred[b * 3] = (out[b * 3] * norm[21] + norm[18]) * n0;
  pred[b * 3 + 1] = out[b * 3 + 1] * norm[22] + norm[19];
  pred[b * 3 + 2] = out[b * 3 + 2] * norm[23] + norm[20];
}

// Fragments of the 32x32x16 bf16 matrix product for the in-step inference:
// for output tile m, k-step s and lane l (half h = l / 32), the eight values
// W[32 m + l % 32][c(e)], e = 0..7, zero outside W.  The first layer takes its
// inputs in natural order, c = 8 h + e.  The hidden and output layers take
// them in the order in which the previous layer's accumulators hold them:
// register r of output tile m' carries unit 32 m' + 8 (r / 4) + 4 h + r % 4,
// so k-step s is made of registers 8 (s % 2) .. 8 (s % 2) + 7 of tile s / 2
// and c = 16 s + 8 (e / 4) + 4 h + e % 4.  The product sums over k, so any
// order shared by both operands gives the same result.
__global__ void k_pack(const float* __restrict__ master, unsigned short* __restrict__ frag,
                       float* __restrict__ biasfrag) {
  const int l = threadIdx.x;  // 64 lanes, one block per (layer, tile, kstep) item
  const int h = l >> 5;
  int item = blockIdx.x;
  for (int L = 0; L < 4; ++L) {
    const int nin = RLBM_MLP_IN[L], nout = RLBM_MLP_OUT[L];
    const int tiles = RLBM_MLP_TILES[L], ks = RLBM_MLP_KSTEPS[L];
    const int n = tiles * ks;
    if (item < n) {
      const int m = item / ks, s = item - m * ks;
      const float* W = master + RLBM_MLP_WOFF[L];
      const int row = 32 * m + (l & 31);
      for (int e = 0; e < 8; ++e) {
        const int col = L == 0 ? 8 * h + e : 16 * s + 8 * (e >> 2) + 4 * h + (e & 3);
        const float w = (row < nout && col < nin) ? W[row * nin + col] : 0.0f;
        const unsigned u = __float_as_uint(w);
        frag[((size_t)(RLBM_MLP_FOFF[L] + item) * 64 + l) * 8 + e] =
            (unsigned short)(((u + 0x7FFFu + ((u >> 16) & 1u)) >> 16) & 0xFFFFu);
      }
      if (s == 0) {
        const float* b = master + RLBM_MLP_BOFF[L];
        for (int r = 0; r < 16; ++r) {
          const int unit = 32 * m + 8 * (r >> 2) + 4 * (l >> 5) + (r & 3);
          biasfrag[((size_t)(RLBM_MLP_BFOFF[L] + m) * 64 + l) * 16 + r] = unit < nout ? b[unit] : 0.0f;
        }
      }
      return;
    }
    item -= n;
  }
}

}  // namespace rlbm_mlp_k

using namespace rlbm_mlp_k;

static int mfail(const char* msg) {
  rlbm_set_global_error(msg);
  return RLBM_EINVAL;
}

#define MHIP(call)                                                                   \
  do {                                                                               \
    hipError_t e_ = (call);                                                          \
    if (e_ != hipSuccess) {                                                          \
      char b_[256];                                                                  \
      snprintf(b_, sizeof(b_), "HIP error: %s", hipGetErrorString(e_));              \
      rlbm_set_global_error(b_);                                                     \
      return RLBM_EHIP;                                                              \
    }                                                                                \
  } while (0)

static dim3 grid_of(long long n) { return dim3((unsigned)((n + kT - 1) / kT)); }

extern "C" int rlbm_mlp_create(rlbm_mlp** out, const float* params, const float* norm, int max_batch) {
  if (!out || !params || !norm || max_batch <= 0) return mfail("rlbm_mlp_create: invalid argument");
  *out = nullptr;
  rlbm_mlp* m = new rlbm_mlp();
  m->max_batch = max_batch;
  size_t P = RLBM_MLP_NPARAM;
  size_t act = (size_t)max_batch * 64;
  float* p = nullptr;
  size_t total = 5 * P + 24 + 2 * (size_t)max_batch * 9 + 2 * (size_t)max_batch * 3 + 6 * act + 1;
  if (hipMalloc((void**)&p, total * sizeof(float)) != hipSuccess) {
    delete m;
    return mfail("rlbm_mlp_create: device allocation failed");
  }
  m->base = p;
  m->master = p; p += P;
  m->bf = p; p += P;
  m->grad = p; p += P;
  m->mom1 = p; p += P;
  m->mom2 = p; p += P;
  m->norm = p; p += 24;
  m->X = p; p += (size_t)max_batch * 9;
  m->Xraw = p; p += (size_t)max_batch * 9;
  m->Y = p; p += (size_t)max_batch * 3;
  m->D4 = p; p += (size_t)max_batch * 3;
  for (int L = 0; L < 3; ++L) {
    m->Z[L] = p; p += act;
    m->A[L] = p; p += act;
  }
  m->loss = p; p += 1;
  if (hipMalloc((void**)&m->frag, sizeof(unsigned short) * 8 * RLBM_MLP_NFRAG * 64) != hipSuccess ||
      hipMalloc((void**)&m->biasfrag, sizeof(float) * 16 * RLBM_MLP_NBFRAG * 64) != hipSuccess ||
      hipMalloc((void**)&m->Z4, sizeof(float) * 3 * (size_t)max_batch) != hipSuccess ||
      hipMalloc((void**)&m->D[0], sizeof(float) * 3 * act) != hipSuccess ||
      hipMalloc((void**)&m->part, sizeof(float) * (size_t)((max_batch + kChunk - 1) / kChunk) * kMaxUnits *
                                      (kMaxUnits + 1)) != hipSuccess) {
    rlbm_mlp_destroy(m);
    return mfail("rlbm_mlp_create: device allocation failed");
  }
  m->D[1] = m->D[0] + act;
  m->D[2] = m->D[1] + act;
  MHIP(hipMemcpy(m->master, params, P * sizeof(float), hipMemcpyHostToDevice));
  MHIP(hipMemset(m->mom1, 0, 2 * P * sizeof(float)));
  MHIP(hipMemcpy(m->norm, norm, 24 * sizeof(float), hipMemcpyHostToDevice));
  memcpy(m->h_norm, norm, sizeof(m->h_norm));
  int rc = rlbm_mlp_refresh(m, nullptr);
  if (rc) return rc;
  MHIP(hipDeviceSynchronize());
  *out = m;
  return RLBM_OK;
}

int rlbm_mlp_refresh(rlbm_mlp* m, hipStream_t s) {
  hipLaunchKernelGGL(k_round, grid_of(RLBM_MLP_NPARAM), dim3(kT), 0, s, m->master, m->bf, RLBM_MLP_NPARAM);
  hipLaunchKernelGGL(k_pack, dim3(RLBM_MLP_NFRAG), dim3(64), 0, s, m->master, m->frag, m->biasfrag);
  MHIP(hipGetLastError());
  return RLBM_OK;
}

extern "C" int rlbm_mlp_destroy(rlbm_mlp* m) {
  if (!m) return RLBM_OK;
  (void)hipDeviceSynchronize();
  if (m->base) (void)hipFree(m->base);
  if (m->frag) (void)hipFree(m->frag);
  if (m->biasfrag) (void)hipFree(m->biasfrag);
  if (m->Z4) (void)hipFree(m->Z4);
  if (m->D[0]) (void)hipFree(m->D[0]);
  if (m->part) (void)hipFree(m->part);
  delete m;
  return RLBM_OK;
}

// forward pass on m->X (standardised), float32 activations, bf16 weights
static void forward(rlbm_mlp* m, int B, hipStream_t s) {
  const float* a = m->X;
  for (int L = 0; L < 4; ++L) {
    const int nin = RLBM_MLP_IN[L], nout = RLBM_MLP_OUT[L];
    float* Z = L < 3 ? m->Z[L] : m->Z4;
    float* A = L < 3 ? m->A[L] : m->Z4;
    hipLaunchKernelGGL(k_fwd, grid_of((long long)B * nout), dim3(kT), 0, s, a, nin, m->bf + RLBM_MLP_WOFF[L],
                       m->bf + RLBM_MLP_BOFF[L], nout, B, L < 3 ? 1 : 0, Z, A);
    a = A;
  }
}

extern "C" int rlbm_mlp_train_step(rlbm_mlp* m, const float* raw9, const float* target, int B, float lr, float* loss,
                                   void* stream) {
  if (!m || !raw9 || !target || B <= 0 || B > m->max_batch) return mfail("rlbm_mlp_train_step: invalid argument");
  hipStream_t s = (hipStream_t)stream;
  hipLaunchKernelGGL(k_standardise, grid_of(B), dim3(kT), 0, s, raw9, target, B, m->norm, m->X, m->Y);
  forward(m, B, s);
  MHIP(hipMemsetAsync(m->loss, 0, sizeof(float), s));
  hipLaunchKernelGGL(k_loss, grid_of((long long)B * 3), dim3(kT), 0, s, m->Z4, m->Y, B, m->D4, m->loss);
  // backward: d = dL/dz of layer L
  const float* d = m->D4;
  for (int L = 3; L >= 0; --L) {
    const int nin = RLBM_MLP_IN[L], nout = RLBM_MLP_OUT[L];
    const float* Aprev = L > 0 ? m->A[L - 1] : m->X;
    const int chunks = (B + kChunk - 1) / kChunk;
    hipLaunchKernelGGL(k_bwd_w_part, dim3(chunks), dim3(kT), 0, s, d, nout, Aprev, nin, B, m->part);
    hipLaunchKernelGGL(k_bwd_w_sum, grid_of((long long)nout * (nin + 1)), dim3(kT), 0, s, m->part, chunks, nout,
                       nin, m->grad + RLBM_MLP_WOFF[L], m->grad + RLBM_MLP_BOFF[L]);
    if (L > 0) {
      hipLaunchKernelGGL(k_bwd_act, grid_of((long long)B * nin), dim3(kT), 0, s, d, nout, m->bf + RLBM_MLP_WOFF[L],
                         nin, m->Z[L - 1], B, m->D[L - 1]);
      d = m->D[L - 1];
    }
  }
  m->t += 1;
  const float c1 = 1.0f - powf(0.9f, (float)m->t), c2 = 1.0f - powf(0.999f, (float)m->t);
  hipLaunchKernelGGL(k_adam, grid_of(RLBM_MLP_NPARAM), dim3(kT), 0, s, m->master, m->grad, m->mom1, m->mom2,
                     RLBM_MLP_NPARAM, lr, c1, c2);
  int rc = rlbm_mlp_refresh(m, s);
  if (rc) return rc;
  MHIP(hipGetLastError());
  if (loss) {
    MHIP(hipMemcpyAsync(loss, m->loss, sizeof(float), hipMemcpyDeviceToHost, s));
    MHIP(hipStreamSynchronize(s));
  }
  return RLBM_OK;
}

extern "C" int rlbm_mlp_predict(rlbm_mlp* m, const float* raw9, int B, float* pred, void* stream) {
  if (!m || !raw9 || !pred || B <= 0 || B > m->max_batch) return mfail("rlbm_mlp_predict: invalid argument");
  hipStream_t s = (hipStream_t)stream;
  hipLaunchKernelGGL(k_standardise, grid_of(B), dim3(kT), 0, s, raw9, (const float*)nullptr, B, m->norm, m->X,
                     (float*)nullptr);
  forward(m, B, s);
  hipLaunchKernelGGL(k_output, grid_of(B), dim3(kT), 0, s, m->Z4, raw9, B, m->norm, pred);
  MHIP(hipGetLastError());
  return RLBM_OK;
}

extern "C" int rlbm_mlp_get_params(rlbm_mlp* m, float* params, float* grads) {
  if (!m) return mfail("rlbm_mlp_get_params: NULL");
  MHIP(hipDeviceSynchronize());
  if (params) MHIP(hipMemcpy(params, m->master, sizeof(float) * RLBM_MLP_NPARAM, hipMemcpyDeviceToHost));
  if (grads) MHIP(hipMemcpy(grads, m->grad, sizeof(float) * RLBM_MLP_NPARAM, hipMemcpyDeviceToHost));
  return RLBM_OK;
}
