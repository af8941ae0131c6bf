// The learned proposal's network outside the sampler: a forward pass in the
// sampler's precision (same device code) and the training step.
//
// Training minimises the mean over rows of -log q_re(t_re) - log q_im(t_im),
// where q_p is the learned proposal of one axis of one antenna: the
// discretised Gaussian over the levels j = 0..Q-1 with natural-log logits
// -kl (j - ml)^2, ml = mu_p + D_p, kl = kappa 2^clamp(b_p, -4, 4), (D_re, D_im,
// b_re, b_im) = network(features).  Derivatives of one axis' term:
//   d/d ml = -2 kl (t - E_q[j]),   d/d kl = (t - ml)^2 - E_q[(j - ml)^2],
//   d/d b  = kl ln 2 * d/d kl inside the clamp, 0 outside.
// The training network is float32 without rounding.  Three kernels:
//   rows:    one thread per row: forward, loss, output gradient, backward to
//            the hidden layers; stores the activations and deltas it needs;
//   partial: per chunk of 256 rows, one wavefront forms the weight gradients
//            dW = sum_r delta_r a_r^T on the matrix cores (float32 16x16x4
//            MFMAs, the rows as the K dimension; a column of ones in the B
//            operand gives the biases) and sums the loss;
//   adam:    one thread per parameter sums the chunks in order and updates
//            the parameter and the two moment estimates (Adam, Kingma & Ba).
// No atomics: the result does not depend on scheduling.
#include <cmath>

#include "../../include/dmala.h"
#include "common.hpp"
#include "host.hpp"
#include "mlp_device.hpp"

namespace dmala {

static_assert(kMlpParams == DMALA_MLP_PARAMS, "parameter count");
static_assert(kTrainRow == DMALA_TRAIN_ROW, "training row size");

// --------------------------------------------------------------- inference

__global__ __launch_bounds__(256) void mlp_forward_kernel(const float* __restrict__ w, const float* __restrict__ rows,
                                                          int n, int stride, float* __restrict__ out) {
  extern __shared__ __attribute__((aligned(16))) unsigned char lds[];
  mlp_stage<false>(w, lds);
  __syncthreads();
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int row = (blockIdx.x * 4 + wave) * 64 + (lane >> 4) * 16 + (lane & 15);
  float f[kMlpIn];
#pragma unroll
  for (int i = 0; i < kMlpIn; ++i) f[i] = row < n ? rows[(size_t)row * stride + i] : 0.f;
  const mlp_f32x4 o = mlp_eval4<false>(lds, 0u, mlp_inputs(f[0], f[1], f[2], f[3], f[4], f[5], f[6]));
  if (row < n) {
#pragma unroll
    for (int i = 0; i < kMlpOut; ++i) out[(size_t)row * kMlpOut + i] = o[i];
  }
}

// --------------------------------------------------------------- training

// Per-row workspace record (floats): a0[8] (inputs and the constant 1), a1[64], a2[64], d1[64], d2[64],
// dout[4], loss[1], 1 pad.
constexpr int kRecA0 = 0, kRecA1 = 8, kRecA2 = 72, kRecD1 = 136, kRecD2 = 200, kRecDo = 264, kRecL = 268;
constexpr int kRec = 272;
constexpr int kChunk = 256;  // rows per partial sum (one wavefront)

__global__ __launch_bounds__(256) void mlp_rows_kernel(const float* __restrict__ w, const float* __restrict__ rows,
                                                       const int32_t* __restrict__ tgt, int n, float inv_n,
                                                       float* __restrict__ rec) {
  __shared__ float W[kMlpParams];
  for (int i = threadIdx.x; i < kMlpParams; i += blockDim.x) W[i] = w[i];
  __syncthreads();
  const int r = blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= n) return;
  const float* row = rows + (size_t)r * kTrainRow;
  float* o = rec + (size_t)r * kRec;
  float x[kMlpIn];
#pragma unroll
  for (int i = 0; i < kMlpIn; ++i) { x[i] = row[i]; o[kRecA0 + i] = x[i]; }
  o[kRecA0 + 7] = 1.f;
  float a1[kMlpHid];
  uint64_t m1 = 0, m2 = 0;
#pragma unroll
  for (int j = 0; j < kMlpHid; ++j) {
    float z = W[kOffB1 + j];
#pragma unroll
    for (int i = 0; i < kMlpIn; ++i) z = fmaf(W[kOffW1 + j * kMlpIn + i], x[i], z);
    m1 |= (z > 0.f ? 1ull : 0ull) << j;
    a1[j] = fmaxf(z, 0.f);
    o[kRecA1 + j] = a1[j];
  }
  float out[kMlpOut];
#pragma unroll
  for (int k = 0; k < kMlpOut; ++k) out[k] = W[kOffB3 + k];
#pragma unroll
  for (int j = 0; j < kMlpHid; ++j) {
    float z = W[kOffB2 + j];
#pragma unroll
    for (int i = 0; i < kMlpHid; ++i) z = fmaf(W[kOffW2 + j * kMlpHid + i], a1[i], z);
    m2 |= (z > 0.f ? 1ull : 0ull) << j;
    const float a = fmaxf(z, 0.f);
    o[kRecA2 + j] = a;
#pragma unroll
    for (int k = 0; k < kMlpOut; ++k) out[k] = fmaf(W[kOffW3 + k * kMlpHid + j], a, out[k]);
  }
  // loss and its gradient with respect to the outputs
  const float qf = row[10];
  const int Q = qf >= 16.f ? 16 : (qf >= 2.f ? (int)qf : 2);
  const float kap = row[9];
  float dout[kMlpOut];
  float loss = 0.f;
  for (int p = 0; p < 2; ++p) {
    const int t = tgt[2 * (size_t)r + p];
    const float b = fminf(fmaxf(out[2 + p], -4.f), 4.f);
    const float ml = row[7 + p] + out[p];
    const float kl = kap * exp2f(b);
    float mx = -INFINITY;
    for (int j = 0; j < Q; ++j) { const float d = j - ml; mx = fmaxf(mx, -kl * d * d); }
    float Z = 0.f, Ej = 0.f, Ed2 = 0.f;
    for (int j = 0; j < Q; ++j) {
      const float d = j - ml;
      const float e = expf(-kl * d * d - mx);
      Z += e; Ej += e * j; Ed2 += e * d * d;
    }
    Ej /= Z; Ed2 /= Z;
    const float dt = t - ml;
    loss += kl * dt * dt + mx + logf(Z);
    dout[p] = -2.f * kl * (t - Ej);
    const float dk = dt * dt - Ed2;
    dout[2 + p] = (fabsf(out[2 + p]) < 4.f) ? dk * kl * 0.69314718055994531f : 0.f;
  }
#pragma unroll
  for (int k = 0; k < kMlpOut; ++k) { dout[k] *= inv_n; o[kRecDo + k] = dout[k]; }
  o[kRecL] = loss * inv_n;
  // backward to the hidden layers
  float d2[kMlpHid];
#pragma unroll
  for (int j = 0; j < kMlpHid; ++j) {
    float v = 0.f;
#pragma unroll
    for (int k = 0; k < kMlpOut; ++k) v = fmaf(dout[k], W[kOffW3 + k * kMlpHid + j], v);
    d2[j] = ((m2 >> j) & 1ull) ? v : 0.f;
    o[kRecD2 + j] = d2[j];
  }
#pragma unroll
  for (int i = 0; i < kMlpHid; ++i) {
    float v = 0.f;
#pragma unroll
    for (int j = 0; j < kMlpHid; ++j) v = fmaf(d2[j], W[kOffW2 + j * kMlpHid + i], v);
    o[kRecD1 + i] = ((m1 >> i) & 1ull) ? v : 0.f;
  }
}

typedef float f32x4 __attribute__((ext_vector_type(4)));

// One wavefront per chunk of kChunk rows.  v_mfma_f32_16x16x4f32 lane layout (checked on the device):
// A (16 x 4) lane l holds A[l % 16][l / 16], B (4 x 16) lane l holds B[l / 16][l % 16], and register j of
// the accumulator holds D[4 (l / 16) + j][l % 16].  With 4 rows per step (row r0 + l / 16):
//   dW2 (64 x 64, bias column): A = d2 tile, B = a1 tile or the ones column;
//   dW1 (64 x 8 = W1 | b1):     A = d1 tile, B = a0 (its 8th entry is the constant 1);
//   dW3 (4 x 64, bias column):  A = dout (rows 0..3 of the tile), B = a2 tile or the ones column.
__global__ __launch_bounds__(64) void mlp_partial_kernel(const float* __restrict__ rec, int n, float* __restrict__ part) {
  const int l = threadIdx.x, c = l & 15, q = l >> 4;
  const int r0 = blockIdx.x * kChunk;
  f32x4 g2[4][5], g1[4], g3[5];
  const f32x4 z = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
  for (int t = 0; t < 4; ++t) {
    g1[t] = z;
#pragma unroll
    for (int u = 0; u < 5; ++u) g2[t][u] = z;
  }
#pragma unroll
  for (int u = 0; u < 5; ++u) g3[u] = z;
  float ls = 0.f;
  for (int kk = 0; kk < kChunk; kk += 4) {
    const int r = r0 + kk + q;
    const bool ok = r < n;
    const float* o = rec + (size_t)(ok ? r : 0) * kRec;
    float a1v[4], a2v[4], d1v[4], d2v[4];
#pragma unroll
    for (int t = 0; t < 4; ++t) {
      a1v[t] = ok ? o[kRecA1 + 16 * t + c] : 0.f;
      a2v[t] = ok ? o[kRecA2 + 16 * t + c] : 0.f;
      d1v[t] = ok ? o[kRecD1 + 16 * t + c] : 0.f;
      d2v[t] = ok ? o[kRecD2 + 16 * t + c] : 0.f;
    }
    const float a0v = (ok && c < 8) ? o[kRecA0 + c] : 0.f;
    const float dov = (ok && c < kMlpOut) ? o[kRecDo + c] : 0.f;
    const float one = (ok && c == 0) ? 1.f : 0.f;
    if (ok && c == 0) ls += o[kRecL];
#pragma unroll
    for (int jt = 0; jt < 4; ++jt) {
#pragma unroll
      for (int it = 0; it < 4; ++it) g2[jt][it] = __builtin_amdgcn_mfma_f32_16x16x4f32(d2v[jt], a1v[it], g2[jt][it], 0, 0, 0);
      g2[jt][4] = __builtin_amdgcn_mfma_f32_16x16x4f32(d2v[jt], one, g2[jt][4], 0, 0, 0);
      g1[jt] = __builtin_amdgcn_mfma_f32_16x16x4f32(d1v[jt], a0v, g1[jt], 0, 0, 0);
    }
#pragma unroll
    for (int it = 0; it < 4; ++it) g3[it] = __builtin_amdgcn_mfma_f32_16x16x4f32(dov, a2v[it], g3[it], 0, 0, 0);
    g3[4] = __builtin_amdgcn_mfma_f32_16x16x4f32(dov, one, g3[4], 0, 0, 0);
  }
  float* out = part + (size_t)blockIdx.x * (kMlpParams + 1);
#pragma unroll
  for (int j = 0; j < 4; ++j) {
    const int row = 4 * q + j;   // row of the accumulator tile
#pragma unroll
    for (int jt = 0; jt < 4; ++jt) {
      const int u = 16 * jt + row;   // hidden unit
#pragma unroll
      for (int it = 0; it < 4; ++it) out[kOffW2 + u * kMlpHid + 16 * it + c] = g2[jt][it][j];
      if (c == 0) out[kOffB2 + u] = g2[jt][4][j];
      if (c < kMlpIn) out[kOffW1 + u * kMlpIn + c] = g1[jt][j];
      if (c == kMlpIn) out[kOffB1 + u] = g1[jt][j];
    }
    if (row < kMlpOut) {
#pragma unroll
      for (int it = 0; it < 4; ++it) out[kOffW3 + row * kMlpHid + 16 * it + c] = g3[it][j];
      if (c == 0) out[kOffB3 + row] = g3[4][j];
    }
  }
  // the loss: the four lanes (c == 0) of the four row slots, in a fixed order
  ls += __shfl_xor(ls, 16);
  ls += __shfl_xor(ls, 32);
  if (l == 0) out[kMlpParams] = ls;
}

__global__ __launch_bounds__(256) void mlp_adam_kernel(float* __restrict__ w, float* __restrict__ m, float* __restrict__ v,
                                                       const float* __restrict__ part, int chunks, int step, float lr,
                                                       float* __restrict__ loss, float* __restrict__ grad) {
  const int p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p > kMlpParams) return;
  float g = 0.f;
  for (int c = 0; c < chunks; ++c) g += part[(size_t)c * (kMlpParams + 1) + p];
  if (p == kMlpParams) {
    if (loss) loss[0] = g;
    return;
  }
  if (grad) grad[p] = g;
  const float b1 = 0.9f, b2 = 0.999f, eps = 1e-8f;
  const float mn = b1 * m[p] + (1.f - b1) * g;
  const float vn = b2 * v[p] + (1.f - b2) * g * g;
  m[p] = mn;
  v[p] = vn;
  const float mh = mn / (1.f - powf(b1, (float)step));
  const float vh = vn / (1.f - powf(b2, (float)step));
  w[p] -= lr * mh / (sqrtf(vh) + eps);
}

}  // namespace dmala

using namespace dmala;
using namespace dmala::host;

extern "C" {

dmala_status dmala_mlp_forward(const float* weights, const float* rows, int32_t n_rows, int32_t row_stride, float* out,
                               dmala_stream_t stream) {
  if (!weights || !rows || !out) return fail(DMALA_ERR_ARG, "weights, rows and out must be non-NULL");
  if (n_rows < 0) return fail(DMALA_ERR_ARG, "n_rows must be >= 0");
  if (row_stride < kMlpIn) return fail(DMALA_ERR_ARG, "row_stride must be >= %d", kMlpIn);
  if (n_rows == 0) return DMALA_OK;
  const int blocks = (n_rows + 255) / 256;
  hipLaunchKernelGGL(mlp_forward_kernel, dim3(blocks), dim3(256), mlp_lds_bytes<false>(), (hipStream_t)stream, weights, rows,
                     n_rows, row_stride, out);
  const hipError_t e = hipGetLastError();
  if (e != hipSuccess) return hip_fail(e, "mlp forward launch");
  g_err.clear();
  return DMALA_OK;
}

size_t dmala_mlp_train_workspace_size(int32_t n_rows) {
  if (n_rows < 1) return 0;
  const size_t chunks = (n_rows + kChunk - 1) / kChunk;
  return round_up((size_t)n_rows * kRec * 4, 256) + round_up(chunks * (kMlpParams + 1) * 4, 256);
}

dmala_status dmala_mlp_train_step(float* weights, float* adam_m, float* adam_v, int32_t step, float lr,
                                  const float* rows, const int32_t* targets, int32_t n_rows, float* loss, float* grad,
                                  void* workspace, size_t workspace_bytes, dmala_stream_t stream) {
  if (!weights || !adam_m || !adam_v || !rows || !targets) return fail(DMALA_ERR_ARG, "NULL argument");
  if (n_rows < 1) return fail(DMALA_ERR_ARG, "n_rows must be >= 1");
  if (step < 1) return fail(DMALA_ERR_ARG, "step counts from 1");
  if (!(lr > 0.f) || !std::isfinite(lr)) return fail(DMALA_ERR_ARG, "lr must be positive and finite");
  if (!workspace) return fail(DMALA_ERR_WORKSPACE, "workspace is NULL");
  const size_t need = dmala_mlp_train_workspace_size(n_rows);
  if (workspace_bytes < need) return fail(DMALA_ERR_WORKSPACE, "workspace too small: %zu < %zu bytes", workspace_bytes, need);
  if (((uintptr_t)workspace & 255) != 0) return fail(DMALA_ERR_WORKSPACE, "workspace must be 256-byte aligned");
  hipStream_t s = (hipStream_t)stream;
  float* rec = (float*)workspace;
  float* part = (float*)((unsigned char*)workspace + round_up((size_t)n_rows * kRec * 4, 256));
  const int chunks = (n_rows + kChunk - 1) / kChunk;
  hipLaunchKernelGGL(mlp_rows_kernel, dim3((n_rows + 255) / 256), dim3(256), 0, s, weights, rows, targets, n_rows,
                     1.0f / (float)n_rows, rec);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return hip_fail(e, "mlp rows launch");
  const int pb = (kMlpParams + 1 + 255) / 256;
  hipLaunchKernelGGL(mlp_partial_kernel, dim3(chunks), dim3(64), 0, s, rec, n_rows, part);
  e = hipGetLastError();
  if (e != hipSuccess) return hip_fail(e, "mlp partial launch");
  hipLaunchKernelGGL(mlp_adam_kernel, dim3(pb), dim3(256), 0, s, weights, adam_m, adam_v, part, chunks, step, lr, loss,
                     grad);
  e = hipGetLastError();
  if (e != hipSuccess) return hip_fail(e, "mlp adam launch");
  g_err.clear();
  return DMALA_OK;
}

}  // extern "C"
