// The learned proposal's per-antenna network on MFMA (device side).
//
// Network: 8 inputs (7 features and a constant 1 that carries the first
// layer's bias) -> 64 -> 64 -> 4, ReLU after both hidden layers.  Inference
// precision: parameters, inputs and hidden activations rounded to bfloat16,
// products summed in fp32 by v_mfma_f32_16x16x32_bf16, second and third layer
// biases added in fp32 (their bf16-rounded values).
//
// Lane layout.  A wavefront evaluates the network for 16 columns (chains) x 4
// rows of antennas at once: lane l = 16 h + c holds the 8 inputs of "its"
// antenna a_h for column c, and receives that antenna's 4 outputs.  No data
// moves between lanes:
//   * layer 1 for the antenna of lane group g is one MFMA per 16 hidden units
//     in which only the K slice 8g..8g+7 -- the inputs that group g supplies --
//     contributes (zero weights or zero inputs elsewhere, see MlpImage);
//   * layers 2 and 3 take their B operand from the lane's own accumulator
//     registers; the K order of the packed weights follows the accumulator
//     layout (lane group h holds hidden units 16 t + 4 h + i);
//   * the output layer of antenna a_g (W3, a per-group copy non-zero only in rows
//     4g..4g+3) writes those rows of one shared accumulator tile, so lane group g
//     ends up with the outputs of a_g.
// 56 MFMAs per 4 x 16 network evaluations.
#pragma once
#include "common.hpp"

namespace dmala {

typedef __bf16 mlp_bf16x8 __attribute__((ext_vector_type(8)));
typedef float mlp_f32x4 __attribute__((ext_vector_type(4)));

constexpr int kMlpIn = 7;
constexpr int kMlpHid = 64;
constexpr int kMlpOut = 4;
constexpr int kMlpParams = kMlpHid * kMlpIn + kMlpHid + kMlpHid * kMlpHid + kMlpHid + kMlpOut * kMlpHid + kMlpOut;
// offsets of the parameter blocks in the flat float32 array
constexpr int kOffW1 = 0;
constexpr int kOffB1 = kOffW1 + kMlpHid * kMlpIn;
constexpr int kOffW2 = kOffB1 + kMlpHid;
constexpr int kOffB2 = kOffW2 + kMlpHid * kMlpHid;
constexpr int kOffW3 = kOffB2 + kMlpHid;
constexpr int kOffB3 = kOffW3 + kMlpOut * kMlpHid;
// LDS image: W1 fragments, W2 fragments [4 out tiles][2 K steps], W3 fragments [4 antenna
// groups][2 K steps] (non-zero only in the group's 4 rows), b2 [64], b3 [4].  W1 comes in one of
// two forms (GW1):
//   false: [4 hidden tiles], the same weights in every K slice; the B operand is masked to the
//          K slice of the antenna group being evaluated (a select per input register);
//   true:  [4 antenna groups][4 hidden tiles], non-zero only in the group's K slice, so the
//          unmasked inputs can be used (12 KiB more LDS, no selects: for the kernels whose
//          register pressure makes the selects' lane masks spill).
template <bool GW1> struct MlpImage {
  static constexpr int kW1 = 0;
  static constexpr int kW2 = GW1 ? 16 : 4;
  static constexpr int kW3 = kW2 + 8;
  static constexpr int kFrags = kW3 + 8;
  static constexpr size_t kBytes = (size_t)kFrags * 1024 + 64 * 4 + 4 * 4;
};
template <bool GW1> constexpr size_t mlp_lds_bytes() { return MlpImage<GW1>::kBytes; }

// Hidden unit that K element j of lane group h feeds in K step s (layers 2, 3).
__device__ __forceinline__ int mlp_kidx(int s, int h, int j) { return 16 * (2 * s + (j >> 2)) + 4 * h + (j & 3); }

__device__ __forceinline__ float bf16_round(float v) { return (float)(__bf16)v; }

// An opaque zero offset (see the sampler's opaque_zero).
__device__ __forceinline__ uint32_t opaque_zero_u32() {
  uint32_t z = 0;
  asm volatile("" : "+s"(z));
  return z;
}

// Build the LDS image of the network from the flat float32 parameters (all
// threads of the block take part; the caller synchronises afterwards).
template <bool GW1>
__device__ inline void mlp_stage(const float* __restrict__ w, unsigned char* lds) {
  using I = MlpImage<GW1>;
  for (int it = threadIdx.x; it < I::kFrags * 64; it += blockDim.x) {
    const int f = it >> 6, l = it & 63, r = l & 15, h = l >> 4;
    mlp_bf16x8 v;
#pragma unroll
    for (int j = 0; j < 8; ++j) {
      float x;
      if (f < I::kW2) {
        const int u = 16 * (f & 3) + r;
        x = (GW1 && h != (f >> 2)) ? 0.0f : (j < kMlpIn ? w[kOffW1 + u * kMlpIn + j] : w[kOffB1 + u]);
      } else if (f < I::kW3) {
        const int ot = (f - I::kW2) >> 1, s = (f - I::kW2) & 1;
        x = w[kOffW2 + (16 * ot + r) * kMlpHid + mlp_kidx(s, h, j)];
      } else {
        const int g = (f - I::kW3) >> 1, s = (f - I::kW3) & 1;
        x = (r >> 2) != g ? 0.0f : w[kOffW3 + (r & 3) * kMlpHid + mlp_kidx(s, h, j)];
      }
      v[j] = (__bf16)x;
    }
    *(mlp_bf16x8*)(lds + (size_t)f * 1024 + l * 16) = v;
  }
  float* bias = (float*)(lds + (size_t)I::kFrags * 1024);
  for (int i = threadIdx.x; i < 64 + 4; i += blockDim.x)
    bias[i] = bf16_round(i < 64 ? w[kOffB2 + i] : w[kOffB3 + i - 64]);
}

// ReLU of 8 hidden values (accumulator registers u then v) rounded to bf16: the packed
// conversion first, then a packed 16-bit signed maximum with 0 (a bf16 with the sign bit set is a
// negative 16-bit integer, so this is max(x, +0) on the bf16 values, -0 and negatives to +0).
__device__ __forceinline__ mlp_bf16x8 relu_bf16x8(mlp_f32x4 u, mlp_f32x4 v) {
  typedef float f32x2 __attribute__((ext_vector_type(2)));
  typedef short s16x2 __attribute__((ext_vector_type(2)));
  typedef __bf16 bf16x2 __attribute__((ext_vector_type(2)));
  typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));
  const f32x2 pr[4] = {{u[0], u[1]}, {u[2], u[3]}, {v[0], v[1]}, {v[2], v[3]}};
  const s16x2 z = {0, 0};
  u32x4 w;
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    const bf16x2 p = __builtin_convertvector(pr[q], bf16x2);
    w[q] = __builtin_bit_cast(uint32_t, __builtin_elementwise_max(__builtin_bit_cast(s16x2, p), z));
  }
  return __builtin_bit_cast(mlp_bf16x8, w);
}

// Inputs of one antenna for this lane (7 features and the constant 1), rounded to bf16.
__device__ __forceinline__ mlp_bf16x8 mlp_inputs(float f0, float f1, float f2, float f3, float f4, float f5, float f6) {
  mlp_bf16x8 x;
  x[0] = (__bf16)f0; x[1] = (__bf16)f1; x[2] = (__bf16)f2; x[3] = (__bf16)f3;
  x[4] = (__bf16)f4; x[5] = (__bf16)f5; x[6] = (__bf16)f6; x[7] = (__bf16)1.0f;
  return x;
}

// Evaluate the network for the 4 antennas x 16 columns held by the wave; the
// lane receives the 4 outputs of its own antenna.  All 64 lanes must call it.
// `lds_off` must be an LDS byte offset hidden from the optimiser (so that the
// fragments are reloaded per call instead of being pinned in registers).
template <bool GW1>
__device__ __forceinline__ mlp_f32x4 mlp_eval4(const unsigned char* lds, uint32_t lds_off, mlp_bf16x8 x) {
  using I = MlpImage<GW1>;
  const int lane = threadIdx.x & 63, h = lane >> 4;
  const float* bias = (const float*)(lds + lds_off + (size_t)I::kFrags * 1024);
  mlp_f32x4 out = *(const mlp_f32x4*)(bias + 64);
#pragma unroll
  for (int g = 0; g < 4; ++g) {
    // fragments are re-read for every antenna group (an opaque offset keeps the
    // compiler from holding all of them in registers across the groups)
    const unsigned char* base = lds + lds_off + opaque_zero_u32() + (uint32_t)lane * 16;
    // only the K slice of antenna group g may contribute: zero weights elsewhere (GW1) or
    // zero inputs of the other groups
    const mlp_bf16x8 zero8 = {};
    const mlp_bf16x8 xg = (GW1 || h == g) ? x : zero8;
    mlp_f32x4 z1[4];
#pragma unroll
    for (int t = 0; t < 4; ++t) {
      const mlp_f32x4 c0 = {0.f, 0.f, 0.f, 0.f};
      const mlp_bf16x8 w1 = *(const mlp_bf16x8*)(base + (I::kW1 + (GW1 ? 4 * g : 0) + t) * 1024);
      z1[t] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(w1, xg, c0, 0, 0, 0);
    }
    mlp_bf16x8 a1[2];
#pragma unroll
    for (int s = 0; s < 2; ++s) a1[s] = relu_bf16x8(z1[2 * s], z1[2 * s + 1]);
    mlp_f32x4 z2[4];
#pragma unroll
    for (int t = 0; t < 4; ++t) {
      z2[t] = *(const mlp_f32x4*)(bias + 16 * t + 4 * h);
#pragma unroll
      for (int s = 0; s < 2; ++s) {
        const mlp_bf16x8 w2 = *(const mlp_bf16x8*)(base + (I::kW2 + 2 * t + s) * 1024);
        z2[t] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(w2, a1[s], z2[t], 0, 0, 0);
      }
    }
    mlp_bf16x8 a2[2];
#pragma unroll
    for (int s = 0; s < 2; ++s) a2[s] = relu_bf16x8(z2[2 * s], z2[2 * s + 1]);
#pragma unroll
    for (int s = 0; s < 2; ++s) {
      const mlp_bf16x8 w3 = *(const mlp_bf16x8*)(base + (I::kW3 + 2 * g + s) * 1024);
      out = __builtin_amdgcn_mfma_f32_16x16x32_bf16(w3, a2[s], out, 0, 0, 0);
    }
  }
  return out;
}

}  // namespace dmala
