// The DMALA chain kernel: Algorithm 1 (on the tempered metric of Algorithm 2)
// for many independent chains per instance, all iterations in one launch.
//
// Work layout.  A wavefront owns 16 chains of one instance.  Lane l handles
// chain l % 16 and, in every 16-row tile rt of the real dimensions, the four
// dimensions n = 16 rt + 4 (l / 16) + i, i = 0..3 -- exactly the rows the
// 16x16x32 MFMA accumulator layout gives that lane.  Per iteration and chain:
//   1. draw x'_n ~ q_n(. | x_n) for the lane's dimensions (inverse CDF of the
//      discretised-Gaussian proposal at one Philox uniform each) and sum
//      log q(x' | x)                                         [Alg. 1: sample, fwd q]
//   2. one batched contraction [P; EG] x lv(x') for the 16 chains on MFMA; the
//      B operand is built from the lane's own proposed levels (no data
//      exchange), the A operands stream from LDS               [Alg. 1: grad f(x')]
//   3. proposal parameters at x' (mode mu', log2 normaliser lz') and
//      log q(x | x')                                          [Alg. 1: reverse q]
//   4. tempered energy difference from the two energy gradients
//      (x' - x)^T (g + g'), the MH log ratio, a 4-lane butterfly sum, and the
//      accept test log ratio > log u                          [eq. acc_prob]
//   5. select, energy bookkeeping for the minimum-residual hard decision.
// The float64 path keeps the same structure with dense double matrices in LDS
// and VALU dot products instead of MFMA.
//
// Learned variant (LRN = 1).  Every transition of every chain uses the plain
// preconditioned kernel with probability eps and otherwise the learned kernel,
// whose proposal is the same discretised Gaussian with the centre and the
// precision of each dimension set by the per-antenna network of
// mlp_device.hpp (features of the antenna at the current state).  Each kernel
// is a complete MH step with its own forward and reverse proposal; the choice
// comes from the chain's random stream (low bytes of words 4, 5, 6), not from
// the state, so the mixture keeps pi_a invariant.  The network runs at every
// proposed state (its output becomes the cached learned proposal when the
// move is accepted), and all Q levels are weighted directly (no window).
#pragma once
#include <type_traits>

#include "common.hpp"
#include "mlp_device.hpp"

namespace dmala {

typedef _Float16 half8 __attribute__((ext_vector_type(8)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

__device__ __forceinline__ float ex2(float x) { return __builtin_amdgcn_exp2f(x); }
__device__ __forceinline__ float lg2(float x) { return __builtin_amdgcn_logf(x); }
__device__ __forceinline__ double ex2(double x) { return exp2(x); }
__device__ __forceinline__ double lg2(double x) { return log2(x); }
// Inverse of the standard normal CDF (the device math library's).
__device__ __forceinline__ float ncdf_inv(float u) { return normcdfinvf(u); }
__device__ __forceinline__ double ncdf_inv(double u) { return normcdfinv(u); }
__device__ __forceinline__ float erfc_(float x) { return erfcf(x); }
__device__ __forceinline__ double erfc_(double x) { return erfc(x); }

// Standard normal deviate Phi^-1(u) of a random word, u = (x + 1/2) 2^-24 with x its high 24 bits.
// The upper half uses Phi^-1(u) = -Phi^-1(1 - u), so that the argument (x + 1/2 or 2^24 - x - 1/2,
// times 2^-24) is exact in fp32 as well.
template <typename R>
__device__ __forceinline__ R gauss_of_word(uint32_t w) {
  const uint32_t x = w >> 8;
  const bool up = x >= (1u << 23);
  const R a = up ? R((1u << 24) - x) - R(0.5) : R(x) + R(0.5);
  const R z = ncdf_inv(a * R(5.9604644775390625e-08));
  return up ? -z : z;
}

// MHGD candidate law of one dimension: log2 of the probability that the nearest level
// of N(mu, sig^2) (index units, levels 0..Q-1, edge cells unbounded) is j.  Each cell
// is integrated on the tail side away from mu, where erfc keeps small cells accurate.
template <int Q, typename R>
__device__ __forceinline__ R mhgd_log2_cell(R j, R mu, R sig) {
  const R r2 = R(0.70710678118654752440) / sig;
  const R lo = (j - R(0.5) - mu) * r2, hi = (j + R(0.5) - mu) * r2;
  const bool first = j == R(0), last = j == R(Q - 1);
  R p;
  if (!first && lo > R(0)) p = R(0.5) * (erfc_(lo) - (last ? R(0) : erfc_(hi)));
  else if (!last && hi < R(0)) p = R(0.5) * (erfc_(-hi) - (first ? R(0) : erfc_(-lo)));
  else p = R(1) - R(0.5) * ((first ? R(0) : erfc_(-lo)) + (last ? R(0) : erfc_(hi)));
  return lg2(p);
}

// Mode of the discretised Gaussian exp2(-kL (j - mu)^2) over j in [0, Q).
template <int Q, typename R>
__device__ __forceinline__ R mode_of(R mu) {
  if constexpr (std::is_same<R, float>::value) {
    return __builtin_amdgcn_fmed3f(rintf(mu), 0.0f, float(Q - 1));   // one v_med3 instead of two compare/selects
  } else {
    R j = rint(mu);
    j = j < R(0) ? R(0) : j;
    j = j > R(Q - 1) ? R(Q - 1) : j;
    return j;
  }
}

// Per-mode coefficient table of the 3-level window (LDS, one row of kCtabStride
// floats per mode js): c_3, c_2, c_1 for the levels js-3 .. js-1, then c_1, c_2,
// c_3 for js+1 .. js+3, with c_o = exp2(-kL o^2) and zero for a level outside
// [0, Q).  Reading the row replaces the per-level range tests of the window.
// The 48-byte stride keeps the rows of an 8-level table on distinct LDS banks.
constexpr int kCtabStride = 12;
constexpr size_t kCtabBytes = 16 * kCtabStride * sizeof(float);  // up to Q = 16
// every layout but one wave of 8 LDS row tiles (whose matrices take all 160 KiB at fp32)
constexpr bool win_table(int rtw, int wd, bool mg) { return !(rtw == 8 && wd == 1 && !mg); }
// form of the network's first-layer weights in LDS: per-group copies for the dimension-split
// kernels (whose register pressure makes the input selects spill), one copy elsewhere (where the
// 12 KiB more would lower the number of workgroups per CU)
constexpr bool mlp_gw1(int wd) { return wd > 1; }

template <int Q>
__device__ __forceinline__ void ctab_fill(float* ctab, float kL) {
  for (int i = threadIdx.x; i < Q * kCtabStride; i += blockDim.x) {
    const int js = i / kCtabStride, sl = i % kCtabStride;
    float v = 0.f;
    if (sl < 3) {
      const int o = 3 - sl;
      v = (js - o >= 0) ? ex2(-kL * float(o * o)) : 0.f;
    } else if (sl < 6) {
      const int o = sl - 2;
      v = (js + o <= Q - 1) ? ex2(-kL * float(o * o)) : 0.f;
    }
    ctab[i] = v;
  }
}

// Weights w_j = exp2(-kL ((j - mu)^2 - (js - mu)^2)) of the proposal over the
// levels j = js - 3 .. js + 3 around the mode js (zero outside [0, Q)), in
// ascending level order.  With delta = js - mu, F = exp2(-2 kL delta) and
// G = 1 / F, the weight of level js + o is c_o F^o above the mode and c_o G^o
// below it: two exponentials per dimension instead of one per level.
// |delta| is bounded by dmax = max(1/2, 12.5 / kL) for the exponentials: |delta|
// exceeds 1/2 only at an edge mode, where the clamped side is out of range (table
// entry zero) and the other side's weights stay below 2^-(kL+25) of the mode either
// way, which leaves every fp32 sum unchanged; the bound keeps F^3 and G^3 finite
// (the window is used only for kL <= 40).
// The window is used only when 12 kL >= 30, so that every omitted level
// weighs less than 2^-30 of the mode -- below the fp32 rounding of the sums,
// i.e. invisible in fp32.
// Coefficients of the window: the LDS table address, or (layouts whose LDS is
// full: one wave with 8 row tiles of matrices) c_o in registers with range tests.
struct WinCoef {
  uint32_t tab;
  float dmax;   // bound on |js - mu| for the two exponentials (table layouts)
  float c[4];
};

// The window's factors: F = exp2(-2 kL delta), G = 1 / F as two exponentials, and the
// coefficients c_1..c_3 of the levels above (cu) and below (cl) the mode, zero outside [0, Q).
template <int Q, int W, bool TAB>
__device__ __forceinline__ void window_coefs(float mu, float kL, const WinCoef& wc, float& F, float& G,
                                             float (&cu)[W], float (&cl)[W], float& jf, float& delta) {
  static_assert(W == 3, "the coefficient table holds a 3-level window");
  // The mode from the clamped centre plus 2^23: the addition rounds to the nearest integer
  // (ties to even, as rint) and leaves the integer in the low 23 bits of the sum's pattern,
  // so that the table row needs no float-to-integer conversion.
  const float jb = __builtin_amdgcn_fmed3f(mu, 0.0f, float(Q - 1)) + 8388608.0f;
  jf = jb - 8388608.0f;
  delta = jf - mu;
  if constexpr (TAB) {
    // the row by its 32-bit LDS address (generic pointer arithmetic would be 64-bit),
    // read before the exponentials so that they cover the LDS latency
    typedef float v4f __attribute__((ext_vector_type(4)));
    typedef float v2f __attribute__((ext_vector_type(2)));
    typedef __attribute__((address_space(3))) const v4f lds_v4f;
    typedef __attribute__((address_space(3))) const v2f lds_v2f;
    // one v_mad_u32_u24, which reads only the low 24 bits (the mode) of jb's pattern
    const uint32_t row = __umul24(__float_as_uint(jb), (uint32_t)(kCtabStride * sizeof(float))) + wc.tab;
    const v4f lo = *(lds_v4f*)(uintptr_t)row;         // c_3, c_2, c_1 below; c_1 above
    const v2f hi = *(lds_v2f*)(uintptr_t)(row + 16);  // c_2, c_3 above
    const float x = 2.0f * kL * __builtin_amdgcn_fmed3f(delta, -wc.dmax, wc.dmax);
    F = ex2(-x);
    G = ex2(x);
    cl[0] = lo.z; cl[1] = lo.y; cl[2] = lo.x;
    cu[0] = lo.w; cu[1] = hi.x; cu[2] = hi.y;
  } else {
    const float x = 2.0f * kL * delta;
    F = ex2(-x);
    G = ex2(x);
#pragma unroll
    for (int o = 1; o <= W; ++o) {
      cu[o - 1] = (jf + float(o) <= float(Q - 1)) ? wc.c[o] : 0.0f;
      cl[o - 1] = (jf - float(o) >= 0.0f) ? wc.c[o] : 0.0f;
    }
  }
}

// The window's weights in ascending level order: c_o F^o above the mode, c_o G^o below it.
template <int Q, int W, bool TAB>
__device__ __forceinline__ void window_weights(float mu, float kL, const WinCoef& wc, float (&e)[2 * W + 1], float& jf,
                                               float& delta) {
  float F, G, cu[W], cl[W];
  window_coefs<Q, W, TAB>(mu, kL, wc, F, G, cu, cl, jf, delta);
  const float F2 = F * F, G2 = G * G;
  e[W] = 1.0f;
  e[W + 1] = cu[0] * F;
  e[W - 1] = cl[0] * G;
  e[W + 2] = cu[1] * F2;
  e[W - 2] = cl[1] * G2;
  e[W + 3] = cu[2] * (F2 * F);
  e[W - 3] = cl[2] * (G2 * G);
}

// All Q weights relative to the mode, one exponential per level (any kL).
template <int Q, typename R>
__device__ __forceinline__ void level_weights(R mu, R kL, R (&e)[Q], R& base) {
  const R js = mode_of<Q>(mu);
  base = (js - mu) * (js - mu);
#pragma unroll
  for (int j = 0; j < Q; ++j) {
    const R t = R(j) - mu;
    e[j] = ex2(kL * (base - t * t));
  }
}

// log2 of the proposal normaliser sum_j exp2(-kL (j - mu)^2) (eq. softmax).
// Its two parts: the weight sum Z relative to the mode (1 <= Z <= Q) and the squared
// mode offset base, log2 normaliser = log2 Z - kL base.
template <int Q, int WIN, int W, bool TAB, typename R>
__device__ __forceinline__ void norm_parts(R mu, R kL, const WinCoef& wc, R& Z, R& base) {
  // the sums start from the first weight, not from zero (0 + x is exact, and a
  // zero start would cost a separate fused multiply-add)
  if constexpr (WIN > 0) {
    // Z = 1 + F (c1 + F (c2 + F c3)) + G (c1' + G (c2' + G c3')): six fused multiply-adds, no powers
    R F, G, cu[W], cl[W], jf;
    window_coefs<Q, W, TAB>(mu, kL, wc, F, G, cu, cl, jf, base);
    const R zu = __builtin_fmaf(F, __builtin_fmaf(F, __builtin_fmaf(F, cu[2], cu[1]), cu[0]), 1.0f);
    Z = __builtin_fmaf(G, __builtin_fmaf(G, __builtin_fmaf(G, cl[2], cl[1]), cl[0]), zu);
    base *= base;
  } else {
    R e[Q];
    level_weights<Q>(mu, kL, e, base);
    Z = e[0];
#pragma unroll
    for (int j = 1; j < Q; ++j) Z += e[j];
  }
}

template <int Q, int WIN, int W, bool TAB, typename R>
__device__ __forceinline__ R log2_norm(R mu, R kL, const WinCoef& wc) {
  R Z, base;
  norm_parts<Q, WIN, W, TAB>(mu, kL, wc, Z, base);
  return lg2(Z) - kL * base;
}

// Inverse-CDF draw: the smallest level j with u Z < sum_{i <= j} w_i
// (ascending levels), Z = sum_i w_i; the level as a floating-point integer.
template <int Q, int WIN, int W, bool TAB, typename R>
__device__ __forceinline__ R draw_level(R mu, R kL, const WinCoef& wc, uint32_t word) {
  if constexpr (WIN > 0) {
    R e[2 * W + 1];
    R jf, delta;
    window_weights<Q, W, TAB>(mu, kL, wc, e, jf, delta);
    R Z = e[0];
#pragma unroll
    for (int i = 1; i <= 2 * W; ++i) Z += e[i];
    // The partial sums above the target, counted in fp32 without compares: with B = 2^100,
    // B (cum - target) is exact in sign and, since target >= 2^-24 Z and cum, target are
    // fp32 numbers, at least B 2^-47 when positive; clamped to [0, 1] it is the 0/1
    // indicator of cum > target (one fused multiply-add with the clamp modifier each).
    constexpr float kB = 0x1p100f;
    const R tB = u23f_x2p100(word) * Z;   // (u Z) 2^100, rounded once as u Z
    R cum = e[0];
    R above = __builtin_amdgcn_fmed3f(0.0f, 1.0f, __builtin_fmaf(cum, kB, -tB));
#pragma unroll
    for (int i = 1; i < 2 * W; ++i) {
      cum += e[i];
      above += __builtin_amdgcn_fmed3f(0.0f, 1.0f, __builtin_fmaf(cum, kB, -tB));
    }
    // js - W + (2 W - above), clamped to the levels
    return __builtin_amdgcn_fmed3f((jf + R(W)) - above, 0.0f, R(Q - 1));
  } else {
    R e[Q], base;
    level_weights<Q>(mu, kL, e, base);
    R Z = R(0);
#pragma unroll
    for (int j = 0; j < Q; ++j) Z += e[j];
    R u;
    if constexpr (std::is_same<R, double>::value) u = u23d(word);
    else u = u23f(word);
    const R target = u * Z;
    R cum = R(0);
    int cnt = 0;
#pragma unroll
    for (int j = 0; j < Q - 1; ++j) {
      cum += e[j];
      cnt += (cum <= target) ? 1 : 0;
    }
    return R(cnt);
  }
}

// Inverse-CDF draw over all Q levels that also returns the log2 normaliser
// (the same arithmetic as log2_norm<Q, 0, .>).
template <int Q>
__device__ __forceinline__ int draw_level_lz(float mu, float kL, float u, float& lz) {
  float e[Q], base;
  level_weights<Q>(mu, kL, e, base);
  float Z = 0.f;
#pragma unroll
  for (int j = 0; j < Q; ++j) Z += e[j];
  const float target = u * Z;
  float cum = 0.f;
  int cnt = 0;
#pragma unroll
  for (int j = 0; j < Q - 1; ++j) {
    cum += e[j];
    cnt += (cum <= target) ? 1 : 0;
  }
  lz = lg2(Z) - kL * base;
  return cnt;
}

// The f16 pair (2 ka - QM1, 2 kb - QM1) of two levels in one word (exact: |2k - QM1| <= 15),
// low half first, by one packing conversion.
template <int QM1, typename R>
__device__ __forceinline__ uint32_t lv_pair(R ka, R kb) {
  const auto h = __builtin_amdgcn_cvt_pkrtz(float(2 * ka - R(QM1)), float(2 * kb - R(QM1)));
  uint32_t u;
  __builtin_memcpy(&u, &h, 4);
  return u;
}

// An opaque zero: added to LDS offsets inside the loop so that the optimiser
// cannot hoist the loop-invariant A-operand fragment loads out of the loop
// (that would pin every fragment in registers and halve the occupancy).
__device__ __forceinline__ uint32_t opaque_zero() {
  uint32_t z = 0;
  asm volatile("" : "+s"(z));
  return z;
}

template <typename R>
__device__ __forceinline__ R bfly4(R v) {
  v += __shfl_xor(v, 16);
  v += __shfl_xor(v, 32);
  return v;
}

// Cross-wave partial sums (dimension-split chain blocks).
struct Red {
  float x, y, z;
  uint32_t h;
};

// Complex-plane layouts: how many half passes (one plane of a pass; proposal passes first, then the
// energy passes) of the packed matrices a workgroup keeps in LDS for all its transitions; the rest
// stream from L2 every transition.  128 dimensions: 3.5 passes of 16 KiB (two workgroups per CU);
// 256 dimensions: 1.5 passes of 64 KiB beside the window layout's two 16-chain blocks, two otherwise
// (one workgroup per CU).
constexpr int cx_lds_halves(int rt, bool win) { return rt <= 8 ? 7 : (win ? 3 : 4); }

// Template parameters: RTW row tiles of 16 dimensions per wave, WD waves per
// chain block splitting the dimensions (RT = RTW * WD tiles in all), MG = the
// packed matrices are read from the instance block in global memory (L2) instead
// of being staged in LDS.
// FULL: the instance has no padding dimensions (N == Npad), so that no dimension needs the
// padding masks (the caller checks; the results are the same either way).
template <typename Real, int RTW, int WD, bool MG, int Q, int PM, bool EVAL, int WIN, int KND, bool CX = false,
          bool FULL = false>
__device__ __forceinline__ void sampler_body(const SamplerArgs& a, const int inst, const int cgy) {
  constexpr bool F64 = std::is_same<Real, double>::value;
  constexpr bool LRN = KND == 1;   // plain/learned kernel mixture
  constexpr bool MHG = KND == 2;   // the MHGD baseline (nearest-point candidate, MH without the proposal ratio)
  static_assert(!F64 || (WD == 1 && !MG), "the float64 path uses one wave per chain block and LDS matrices");
  static_assert(!LRN || (!F64 && PM != PM_NAIVE && WIN == 0 && RTW <= 4), "learned variant: float, preconditioned, no window");
  static_assert(!MHG || (PM != PM_NAIVE && WIN == 0), "MHGD: the preconditioned gradient step, no proposal window");
  static_assert(!CX || (!F64 && !LRN && RTW % 4 == 0 && (MG ? RTW * WD >= 8 : RTW * WD == 4)),
                "complex-plane matrices: float, whole 32-antenna K blocks per wave, from L2 or (64 dimensions) LDS");
  static_assert(WD == 1 || RTW % 2 == 0, "dimension-split waves own whole K blocks");
  constexpr int RT = RTW * WD;
  constexpr int D = 4 * RTW;
  constexpr int KB = RT / 2;
  constexpr int KBW = RTW / 2;
  constexpr int NPP = p_passes(PM);
  constexpr int QM1 = Q - 1;
  constexpr int W = WIN > 0 ? WIN : Q - 1;
  // one-wave layouts with up to 4 row tiles: the next transition's random words are
  // generated beside the contraction, with three-input xors in the Philox rounds
  constexpr bool PIPE = !LRN && !F64 && WD == 1 && RTW <= 4;
  extern __shared__ __attribute__((aligned(16))) unsigned char smem[];

  // inst: index within the class (workspace slot); cgy: group of 16-chain blocks
  const int N = a.N, Npad = a.Npad;
  const unsigned char* blk = a.ws_inst + (size_t)inst * a.inst_stride;
  // the caller's instance index (RNG counter, per-instance outputs) and final-state offset
  const uint32_t rid = a.desc ? (uint32_t)a.desc[inst].orig : (uint32_t)inst;
  const uint32_t rctr = rid + a.ctr_base;                 // instance word of the random counter
  const size_t fs_base = a.desc ? (size_t)a.desc[inst].fs_off : (size_t)inst * a.C * N;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6, nwaves = blockDim.x >> 6;
  const int cl = lane & 15, h = lane >> 4;
  // dimension-split layouts: WD consecutive waves share one 16-chain block (a "slot"), and a
  // workgroup holds nwaves / WD slots (chain blocks of the same instance, so that the waves
  // owning the same row tiles read the same matrix fragments at the same time)
  const int wd = WD > 1 ? wave % WD : 0;                  // dimension slice of this wave
  const int slot = WD > 1 ? wave / WD : 0;
  const int cblock = WD > 1 ? cgy * (nwaves / WD) + slot : cgy * nwaves + wave;
  const int chain = cblock * 16 + cl;
  const bool live = chain < a.C;
  const int rt0 = wd * RTW;                               // first row tile owned

  // A flagged instance (a non-finite entry in H or y, or sigma^2 not positive and finite):
  // no chain runs; the optional per-chain outputs are written as zeros (evaluation: NaN).
  // The flag belongs to the workgroup's one instance, so every thread leaves here.
  if (((const InstParams*)blk)->nonfinite) {
    if (live && h == 0 && wd == 0) {
      if constexpr (EVAL) {
        double* o = a.eval_out + ((size_t)inst * a.C + chain) * 4;
        for (int i = 0; i < 4; ++i) o[i] = __builtin_nan("");
        if (a.eval_dim)
          for (int n = 0; n < N; ++n) a.eval_dim[((size_t)inst * a.C + chain) * N + n] = __builtin_nan("");
      } else {
        const size_t trow = (size_t)rid * a.C + chain;
        if (a.accept_count) a.accept_count[trow] = 0;
        if (a.final_state)
          for (int n = 0; n < N; ++n) a.final_state[fs_base + (size_t)chain * N + n] = 0;
        if (a.trace_accept)
          for (int w = 0; w < a.trace_words; ++w) a.trace_accept[trow * a.trace_words + w] = 0u;
        if (a.trace_hash)
          for (int t = 0; t < a.T; ++t) a.trace_hash[trow * a.T + t] = 0u;
        if (a.train_rows) {
          const int Nt = N >> 1;
          const int64_t sym0 = a.desc ? a.desc[inst].sym_off : (int64_t)inst * Nt;
          float* row = a.train_rows + ((size_t)sym0 * a.C + (size_t)chain * Nt) * kTrainRow;
          for (int i = 0; i < Nt * kTrainRow; ++i) row[i] = 0.f;
        }
      }
    }
    return;
  }

  // stage the instance's packed matrices and vectors in LDS
  // bytes of one split term (pass) of a packed matrix: RT x KB real-equivalent fragments, or (complex
  // planes) 2 planes x RT/2 antenna tiles x RT/4 K blocks of 32 antennas
  constexpr size_t PASS = CX ? (size_t)RT * RT / 4 * 1024 : (size_t)RT * KB * 1024;
  const size_t mat_bytes = F64 ? 0 : (size_t)(NPP + kEPasses) * PASS;
  // complex planes: passes staged in LDS (every pass when the matrices are not read from L2)
  constexpr int SPH = CX ? (MG ? (cx_lds_halves(RT, WIN > 0) < 2 * (NPP + kEPasses) ? cx_lds_halves(RT, WIN > 0)
                                                                          : 2 * (NPP + kEPasses))
                              : 2 * (NPP + kEPasses))
                       : 0;
  size_t staged = 0;
  if constexpr (F64) staged = a.frag_bytes;
  else if constexpr (!MG) staged = (RT <= 4) ? (size_t)a.frag_bytes : mat_bytes;
  else if constexpr (CX) staged = (size_t)SPH * (PASS / 2);
  for (size_t o = threadIdx.x * 16; o < staged; o += blockDim.x * 16)
    *(uint4*)(smem + o) = *(const uint4*)(blk + kParamBytes + o);
  const InstParams ip = *(const InstParams*)blk;
  const int nslots = WD > 1 ? nwaves / WD : 0;
  unsigned char* xbuf = smem + ((staged + 15) & ~(size_t)15);      // per slot 2 x KB x 1 KiB (WD > 1)
  Red* rbuf = (Red*)(xbuf + (size_t)nslots * 2 * KB * 1024);        // per slot 2 x WD x 16
  unsigned char* mlp_lds = (unsigned char*)(rbuf + (size_t)nslots * 2 * WD * 16);   // network image (LRN)
  xbuf += (size_t)slot * 2 * KB * 1024;
  rbuf += (size_t)slot * 2 * WD * 16;
  // window coefficients: a per-mode LDS table, except where the matrices fill the LDS
  constexpr bool TAB = WIN > 0 && win_table(RTW, WD, MG);
  float* ctab_p = (float*)(mlp_lds + (LRN ? mlp_lds_bytes<mlp_gw1(WD)>() : 0));
  WinCoef wc;
  wc.tab = (uint32_t)(uintptr_t)(__attribute__((address_space(3))) float*)ctab_p;
  wc.dmax = fmaxf(0.5f, 12.5f / (float)ip.kL);
#pragma unroll
  for (int o = 0; o < 4; ++o) wc.c[o] = ex2(-(float)ip.kL * float(o * o));
  if constexpr (LRN) mlp_stage<mlp_gw1(WD)>(a.mlp, mlp_lds);
  if constexpr (TAB) ctab_fill<Q>(ctab_p, (float)ip.kL);
  __syncthreads();

  const Real kL = (Real)ip.kL;
  const Real rho = (Real)ip.rho;
  // MHGD: standard deviation of the random walk in index units, sqrt(alpha beta) / (2 s)
  // = sqrt(log2(e) / (2 kL))
  const Real msig = (Real)sqrt(kLog2e / (2.0 * ip.kL));
  const Real sP = (Real)ip.scaleP, sE = (Real)ip.scaleE;
  const Real* pbv;
  const Real* ezv;
  const double* Pd = nullptr;
  const double* EGd = nullptr;
  double* lvbuf = nullptr;
  if constexpr (F64) {
    Pd = (const double*)smem;
    EGd = Pd + (size_t)Npad * Npad;
    pbv = (const Real*)(EGd + (size_t)Npad * Npad);
    ezv = pbv + Npad;
    lvbuf = (double*)(smem + a.frag_bytes) + (size_t)wave * 16 * Npad;
  } else {
    // the two per-dimension vectors follow the fragments (in LDS only when small)
    if (!MG && RT <= 4) pbv = (const Real*)(smem + mat_bytes);
    else pbv = (const Real*)(blk + kParamBytes + mat_bytes);
    ezv = pbv + Npad;
  }
  // per-antenna network features (dimension 2m: LS variance, 2m+1: conditional variance)
  const float* afv = (const float*)ezv + Npad;

  // The lane's dimensions come in GR = RTW groups of 4 consecutive real dimensions: group g is
  // dimensions 16 (rt0 + g) + 4 h + 0..3 (real-equivalent rows of row tile rt0 + g), or, with
  // complex planes, 32 (rt0/2 + g/2) + 8 h + 4 (g%2) + 0..3 (Re and Im of the lane's 4 antennas
  // 16 at + 4 h + 0..3 of antenna tile at = rt0/2 + g/2).  Group g draws from random block gdim(g)/4.
  auto gdim = [&](int g) {
    if constexpr (CX) return 32 * ((rt0 >> 1) + (g >> 1)) + 8 * h + 4 * (g & 1);
    else return 16 * (rt0 + g) + 4 * h;
  };
  auto dim_of = [&](int d) { return gdim(d >> 2) + (d & 3); };
  int xphase = 0, rphase = 0;

  // Sum of per-lane partials over the chain's 4 lanes and (WD > 1) its WD waves;
  // every lane of the chain gets bitwise the same totals.
  auto chain_sum = [&](Red v) {
    v.x = bfly4(v.x); v.y = bfly4(v.y); v.z = bfly4(v.z);
    v.h += __shfl_xor(v.h, 16);
    v.h += __shfl_xor(v.h, 32);
    if constexpr (WD > 1) {
      Red* rb = rbuf + (rphase & 1) * WD * 16;
      ++rphase;
      if (h == 0) rb[wd * 16 + cl] = v;
      __syncthreads();
      Red t = rb[cl];
#pragma unroll
      for (int w2 = 1; w2 < WD; ++w2) {
        const Red u = rb[w2 * 16 + cl];
        t.x += u.x; t.y += u.y; t.z += u.z; t.h += u.h;
      }
      v = t;
    }
    return v;
  };

  // [P; EG] x lv(k): accP/accE hold the lane's D outputs.  hook(rt) runs after the
  // products of row tile rt are issued (independent work placed there overlaps them).
  auto contract = [&](const Real (&k)[D], Real (&accP)[D], Real (&accE)[D], auto&& hook) {
    if constexpr (F64) {
      __syncthreads();
#pragma unroll
      for (int d = 0; d < D; ++d) {
        const int n = dim_of(d);
        lvbuf[cl * Npad + n] = (n < N) ? (double)(2 * k[d] - QM1) : 0.0;
      }
      __syncthreads();
#pragma unroll
      for (int d = 0; d < D; ++d) {
        const int n = dim_of(d);
        double sp = 0.0, se = 0.0;
        for (int n2 = 0; n2 < Npad; ++n2) {
          const double lv = lvbuf[cl * Npad + n2];
          sp = fma(Pd[(size_t)n * Npad + n2], lv, sp);
          se = fma(EGd[(size_t)n * Npad + n2], lv, se);
        }
        accP[d] = sp;
        accE[d] = se;
      }
#pragma unroll
      for (int rt = 0; rt < RTW; ++rt) hook(rt);
    } else if constexpr (CX) {
      // Complex planes: the matrix X (Nt x Nt) is stored as its real and imaginary planes, and
      //   V_re = Re(X) x_re - Im(X) x_im,   V_im = Im(X) x_re + Re(X) x_im
      // (the real-equivalent product of eq. sys_model, row 2m = V_re of antenna m, 2m+1 = V_im):
      // four products per (antenna tile, K block of 32 antennas), each plane fragment used twice.
      // K block kb, element j of lane l: antenna 16 (2 kb + j/4) + 4 (l/16) + j%4, which is the
      // lane's own antenna (Re in group dimension 2 i, Im in 2 i + 1) of antenna tile 2 kb + j/4.
      constexpr int KBX = RT / 4, KBWX = RTW / 4, ATW = RTW / 2, AT = RT / 2;
      half8 xr[KBX], xi[KBX], xn[KBX];
      bf16x8 br[KBX], bi[KBX], bn[KBX];
      // the wave's own K blocks (its antenna tiles), built from its registers
      half8 ownr[KBWX], owni[KBWX];
#pragma unroll
      for (int kbl = 0; kbl < KBWX; ++kbl) {
        uint32_t wr[4], wi[4];
#pragma unroll
        for (int q = 0; q < 4; ++q) {
          // elements j = 2q, 2q + 1: dimensions d and d + 2 (Re), d + 1 and d + 3 (Im)
          const int d = ((2 * kbl + (q >> 1)) * 4 + 2 * (q & 1)) * 2;
          wr[q] = lv_pair<QM1>(k[d], k[d + 2]);
          wi[q] = lv_pair<QM1>(k[d + 1], k[d + 3]);
        }
        __builtin_memcpy(&ownr[kbl], wr, 16);
        __builtin_memcpy(&owni[kbl], wi, 16);
      }
      if constexpr (WD > 1) {
        // every wave's K blocks of both planes through LDS (no register array indexed by the
        // wave's slice number)
        unsigned char* xb = xbuf + (xphase & 1) * 2 * KBX * 1024;
        ++xphase;
#pragma unroll
        for (int kbl = 0; kbl < KBWX; ++kbl) {
          const int kb = wd * KBWX + kbl;
          *(half8*)(xb + (size_t)kb * 1024 + lane * 16) = ownr[kbl];
          *(half8*)(xb + (size_t)(KBX + kb) * 1024 + lane * 16) = owni[kbl];
        }
        __syncthreads();
#pragma unroll
        for (int kb = 0; kb < KBX; ++kb) {
          xr[kb] = *(const half8*)(xb + (size_t)kb * 1024 + lane * 16);
          xi[kb] = *(const half8*)(xb + (size_t)(KBX + kb) * 1024 + lane * 16);
        }
      } else {
#pragma unroll
        for (int kb = 0; kb < KBX; ++kb) {
          xr[kb] = ownr[kb];
          xi[kb] = owni[kb];
        }
      }
#pragma unroll
      for (int kb = 0; kb < KBX; ++kb) {
        uint32_t u[4];
        __builtin_memcpy(u, &xi[kb], 16);
#pragma unroll
        for (int q = 0; q < 4; ++q) u[q] ^= 0x80008000u;                          // -x_im
        __builtin_memcpy(&xn[kb], u, 16);
        if constexpr (PM == PM_BF16X1) {
#pragma unroll
          for (int j = 0; j < 8; ++j) {
            br[kb][j] = (__bf16)(float)xr[kb][j];
            bi[kb][j] = (__bf16)(float)xi[kb][j];
          }
          // -x_im: the sign bits of the converted values (exact, as for the fp16 form)
          uint32_t ub[4];
          __builtin_memcpy(ub, &bi[kb], 16);
#pragma unroll
          for (int q = 0; q < 4; ++q) ub[q] ^= 0x80008000u;
          __builtin_memcpy(&bn[kb], ub, 16);
        }
      }
      const uint32_t fo = opaque_zero() + (uint32_t)lane * 16;
      // the first SPH half passes (planes) from LDS (p, pl are compile-time indices at every call), the others from L2
      auto frag = [&](int p, int pl, int atg, int kb) -> const unsigned char* {
        const uint32_t off = fo + (uint32_t)(((p * 2 + pl) * AT + atg) * KBX + kb) * 1024u;
        if (p * 2 + pl < SPH) return smem + off;
        return blk + kParamBytes + off;
      };
#pragma unroll
      for (int at = 0; at < ATW; ++at) {
        const int atg = (rt0 >> 1) + at;
        // the energy matrix's fragments of the antenna tile, all loads issued before the products
        uint4 fe[kEPasses][2][KBX];
#pragma unroll
        for (int p = 0; p < kEPasses; ++p)
#pragma unroll
          for (int pl = 0; pl < 2; ++pl)
#pragma unroll
            for (int kb = 0; kb < KBX; ++kb) fe[p][pl][kb] = *(const uint4*)frag(NPP + p, pl, atg, kb);
        f32x4 er = {0.f, 0.f, 0.f, 0.f}, ei = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
        for (int p = 0; p < kEPasses; ++p)
#pragma unroll
          for (int kb = 0; kb < KBX; ++kb) {
            half8 re, im;
            __builtin_memcpy(&re, &fe[p][0][kb], 16);
            __builtin_memcpy(&im, &fe[p][1][kb], 16);
            er = __builtin_amdgcn_mfma_f32_16x16x32_f16(re, xr[kb], er, 0, 0, 0);
            er = __builtin_amdgcn_mfma_f32_16x16x32_f16(im, xn[kb], er, 0, 0, 0);
            ei = __builtin_amdgcn_mfma_f32_16x16x32_f16(im, xr[kb], ei, 0, 0, 0);
            ei = __builtin_amdgcn_mfma_f32_16x16x32_f16(re, xi[kb], ei, 0, 0, 0);
          }
#pragma unroll
        for (int i = 0; i < 4; ++i) {
          accE[(at * 4 + i) * 2] = er[i];
          accE[(at * 4 + i) * 2 + 1] = ei[i];
        }
        if constexpr (PM != PM_NAIVE) {
          // then the proposal matrix's (its loads issue behind the energy products)
          uint4 fp[NPP > 0 ? NPP : 1][2][KBX];
#pragma unroll
          for (int p = 0; p < NPP; ++p)
#pragma unroll
            for (int pl = 0; pl < 2; ++pl)
#pragma unroll
              for (int kb = 0; kb < KBX; ++kb) fp[p][pl][kb] = *(const uint4*)frag(p, pl, atg, kb);
          f32x4 pr = {0.f, 0.f, 0.f, 0.f}, pi = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
          for (int p = 0; p < NPP; ++p)
#pragma unroll
            for (int kb = 0; kb < KBX; ++kb) {
              if constexpr (PM == PM_BF16X1) {
                bf16x8 re, im;
                __builtin_memcpy(&re, &fp[p][0][kb], 16);
                __builtin_memcpy(&im, &fp[p][1][kb], 16);
                pr = __builtin_amdgcn_mfma_f32_16x16x32_bf16(re, br[kb], pr, 0, 0, 0);
                pr = __builtin_amdgcn_mfma_f32_16x16x32_bf16(im, bn[kb], pr, 0, 0, 0);
                pi = __builtin_amdgcn_mfma_f32_16x16x32_bf16(im, br[kb], pi, 0, 0, 0);
                pi = __builtin_amdgcn_mfma_f32_16x16x32_bf16(re, bi[kb], pi, 0, 0, 0);
              } else {
                half8 re, im;
                __builtin_memcpy(&re, &fp[p][0][kb], 16);
                __builtin_memcpy(&im, &fp[p][1][kb], 16);
                pr = __builtin_amdgcn_mfma_f32_16x16x32_f16(re, xr[kb], pr, 0, 0, 0);
                pr = __builtin_amdgcn_mfma_f32_16x16x32_f16(im, xn[kb], pr, 0, 0, 0);
                pi = __builtin_amdgcn_mfma_f32_16x16x32_f16(im, xr[kb], pi, 0, 0, 0);
                pi = __builtin_amdgcn_mfma_f32_16x16x32_f16(re, xi[kb], pi, 0, 0, 0);
              }
            }
#pragma unroll
          for (int i = 0; i < 4; ++i) {
            accP[(at * 4 + i) * 2] = pr[i];
            accP[(at * 4 + i) * 2 + 1] = pi[i];
          }
        }
        hook(2 * at);
        hook(2 * at + 1);
        __builtin_amdgcn_sched_barrier(0);   // one antenna tile's fragments in registers at a time
      }
    } else {
      // B operand: this wave's K blocks from its own registers.  The packed
      // matrices are zero in the padding columns, so a padding dimension's
      // level (any in-range value) contributes nothing and needs no mask.
      half8 bh[KB];
      bf16x8 bb[KB];
#pragma unroll
      for (int kb = 0; kb < KBW; ++kb) {
        uint32_t wh[4];
#pragma unroll
        for (int q = 0; q < 4; ++q) {
          const int d = (2 * kb + (q >> 1)) * 4 + 2 * (q & 1);   // elements 2q, 2q + 1
          wh[q] = lv_pair<QM1>(k[d], k[d + 1]);
        }
        __builtin_memcpy(&bh[wd * KBW + kb], wh, 16);
        if constexpr (PM == PM_BF16X1) {
#pragma unroll
          for (int j = 0; j < 8; ++j) {
            const int d = (2 * kb + (j >> 2)) * 4 + (j & 3);
            bb[wd * KBW + kb][j] = (__bf16)(float)(2 * k[d] - QM1);
          }
        }
      }
      if constexpr (WD > 1) {
        // exchange the K blocks of the other waves through LDS
        unsigned char* xb = xbuf + (xphase & 1) * KB * 1024;
        ++xphase;
#pragma unroll
        for (int kb = 0; kb < KBW; ++kb) *(half8*)(xb + (size_t)(wd * KBW + kb) * 1024 + lane * 16) = bh[wd * KBW + kb];
        __syncthreads();
#pragma unroll
        for (int kb = 0; kb < KB; ++kb) {
          bh[kb] = *(const half8*)(xb + (size_t)kb * 1024 + lane * 16);
          if constexpr (PM == PM_BF16X1) {
#pragma unroll
            for (int j = 0; j < 8; ++j) bb[kb][j] = (__bf16)(float)bh[kb][j];
          }
        }
      }
      const uint32_t fo = opaque_zero() + (uint32_t)lane * 16;
      auto frag = [&](int p, int rtg, int kb) -> const unsigned char* {
        const uint32_t off = fo + (uint32_t)((p * RT + rtg) * KB + kb) * 1024u;
        if constexpr (MG) return blk + kParamBytes + off;
        else return smem + off;
      };
#pragma unroll
      for (int rt = 0; rt < RTW; ++rt) {
        const int rtg = rt0 + rt;
        f32x4 e = {0.f, 0.f, 0.f, 0.f};
        if constexpr (MG && RT >= 8) {
          // matrices from L2 at one wave per SIMD: issue every fragment load of the row tile
          // before the first product, so the loads overlap instead of waiting one by one
          uint4 fr[kEPasses + NPP][KB];
#pragma unroll
          for (int p = 0; p < kEPasses + NPP; ++p)
#pragma unroll
            for (int kb = 0; kb < KB; ++kb)
              fr[p][kb] = *(const uint4*)frag(p < kEPasses ? NPP + p : p - kEPasses, rtg, kb);
#pragma unroll
          for (int p = 0; p < kEPasses; ++p)
#pragma unroll
            for (int kb = 0; kb < KB; ++kb) {
              half8 av;
              __builtin_memcpy(&av, &fr[p][kb], 16);
              e = __builtin_amdgcn_mfma_f32_16x16x32_f16(av, bh[kb], e, 0, 0, 0);
            }
#pragma unroll
          for (int i = 0; i < 4; ++i) accE[rt * 4 + i] = e[i];
          if constexpr (PM != PM_NAIVE) {
            f32x4 q = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
            for (int p = 0; p < NPP; ++p)
#pragma unroll
              for (int kb = 0; kb < KB; ++kb) {
                if constexpr (PM == PM_BF16X1) {
                  bf16x8 av;
                  __builtin_memcpy(&av, &fr[kEPasses + p][kb], 16);
                  q = __builtin_amdgcn_mfma_f32_16x16x32_bf16(av, bb[kb], q, 0, 0, 0);
                } else {
                  half8 av;
                  __builtin_memcpy(&av, &fr[kEPasses + p][kb], 16);
                  q = __builtin_amdgcn_mfma_f32_16x16x32_f16(av, bh[kb], q, 0, 0, 0);
                }
              }
#pragma unroll
            for (int i = 0; i < 4; ++i) accP[rt * 4 + i] = q[i];
          }
          hook(rt);
          continue;
        }
#pragma unroll
        for (int p = 0; p < kEPasses; ++p)
#pragma unroll
          for (int kb = 0; kb < KB; ++kb)
            e = __builtin_amdgcn_mfma_f32_16x16x32_f16(*(const half8*)frag(NPP + p, rtg, kb), bh[kb], e, 0, 0, 0);
#pragma unroll
        for (int i = 0; i < 4; ++i) accE[rt * 4 + i] = e[i];
        if constexpr (PM != PM_NAIVE) {
          f32x4 q = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
          for (int p = 0; p < NPP; ++p)
#pragma unroll
            for (int kb = 0; kb < KB; ++kb) {
              if constexpr (PM == PM_BF16X1)
                q = __builtin_amdgcn_mfma_f32_16x16x32_bf16(*(const bf16x8*)frag(p, rtg, kb), bb[kb], q, 0, 0, 0);
              else
                q = __builtin_amdgcn_mfma_f32_16x16x32_f16(*(const half8*)frag(p, rtg, kb), bh[kb], q, 0, 0, 0);
            }
#pragma unroll
          for (int i = 0; i < 4; ++i) accP[rt * 4 + i] = q[i];
        }
        hook(rt);
        __builtin_amdgcn_sched_barrier(0);   // keep the hook's work beside this tile's products
      }
    }
  };

  // Proposal centre and energy gradient at state k from the contraction.
  auto nohook = [](int) {};
  auto grad_at = [&](const Real (&k)[D], Real (&mu)[D], Real (&eg)[D], auto&& hook) {
    Real accP[D], accE[D];
    contract(k, accP, accE, hook);
#pragma unroll
    for (int d = 0; d < D; ++d) {
      const int n = dim_of(d);
      const Real g = accE[d] * sE - ezv[n];
      Real shift;
      if constexpr (PM == PM_NAIVE) shift = rho * g;
      else shift = accP[d] * sP - pbv[n];
      eg[d] = g;
      mu[d] = Real(k[d]) - shift;
    }
  };
  // ... and the log2 normalisers.
  auto proposal_at = [&](const Real (&k)[D], Real (&mu)[D], Real (&lz)[D], Real (&eg)[D]) {
    grad_at(k, mu, eg, nohook);
#pragma unroll
    for (int d = 0; d < D; ++d) lz[d] = log2_norm<Q, WIN, W, TAB>(mu[d], kL, wc);
  };

  // Network features of the lane's antenna in slot (rt, i2) at state k with plain centre mu.
  constexpr float kCq = 0.5f * (Q - 1), kIhq = 2.0f / Q;
  const float lq4 = 0.25f * (Q == 2 ? 1.f : Q == 4 ? 2.f : Q == 8 ? 3.f : 4.f);
  auto feats = [&](const Real (&k)[D], const Real (&m)[D], int rt, int i2, float (&f)[kMlpIn]) {
    const int d0 = rt * 4 + 2 * i2;
    const int n0 = dim_of(d0);
    f[0] = ((float)m[d0] - kCq) * kIhq;
    f[1] = ((float)m[d0 + 1] - kCq) * kIhq;
    f[2] = ((float)k[d0] - kCq) * kIhq;
    f[3] = ((float)k[d0 + 1] - kCq) * kIhq;
    f[4] = afv[n0];
    f[5] = afv[n0 + 1];
    f[6] = lq4;
  };
  // Learned proposal (centre muL, log2 precision kLL) at state k with plain centre m.
  auto learned_at = [&](const Real (&k)[D], const Real (&m)[D], Real (&muL)[D], Real (&kLL)[D]) {
    const uint32_t mo = opaque_zero();
#pragma unroll
    for (int rt = 0; rt < RTW; ++rt)
#pragma unroll
      for (int i2 = 0; i2 < 2; ++i2) {
        float f[kMlpIn];
        feats(k, m, rt, i2, f);
        const mlp_f32x4 o = mlp_eval4<mlp_gw1(WD)>(mlp_lds, mo, mlp_inputs(f[0], f[1], f[2], f[3], f[4], f[5], f[6]));
#pragma unroll
        for (int p = 0; p < 2; ++p) {
          const int d = rt * 4 + 2 * i2 + p;
          const float b = fminf(fmaxf(o[2 + p], -4.0f), 4.0f);
          muL[d] = m[d] + o[p];
          kLL[d] = kL * ex2(b);
        }
      }
  };
  // Training rows (features, plain centre, natural-log precision, Q) of the lane's antennas at k.
  auto write_rows = [&](const Real (&k)[D], const Real (&m)[D]) {
    const int Nt = N >> 1;
    const int64_t sym0 = a.desc ? a.desc[inst].sym_off : (int64_t)inst * Nt;
#pragma unroll
    for (int rt = 0; rt < RTW; ++rt)
#pragma unroll
      for (int i2 = 0; i2 < 2; ++i2) {
        const int d0 = rt * 4 + 2 * i2;
        const int ant = dim_of(d0) >> 1;
        if (ant < Nt) {
          float f[kMlpIn];
          feats(k, m, rt, i2, f);
          float* row = a.train_rows + ((size_t)sym0 * a.C + (size_t)chain * Nt + ant) * kTrainRow;
#pragma unroll
          for (int i = 0; i < kMlpIn; ++i) row[i] = f[i];
          row[7] = (float)m[d0];
          row[8] = (float)m[d0 + 1];
          row[9] = (float)(kL / Real(kLog2e));
          row[10] = (float)Q;
          row[11] = 0.f;
        }
      }
  };

  // log2 q_n(j | .) for a level j given the cached mode and normaliser
  auto lq = [&](Real j, Real mu, Real lz) {
    const Real t = j - mu;
    return -kL * t * t - lz;
  };

  Real kc[D];   // levels (small integers, exact in Real)
  Real mu[D], lz[D], eg[D];
  bool valid[D];
#pragma unroll
  for (int d = 0; d < D; ++d) valid[d] = FULL || dim_of(d) < N;

  if constexpr (EVAL) {
    // transition quantities for a given pair (x_from -> x_to)
    const size_t row = ((size_t)inst * a.C + (live ? chain : 0)) * N;
    Real kt[D];
#pragma unroll
    for (int d = 0; d < D; ++d) {
      const int n = dim_of(d);
      kc[d] = (live && valid[d]) ? Real(a.x_from[row + n]) : Real(0);
      kt[d] = (live && valid[d]) ? Real(a.x_to[row + n]) : Real(0);
    }
    Real lqf = 0, lqr = 0, T2 = 0;
    Real mup[D], lzp[D], egp[D];
    // per-dimension forward terms (log2 units) for the optional per-dimension output
    auto dim_out = [&](int d, Real v) {
      if (a.eval_dim && live && valid[d])
        a.eval_dim[((size_t)inst * a.C + chain) * N + dim_of(d)] = (double)v * (1.0 / kLog2e);
    };
    if constexpr (MHG) {
      grad_at(kc, mu, eg, nohook);
      grad_at(kt, mup, egp, nohook);
#pragma unroll
      for (int d = 0; d < D; ++d)
        if (valid[d]) {
          const Real fd = mhgd_log2_cell<Q>(kt[d], mu[d], msig);
          lqf += fd;
          lqr += mhgd_log2_cell<Q>(kc[d], mup[d], msig);
          T2 -= Real(kt[d] - kc[d]) * (eg[d] + egp[d]);
          dim_out(d, fd);
        }
    } else if constexpr (LRN) {
      // the learned kernel alone (the mixture's other component is the plain kernel)
      Real muL[D], kLL[D], muLp[D], kLLp[D];
      grad_at(kc, mu, eg, nohook);
      learned_at(kc, mu, muL, kLL);
      grad_at(kt, mup, egp, nohook);
      learned_at(kt, mup, muLp, kLLp);
#pragma unroll
      for (int d = 0; d < D; ++d)
        if (valid[d]) {
          const Real tf = Real(kt[d]) - muL[d], tr = Real(kc[d]) - muLp[d];
          const Real fd = -kLL[d] * tf * tf - log2_norm<Q, 0, W, false>(muL[d], kLL[d], wc);
          lqf += fd;
          lqr += -kLLp[d] * tr * tr - log2_norm<Q, 0, W, false>(muLp[d], kLLp[d], wc);
          T2 -= Real(kt[d] - kc[d]) * (eg[d] + egp[d]);
          dim_out(d, fd);
        }
    } else {
      proposal_at(kc, mu, lz, eg);
#pragma unroll
      for (int d = 0; d < D; ++d)
        if (valid[d]) {
          const Real fd = lq(kt[d], mu[d], lz[d]);
          lqf += fd;
          dim_out(d, fd);
        }
      proposal_at(kt, mup, lzp, egp);
#pragma unroll
      for (int d = 0; d < D; ++d)
        if (valid[d]) {
          lqr += lq(kc[d], mup[d], lzp[d]);
          T2 -= Real(kt[d] - kc[d]) * (eg[d] + egp[d]);
        }
    }
    if constexpr (WD > 1) {
      const Red r = chain_sum(Red{(float)lqf, (float)lqr, (float)T2, 0u});
      lqf = r.x; lqr = r.y; T2 = r.z;
    } else {
      lqf = bfly4(lqf); lqr = bfly4(lqr); T2 = bfly4(T2);
    }
    if (live && h == 0 && wd == 0) {
      double* o = a.eval_out + ((size_t)inst * a.C + chain) * 4;
      const double ln2 = 1.0 / kLog2e;
      o[0] = (double)lqf * ln2;
      o[1] = (double)lqr * ln2;
      o[2] = (double)T2 * ln2;
      // MHGD's test leaves the proposal ratio out
      o[3] = (MHG ? (double)T2 : ((double)T2 + (double)lqr - (double)lqf)) * ln2;
    }
    return;
  } else {
    const uint32_t key0 = a.key0, key1 = a.key1;
    // initial state from the t = 0 words
#pragma unroll
    for (int rt = 0; rt < RTW; ++rt) {
      uint32_t c[4] = {(uint32_t)(gdim(rt) >> 2), 0u, (uint32_t)chain, rctr};
      philox4x32_10<true>(c, key0, key1);
#pragma unroll
      for (int i = 0; i < 4; ++i) kc[rt * 4 + i] = Real((int)(((uint64_t)(c[i] >> 8) * Q) >> 24));
    }
    Real muL[D], kLL[D];  // cached learned proposal (LRN)
    Real lzs = 0;         // sum of the lane's log2 normalisers at the current state (plain kernel)
    if constexpr (LRN) {
      grad_at(kc, mu, eg, nohook);
      learned_at(kc, mu, muL, kLL);
    } else {
      grad_at(kc, mu, eg, nohook);
      if constexpr (KND == 0) {
#pragma unroll
        for (int d = 0; d < D; ++d) lzs += log2_norm<Q, WIN, W, TAB>(mu[d], kL, wc);
      }
    }
    // E(x) = ||y||^2 + x^T g - z^T x = ||y||^2 + (eunit/2) sum_n lv_n (eg_n - ez_n)
    Real ep = 0;
#pragma unroll
    for (int d = 0; d < D; ++d) {
      const int n = dim_of(d);
      ep += valid[d] ? Real(2 * kc[d] - QM1) * (eg[d] - ezv[n]) : Real(0);
    }
    if constexpr (WD > 1) ep = chain_sum(Red{(float)ep, 0.f, 0.f, 0u}).x;
    else ep = bfly4(ep);
    const Real eunit = (Real)ip.eunit;
    Real E = (Real)ip.yy + Real(0.5) * eunit * ep;
    Real Ebest = E;
    // the levels of group rt as 4 bytes
    // (the conversions stay in the branches that use them: an empty asm per value keeps the
    // compiler from hoisting them into every transition)
    auto pack4 = [&](int rt) {
      Real v[4];
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        v[i] = kc[rt * 4 + i];
        asm volatile("" : "+v"(v[i]));
      }
      return (uint32_t)v[0] | ((uint32_t)v[1] << 8) | ((uint32_t)v[2] << 16) | ((uint32_t)v[3] << 24);
    };
    uint32_t kbest[RTW];
#pragma unroll
    for (int rt = 0; rt < RTW; ++rt) kbest[rt] = pack4(rt);
    int nacc = 0;
    uint32_t abits = 0;
    const size_t trow = (size_t)rid * a.C + (live ? chain : 0);

    // Random words of transition t (counter (4 rt + h, t, chain, instance)).  They do not
    // depend on the chain: on the one-wave layouts with up to 4 row tiles the words of
    // t + 1 are generated while the contraction of t runs on the matrix cores (elsewhere
    // the registers they would hold meanwhile are not free).
    uint32_t w[RTW][4];
    auto word_block = [&](int rt, int tt) {
      w[rt][0] = (uint32_t)(gdim(rt) >> 2); w[rt][1] = (uint32_t)tt; w[rt][2] = (uint32_t)chain; w[rt][3] = rctr;
      philox4x32_10<true>(w[rt], key0, key1);
    };
    if constexpr (PIPE) {
#pragma unroll
      for (int rt = 0; rt < RTW; ++rt) word_block(rt, 1);
    }
    for (int t = 1; t <= a.T; ++t) {
      if constexpr (!PIPE) {
#pragma unroll
        for (int rt = 0; rt < RTW; ++rt) word_block(rt, t);
      }
      // kernel choice of the mixture (LRN): learned unless the uniform from the
      // low bytes of words 4, 5, 6 falls below eps; every lane of the chain
      // regenerates block 1 of the stream, so no lane has to broadcast it
      bool useL = false;
      if constexpr (LRN) {
        uint32_t wm[4] = {1u, (uint32_t)t, (uint32_t)chain, rctr};
        philox4x32_10<true>(wm, key0, key1);
        useL = low_bytes24(wm[0], wm[1], wm[2]) >= a.mix_thr;
      }
      // 1. draw x' (padding dimensions never move) and -log q(x'|x); the plain
      // kernel's terms are collected as kL sum (x'_n - mu_n)^2 + sum lz_n
      Real kp[D];
      Real S = 0, tq = 0;
#pragma unroll
      for (int d = 0; d < D; ++d) {
        if constexpr (MHG) {
          // gradient step + Gaussian random walk, mapped to the nearest level (rint, clamped)
          const Real kd = mode_of<Q>(mu[d] + msig * gauss_of_word<Real>(w[d >> 2][d & 3]));
          kp[d] = valid[d] ? kd : kc[d];
        } else if constexpr (LRN) {
          const float ms = useL ? muL[d] : mu[d], ks = useL ? kLL[d] : (float)kL;
          float lzf;
          const float kd = (float)draw_level_lz<Q>(ms, ks, u23f(w[d >> 2][d & 3]), lzf);
          kp[d] = valid[d] ? kd : kc[d];
          const float t0 = float(kp[d]) - ms;
          S -= valid[d] ? (-ks * t0 * t0 - lzf) : 0.f;
        } else {
          const Real kd = draw_level<Q, WIN, W, TAB>(mu[d], kL, wc, w[d >> 2][d & 3]);
          kp[d] = valid[d] ? kd : kc[d];
          const Real t0 = Real(kp[d]) - mu[d];
          tq += t0 * t0;
        }
      }
      if constexpr (KND == 0) S = kL * tq + lzs;
      // the MH word is held by the lanes that own dimensions 0..3 (h = 0 of the first slice)
      const uint32_t um = low_bytes24(w[0][0], w[0][1], w[0][2]);
      auto next_words = [&](int rt) {
        if constexpr (PIPE) {
          word_block(rt, t + 1);
          // pin the block here: otherwise it is sunk to the end of the iteration
          asm volatile("" : "+v"(w[rt][0]), "+v"(w[rt][1]), "+v"(w[rt][2]), "+v"(w[rt][3]));
        }
      };
      // 2-3. gradient at x', proposal at x', + log q(x|x'), energy term.
      // A padding dimension contributes nothing: its contraction rows are zero,
      // so mu' = mu, lz' = lz and its two log q terms cancel.
      Real mup[D], egp[D], lzps = 0;
      Real muLp[D], kLLp[D];
      Real T2 = 0;
      if constexpr (MHG) {
        grad_at(kp, mup, egp, next_words);
#pragma unroll
        for (int d = 0; d < D; ++d) T2 -= (Real(kp[d]) - Real(kc[d])) * (eg[d] + egp[d]);
      } else if constexpr (LRN) {
        grad_at(kp, mup, egp, next_words);
        learned_at(kp, mup, muLp, kLLp);
#pragma unroll
        for (int d = 0; d < D; ++d) {
          const float mr = useL ? muLp[d] : mup[d], kr = useL ? kLLp[d] : (float)kL;
          const float lzr = log2_norm<Q, 0, W, false>(mr, kr, wc);
          const float t0 = float(kc[d]) - mr;
          S += valid[d] ? (-kr * t0 * t0 - lzr) : 0.f;
          T2 -= (Real(kp[d]) - Real(kc[d])) * (eg[d] + egp[d]);
        }
      } else {
        grad_at(kp, mup, egp, next_words);
        // sum of the lane's log2 normalisers as log2 of the product of the weight sums
        // (each in [1, Q], so the product of D of them stays far inside the exponent
        // range): one logarithm per lane instead of one per dimension
        Real tr = 0, zp = 1, bs = 0;
#pragma unroll
        for (int d = 0; d < D; ++d) {
          Real Z, b2;
          norm_parts<Q, WIN, W, TAB>(mup[d], kL, wc, Z, b2);
          zp *= Z;
          bs += b2;
          const Real t0 = Real(kc[d]) - mup[d];
          tr += t0 * t0;
          T2 -= (Real(kp[d]) - Real(kc[d])) * (eg[d] + egp[d]);
        }
        lzps = lg2(zp) - kL * bs;
        S -= kL * tr + lzps;
      }
      S += T2;
      // 4. MH: accept iff  log ratio > log u  (eq. acc_prob: A > u)
      {
        Real lu;
        if constexpr (F64) lu = lg2((double)um * 5.9604644775390625e-08);
        else lu = lg2((float)um * 5.9604644775390625e-08f);
        S -= (h == 0 && wd == 0) ? lu : Real(0);
      }
      if constexpr (WD > 1) {
        const Red r = chain_sum(Red{(float)S, (float)T2, 0.f, 0u});
        S = r.x; T2 = r.y;
      } else {
        S = bfly4(S);
        T2 = bfly4(T2);
      }
      const bool acc = S > Real(0);
      // 5. select
#pragma unroll
      for (int d = 0; d < D; ++d) {
        kc[d] = acc ? kp[d] : kc[d];
        mu[d] = acc ? mup[d] : mu[d];
        eg[d] = acc ? egp[d] : eg[d];
        if constexpr (LRN) {
          muL[d] = acc ? muLp[d] : muL[d];
          kLL[d] = acc ? kLLp[d] : kLL[d];
        }
      }
      if constexpr (KND == 0) lzs = acc ? lzps : lzs;
      E = acc ? E - T2 * eunit : E;
      nacc += acc ? 1 : 0;
      if (E < Ebest) {
        Ebest = E;
#pragma unroll
        for (int rt = 0; rt < RTW; ++rt) kbest[rt] = pack4(rt);
      }
      if (a.trace_accept) {
        abits |= (acc ? 1u : 0u) << ((t - 1) & 31);
        if (((t & 31) == 0 || t == a.T) && live && h == 0 && wd == 0) {
          a.trace_accept[trow * a.trace_words + ((t - 1) >> 5)] = abits;
        }
        if ((t & 31) == 0) abits = 0;
      }
      if (a.trace_hash) {
        uint32_t hs = 0;
#pragma unroll
        for (int d = 0; d < D; ++d) {
          Real v = kc[d];
          asm volatile("" : "+v"(v));
          hs += valid[d] ? ((uint32_t)v + 1u) * hash_mult(dim_of(d)) : 0u;
        }
        if constexpr (WD > 1) {
          hs = chain_sum(Red{0.f, 0.f, 0.f, hs}).h;
        } else {
          hs += __shfl_xor(hs, 16);
          hs += __shfl_xor(hs, 32);
        }
        if (live && h == 0 && wd == 0) a.trace_hash[trow * a.T + (t - 1)] = hs;
      }
    }

    // results for the estimator and the optional outputs
    if constexpr (!F64 && PM != PM_NAIVE) {
      if (a.train_rows && live) write_rows(kc, mu);
    }
    if (live) {
      const StateOff so = state_offsets(a.Cpad, Npad);
      unsigned char* st = a.ws_state + (size_t)inst * a.state_stride;
      if constexpr (!F64) {
        // the energy gradient at the final state: the estimator's H^H r comes from it
        float* egs = (float*)(st + so.eg) + (size_t)chain * Npad;
#pragma unroll
        for (int d = 0; d < D; ++d) egs[dim_of(d)] = valid[d] ? (float)eg[d] : 0.0f;
      }
#pragma unroll
      for (int rt = 0; rt < RTW; ++rt) {
        const int n0 = gdim(rt);
        const uint32_t cur = pack4(rt);
        *(uint32_t*)(st + so.k + (size_t)chain * Npad + n0) = cur;
        *(uint32_t*)(st + so.kbest + (size_t)chain * Npad + n0) = kbest[rt];
        if (a.final_state) {
#pragma unroll
          for (int i = 0; i < 4; ++i)
            if (n0 + i < N) a.final_state[fs_base + (size_t)chain * N + n0 + i] = (int8_t)(int)kc[rt * 4 + i];
        }
      }
      if (h == 0 && wd == 0) {
        ((double*)(st + so.ebest))[chain] = (double)Ebest;
        ((int32_t*)(st + so.nacc))[chain] = nacc;
        if (a.accept_count) a.accept_count[(size_t)rid * a.C + chain] = nacc;
      }
    }
  }
}

// Direct launch (PERS false): instance blockIdx.x, chain group blockIdx.y.  Persistent launch:
// items from the list until it is exhausted, each with its class's arguments (a separate
// instantiation, so that the direct kernels keep their registers).
template <typename Real, int RTW, int WD, bool MG, int Q, int PM, bool EVAL, int WIN, int KND, bool CX, bool PERS,
          bool FULL = false>
__device__ __forceinline__ void sampler_entry(const SamplerArgs& a, const Persist& p) {
  if constexpr (!PERS) {
    sampler_body<Real, RTW, WD, MG, Q, PM, EVAL, WIN, KND, CX, FULL>(a, blockIdx.x, blockIdx.y);
  } else {
    extern __shared__ __attribute__((aligned(16))) unsigned char smem[];
    for (;;) {
      const int it = persist_take(p, smem);
      if (it >= p.n_items) break;
      const WorkItem w = p.items[it];
      const SamplerArgs ca = ((const SamplerArgs*)p.cls)[__builtin_amdgcn_readfirstlane(w.cls)];
      sampler_body<Real, RTW, WD, MG, Q, PM, EVAL, WIN, KND, CX>(ca, __builtin_amdgcn_readfirstlane(w.inst),
                                                                 __builtin_amdgcn_readfirstlane(w.cg));
    }
    persist_done(p);
  }
}

template <typename Real, int RTW, int WD, bool MG, int Q, int PM, bool EVAL, int WIN, int KND, bool CX = false,
          bool PERS = false>
__global__ __launch_bounds__(256) void sampler_kernel(SamplerArgs a, Persist p) {
  sampler_entry<Real, RTW, WD, MG, Q, PM, EVAL, WIN, KND, CX, PERS>(a, p);
}

// The same kernel held to two waves per SIMD (at most 256 registers): the
// learned variant with two row tiles per wave fits without spilling.
template <typename Real, int RTW, int WD, bool MG, int Q, int PM, bool EVAL, int WIN, int KND, bool CX = false,
          bool PERS = false, bool FULL = false>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(2))) void sampler_kernel_w2(SamplerArgs a, Persist p) {
  sampler_entry<Real, RTW, WD, MG, Q, PM, EVAL, WIN, KND, CX, PERS, FULL>(a, p);
}

// ... in 512-thread workgroups (two chain blocks of the four-wave layout).
template <typename Real, int RTW, int WD, bool MG, int Q, int PM, bool EVAL, int WIN, int KND, bool CX = false,
          bool PERS = false, bool FULL = false>
__global__ __launch_bounds__(512) __attribute__((amdgpu_waves_per_eu(2))) void sampler_kernel_w2_512(SamplerArgs a, Persist p) {
  sampler_entry<Real, RTW, WD, MG, Q, PM, EVAL, WIN, KND, CX, PERS, FULL>(a, p);
}

// LDS bytes of a configuration.
// Whether the four-wave layout runs its two-waves-per-SIMD kernel (the windowed preconditioned
// float chain), which then holds two 16-chain blocks in a 512-thread workgroup.
inline bool split4_wide(const Shape& sh) {
  return !sh.fp64 && !sh.lrn && !sh.mhgd && sh.pm != PM_NAIVE && sh.win > 0;
}

// 16-chain blocks per workgroup of a dimension-split layout (wd waves each): up to 4 waves, or
// 8 for the wide four-wave case.
inline int split_slots(const Shape& sh, int wd) {
  const int cb = sh.cbw > 0 ? sh.cbw : 4, blocks = sh.Cpad / 16;
  const int cap = (wd == 4 && split4_wide(sh)) ? 2 : 4 / wd;
  int n = cb < cap ? cb : cap;
  return n < blocks ? n : blocks;
}

inline size_t sampler_cfg_lds(const Shape& sh, int rtw, int wd, bool mg, int waves, bool cx = false) {
  if (sh.fp64) return sh.frag_bytes + (size_t)waves * 16 * sh.Npad * sizeof(double);
  const int RT = rtw * wd, KB = RT / 2;
  const size_t mat = (size_t)(p_passes(sh.pm) + kEPasses) * RT * KB * 1024;
  size_t staged = mg ? 0 : (RT <= 4 ? sh.frag_bytes : mat);
  if (cx && mg) {
    const int halves = cx_lds_halves(RT, sh.win > 0), all = 2 * (p_passes(sh.pm) + kEPasses);
    staged = (size_t)(halves < all ? halves : all) * RT * RT / 8 * 1024;
  }
  staged = (staged + 15) & ~(size_t)15;
  if (wd > 1) staged += (size_t)(waves / wd) * (2 * (size_t)KB * 1024 + 2 * (size_t)wd * 16 * sizeof(Red));
  if (sh.lrn) staged += wd > 1 ? mlp_lds_bytes<mlp_gw1(2)>() : mlp_lds_bytes<mlp_gw1(1)>();
  if (sh.win > 0 && win_table(rtw, wd, mg)) staged += kCtabBytes;
  return staged;
}

template <typename Real, int RTW, int WD, bool MG, int Q, int PM, int WIN, int KND = 0, bool CX = false>
hipError_t launch_t(const Shape& sh, const SamplerArgs& a, bool eval, hipStream_t s, const Persist* p, int gn,
                    KernelCfg* cfg) {
  constexpr bool LRN = KND == 1;
  const int chain_blocks = sh.Cpad / 16;
  int waves, gy;
  if (WD > 1) {
    const int slots = eval ? 1 : split_slots(sh, WD);   // evaluation kernels keep 256-thread workgroups
    waves = WD * slots;
    gy = (chain_blocks + slots - 1) / slots;
  }
  else {
    const int cb = sh.cbw > 0 ? sh.cbw : 4;
    waves = chain_blocks < cb ? chain_blocks : cb;
    gy = (chain_blocks + waves - 1) / waves;
  }
  const dim3 grid(a.n_inst, gy);
  const size_t lds = sampler_cfg_lds(sh, RTW, WD, MG, waves, CX);
  // two waves per SIMD where the chain loop fits 256 registers without spilling: the learned
  // two-tile layouts, and the plain four-tile layouts except the naive proposal's four-wave one
  // (the evaluation kernels keep the default).  The four-wave layout without the window table
  // (Q <= 4) needs ~270 registers unbounded: bounded it is faster alone, but beside other
  // classes' kernels (graph branches) the unbounded variant's spare registers serve them better
  constexpr bool kW2Eval = LRN && RTW == 2;
  constexpr bool kW2 = kW2Eval || (!LRN && RTW == 4 && !std::is_same<Real, double>::value && (WD < 4 || (WIN > 0 && PM != PM_NAIVE)));
  constexpr bool kW2Alone = !LRN && RTW == 4 && !std::is_same<Real, double>::value && WD == 4 && WIN == 0 && PM != PM_NAIVE;
  void (*k)(SamplerArgs, Persist);
  // persistent instantiations (plans): the plain float chains
  constexpr bool kPersOK = KND == 0 && !std::is_same<Real, double>::value;
  // direct launches of the plain float complex-plane chains: a variant without the padding masks
  // for instances whose dimensions fill the tiles (fewer instructions per transition)
  constexpr bool kFull = KND == 0 && CX && !std::is_same<Real, double>::value;
  const bool full = sh.N == sh.Npad;
  const bool pers = (p != nullptr || cfg != nullptr) && !eval;
  if (pers) {
    if constexpr (kPersOK) {
      if (waves > 4) {
        if constexpr (kW2 && WD == 4) k = sampler_kernel_w2_512<Real, RTW, WD, MG, Q, PM, false, WIN, KND, CX, true>;
        else return hipErrorInvalidConfiguration;
      } else if constexpr (kW2) {
        k = sampler_kernel_w2<Real, RTW, WD, MG, Q, PM, false, WIN, KND, CX, true>;
      } else {
        k = sampler_kernel<Real, RTW, WD, MG, Q, PM, false, WIN, KND, CX, true>;
      }
    } else {
      return hipErrorNotSupported;
    }
  } else if (eval) {
    if constexpr (kW2Eval) k = sampler_kernel_w2<Real, RTW, WD, MG, Q, PM, true, WIN, KND, CX>;
    else k = sampler_kernel<Real, RTW, WD, MG, Q, PM, true, WIN, KND, CX>;
  } else if (waves > 4) {
    if constexpr (kW2 && WD == 4 && !LRN) {
      if constexpr (kFull) k = full ? sampler_kernel_w2_512<Real, RTW, WD, MG, Q, PM, false, WIN, KND, CX, false, true>
                                    : sampler_kernel_w2_512<Real, RTW, WD, MG, Q, PM, false, WIN, KND, CX>;
      else k = sampler_kernel_w2_512<Real, RTW, WD, MG, Q, PM, false, WIN, KND, CX>;
    } else {
      return hipErrorInvalidConfiguration;
    }
  } else {
    if constexpr (kW2 && kFull) k = full ? sampler_kernel_w2<Real, RTW, WD, MG, Q, PM, false, WIN, KND, CX, false, true>
                                         : sampler_kernel_w2<Real, RTW, WD, MG, Q, PM, false, WIN, KND, CX>;
    else if constexpr (kW2) k = sampler_kernel_w2<Real, RTW, WD, MG, Q, PM, false, WIN, KND, CX>;
    else if constexpr (kW2Alone) k = sh.share ? sampler_kernel<Real, RTW, WD, MG, Q, PM, false, WIN, KND, CX>
                                              : sampler_kernel_w2<Real, RTW, WD, MG, Q, PM, false, WIN, KND, CX>;
    else k = sampler_kernel<Real, RTW, WD, MG, Q, PM, false, WIN, KND, CX>;
  }
  if (cfg) {
    cfg->k = (const void*)k;
    cfg->threads = 64 * waves;
    cfg->lds = lds;
    cfg->gx = (int)grid.x;
    cfg->gy = (int)grid.y;
    return hipSuccess;
  }
  // a persistent launch keeps one more aligned word after the body's LDS (the item broadcast)
  const size_t lds_run = p ? ((p->lds_off + 4 + 15) & ~(size_t)15) : lds;
  if (lds_run > 65536) {
    hipError_t e = hipFuncSetAttribute((const void*)k, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds_run);
    if (e != hipSuccess) return e;
  }
  if (p) hipLaunchKernelGGL(k, dim3(gn), dim3(64 * waves), lds_run, s, a, *p);
  else hipLaunchKernelGGL(k, grid, dim3(64 * waves), lds, s, a, Persist{});
  return hipGetLastError();
}

template <typename Real, int RTW, int WD, bool MG, int PM, bool CX = false>
hipError_t launch_q(const Shape& sh, const SamplerArgs& a, bool eval, hipStream_t s, const Persist* p, int gn,
                    KernelCfg* cfg) {
  // the 3-level window is used only for Q >= 8 (it would not be smaller otherwise)
  constexpr int WN = std::is_same<Real, double>::value ? 0 : 3;   // the float path only
  const bool win = WN > 0 && sh.win == 3;
  switch (sh.Q) {
    case 2: return launch_t<Real, RTW, WD, MG, 2, PM, 0, 0, CX>(sh, a, eval, s, p, gn, cfg);
    case 4: return launch_t<Real, RTW, WD, MG, 4, PM, 0, 0, CX>(sh, a, eval, s, p, gn, cfg);
    case 8: return win ? launch_t<Real, RTW, WD, MG, 8, PM, WN, 0, CX>(sh, a, eval, s, p, gn, cfg)
                       : launch_t<Real, RTW, WD, MG, 8, PM, 0, 0, CX>(sh, a, eval, s, p, gn, cfg);
    case 16: return win ? launch_t<Real, RTW, WD, MG, 16, PM, WN, 0, CX>(sh, a, eval, s, p, gn, cfg)
                        : launch_t<Real, RTW, WD, MG, 16, PM, 0, 0, CX>(sh, a, eval, s, p, gn, cfg);
  }
  return hipErrorInvalidValue;
}

// Configurations (row tiles per wave, waves per chain block, matrices in L2):
//   cfg 0: RT 2, 1 wave, LDS     cfg 1: RT 4, 1 wave, LDS     cfg 2: RT 8, 1 wave, LDS
//   cfg 3: RT 8 as 2 waves x 4, L2     cfg 4: RT 16 as 4 waves x 4, L2
//   cfg 7, 8: cfg 3, 4 with the matrices stored as complex planes
//   cfg 9: cfg 1 with complex-plane matrices (half the LDS: four workgroups per CU at fp32)
template <typename Real, int PM>
hipError_t launch_rt(const Shape& sh, const SamplerArgs& a, bool eval, hipStream_t s, const Persist* p, int gn,
                    KernelCfg* cfg) {
  if constexpr (std::is_same<Real, double>::value) {
    switch (sh.RT) {
      case 2: return launch_q<Real, 2, 1, false, PM>(sh, a, eval, s, p, gn, cfg);
      case 4: return launch_q<Real, 4, 1, false, PM>(sh, a, eval, s, p, gn, cfg);
    }
    return hipErrorInvalidValue;
  } else {
    switch (sh.cfg) {
      case 0: return launch_q<Real, 2, 1, false, PM>(sh, a, eval, s, p, gn, cfg);
      case 1: return launch_q<Real, 4, 1, false, PM>(sh, a, eval, s, p, gn, cfg);
      case 2: return launch_q<Real, 8, 1, false, PM>(sh, a, eval, s, p, gn, cfg);
      case 3: return launch_q<Real, 4, 2, true, PM>(sh, a, eval, s, p, gn, cfg);
      case 4: return launch_q<Real, 4, 4, true, PM>(sh, a, eval, s, p, gn, cfg);
      case 7: return launch_q<Real, 4, 2, true, PM, true>(sh, a, eval, s, p, gn, cfg);
      case 8: return launch_q<Real, 4, 4, true, PM, true>(sh, a, eval, s, p, gn, cfg);
      case 9: return launch_q<Real, 4, 1, false, PM, true>(sh, a, eval, s, p, gn, cfg);
    }
    return hipErrorInvalidValue;
  }
}

// The MHGD baseline on the plain layouts (every Q weighted directly: there is no window).
template <typename Real, int RTW, int WD, bool MG, int PM, bool CX = false>
hipError_t launch_q_mhg(const Shape& sh, const SamplerArgs& a, bool eval, hipStream_t s, const Persist* p, int gn,
                    KernelCfg* cfg) {
  switch (sh.Q) {
    case 2: return launch_t<Real, RTW, WD, MG, 2, PM, 0, 2, CX>(sh, a, eval, s, p, gn, cfg);
    case 4: return launch_t<Real, RTW, WD, MG, 4, PM, 0, 2, CX>(sh, a, eval, s, p, gn, cfg);
    case 8: return launch_t<Real, RTW, WD, MG, 8, PM, 0, 2, CX>(sh, a, eval, s, p, gn, cfg);
    case 16: return launch_t<Real, RTW, WD, MG, 16, PM, 0, 2, CX>(sh, a, eval, s, p, gn, cfg);
  }
  return hipErrorInvalidValue;
}

template <typename Real, int PM>
hipError_t launch_rt_mhg(const Shape& sh, const SamplerArgs& a, bool eval, hipStream_t s, const Persist* p, int gn,
                    KernelCfg* cfg) {
  if constexpr (std::is_same<Real, double>::value) {
    switch (sh.RT) {
      case 2: return launch_q_mhg<Real, 2, 1, false, PM>(sh, a, eval, s, p, gn, cfg);
      case 4: return launch_q_mhg<Real, 4, 1, false, PM>(sh, a, eval, s, p, gn, cfg);
    }
  } else {
    switch (sh.cfg) {
      case 0: return launch_q_mhg<Real, 2, 1, false, PM>(sh, a, eval, s, p, gn, cfg);
      case 1: return launch_q_mhg<Real, 4, 1, false, PM>(sh, a, eval, s, p, gn, cfg);
      case 2: return launch_q_mhg<Real, 8, 1, false, PM>(sh, a, eval, s, p, gn, cfg);
      case 3: return launch_q_mhg<Real, 4, 2, true, PM>(sh, a, eval, s, p, gn, cfg);
      case 4: return launch_q_mhg<Real, 4, 4, true, PM>(sh, a, eval, s, p, gn, cfg);
      case 7: return launch_q_mhg<Real, 4, 2, true, PM, true>(sh, a, eval, s, p, gn, cfg);
      case 8: return launch_q_mhg<Real, 4, 4, true, PM, true>(sh, a, eval, s, p, gn, cfg);
      case 9: return launch_q_mhg<Real, 4, 1, false, PM, true>(sh, a, eval, s, p, gn, cfg);
    }
  }
  return hipErrorInvalidValue;
}

// Learned-mixture instances: layouts with at most 4 row tiles per wave (cfg 0, 1, 3, 4) and the
// two-tile dimension splits 5 (64 dims, 2 waves, LDS matrices) and 6 (128 dims, 4 waves, L2), which
// keep the network, the two cached proposals and the state within 256 registers.
template <int RTW, int WD, bool MG, int PM>
hipError_t launch_q_lrn(const Shape& sh, const SamplerArgs& a, bool eval, hipStream_t s, const Persist* p, int gn,
                    KernelCfg* cfg) {
  switch (sh.Q) {
    case 2: return launch_t<float, RTW, WD, MG, 2, PM, 0, 1>(sh, a, eval, s, p, gn, cfg);
    case 4: return launch_t<float, RTW, WD, MG, 4, PM, 0, 1>(sh, a, eval, s, p, gn, cfg);
    case 8: return launch_t<float, RTW, WD, MG, 8, PM, 0, 1>(sh, a, eval, s, p, gn, cfg);
    case 16: return launch_t<float, RTW, WD, MG, 16, PM, 0, 1>(sh, a, eval, s, p, gn, cfg);
  }
  return hipErrorInvalidValue;
}

template <int PM>
hipError_t launch_rt_lrn(const Shape& sh, const SamplerArgs& a, bool eval, hipStream_t s, const Persist* p, int gn,
                    KernelCfg* cfg) {
  switch (sh.cfg) {
    case 0: return launch_q_lrn<2, 1, false, PM>(sh, a, eval, s, p, gn, cfg);
    case 1: return launch_q_lrn<4, 1, false, PM>(sh, a, eval, s, p, gn, cfg);
    case 3: return launch_q_lrn<4, 2, true, PM>(sh, a, eval, s, p, gn, cfg);
    case 4: return launch_q_lrn<4, 4, true, PM>(sh, a, eval, s, p, gn, cfg);
    case 5: return launch_q_lrn<2, 2, false, PM>(sh, a, eval, s, p, gn, cfg);
    case 6: return launch_q_lrn<2, 4, true, PM>(sh, a, eval, s, p, gn, cfg);
  }
  return hipErrorInvalidValue;
}

}  // namespace dmala
