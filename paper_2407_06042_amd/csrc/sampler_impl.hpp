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
#pragma once
#include <type_traits>

#include "common.hpp"

namespace dmala {

typedef _Float16 half8 __attribute__((ext_vector_type(8)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

__device__ __forceinline__ float ex2(float x) { return __builtin_amdgcn_exp2f(x); }
__device__ __forceinline__ float lg2(float x) { return __builtin_amdgcn_logf(x); }
__device__ __forceinline__ double ex2(double x) { return exp2(x); }
__device__ __forceinline__ double lg2(double x) { return log2(x); }

// Mode of the discretised Gaussian exp2(-kL (j - mu)^2) over j in [0, Q).
template <int Q, typename R>
__device__ __forceinline__ R mode_of(R mu) {
  R j = rint(mu);
  j = j < R(0) ? R(0) : j;
  j = j > R(Q - 1) ? R(Q - 1) : j;
  return j;
}

// log2 of the proposal normaliser sum_j exp2(-kL (j - mu)^2) (eq. softmax),
// summed relative to the mode so that it never underflows.
template <int Q, typename R>
__device__ __forceinline__ R log2_norm(R mu, R kL) {
  const R js = mode_of<Q>(mu);
  const R base = (js - mu) * (js - mu);
  R W = R(0);
#pragma unroll
  for (int j = 0; j < Q; ++j) {
    const R t = R(j) - mu;
    W += ex2(kL * (base - t * t));
  }
  return lg2(W) - kL * base;
}

// Inverse-CDF draw: the smallest j with u W < sum_{i <= j} w_i (ascending
// levels), w_i = exp2(-kL (i - mu)^2) relative to the mode, W = sum w.
template <int Q, typename R>
__device__ __forceinline__ int draw_level(R mu, R kL, R u) {
  const R js = mode_of<Q>(mu);
  const R base = (js - mu) * (js - mu);
  R w[Q];
  R W = R(0);
#pragma unroll
  for (int j = 0; j < Q; ++j) {
    const R t = R(j) - mu;
    w[j] = ex2(kL * (base - t * t));
    W += w[j];
  }
  const R target = u * W;
  R cum = R(0);
  int cnt = 0;
#pragma unroll
  for (int j = 0; j < Q - 1; ++j) {
    cum += w[j];
    cnt += (cum <= target) ? 1 : 0;
  }
  return cnt;
}

// Hide a loop-invariant LDS base from the optimiser so that the A-operand
// fragments are re-read from LDS every iteration instead of being hoisted into
// (and permanently occupying) registers.
__device__ __forceinline__ const unsigned char* opaque(const unsigned char* p) {
  asm volatile("" : "+s"(p));
  return p;
}

template <typename R>
__device__ __forceinline__ R bfly4(R v) {
  v += __shfl_xor(v, 16);
  v += __shfl_xor(v, 32);
  return v;
}

template <typename Real, int RT, int Q, int PM, bool EVAL>
__global__ __launch_bounds__(256) void sampler_kernel(SamplerArgs a) {
  constexpr bool F64 = std::is_same<Real, double>::value;
  constexpr int D = 4 * RT;
  constexpr int KB = RT / 2;
  constexpr int NPP = p_passes(PM);
  constexpr int QM1 = Q - 1;
  extern __shared__ __attribute__((aligned(16))) unsigned char smem[];

  const int inst = blockIdx.x;
  const int N = a.N, Npad = a.Npad;
  const unsigned char* blk = a.ws_inst + (size_t)inst * a.inst_stride;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6, nwaves = blockDim.x >> 6;
  const int cl = lane & 15, h = lane >> 4;
  const int chain = (blockIdx.y * nwaves + wave) * 16 + cl;
  const bool live = chain < a.C;

  // stage the instance's packed matrices and vectors in LDS
  {
    const int total = (!F64 && RT > 4) ? a.frag_bytes - 2 * Npad * 4 : a.frag_bytes;  // bytes staged in LDS
    for (int o = threadIdx.x * 16; o < total; o += blockDim.x * 16)
      *(uint4*)(smem + o) = *(const uint4*)(blk + kParamBytes + o);
  }
  const InstParams ip = *(const InstParams*)blk;
  __syncthreads();

  const Real kL = (Real)ip.kL;
  const Real rho = (Real)ip.rho;
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
    // the two per-dimension vectors follow the fragments; with 8 row tiles the
    // fragments alone can fill the LDS, so the vectors are then read from the
    // instance block (they stay in the L1/L2 caches)
    const size_t mat = (size_t)(NPP + kEPasses) * RT * KB * 1024;
    if constexpr (RT <= 4) pbv = (const Real*)(smem + mat);
    else pbv = (const Real*)(blk + kParamBytes + mat);
    ezv = pbv + Npad;
  }

  auto dim_of = [&](int d) { return 16 * (d >> 2) + 4 * h + (d & 3); };

  // [P; EG] x lv(k): accP/accE hold the lane's D outputs.
  auto contract = [&](const int (&k)[D], Real (&accP)[D], Real (&accE)[D]) {
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
    } else {
      const unsigned char* fb = opaque(smem);
      half8 bh[KB];
      bf16x8 bb[KB];
#pragma unroll
      for (int kb = 0; kb < KB; ++kb) {
#pragma unroll
        for (int j = 0; j < 8; ++j) {
          const int d = (2 * kb + (j >> 2)) * 4 + (j & 3);
          const int lv = (dim_of(d) < N) ? (2 * k[d] - QM1) : 0;
          bh[kb][j] = (_Float16)(float)lv;
          if constexpr (PM == PM_BF16X1) bb[kb][j] = (__bf16)(float)lv;
        }
      }
#pragma unroll
      for (int rt = 0; rt < RT; ++rt) {
        f32x4 e = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
        for (int p = 0; p < kEPasses; ++p)
#pragma unroll
          for (int kb = 0; kb < KB; ++kb) {
            const half8 fa = *(const half8*)(fb + (size_t)(((NPP + p) * RT + rt) * KB + kb) * 1024 + lane * 16);
            e = __builtin_amdgcn_mfma_f32_16x16x32_f16(fa, bh[kb], e, 0, 0, 0);
          }
#pragma unroll
        for (int i = 0; i < 4; ++i) accE[rt * 4 + i] = e[i];
        if constexpr (PM != PM_NAIVE) {
          f32x4 q = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
          for (int p = 0; p < NPP; ++p)
#pragma unroll
            for (int kb = 0; kb < KB; ++kb) {
              const unsigned char* src = fb + (size_t)((p * RT + rt) * KB + kb) * 1024 + lane * 16;
              if constexpr (PM == PM_BF16X1)
                q = __builtin_amdgcn_mfma_f32_16x16x32_bf16(*(const bf16x8*)src, bb[kb], q, 0, 0, 0);
              else
                q = __builtin_amdgcn_mfma_f32_16x16x32_f16(*(const half8*)src, bh[kb], q, 0, 0, 0);
            }
#pragma unroll
          for (int i = 0; i < 4; ++i) accP[rt * 4 + i] = q[i];
        }
      }
    }
  };

  // Proposal parameters and energy gradient at state k from the contraction.
  auto proposal_at = [&](const int (&k)[D], Real (&mu)[D], Real (&lz)[D], Real (&eg)[D]) {
    Real accP[D], accE[D];
    contract(k, accP, accE);
#pragma unroll
    for (int d = 0; d < D; ++d) {
      const int n = dim_of(d);
      const Real g = accE[d] * sE - ezv[n];
      Real shift;
      if constexpr (PM == PM_NAIVE) shift = rho * g;
      else shift = accP[d] * sP - pbv[n];
      eg[d] = g;
      mu[d] = Real(k[d]) - shift;
      lz[d] = log2_norm<Q>(mu[d], kL);
    }
  };

  int kc[D];
  Real mu[D], lz[D], eg[D];

  if constexpr (EVAL) {
    // transition quantities for a given pair (x_from -> x_to)
    const size_t row = ((size_t)inst * a.C + (live ? chain : 0)) * N;
    int kt[D];
#pragma unroll
    for (int d = 0; d < D; ++d) {
      const int n = dim_of(d);
      kc[d] = (live && n < N) ? (int)a.x_from[row + n] : 0;
      kt[d] = (live && n < N) ? (int)a.x_to[row + n] : 0;
    }
    proposal_at(kc, mu, lz, eg);
    Real lqf = 0;
#pragma unroll
    for (int d = 0; d < D; ++d)
      if (dim_of(d) < N) { const Real t = Real(kt[d]) - mu[d]; lqf += -kL * t * t - lz[d]; }
    Real mup[D], lzp[D], egp[D];
    proposal_at(kt, mup, lzp, egp);
    Real lqr = 0, T2 = 0;
#pragma unroll
    for (int d = 0; d < D; ++d)
      if (dim_of(d) < N) {
        const Real t = Real(kc[d]) - mup[d];
        lqr += -kL * t * t - lzp[d];
        T2 -= Real(kt[d] - kc[d]) * (eg[d] + egp[d]);
      }
    lqf = bfly4(lqf); lqr = bfly4(lqr); T2 = bfly4(T2);
    if (live && h == 0) {
      double* o = a.eval_out + ((size_t)inst * a.C + chain) * 4;
      const double ln2 = 1.0 / kLog2e;
      o[0] = (double)lqf * ln2;
      o[1] = (double)lqr * ln2;
      o[2] = (double)T2 * ln2;
      o[3] = ((double)T2 + (double)lqr - (double)lqf) * ln2;
    }
    return;
  } else {
    const uint32_t key0 = a.key0, key1 = a.key1;
    // initial state from the t = 0 words
#pragma unroll
    for (int rt = 0; rt < RT; ++rt) {
      uint32_t c[4] = {(uint32_t)(4 * rt + h), 0u, (uint32_t)chain, (uint32_t)inst};
      philox4x32_10(c, key0, key1);
#pragma unroll
      for (int i = 0; i < 4; ++i) kc[rt * 4 + i] = (int)(((uint64_t)(c[i] >> 8) * Q) >> 24);
    }
    proposal_at(kc, mu, lz, eg);
    // E(x) = ||y||^2 + x^T g - z^T x = ||y||^2 + (eunit/2) sum_n lv_n (eg_n - ez_n)
    Real ep = 0;
#pragma unroll
    for (int d = 0; d < D; ++d) {
      const int n = dim_of(d);
      if (n < N) ep += Real(2 * kc[d] - QM1) * (eg[d] - ezv[n]);
    }
    ep = bfly4(ep);
    const Real eunit = (Real)ip.eunit;
    Real E = (Real)ip.yy + Real(0.5) * eunit * ep;
    Real Ebest = E;
    uint32_t kbest[RT];
#pragma unroll
    for (int rt = 0; rt < RT; ++rt)
      kbest[rt] = (uint32_t)kc[rt * 4] | ((uint32_t)kc[rt * 4 + 1] << 8) | ((uint32_t)kc[rt * 4 + 2] << 16) | ((uint32_t)kc[rt * 4 + 3] << 24);
    int nacc = 0;
    uint32_t abits = 0;
    const size_t trow = (size_t)inst * a.C + (live ? chain : 0);

    for (int t = 1; t <= a.T; ++t) {
      uint32_t w[RT][4];
#pragma unroll
      for (int rt = 0; rt < RT; ++rt) {
        w[rt][0] = (uint32_t)(4 * rt + h); w[rt][1] = (uint32_t)t; w[rt][2] = (uint32_t)chain; w[rt][3] = (uint32_t)inst;
        philox4x32_10(w[rt], key0, key1);
      }
      // 1. draw x' and log q(x'|x)
      int kp[D];
      Real lqf = 0;
#pragma unroll
      for (int d = 0; d < D; ++d) {
        Real u;
        if constexpr (F64) u = u24d(w[d >> 2][d & 3]);
        else u = u24f(w[d >> 2][d & 3]);
        kp[d] = draw_level<Q>(mu[d], kL, u);
        if (dim_of(d) < N) { const Real tt = Real(kp[d]) - mu[d]; lqf += -kL * tt * tt - lz[d]; }
      }
      // 2-3. gradient at x', proposal at x', log q(x|x')
      Real mup[D], lzp[D], egp[D];
      proposal_at(kp, mup, lzp, egp);
      Real lqr = 0, T2 = 0;
#pragma unroll
      for (int d = 0; d < D; ++d)
        if (dim_of(d) < N) {
          const Real tt = Real(kc[d]) - mup[d];
          lqr += -kL * tt * tt - lzp[d];
          T2 -= Real(kp[d] - kc[d]) * (eg[d] + egp[d]);
        }
      // 4. MH: accept iff  log ratio > log u  (eq. acc_prob: A > u)
      Real S = T2 + lqr - lqf;
      if (h == 0) {
        const uint32_t um = low_bytes24(w[0][0], w[0][1], w[0][2]);
        Real lu;
        if constexpr (F64) lu = lg2((double)um * 5.9604644775390625e-08);
        else lu = lg2((float)um * 5.9604644775390625e-08f);
        S -= lu;
      }
      S = bfly4(S);
      T2 = bfly4(T2);
      const bool acc = S > Real(0);
      // 5. select
#pragma unroll
      for (int d = 0; d < D; ++d) {
        kc[d] = acc ? kp[d] : kc[d];
        mu[d] = acc ? mup[d] : mu[d];
        lz[d] = acc ? lzp[d] : lz[d];
        eg[d] = acc ? egp[d] : eg[d];
      }
      if (acc) { E -= T2 * eunit; ++nacc; }
      if (E < Ebest) {
        Ebest = E;
#pragma unroll
        for (int rt = 0; rt < RT; ++rt)
          kbest[rt] = (uint32_t)kc[rt * 4] | ((uint32_t)kc[rt * 4 + 1] << 8) | ((uint32_t)kc[rt * 4 + 2] << 16) | ((uint32_t)kc[rt * 4 + 3] << 24);
      }
      if (a.trace_accept) {
        abits |= (acc ? 1u : 0u) << ((t - 1) & 31);
        if (((t & 31) == 0 || t == a.T) && live && h == 0) {
          a.trace_accept[trow * a.trace_words + ((t - 1) >> 5)] = abits;
        }
        if ((t & 31) == 0) abits = 0;
      }
      if (a.trace_hash) {
        uint32_t hs = 0;
#pragma unroll
        for (int d = 0; d < D; ++d) {
          const int n = dim_of(d);
          if (n < N) hs += (uint32_t)(kc[d] + 1) * hash_mult(n);
        }
        hs += __shfl_xor(hs, 16);
        hs += __shfl_xor(hs, 32);
        if (live && h == 0) a.trace_hash[trow * a.T + (t - 1)] = hs;
      }
    }

    // results for the estimator and the optional outputs
    if (live) {
      const StateOff so = state_offsets(a.Cpad, Npad);
      unsigned char* st = a.ws_state + (size_t)inst * a.state_stride;
#pragma unroll
      for (int rt = 0; rt < RT; ++rt) {
        const int n0 = 16 * rt + 4 * h;
        const uint32_t cur = (uint32_t)kc[rt * 4] | ((uint32_t)kc[rt * 4 + 1] << 8) | ((uint32_t)kc[rt * 4 + 2] << 16) | ((uint32_t)kc[rt * 4 + 3] << 24);
        *(uint32_t*)(st + so.k + (size_t)chain * Npad + n0) = cur;
        *(uint32_t*)(st + so.kbest + (size_t)chain * Npad + n0) = kbest[rt];
        if (a.final_state) {
#pragma unroll
          for (int i = 0; i < 4; ++i)
            if (n0 + i < N) a.final_state[((size_t)inst * a.C + chain) * N + n0 + i] = (int8_t)kc[rt * 4 + i];
        }
      }
      if (h == 0) {
        ((double*)(st + so.ebest))[chain] = (double)Ebest;
        ((int32_t*)(st + so.nacc))[chain] = nacc;
        if (a.accept_count) a.accept_count[(size_t)inst * a.C + chain] = nacc;
      }
    }
  }
}

template <typename Real, int RT, int Q, int PM>
hipError_t launch_t(const Shape& sh, const SamplerArgs& a, bool eval, hipStream_t s) {
  const int chain_blocks = sh.Cpad / 16;
  const int waves = chain_blocks < 4 ? chain_blocks : 4;
  const dim3 grid(a.n_inst, (chain_blocks + waves - 1) / waves);
  const size_t lds = sampler_lds_bytes(sh);
  auto k = eval ? sampler_kernel<Real, RT, Q, PM, true> : sampler_kernel<Real, RT, Q, PM, false>;
  if (lds > 65536) {
    hipError_t e = hipFuncSetAttribute((const void*)k, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (e != hipSuccess) return e;
  }
  hipLaunchKernelGGL(k, grid, dim3(64 * waves), lds, s, a);
  return hipGetLastError();
}

template <typename Real, int RT, int PM>
hipError_t launch_q(const Shape& sh, const SamplerArgs& a, bool eval, hipStream_t s) {
  switch (sh.Q) {
    case 2: return launch_t<Real, RT, 2, PM>(sh, a, eval, s);
    case 4: return launch_t<Real, RT, 4, PM>(sh, a, eval, s);
    case 8: return launch_t<Real, RT, 8, PM>(sh, a, eval, s);
    case 16: return launch_t<Real, RT, 16, PM>(sh, a, eval, s);
  }
  return hipErrorInvalidValue;
}

template <typename Real, int PM>
hipError_t launch_rt(const Shape& sh, const SamplerArgs& a, bool eval, hipStream_t s) {
  switch (sh.RT) {
    case 2: return launch_q<Real, 2, PM>(sh, a, eval, s);
    case 4: return launch_q<Real, 4, PM>(sh, a, eval, s);
    case 8: return launch_q<Real, 8, PM>(sh, a, eval, s);
  }
  return hipErrorInvalidValue;
}

}  // namespace dmala
