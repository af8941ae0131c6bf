// Shared declarations of the DMALA HIP library (host launchers and device helpers).
//
// Notation (index units): a chain state is a vector of level indices k_n in
// [0, Q), real dimension n = 2m (Re x_m) or 2m+1 (Im x_m); the real value is
// s * lv_n with lv_n = 2 k_n - Q + 1 an odd integer.  All log-probabilities in
// the kernels are base-2 (exp2/log2 are the native transcendental ops).
//
// With the parameters of the preconditioned proposal (Remark after Algorithm
// 1, tempered as in Algorithm 2) the factorised proposal of eq. dis_prop_fac2
// over the levels j of dimension n is a discretised Gaussian in j:
//     log2 q_n(j | x) = -kL (j - mu_n)^2 - lz_n,
//     mu_n = k_n - shift_n,   shift = c_m (A x - b),   A = M G,  b = M z,
// with G = H^T H, z = H^T y, M = (G + gamma I)^-1, c_m = alpha / (2 tau sigma^2 s),
// kL = log2(e) * 2 s^2 / (alpha beta) and lz_n the log2 normaliser.  The naive
// proposal (eq. exp_fac) is the same with A = G, b = z and beta -> 1.  The
// tempered log acceptance ratio of eq. acc_prob uses the exact identity
//     E(x') - E(x) = (x' - x)^T (g(x) + g(x')),   g = G x - z,   E = ||y - Hx||^2,
// so the sampler carries the energy gradient eg = (2 s log2(e) / (tau sigma^2)) g
// (in log2 units) and never forms a residual inside the loop.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace dmala {

constexpr double kLog2e = 1.4426950408889634074;

// Per-instance constants written by the setup kernel (first 256 bytes of each
// instance block of the workspace).
struct InstParams {
  double yy;       // ||y||^2
  double eunit;    // tau sigma^2 / log2(e): energy per log2 unit of the tempered metric
  double kL;       // log2(e) * 2 s^2 / (alpha beta')
  double rho;      // naive proposal: shift = rho * eg
  double sigma2;
  double s;        // level step
  double tau;
  float scaleP;    // 2^-e of the packed proposal matrix
  float scaleE;    // 2^-e of the packed energy matrix
  int32_t nonfinite;  // 1: H or y has a non-finite entry, or sigma^2 is not positive and finite (Lemma 1
                      // needs sigma^2 > 0); the sampler and the estimator then skip the instance
  int32_t pad_[3];
};
static_assert(sizeof(InstParams) <= 256, "params block");
constexpr int kParamBytes = 256;
// Per-instance status written by the setup kernel for a flagged instance (the C ABI's DMALA_ERR_NONFINITE).
constexpr int32_t kStatusNonfinite = -3;

// Floats per exported training row: 7 network features, the plain centre (Re, Im),
// the plain precision (natural-log units), Q, 0.
constexpr int kTrainRow = 12;

// Packing modes of the proposal matrix in the MFMA path.
enum PMode : int { PM_NAIVE = 0, PM_F16X2 = 1, PM_F16X1 = 2, PM_BF16X1 = 3 };
constexpr int kEPasses = 3;  // energy matrix: hi/mid/lo fp16 split

__host__ __device__ constexpr int p_passes(int pm) { return pm == PM_NAIVE ? 0 : (pm == PM_F16X2 ? 2 : 1); }

// Geometry of one problem shape.
struct Shape {
  int nt, nr, M, Q, N, Npad, RT, KB, C, Cpad, T;
  int fp64;        // 1: double path
  int pm;          // PMode (MFMA path)
  int win;         // proposal window half-width (0 = all levels), see the sampler
  int cfg;         // sampler work layout (see sampler_impl.hpp launch_rt)
  int cbw;         // 16-chain blocks per workgroup for the one-wave layouts (1, 2 or 4)
  int lrn;         // 1: plain/learned kernel mixture (learned proposal network in the sampler)
  int share;       // 1: launched beside other classes' kernels (an uneven batch's graph branches)
  int mhgd;        // 1: the MHGD baseline kernel (nearest-point candidate, MH without the proposal ratio)
  int cx;          // 1: matrices packed as complex planes (layouts 7, 8)
  size_t inst_bytes;   // per-instance setup block
  size_t frag_bytes;   // MFMA fragments (MFMA path)
  size_t state_bytes;  // per-instance sampler->estimator block
  size_t wscratch_bytes;  // per-instance setup working matrix (large nt)
};

// Offsets inside the per-instance state block.
struct StateOff {
  size_t k, kbest, ebest, nacc, eg, end;
};
__host__ __device__ inline StateOff state_offsets(int Cpad, int Npad) {
  StateOff o;
  o.k = 0;
  o.kbest = o.k + (size_t)Cpad * Npad;
  o.ebest = (o.kbest + (size_t)Cpad * Npad + 15) & ~(size_t)15;
  o.nacc = o.ebest + (size_t)Cpad * 8;
  // the float chains' energy gradient at the final state (Cpad x Npad floats), for the estimator
  o.eg = (o.nacc + (size_t)Cpad * 4 + 255) & ~(size_t)255;
  o.end = (o.eg + (size_t)Cpad * Npad * 4 + 255) & ~(size_t)255;
  return o;
}

// Where one instance's inputs and outputs live in the caller's buffers.  A
// uniform batch uses no table (offsets follow from the instance index); an
// uneven batch passes one entry per instance, grouped by shape class.
struct InstDesc {
  int64_t h_off;     // complex elements into H
  int64_t y_off;     // complex elements into y
  int64_t sym_off;   // antennas into symbols (sum of Nt over the preceding instances)
  int64_t marg_off;  // floats into marginals / marginals_mc (sum of Nt * M)
  int64_t llr_off;   // floats into llrs (sum of Nt * log2 M)
  int64_t fs_off;    // bytes into final_state (sum of n_chains * 2 Nt)
  int32_t orig;      // instance index in the caller's batch: sigma2, best_energy, accept_count, RNG counter
  int32_t pad_;
};

__host__ __device__ inline InstDesc inst_desc(const InstDesc* d, int b, int nt, int nr, int M, int C) {
  if (d) return d[b];
  int nb = 0;
  while ((1 << nb) < M) ++nb;
  InstDesc r;
  r.h_off = (int64_t)b * nt * nr;
  r.y_off = (int64_t)b * nr;
  r.sym_off = (int64_t)b * nt;
  r.marg_off = (int64_t)b * nt * M;
  r.llr_off = (int64_t)b * nt * nb;
  r.fs_off = (int64_t)b * C * 2 * nt;
  r.orig = b;
  r.pad_ = 0;
  return r;
}

struct SetupArgs {
  const InstDesc* desc;
  const void* H; const void* y; const void* sigma2;
  double sigma2_val;   // the noise variance of every instance when sigma2 is NULL
  int32_t* status;     // optional [caller's instance index]: 0, or DMALA_ERR_NONFINITE for a flagged instance
  unsigned char* ws_inst; size_t inst_stride;
  unsigned char* wscratch; size_t wscratch_stride;  // per-instance working matrix when nt > 32
  int n_inst, nt, nr, Q, N, Npad, RT, KB, fp64, pm, naive;
  int cx;              // 1: pack the matrices as complex planes (the sampler's complex-plane layouts)
  double tau, alpha_mult, beta_mult, gamma_mult;
};

struct SamplerArgs {
  const InstDesc* desc;
  const unsigned char* ws_inst; size_t inst_stride;
  unsigned char* ws_state; size_t state_stride;
  int n_inst, N, Npad, C, Cpad, T;
  uint32_t key0, key1;
  uint32_t ctr_base;      // the random counter's instance word is ctr_base + the caller's instance index
  int frag_bytes;
  int8_t* final_state; int32_t* accept_count; uint32_t* trace_accept; uint32_t* trace_hash;
  int trace_words;
  // learned-proposal mixture and training-row export
  const float* mlp;       // network parameters (flat float32, see mlp_device.hpp)
  uint32_t mix_thr;       // plain kernel iff the 24-bit mixture uniform < mix_thr (= ceil(eps 2^24))
  float* train_rows;      // [sum Nt][n_chains] rows of kTrainRow floats at the final state
  // debug-eval mode
  const int8_t* x_from; const int8_t* x_to; double* eval_out;
  double* eval_dim;       // optional per-dimension forward log q terms [n_inst][n_pairs][N]
};

struct EstArgs {
  const InstDesc* desc;
  const void* H; const void* y; const void* sigma2;
  const unsigned char* ws_inst; size_t inst_stride;
  const unsigned char* ws_state; size_t state_stride;
  int n_inst, nt, nr, Q, N, Npad, C, Cpad, fp64;
  int chunk;       // chains staged in LDS at a time
  int32_t* symbols; float* marginals; float* llrs; float* best_energy; float* marginals_mc;
  int llr_mode;    // 0: IS (eq. llr_is), 1: list (eq. llr_approx_app), 2: Monte Carlo bit frequencies (eq. mc)
  float llr_clip;  // |LLR| limit of the list and Monte Carlo forms
};

// Persistent launches (uneven-batch plans).  A work item is one instance (workspace slot) of one
// class of the plan and, for the sampler, one group of 16-chain blocks; a persistent launch keeps
// its workgroups resident and each takes the next item of a list (longest classes first) from a
// global atomic counter until the list is exhausted.  The workgroup that finishes last returns
// both counters to 0, so a captured graph can replay the launch.
struct WorkItem {
  int32_t cls, inst, cg, pad_;
};

struct Persist {
  const WorkItem* items;   // NULL: a direct launch (instance blockIdx.x, chain group blockIdx.y)
  int32_t n_items;
  int32_t lds_off;         // byte offset of the item broadcast word in the dynamic LDS
  int32_t* counter;        // [0] next item, [1] workgroups finished
  const void* cls;         // per-class argument structs (SetupArgs, SamplerArgs or EstArgs)
};

#ifdef __HIPCC__
// Next item index for the whole workgroup (after a barrier that ends the previous item's LDS use).
__device__ inline int persist_take(const Persist& p, unsigned char* lds) {
  int* slot = (int*)(lds + p.lds_off);
  __syncthreads();
  if (threadIdx.x == 0) slot[0] = __hip_atomic_fetch_add(p.counter, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  __syncthreads();
  return __builtin_amdgcn_readfirstlane(slot[0]);
}

// The workgroup has taken its last item; the last one to get here resets the counters.
__device__ inline void persist_done(const Persist& p) {
  if (threadIdx.x == 0) {
    const int f = __hip_atomic_fetch_add(p.counter + 1, 1, __ATOMIC_ACQ_REL, __HIP_MEMORY_SCOPE_AGENT);
    if (f == (int)gridDim.x - 1) {
      __hip_atomic_store(p.counter, 0, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      __hip_atomic_store(p.counter + 1, 0, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
    }
  }
}
#endif

// Launch geometry of one class's kernel: the kernel (identity of a persistent family), threads per
// workgroup, dynamic LDS bytes and the direct grid.
struct KernelCfg {
  const void* k = nullptr;
  int threads = 0;
  size_t lds = 0;
  int gx = 0, gy = 0;
};

// Host launchers (defined in the .hip translation units).
// With cfg != NULL the launchers only fill in the class's launch geometry; with p != NULL (and
// p->items set) they make a persistent launch of p->n_items items on `grid` workgroups.
hipError_t launch_setup(const SetupArgs& a, hipStream_t s, const Persist* p = nullptr, int grid = 0,
                        KernelCfg* cfg = nullptr);
bool setup_w_global(int nt);
hipError_t launch_sampler(const Shape& sh, const SamplerArgs& a, bool eval, hipStream_t s, const Persist* p = nullptr,
                          int grid = 0, KernelCfg* cfg = nullptr);
hipError_t launch_estimate(const EstArgs& a, hipStream_t s, const Persist* p = nullptr, int grid = 0,
                           KernelCfg* cfg = nullptr);
size_t sampler_lds_bytes(const Shape& sh);
bool sampler_cfg_valid(const Shape& sh, int cfg);
int sampler_default_cfg(const Shape& sh);
int estimate_chunk(int nt, int nr, int M, int N, int C, bool fp64);

// ------------------------------------------------------------------ device helpers

// a ^ b ^ k as one three-input bit operation (v_bitop3_b32, truth table 0x96; from two
// xors the compiler emits two instructions).
__device__ __forceinline__ uint32_t xor3(uint32_t a, uint32_t b, uint32_t k) {
  return __builtin_amdgcn_bitop3_b32(a, b, k, 0x96);
}

// Philox4x32-10 (Salmon et al., SC'11): 10 rounds of the 4x32 S-box, key bumped
// by the Weyl constants between rounds.  BITOP3: the xors as three-input bit
// operations.
template <bool BITOP3>
__device__ __forceinline__ void philox4x32_10(uint32_t c[4], uint32_t k0, uint32_t k1) {
#pragma unroll
  for (int r = 0; r < 10; ++r) {
    if (r) { k0 += 0x9E3779B9u; k1 += 0xBB67AE85u; }
    const uint64_t p0 = (uint64_t)0xD2511F53u * c[0];
    const uint64_t p1 = (uint64_t)0xCD9E8D57u * c[2];
    uint32_t n0, n2;
    if constexpr (BITOP3) {
      n0 = xor3((uint32_t)(p1 >> 32), c[1], k0);
      n2 = xor3((uint32_t)(p0 >> 32), c[3], k1);
    } else {
      n0 = (uint32_t)(p1 >> 32) ^ c[1] ^ k0;
      n2 = (uint32_t)(p0 >> 32) ^ c[3] ^ k1;
    }
    c[0] = n0; c[1] = (uint32_t)p1; c[2] = n2; c[3] = (uint32_t)p0;
  }
}

__device__ __forceinline__ float u24f(uint32_t w) { return (float)(w >> 8) * 5.9604644775390625e-08f; }
__device__ __forceinline__ double u24d(uint32_t w) { return (double)(w >> 8) * 5.9604644775390625e-08; }
// Uniform of a proposal draw: the midpoint (x + 1/2) 2^-23 of the cell of x = w >> 9, in (0, 1) and
// exact in fp32: the bits of 1 + x 2^-23 (one funnel shift) minus 1 - 2^-24.
__device__ __forceinline__ float u23f(uint32_t w) {
  return __uint_as_float(__builtin_amdgcn_alignbit(0x7Fu, w, 9)) - 0.999999940395355224609375f;
}
__device__ __forceinline__ double u23d(uint32_t w) { return ((double)(w >> 9) + 0.5) * 1.1920928955078125e-07; }
// The same uniform times 2^100, in one fused multiply-add (exact: (x + 1/2) 2^77).
__device__ __forceinline__ float u23f_x2p100(uint32_t w) {
  return __builtin_fmaf(__uint_as_float(__builtin_amdgcn_alignbit(0x7Fu, w, 9)), 0x1p100f,
                        -0.999999940395355224609375f * 0x1p100f);
}
__device__ __forceinline__ uint32_t low_bytes24(uint32_t a, uint32_t b, uint32_t c) {
  return (a & 0xFFu) | ((b & 0xFFu) << 8) | ((c & 0xFFu) << 16);
}
__device__ __forceinline__ uint32_t hash_mult(int n) { return (uint32_t)(2 * n + 1) * 0x9E3779B1u; }

}  // namespace dmala
