// The gradient contraction alone, looped: V = P lv(X) on MFMA with a synthetic state update.
//
// Measurement kernel for the G.X stage of the chain -- the preconditioned gradient of
// Algorithm 1 as one bf16 or fp16 MFMA pass with fp32 accumulation (v_mfma_f32_16x16x32_*),
// 8 Nt^2 flops per chain and transition.  It reads the A-operand fragments the setup kernel
// packs for the sampler and uses the sampler's lane layout (lane l: chain l % 16 and, in row
// tile rt, the dimensions 16 rt + 4 (l / 16) + i of its accumulator rows), but keeps the matrix
// in registers for the whole loop and replaces the rest of a transition by a cheap update that
// depends on the product: every level whose gradient entry is negative changes sign (the B
// operand stays exact odd integers).  A wave takes NB blocks of 16 chains of one instance; WD
// waves split the row tiles of larger matrices and exchange their halves of X through LDS.
#include "../../include/dmala.h"
#include "common.hpp"
#include "host.hpp"

namespace dmala {
namespace {

typedef _Float16 gx_half8 __attribute__((ext_vector_type(8)));
typedef __bf16 gx_bf16x8 __attribute__((ext_vector_type(8)));
typedef float gx_f32x4 __attribute__((ext_vector_type(4)));

struct GxArgs {
  const unsigned char* ws_inst;
  size_t inst_stride;
  int n_inst, Q, n_groups;  // n_groups: chain groups (NB blocks of 16) per instance
  int n_loops;
  float* sink;              // [n_inst * n_groups * WD * 64] per-lane sums of the last products
};

template <int RTW, int WD, int NB, bool BF>
__global__ __launch_bounds__(256) void gx_loop_kernel(GxArgs a) {
  constexpr int RT = RTW * WD, KB = RT / 2, KBW = RTW / 2;
  constexpr int IPW = 4 / WD;  // items per workgroup of 4 waves
  static_assert(RTW % 2 == 0 && 4 % WD == 0, "whole K blocks per wave, waves divide the workgroup");
  __shared__ __attribute__((aligned(16))) uint4 xch[WD > 1 ? 2 * IPW * NB * KB * 64 : 1];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int h = lane >> 4, cl = lane & 15;
  const int slot = wave / WD, wd = wave % WD;
  const int item = blockIdx.x * IPW + slot;
  const bool active = item < a.n_inst * a.n_groups;          // uniform per slot (the WD waves of an item)
  const int inst = active ? item / a.n_groups : 0;
  const int grp = active ? item % a.n_groups : 0;
  const int rt0 = wd * RTW;
  const unsigned char* frag = a.ws_inst + (size_t)inst * a.inst_stride + kParamBytes;

  // the wave's row tiles of the packed proposal matrix, in registers for the whole loop
  uint4 A[RTW][KB];
#pragma unroll
  for (int rt = 0; rt < RTW; ++rt)
#pragma unroll
    for (int kb = 0; kb < KB; ++kb) A[rt][kb] = *(const uint4*)(frag + ((size_t)(rt0 + rt) * KB + kb) * 1024 + lane * 16);

  // B operands: levels lv = 2 k - Q + 1 of a fixed starting state, all K blocks
  uint4 B[NB][KB];
#pragma unroll
  for (int nb = 0; nb < NB; ++nb)
#pragma unroll
    for (int kb = 0; kb < KB; ++kb) {
      union { _Float16 hv[8]; __bf16 bv[8]; uint4 u; } v;
#pragma unroll
      for (int j = 0; j < 8; ++j) {
        const int n = 16 * (2 * kb + (j >> 2)) + 4 * h + (j & 3);
        const int chain = (grp * NB + nb) * 16 + cl;
        const int lv = 2 * ((n * 5 + chain * 3) % a.Q) - a.Q + 1;
        if constexpr (BF) v.bv[j] = (__bf16)(float)lv;
        else v.hv[j] = (_Float16)(float)lv;
      }
      B[nb][kb] = v.u;
    }

  gx_f32x4 acc[NB][RTW];
  int phase = 0;
  for (int it = 0; it < a.n_loops; ++it) {
#pragma unroll
    for (int nb = 0; nb < NB; ++nb)
#pragma unroll
      for (int rt = 0; rt < RTW; ++rt) {
        gx_f32x4 c = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
        for (int kb = 0; kb < KB; ++kb) {
          if constexpr (BF) {
            gx_bf16x8 av, bv;
            __builtin_memcpy(&av, &A[rt][kb], 16);
            __builtin_memcpy(&bv, &B[nb][kb], 16);
            c = __builtin_amdgcn_mfma_f32_16x16x32_bf16(av, bv, c, 0, 0, 0);
          } else {
            gx_half8 av, bv;
            __builtin_memcpy(&av, &A[rt][kb], 16);
            __builtin_memcpy(&bv, &B[nb][kb], 16);
            c = __builtin_amdgcn_mfma_f32_16x16x32_f16(av, bv, c, 0, 0, 0);
          }
        }
        acc[nb][rt] = c;
      }
    // synthetic update of the wave's own dimensions: row tile rt fills half of K block rt / 2,
    // element pairs (2q, 2q + 1) take the sign bits of accumulator entries (2q', 2q' + 1)
#pragma unroll
    for (int nb = 0; nb < NB; ++nb)
#pragma unroll
      for (int rt = 0; rt < RTW; ++rt) {
        const int kb = (rt0 + rt) >> 1, half = (rt0 + rt) & 1;
        uint32_t w[4];
        __builtin_memcpy(w, &B[nb][kb], 16);
#pragma unroll
        for (int q = 0; q < 2; ++q) {
          const uint32_t m = ((__float_as_uint(acc[nb][rt][2 * q]) >> 16) & 0x8000u) |
                             (__float_as_uint(acc[nb][rt][2 * q + 1]) & 0x80000000u);
          w[2 * half + q] ^= m;
        }
        __builtin_memcpy(&B[nb][kb], w, 16);
      }
    if constexpr (WD > 1) {
      // exchange the K blocks through LDS (double-buffered: one barrier per iteration)
      uint4* xb = xch + ((size_t)(phase & 1) * IPW + slot) * NB * KB * 64;
      ++phase;
#pragma unroll
      for (int nb = 0; nb < NB; ++nb)
#pragma unroll
        for (int kb = 0; kb < KBW; ++kb) xb[((size_t)nb * KB + wd * KBW + kb) * 64 + lane] = B[nb][wd * KBW + kb];
      __syncthreads();
#pragma unroll
      for (int nb = 0; nb < NB; ++nb)
#pragma unroll
        for (int kb = 0; kb < KB; ++kb) B[nb][kb] = xb[((size_t)nb * KB + kb) * 64 + lane];
    }
  }
  if (active) {
    float s = 0.f;
#pragma unroll
    for (int nb = 0; nb < NB; ++nb)
#pragma unroll
      for (int rt = 0; rt < RTW; ++rt) s += acc[nb][rt][0] + acc[nb][rt][1] + acc[nb][rt][2] + acc[nb][rt][3];
    a.sink[((size_t)item * WD + wd) * 64 + lane] = s;
  }
}

template <int RTW, int WD, int NB>
hipError_t launch_gx(const GxArgs& a, bool bf, hipStream_t s) {
  constexpr int IPW = 4 / WD;
  const int items = a.n_inst * a.n_groups;
  const dim3 grid((items + IPW - 1) / IPW);
  if (bf) hipLaunchKernelGGL((gx_loop_kernel<RTW, WD, NB, true>), grid, dim3(256), 0, s, a);
  else hipLaunchKernelGGL((gx_loop_kernel<RTW, WD, NB, false>), grid, dim3(256), 0, s, a);
  return hipGetLastError();
}

// Chain blocks per wave and row-tile split per matrix size (registers: RTW KB + NB KB fragments).
int gx_nb(int Npad) { return Npad <= 64 ? 2 : 1; }
int gx_wd(int Npad) { return Npad >= 256 ? 4 : 1; }

}  // namespace
}  // namespace dmala

using namespace dmala;
using namespace dmala::host;

extern "C" {

size_t dmala_gx_loop_sink_size(int32_t n_inst, int32_t nt, int32_t n_chains) {
  if (n_inst < 1 || nt < 1 || nt > 128 || n_chains < 1) return 0;
  int Npad = 32;
  while (Npad < 2 * nt) Npad *= 2;
  const int nb = gx_nb(Npad), groups = ((n_chains + 15) / 16 + nb - 1) / nb;
  return (size_t)n_inst * groups * gx_wd(Npad) * 64;
}

dmala_status dmala_gx_loop(const void* H, const void* y, const void* sigma2, int32_t n_inst, int32_t nt, int32_t nr,
                           int32_t qam_order, const dmala_params* params, int32_t n_loops, int32_t run_setup,
                           float* sink, void* workspace, size_t workspace_bytes, dmala_stream_t stream) {
  if (!params) return fail(DMALA_ERR_ARG, "params is NULL");
  // the loop reads real-equivalent fragments: pin the matching layout (1 + layout 0, 1, 3 or 4)
  dmala_params prm = *params;
  {
    int npad = 32;
    while (npad < 2 * nt) npad *= 2;
    prm.tile_config = npad == 32 ? 1 : (npad == 64 ? 2 : (npad == 128 ? 4 : 5));
  }
  params = &prm;
  Plan pl;
  dmala_status st = make_plan(n_inst, nt, nr, qam_order, params, pl);
  if (st != DMALA_OK) return st;
  if (params->proposal != DMALA_PRECOND || (params->precision != DMALA_BF16 && params->precision != DMALA_FP16))
    return fail(DMALA_ERR_UNSUPPORTED, "the gradient loop runs the single-pass DMALA_BF16 / DMALA_FP16 DMALA_PRECOND form");
  if (n_loops < 1) return fail(DMALA_ERR_ARG, "n_loops must be >= 1");
  if (!sink) return fail(DMALA_ERR_ARG, "sink must be non-NULL");
  if (!workspace) return fail(DMALA_ERR_WORKSPACE, "workspace is NULL");
  if (workspace_bytes < pl.total) return fail(DMALA_ERR_WORKSPACE, "workspace too small: %zu < %zu bytes", workspace_bytes, pl.total);
  if (((uintptr_t)workspace & 255) != 0) return fail(DMALA_ERR_WORKSPACE, "workspace must be 256-byte aligned");
  hipStream_t s = (hipStream_t)stream;
  const Shape& sh = pl.sh;
  unsigned char* base = (unsigned char*)workspace;
  if (run_setup) {
    if (!H || !y || !sigma2) return fail(DMALA_ERR_ARG, "H, y and sigma2 must be non-NULL");
    SetupArgs sa{};
    sa.H = H; sa.y = y; sa.sigma2 = sigma2;
    sa.ws_inst = base + pl.inst_off; sa.inst_stride = sh.inst_bytes;
    sa.wscratch = base + pl.wscratch_off; sa.wscratch_stride = sh.wscratch_bytes;
    sa.n_inst = n_inst; sa.nt = sh.nt; sa.nr = sh.nr; sa.Q = sh.Q; sa.N = sh.N; sa.Npad = sh.Npad;
    sa.RT = sh.RT; sa.KB = sh.KB; sa.fp64 = 0; sa.pm = sh.pm; sa.naive = 0;
    sa.tau = pl.tau; sa.alpha_mult = pl.am; sa.beta_mult = pl.bm; sa.gamma_mult = pl.gm;
    const hipError_t e = launch_setup(sa, s);
    if (e != hipSuccess) return hip_fail(e, "setup launch");
  }
  GxArgs ga{};
  ga.ws_inst = base + pl.inst_off;
  ga.inst_stride = sh.inst_bytes;
  ga.n_inst = n_inst;
  ga.Q = sh.Q;
  const int nb = gx_nb(sh.Npad);
  ga.n_groups = (sh.Cpad / 16 + nb - 1) / nb;
  ga.n_loops = n_loops;
  ga.sink = sink;
  const bool bf = params->precision == DMALA_BF16;
  hipError_t e;
  switch (sh.Npad) {
    case 32: e = launch_gx<2, 1, 2>(ga, bf, s); break;
    case 64: e = launch_gx<4, 1, 2>(ga, bf, s); break;
    case 128: e = launch_gx<8, 1, 1>(ga, bf, s); break;
    default: e = launch_gx<4, 4, 1>(ga, bf, s); break;
  }
  if (e != hipSuccess) return hip_fail(e, "gradient loop launch");
  g_err.clear();
  return DMALA_OK;
}

}  // extern "C"
