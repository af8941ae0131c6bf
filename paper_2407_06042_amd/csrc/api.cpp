// C ABI of the DMALA library: argument validation, workspace layout, launches.
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <string>

#include "../../include/dmala.h"
#include "common.hpp"
#include "host.hpp"

static_assert((int)DMALA_ERR_NONFINITE == dmala::kStatusNonfinite, "status code of a flagged instance");

namespace dmala {
namespace host {

thread_local std::string g_err;

dmala_status fail(dmala_status st, const char* fmt, ...) __attribute__((format(printf, 2, 3)));
dmala_status fail(dmala_status st, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof buf, fmt, ap);
  va_end(ap);
  g_err = buf;
  return st;
}

size_t round_up(size_t v, size_t a) { return (v + a - 1) / a * a; }

dmala_status make_plan(int32_t n_inst, int32_t nt, int32_t nr, int32_t M, const dmala_params* p, Plan& pl) {
  if (!p) return fail(DMALA_ERR_ARG, "params is NULL");
  if (n_inst < 1) return fail(DMALA_ERR_ARG, "n_inst must be >= 1 (got %d)", n_inst);
  if (nt < 1 || nr < 1) return fail(DMALA_ERR_ARG, "nt and nr must be >= 1 (got %d, %d)", nt, nr);
  if (p->n_chains < 1 || p->n_chains > 1024) return fail(DMALA_ERR_ARG, "n_chains must be in [1, 1024] (got %d)", p->n_chains);
  if (p->n_iters < 0 || p->n_iters > 65535) return fail(DMALA_ERR_ARG, "n_iters must be in [0, 65535] (got %d)", p->n_iters);
  if (p->precision < DMALA_FP64 || p->precision > DMALA_FP16) return fail(DMALA_ERR_ARG, "unknown precision %d", (int)p->precision);
  if (p->proposal != DMALA_PRECOND && p->proposal != DMALA_NAIVE && p->proposal != DMALA_LEARNED &&
      p->proposal != DMALA_MHGD)
    return fail(DMALA_ERR_ARG, "unknown proposal %d", (int)p->proposal);
  const bool lrn = p->proposal == DMALA_LEARNED;
  const bool mhgd = p->proposal == DMALA_MHGD;
  if (mhgd && p->precision == DMALA_FP16)
    return fail(DMALA_ERR_UNSUPPORTED, "DMALA_MHGD runs with DMALA_FP64, DMALA_FP32 or DMALA_BF16");
  if (p->llr_mode < DMALA_LLR_IS || p->llr_mode > DMALA_LLR_MC) return fail(DMALA_ERR_ARG, "unknown llr_mode %d", (int)p->llr_mode);
  if (lrn) {
    if (p->precision == DMALA_FP64) return fail(DMALA_ERR_UNSUPPORTED, "DMALA_LEARNED is not available with DMALA_FP64");
    if (!p->mlp_weights) return fail(DMALA_ERR_ARG, "DMALA_LEARNED needs mlp_weights");
    if (!(p->mix_eps >= 0.0 && p->mix_eps <= 1.0)) return fail(DMALA_ERR_ARG, "mix_eps must be in [0, 1]");
  }
  if (!(std::isfinite(p->tau) && std::isfinite(p->alpha_mult) && std::isfinite(p->beta_mult) && std::isfinite(p->gamma_mult)))
    return fail(DMALA_ERR_ARG, "non-finite tau/alpha/beta/gamma multiplier");
  int Q = 0;
  if (M == 4) Q = 2; else if (M == 16) Q = 4; else if (M == 64) Q = 8; else if (M == 256) Q = 16;
  else return fail(DMALA_ERR_UNSUPPORTED, "qam_order must be 4, 16, 64 or 256 (got %d)", M);
  if (nr > 4096) return fail(DMALA_ERR_UNSUPPORTED, "nr > 4096 is not supported (got %d)", nr);
  const bool fp64 = p->precision == DMALA_FP64;
  if (nt > 128) return fail(DMALA_ERR_UNSUPPORTED, "nt > 128 is not supported (got %d)", nt);
  if (fp64 && nt > 32) return fail(DMALA_ERR_UNSUPPORTED, "DMALA_FP64 supports nt <= 32 (got %d)", nt);
  Shape& sh = pl.sh;
  sh.nt = nt; sh.nr = nr; sh.M = M; sh.Q = Q; sh.N = 2 * nt;
  sh.Npad = 32;  // the sampler layouts cover 32, 64, 128 or 256 real dimensions
  while (sh.Npad < sh.N) sh.Npad *= 2;
  sh.RT = sh.Npad / 16; sh.KB = sh.RT / 2;
  sh.C = p->n_chains; sh.Cpad = 16 * ((sh.C + 15) / 16); sh.T = p->n_iters;
  sh.fp64 = fp64 ? 1 : 0;
  sh.lrn = lrn ? 1 : 0;
  sh.mhgd = mhgd ? 1 : 0;
  sh.share = 0;
  pl.naive = p->proposal == DMALA_NAIVE;
  if (pl.naive) sh.pm = PM_NAIVE;
  else if (p->precision == DMALA_BF16) sh.pm = PM_BF16X1;
  else if (p->precision == DMALA_FP16) sh.pm = PM_F16X1;
  else sh.pm = PM_F16X2;
  // Proposal window: with the preconditioned parameters kL = 2 log2(e) / (alpha_mult beta_mult)
  // is the same for every instance; a 3-level window is exact to fp32 when kL * 3 * 4 >= 30, and
  // its factorised weights (powers up to exp2(3 kL)) stay finite in fp32 for kL <= 40.
  {
    const double am = p->alpha_mult > 0 ? p->alpha_mult : 1.0, bm = p->beta_mult > 0 ? p->beta_mult : 1.0;
    const double kL = 2.0 * 1.4426950408889634 / (am * bm);
    sh.win = (!fp64 && !pl.naive && !lrn && !mhgd && Q >= 8 && kL * 12.0 >= 30.0 && kL <= 40.0) ? 3 : 0;
  }
  auto set_frag_bytes = [&]() {
    if (fp64) {
      sh.frag_bytes = round_up((2 * (size_t)sh.Npad * sh.Npad + 2 * (size_t)sh.Npad) * 8, 16);
    } else {
      // fragments (real-equivalent RT x KB, or complex planes 2 x RT/2 x RT/4 KiB per split term), then
      // the vectors pb, ez and the per-antenna network features
      const size_t pass = sh.cx ? (size_t)sh.RT * sh.RT / 4 * 1024 : (size_t)sh.RT * sh.KB * 1024;
      sh.frag_bytes = (size_t)(p_passes(sh.pm) + kEPasses) * pass + 3 * (size_t)sh.Npad * 4;
    }
  };
  sh.cx = 0;
  set_frag_bytes();
  if (p->tile_config < 0 || p->tile_config > 10) return fail(DMALA_ERR_ARG, "tile_config must be in [0, 10]");
  if (p->wg_chain_blocks != 0 && p->wg_chain_blocks != 1 && p->wg_chain_blocks != 2 && p->wg_chain_blocks != 4)
    return fail(DMALA_ERR_ARG, "wg_chain_blocks must be 0, 1, 2 or 4");
  sh.cbw = p->wg_chain_blocks ? p->wg_chain_blocks : 4;
  if (fp64 || p->tile_config == 0) {
      sh.cfg = fp64 ? 0 : sampler_default_cfg(sh);
  } else {
    if (!sampler_cfg_valid(sh, p->tile_config - 1))
      return fail(DMALA_ERR_UNSUPPORTED, "tile_config %d does not fit this shape", p->tile_config);
    sh.cfg = p->tile_config - 1;
  }
  sh.cx = (sh.cfg == 7 || sh.cfg == 8 || sh.cfg == 9) ? 1 : 0;
  set_frag_bytes();
  if (sampler_lds_bytes(sh) > 160 * 1024)
    return fail(DMALA_ERR_UNSUPPORTED, "shape needs %zu bytes of LDS (> 160 KiB)", sampler_lds_bytes(sh));
  sh.inst_bytes = round_up(kParamBytes + sh.frag_bytes, 256);
  sh.state_bytes = state_offsets(sh.Cpad, sh.Npad).end;
  sh.wscratch_bytes = setup_w_global(nt) ? round_up((size_t)nt * (nt + 1) * 16, 256) : 0;
  pl.inst_off = 0;
  pl.state_off = round_up((size_t)n_inst * sh.inst_bytes, 256);
  pl.wscratch_off = round_up(pl.state_off + (size_t)n_inst * sh.state_bytes, 256);
  pl.total = pl.wscratch_off + (size_t)n_inst * sh.wscratch_bytes;
  pl.tau = p->tau > 0 ? p->tau : 2.0;
  pl.am = p->alpha_mult > 0 ? p->alpha_mult : 1.0;
  pl.bm = p->beta_mult > 0 ? p->beta_mult : 1.0;
  pl.gm = p->gamma_mult > 0 ? p->gamma_mult : 1.0;
  pl.mix_thr = 0;
  if (lrn) {
    const double t = std::ceil(p->mix_eps * 16777216.0);
    pl.mix_thr = (uint32_t)(t < 0 ? 0 : (t > 16777216.0 ? 16777216.0 : t));
  }
  return DMALA_OK;
}

bool canonical_qam(const float* pts, int M) {
  const int Q = (int)std::lround(std::sqrt((double)M));
  const double s = std::sqrt(3.0 / (2.0 * (M - 1)));
  for (int a = 0; a < M; ++a) {
    const double re = s * (2 * (a / Q) - Q + 1), im = s * (2 * (a % Q) - Q + 1);
    if (std::fabs(pts[2 * a] - re) > 1e-6 || std::fabs(pts[2 * a + 1] - im) > 1e-6) return false;
  }
  return true;
}

dmala_status hip_fail(hipError_t e, const char* what) {
  return fail(DMALA_ERR_HIP, "%s: %s", what, hipGetErrorString(e));
}

void make_args(const void* H, const void* y, const void* sigma2, int32_t n_inst, const Plan& pl, const dmala_params* p,
               const dmala_outputs* out, const InstDesc* desc, unsigned char* base, const int8_t* x_from,
               const int8_t* x_to, double* eval_out, double* eval_dim, double sigma2_val, SetupArgs& sa,
               SamplerArgs& ka, EstArgs& ea) {
  const Shape& sh = pl.sh;
  sa = SetupArgs{};
  sa.desc = desc;
  sa.H = H; sa.y = y; sa.sigma2 = sigma2;
  sa.sigma2_val = sigma2_val;
  sa.status = (!eval_out && out) ? out->status : nullptr;
  sa.ws_inst = base + pl.inst_off; sa.inst_stride = sh.inst_bytes;
  sa.wscratch = base + pl.wscratch_off; sa.wscratch_stride = sh.wscratch_bytes;
  sa.n_inst = n_inst; sa.nt = sh.nt; sa.nr = sh.nr; sa.Q = sh.Q; sa.N = sh.N; sa.Npad = sh.Npad;
  sa.RT = sh.RT; sa.KB = sh.KB; sa.fp64 = sh.fp64; sa.pm = sh.pm; sa.naive = pl.naive ? 1 : 0; sa.cx = sh.cx;
  sa.tau = pl.tau; sa.alpha_mult = pl.am; sa.beta_mult = pl.bm; sa.gamma_mult = pl.gm;

  ka = SamplerArgs{};
  ka.desc = desc;
  ka.ws_inst = base + pl.inst_off; ka.inst_stride = sh.inst_bytes;
  ka.ws_state = base + pl.state_off; ka.state_stride = sh.state_bytes;
  ka.n_inst = n_inst; ka.N = sh.N; ka.Npad = sh.Npad; ka.C = sh.C; ka.Cpad = sh.Cpad; ka.T = sh.T;
  ka.key0 = (uint32_t)(p->seed & 0xFFFFFFFFu); ka.key1 = (uint32_t)(p->seed >> 32);
  ka.ctr_base = p->counter_base;
  ka.frag_bytes = (int)sh.frag_bytes;
  if (eval_out) {
    ka.x_from = x_from; ka.x_to = x_to; ka.eval_out = eval_out; ka.eval_dim = eval_dim;
  } else if (out) {
    ka.final_state = out->final_state; ka.accept_count = out->accept_count;
    ka.trace_accept = out->trace_accept; ka.trace_hash = out->trace_hash;
    ka.trace_words = (sh.T + 31) / 32;
    ka.train_rows = out->train_rows;
  }
  ka.mlp = sh.lrn ? p->mlp_weights : nullptr;
  ka.mix_thr = pl.mix_thr;

  ea = EstArgs{};
  ea.desc = desc;
  ea.H = H; ea.y = y; ea.sigma2 = sigma2;
  ea.ws_inst = base + pl.inst_off; ea.inst_stride = sh.inst_bytes;
  ea.ws_state = base + pl.state_off; ea.state_stride = sh.state_bytes;
  ea.n_inst = n_inst; ea.nt = sh.nt; ea.nr = sh.nr; ea.Q = sh.Q; ea.N = sh.N; ea.Npad = sh.Npad;
  ea.C = sh.C; ea.Cpad = sh.Cpad; ea.fp64 = sh.fp64;
  ea.chunk = estimate_chunk(sh.nt, sh.nr, sh.M, sh.N, sh.C, sh.fp64 != 0);
  ea.llr_mode = (int)p->llr_mode;
  ea.llr_clip = 20.0f;
  if (out) {
    ea.symbols = out->symbols; ea.marginals = out->marginals; ea.llrs = out->llrs;
    ea.best_energy = out->best_energy; ea.marginals_mc = out->marginals_mc;
  }
}

bool wants_estimates(const dmala_outputs* out) {
  return out && (out->symbols || out->marginals || out->llrs || out->best_energy || out->marginals_mc);
}

dmala_status enqueue(const void* H, const void* y, const void* sigma2, int32_t n_inst, const Plan& pl,
                     const dmala_params* p, const dmala_outputs* out, const InstDesc* desc, unsigned char* base,
                     const int8_t* x_from, const int8_t* x_to, double* eval_out, hipStream_t stream,
                     double* eval_dim, double sigma2_val) {
  const Shape& sh = pl.sh;
  SetupArgs sa;
  SamplerArgs ka;
  EstArgs ea;
  make_args(H, y, sigma2, n_inst, pl, p, out, desc, base, x_from, x_to, eval_out, eval_dim, sigma2_val, sa, ka, ea);
  auto mark = [&](int i) {
    if (!eval_out && out && out->stage_events[i]) (void)hipEventRecord((hipEvent_t)out->stage_events[i], stream);
  };
  mark(0);
  hipError_t e = launch_setup(sa, stream);
  if (e != hipSuccess) return hip_fail(e, "setup launch");
  const bool eval = eval_out != nullptr;
  mark(1);
  e = launch_sampler(sh, ka, eval, stream);
  if (e != hipSuccess) return hip_fail(e, "sampler launch");
  mark(2);
  if (eval || !out) return DMALA_OK;
  if (wants_estimates(out)) {
    e = launch_estimate(ea, stream);
    if (e != hipSuccess) return hip_fail(e, "estimator launch");
  }
  mark(3);
  return DMALA_OK;
}

dmala_status run(const void* H, const void* y, const void* sigma2, int32_t n_inst, const Plan& pl,
                 const dmala_params* p, const dmala_outputs* out, const int8_t* x_from, const int8_t* x_to,
                 double* eval_out, double* eval_dim, void* ws, size_t ws_bytes, hipStream_t stream) {
  if (!H || !y || !sigma2) return fail(DMALA_ERR_ARG, "H, y and sigma2 must be non-NULL");
  if (!ws) return fail(DMALA_ERR_WORKSPACE, "workspace is NULL");
  if (ws_bytes < pl.total) return fail(DMALA_ERR_WORKSPACE, "workspace too small: %zu < %zu bytes", ws_bytes, pl.total);
  if (((uintptr_t)ws & 255) != 0) return fail(DMALA_ERR_WORKSPACE, "workspace must be 256-byte aligned");
  if (out && out->train_rows && (pl.naive || pl.sh.fp64 || pl.sh.mhgd))
    return fail(DMALA_ERR_UNSUPPORTED, "train_rows needs the PRECOND or LEARNED proposal without DMALA_FP64");
  return enqueue(H, y, sigma2, n_inst, pl, p, out, nullptr, (unsigned char*)ws, x_from, x_to, eval_out, stream,
                 eval_dim, 0.0);
}

}  // namespace host
}  // namespace dmala

using namespace dmala;
using namespace dmala::host;

extern "C" {

size_t dmala_workspace_size(int32_t n_inst, int32_t nt, int32_t nr, int32_t qam_order, const dmala_params* params) {
  Plan pl;
  if (make_plan(n_inst, nt, nr, qam_order, params, pl) != DMALA_OK) return 0;
  g_err.clear();
  return pl.total;
}

dmala_status dmala_detect(const void* H, const void* y, const void* sigma2, int32_t n_inst, int32_t nt, int32_t nr,
                          int32_t qam_order, const float* constellation, const dmala_params* params,
                          const dmala_outputs* out, void* workspace, size_t workspace_bytes, dmala_stream_t stream) {
  Plan pl;
  dmala_status st = make_plan(n_inst, nt, nr, qam_order, params, pl);
  if (st != DMALA_OK) return st;
  if (constellation && !canonical_qam(constellation, qam_order))
    return fail(DMALA_ERR_UNSUPPORTED, "constellation is not the canonical unit-energy square %d-QAM", qam_order);
  st = run(H, y, sigma2, n_inst, pl, params, out, nullptr, nullptr, nullptr, nullptr, workspace, workspace_bytes,
           (hipStream_t)stream);
  if (st == DMALA_OK) g_err.clear();
  return st;
}

dmala_status dmala_debug_eval(const void* H, const void* y, const void* sigma2, int32_t n_inst, int32_t nt, int32_t nr,
                              int32_t qam_order, const dmala_params* params, const int8_t* x_from, const int8_t* x_to,
                              int32_t n_pairs, double* out, double* out_dim, void* workspace, size_t workspace_bytes,
                              dmala_stream_t stream) {
  if (!params) return fail(DMALA_ERR_ARG, "params is NULL");
  if (!x_from || !x_to || !out) return fail(DMALA_ERR_ARG, "x_from, x_to and out must be non-NULL");
  dmala_params p = *params;
  p.n_chains = n_pairs;
  p.n_iters = 0;
  Plan pl;
  dmala_status st = make_plan(n_inst, nt, nr, qam_order, &p, pl);
  if (st != DMALA_OK) return st;
  st = run(H, y, sigma2, n_inst, pl, &p, nullptr, x_from, x_to, out, out_dim, workspace, workspace_bytes,
           (hipStream_t)stream);
  if (st == DMALA_OK) g_err.clear();
  return st;
}

dmala_status dmala_sync_status(const int32_t* status, int32_t n_inst, dmala_stream_t stream) {
  if (!status || n_inst < 1) return fail(DMALA_ERR_ARG, "status must be non-NULL and n_inst >= 1");
  hipError_t e = hipStreamSynchronize((hipStream_t)stream);
  if (e != hipSuccess) return hip_fail(e, "stream synchronize");
  int32_t buf[1024];
  int32_t flagged = 0, first = -1;
  for (int32_t b0 = 0; b0 < n_inst; b0 += 1024) {
    const int32_t n = n_inst - b0 < 1024 ? n_inst - b0 : 1024;
    e = hipMemcpy(buf, status + b0, (size_t)n * sizeof(int32_t), hipMemcpyDeviceToHost);
    if (e != hipSuccess) return hip_fail(e, "status copy");
    for (int32_t i = 0; i < n; ++i)
      if (buf[i] != DMALA_OK) {
        ++flagged;
        if (first < 0) first = b0 + i;
      }
  }
  if (flagged)
    return fail(DMALA_ERR_NONFINITE, "%d of %d instances have a non-finite entry in H or y, or sigma^2 not positive "
                "and finite (first: instance %d)", flagged, n_inst, first);
  g_err.clear();
  return DMALA_OK;
}

namespace {
dmala_params one_params(int32_t n_chains, int32_t n_iters, uint64_t seed) {
  dmala_params p{};
  p.n_chains = n_chains;
  p.n_iters = n_iters;
  p.seed = seed;
  p.precision = DMALA_FP32;
  p.proposal = DMALA_PRECOND;
  p.llr_mode = DMALA_LLR_IS;
  return p;
}
}  // namespace

size_t dmala_detect_one_workspace_size(int32_t nt, int32_t nr, int32_t qam_order, int32_t n_chains) {
  const dmala_params p = one_params(n_chains, 0, 0);
  Plan pl;
  if (make_plan(1, nt, nr, qam_order, &p, pl) != DMALA_OK) return 0;
  g_err.clear();
  return round_up(pl.total, 256) + 256;   // + the instance's status word
}

dmala_status dmala_detect_one(const void* H, const void* y, float sigma2, int32_t nt, int32_t nr,
                              const float* constellation, int32_t qam_order, int32_t n_chains, int32_t n_iters,
                              uint64_t seed, int32_t* symbols, float* marginals, void* workspace,
                              size_t workspace_bytes, dmala_stream_t stream) {
  const dmala_params p = one_params(n_chains, n_iters, seed);
  Plan pl;
  dmala_status st = make_plan(1, nt, nr, qam_order, &p, pl);
  if (st != DMALA_OK) return st;
  if (constellation && !canonical_qam(constellation, qam_order))
    return fail(DMALA_ERR_UNSUPPORTED, "constellation is not the canonical unit-energy square %d-QAM", qam_order);
  if (!H || !y || !symbols) return fail(DMALA_ERR_ARG, "H, y and symbols must be non-NULL");
  if (!(sigma2 > 0.f) || !std::isfinite(sigma2))
    return fail(DMALA_ERR_NONFINITE, "sigma^2 must be positive and finite (got %g)", (double)sigma2);
  const size_t status_off = round_up(pl.total, 256);
  if (!workspace) return fail(DMALA_ERR_WORKSPACE, "workspace is NULL");
  if (workspace_bytes < status_off + 256)
    return fail(DMALA_ERR_WORKSPACE, "workspace too small: %zu < %zu bytes", workspace_bytes, status_off + 256);
  if (((uintptr_t)workspace & 255) != 0) return fail(DMALA_ERR_WORKSPACE, "workspace must be 256-byte aligned");
  dmala_outputs o{};
  o.symbols = symbols;
  o.marginals = marginals;
  o.status = (int32_t*)((unsigned char*)workspace + status_off);
  hipStream_t s = (hipStream_t)stream;
  st = enqueue(H, y, nullptr, 1, pl, &p, &o, nullptr, (unsigned char*)workspace, nullptr, nullptr, nullptr, s, nullptr,
               (double)sigma2);
  if (st != DMALA_OK) return st;
  return dmala_sync_status(o.status, 1, stream);
}

const char* dmala_last_error(void) { return g_err.c_str(); }

const char* dmala_version(void) { return "dmala-mi355x 0.1 (gfx950)"; }

}  // extern "C"
