// Host-side planning shared by the uniform-batch API and uneven-batch plans.
#pragma once

#include <string>

#include "../../include/dmala.h"
#include "common.hpp"

namespace dmala {
namespace host {

// Workspace layout and launch geometry of one uniform batch (one shape class).
struct Plan {
  Shape sh;
  size_t inst_off, state_off, wscratch_off, total;
  double tau, am, bm, gm;
  bool naive;
  uint32_t mix_thr;   // learned mixture: plain kernel iff the 24-bit uniform < mix_thr
};

extern thread_local std::string g_err;
dmala_status fail(dmala_status st, const char* fmt, ...) __attribute__((format(printf, 2, 3)));
dmala_status hip_fail(hipError_t e, const char* what);
size_t round_up(size_t v, size_t a);
// Whether pts (M complex floats) is the canonical unit-energy square M-QAM.
bool canonical_qam(const float* pts, int M);

// Validate a uniform shape and compute its layout (workspace relative to 0).
dmala_status make_plan(int32_t n_inst, int32_t nt, int32_t nr, int32_t M, const dmala_params* p, Plan& pl);

// Enqueue setup, sampler and estimator for n_inst instances of one class whose
// workspace region starts at base (256-byte aligned); desc (device, may be NULL)
// maps the instances to the caller's buffers.
// sigma2 NULL: every instance has noise variance sigma2_val.  eval_dim: per-dimension forward
// log q terms of the evaluation mode (may be NULL).
dmala_status enqueue(const void* H, const void* y, const void* sigma2, int32_t n_inst, const Plan& pl,
                     const dmala_params* p, const dmala_outputs* out, const InstDesc* desc, unsigned char* base,
                     const int8_t* x_from, const int8_t* x_to, double* eval_out, hipStream_t stream,
                     double* eval_dim = nullptr, double sigma2_val = 0.0);

// The three kernels' arguments for one class (as enqueue passes them).
void make_args(const void* H, const void* y, const void* sigma2, int32_t n_inst, const Plan& pl, const dmala_params* p,
               const dmala_outputs* out, const InstDesc* desc, unsigned char* base, const int8_t* x_from,
               const int8_t* x_to, double* eval_out, double* eval_dim, double sigma2_val, SetupArgs& sa,
               SamplerArgs& ka, EstArgs& ea);
// Whether any estimator output is requested.
bool wants_estimates(const dmala_outputs* out);

}  // namespace host
}  // namespace dmala
