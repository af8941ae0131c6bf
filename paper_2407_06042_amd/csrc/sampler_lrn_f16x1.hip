// Sampler instances: plain/learned kernel mixture, proposal mode PM_F16X1.
#include "sampler_impl.hpp"

namespace dmala {
hipError_t launch_sampler_lrn_f16x1(const Shape& sh, const SamplerArgs& a, bool eval, hipStream_t s, const Persist* p, int gn,
                    KernelCfg* cfg) {
  return launch_rt_lrn<PM_F16X1>(sh, a, eval, s, p, gn, cfg);
}
}  // namespace dmala
