// Sampler instances: double arithmetic, proposal mode PM_F16X2.
#include "sampler_impl.hpp"

namespace dmala {
hipError_t launch_sampler_f64_pre(const Shape& sh, const SamplerArgs& a, bool eval, hipStream_t s, const Persist* p, int gn,
                    KernelCfg* cfg) {
  return launch_rt<double, PM_F16X2>(sh, a, eval, s, p, gn, cfg);
}
}  // namespace dmala
