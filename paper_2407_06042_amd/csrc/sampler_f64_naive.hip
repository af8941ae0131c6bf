// Sampler instances: double arithmetic, proposal mode PM_NAIVE.
#include "sampler_impl.hpp"

namespace dmala {
hipError_t launch_sampler_f64_naive(const Shape& sh, const SamplerArgs& a, bool eval, hipStream_t s, const Persist* p, int gn,
                    KernelCfg* cfg) {
  return launch_rt<double, PM_NAIVE>(sh, a, eval, s, p, gn, cfg);
}
}  // namespace dmala
