// Sampler dispatch: picks the compiled instance for a shape (the kernel
// templates live in sampler_impl.hpp, instantiated per proposal mode in
// sampler_<mode>.hip so that they compile in parallel).
#include "common.hpp"

namespace dmala {

hipError_t launch_sampler_f64_naive(const Shape&, const SamplerArgs&, bool, hipStream_t);
hipError_t launch_sampler_f64_pre(const Shape&, const SamplerArgs&, bool, hipStream_t);
hipError_t launch_sampler_naive(const Shape&, const SamplerArgs&, bool, hipStream_t);
hipError_t launch_sampler_f16x2(const Shape&, const SamplerArgs&, bool, hipStream_t);
hipError_t launch_sampler_f16x1(const Shape&, const SamplerArgs&, bool, hipStream_t);
hipError_t launch_sampler_bf16x1(const Shape&, const SamplerArgs&, bool, hipStream_t);

size_t sampler_lds_bytes(const Shape& sh) {
  if (sh.fp64) {
    const int waves = sh.Cpad / 16 < 4 ? sh.Cpad / 16 : 4;
    return sh.frag_bytes + (size_t)waves * 16 * sh.Npad * sizeof(double);
  }
  return sh.RT > 4 ? sh.frag_bytes - 2 * (size_t)sh.Npad * 4 : sh.frag_bytes;
}

hipError_t launch_sampler(const Shape& sh, const SamplerArgs& a, bool eval, hipStream_t s) {
  if (sh.fp64) return sh.pm == PM_NAIVE ? launch_sampler_f64_naive(sh, a, eval, s) : launch_sampler_f64_pre(sh, a, eval, s);
  switch (sh.pm) {
    case PM_NAIVE: return launch_sampler_naive(sh, a, eval, s);
    case PM_F16X2: return launch_sampler_f16x2(sh, a, eval, s);
    case PM_F16X1: return launch_sampler_f16x1(sh, a, eval, s);
    case PM_BF16X1: return launch_sampler_bf16x1(sh, a, eval, s);
  }
  return hipErrorInvalidValue;
}

}  // namespace dmala
