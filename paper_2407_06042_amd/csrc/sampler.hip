// Sampler dispatch: picks the compiled instance for a shape (the kernel
// templates live in sampler_impl.hpp, instantiated per proposal mode in
// sampler_<mode>.hip so that they compile in parallel).
#include "sampler_impl.hpp"

namespace dmala {

hipError_t launch_sampler_f64_naive(const Shape&, const SamplerArgs&, bool, hipStream_t, const Persist*, int, KernelCfg*);
hipError_t launch_sampler_f64_pre(const Shape&, const SamplerArgs&, bool, hipStream_t, const Persist*, int, KernelCfg*);
hipError_t launch_sampler_naive(const Shape&, const SamplerArgs&, bool, hipStream_t, const Persist*, int, KernelCfg*);
hipError_t launch_sampler_f16x2(const Shape&, const SamplerArgs&, bool, hipStream_t, const Persist*, int, KernelCfg*);
hipError_t launch_sampler_f16x1(const Shape&, const SamplerArgs&, bool, hipStream_t, const Persist*, int, KernelCfg*);
hipError_t launch_sampler_bf16x1(const Shape&, const SamplerArgs&, bool, hipStream_t, const Persist*, int, KernelCfg*);
hipError_t launch_sampler_lrn_f16x2(const Shape&, const SamplerArgs&, bool, hipStream_t, const Persist*, int, KernelCfg*);
hipError_t launch_sampler_lrn_f16x1(const Shape&, const SamplerArgs&, bool, hipStream_t, const Persist*, int, KernelCfg*);
hipError_t launch_sampler_lrn_bf16x1(const Shape&, const SamplerArgs&, bool, hipStream_t, const Persist*, int, KernelCfg*);
hipError_t launch_sampler_mhgd_f64(const Shape&, const SamplerArgs&, bool, hipStream_t, const Persist*, int, KernelCfg*);
hipError_t launch_sampler_mhgd_f16x2(const Shape&, const SamplerArgs&, bool, hipStream_t, const Persist*, int, KernelCfg*);
hipError_t launch_sampler_mhgd_bf16x1(const Shape&, const SamplerArgs&, bool, hipStream_t, const Persist*, int, KernelCfg*);

size_t sampler_lds_bytes(const Shape& sh) {
  if (sh.fp64) {
    const int cb = sh.cbw > 0 ? sh.cbw : 4;
    const int waves = sh.Cpad / 16 < cb ? sh.Cpad / 16 : cb;
    return sampler_cfg_lds(sh, sh.RT, 1, false, waves);
  }
  switch (sh.cfg) {
    case 0: return sampler_cfg_lds(sh, 2, 1, false, 4);
    case 1: return sampler_cfg_lds(sh, 4, 1, false, 4);
    case 2: return sampler_cfg_lds(sh, 8, 1, false, 4);
    case 3: return sampler_cfg_lds(sh, 4, 2, true, 2 * split_slots(sh, 2));
    case 4: return sampler_cfg_lds(sh, 4, 4, true, 4 * split_slots(sh, 4));
    case 5: return sampler_cfg_lds(sh, 2, 2, false, 2 * split_slots(sh, 2));
    case 6: return sampler_cfg_lds(sh, 2, 4, true, 4 * split_slots(sh, 4));
    case 7: return sampler_cfg_lds(sh, 4, 2, true, 2 * split_slots(sh, 2), true);
    case 8: return sampler_cfg_lds(sh, 4, 4, true, 4 * split_slots(sh, 4), true);
    case 9: return sampler_cfg_lds(sh, 4, 1, false, 4, true);
  }
  return ~(size_t)0;
}

bool sampler_cfg_valid(const Shape& sh, int cfg) {
  static const int rt_of[10] = {2, 4, 8, 8, 16, 4, 8, 8, 16, 4};
  if (cfg < 0 || cfg > 9 || rt_of[cfg] != sh.RT) return false;
  if (sh.lrn && cfg == 2) return false;   // the learned variant keeps at most 4 row tiles per wave
  if ((sh.lrn || sh.fp64) && cfg >= 7) return false;   // complex planes: the plain and MHGD float chains
  if (!sh.lrn && (cfg == 5 || cfg == 6)) return false;  // layouts 5, 6 are built for the learned variant only
  Shape t = sh;
  t.cfg = cfg;
  return sampler_lds_bytes(t) <= 160 * 1024;
}

int sampler_default_cfg(const Shape& sh) {
  // 64, 128 and 256 dimensions: the complex-plane layouts (half the fragment bytes) for the
  // preconditioned and MHGD chains (64x64 64-QAM fp32 sampler 18.7 -> 15.1 ms, 128x128 256-QAM
  // 9.7 -> 6.9 ms; at 64 dimensions the halved LDS copy lets four workgroups share a CU); two
  // waves of 4 tiles at two waves per SIMD beat one wave of 8 tiles
  const bool cx = !sh.lrn && sh.pm != PM_NAIVE;
  switch (sh.RT) {
    case 2: return 0;
    case 4: return sh.lrn ? 5 : (cx ? 9 : 1);   // 32x32 64-QAM fp32 sampler 4.63 -> 3.47 ms (4 workgroups per CU)
    case 8: return sh.lrn ? 6 : (cx ? 7 : 3);
    case 16: return cx ? 8 : 4;
  }
  return -1;
}

hipError_t launch_sampler(const Shape& sh, const SamplerArgs& a, bool eval, hipStream_t s, const Persist* p, int gn,
                    KernelCfg* cfg) {
  if (sh.mhgd) {
    if (sh.fp64) return launch_sampler_mhgd_f64(sh, a, eval, s, p, gn, cfg);
    if (sh.pm == PM_F16X2) return launch_sampler_mhgd_f16x2(sh, a, eval, s, p, gn, cfg);
    if (sh.pm == PM_BF16X1) return launch_sampler_mhgd_bf16x1(sh, a, eval, s, p, gn, cfg);
    return hipErrorInvalidValue;
  }
  if (sh.fp64) return sh.pm == PM_NAIVE ? launch_sampler_f64_naive(sh, a, eval, s, p, gn, cfg) : launch_sampler_f64_pre(sh, a, eval, s, p, gn, cfg);
  if (sh.lrn) {
    switch (sh.pm) {
      case PM_F16X2: return launch_sampler_lrn_f16x2(sh, a, eval, s, p, gn, cfg);
      case PM_F16X1: return launch_sampler_lrn_f16x1(sh, a, eval, s, p, gn, cfg);
      case PM_BF16X1: return launch_sampler_lrn_bf16x1(sh, a, eval, s, p, gn, cfg);
    }
    return hipErrorInvalidValue;
  }
  switch (sh.pm) {
    case PM_NAIVE: return launch_sampler_naive(sh, a, eval, s, p, gn, cfg);
    case PM_F16X2: return launch_sampler_f16x2(sh, a, eval, s, p, gn, cfg);
    case PM_F16X1: return launch_sampler_f16x1(sh, a, eval, s, p, gn, cfg);
    case PM_BF16X1: return launch_sampler_bf16x1(sh, a, eval, s, p, gn, cfg);
  }
  return hipErrorInvalidValue;
}

}  // namespace dmala
