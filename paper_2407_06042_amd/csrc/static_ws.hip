// dmala_detect_static: dmala_detect with its workspace in a fixed device array.
//
// For callers that cannot allocate device memory.  The array below lives in
// every GPU's copy of the code object for as long as the process runs; host code
// reaches it only through the device address hipGetSymbolAddress returns for the
// current device (the array's name in host code is a host-side stand-in, not a
// device address).  The kernels are the ones dmala_detect launches, given that
// address as their workspace.  They write every workspace byte they read before
// reading it, so nothing has to start at zero, and a call leaves the previous
// call's contents irrelevant.
#include <mutex>

#include "../../include/dmala.h"
#include "common.hpp"
#include "host.hpp"

namespace dmala {

static __device__ __align__(256) unsigned char scratch[DMALA_STATIC_SCRATCH_BYTES];

namespace {

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxDevices] = {};

// Device address of this device's scratch array (looked up once per device, with
// that device current).
dmala_status scratch_for_current_device(unsigned char** out) {
  int dev = -1;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return host::hip_fail(e, "hipGetDevice");
  if (dev < 0 || dev >= kMaxDevices) return host::fail(DMALA_ERR_UNSUPPORTED, "device index %d out of range", dev);
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void* p = nullptr;
    e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return host::hip_fail(e, "hipGetSymbolAddress(scratch)");
    if (!p || ((uintptr_t)p & 255) != 0) return host::fail(DMALA_ERR_HIP, "static scratch address %p is not 256-byte aligned", p);
    g_scratch_ptr[dev] = p;
  }
  *out = (unsigned char*)g_scratch_ptr[dev];
  return DMALA_OK;
}

}  // namespace
}  // namespace dmala

using namespace dmala;
using namespace dmala::host;

extern "C" dmala_status dmala_detect_static(const void* H, const void* y, const void* sigma2, int32_t n_inst, int32_t nt,
                                            int32_t nr, int32_t qam_order, const float* constellation,
                                            const dmala_params* params, const dmala_outputs* out,
                                            dmala_stream_t stream) {
  Plan pl;
  dmala_status st = make_plan(n_inst, nt, nr, qam_order, params, pl);
  if (st != DMALA_OK) return st;
  if (constellation && !canonical_qam(constellation, qam_order))
    return fail(DMALA_ERR_UNSUPPORTED, "constellation is not the canonical unit-energy square %d-QAM", qam_order);
  if (pl.total > (size_t)DMALA_STATIC_SCRATCH_BYTES)
    return fail(DMALA_ERR_WORKSPACE, "this batch needs %zu bytes of workspace; the static scratch holds %zu bytes "
                "(use dmala_detect with a caller workspace, or fewer instances per call)",
                pl.total, (size_t)DMALA_STATIC_SCRATCH_BYTES);
  if (!H || !y || !sigma2) return fail(DMALA_ERR_ARG, "H, y and sigma2 must be non-NULL");
  if (out && out->train_rows && (pl.naive || pl.sh.fp64 || pl.sh.mhgd))
    return fail(DMALA_ERR_UNSUPPORTED, "train_rows needs the PRECOND or LEARNED proposal without DMALA_FP64");
  unsigned char* base = nullptr;
  st = scratch_for_current_device(&base);
  if (st != DMALA_OK) return st;
  st = enqueue(H, y, sigma2, n_inst, pl, params, out, nullptr, base, nullptr, nullptr, nullptr, (hipStream_t)stream);
  if (st == DMALA_OK) g_err.clear();
  return st;
}
