// fx_tape_eval_static: fx_tape_eval for callers that cannot allocate.
//
// The reductions of a tape need a workspace (per-block partials and the
// finish counters).  Here it is one file-scope device array, `scratch`, of
// kStaticScratchBytes; every GPU holds its own copy for the life of the
// process.  In host code the array's name is only a stand-in for the symbol,
// so the first call on a device looks its device address up
// (hipGetSymbolAddress) and clears the array with a fill kernel on the
// caller's stream; after that the finish counters are left at zero by every
// call, like a caller's workspace.  No call allocates device or pinned
// memory.  Calls that overlap on one GPU share the array and race.
#include <mutex>

#include "fx_tape.hpp"

namespace fx {

constexpr size_t kStaticScratchBytes = size_t(16) << 20;
constexpr int kMaxDevices = 64;

static __device__ __align__(256) unsigned char scratch[kStaticScratchBytes];

namespace {

std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxDevices] = {};

// The device address of this device's scratch (looked up and cleared on the
// first call on the device, in stream order before the call's own kernels).
int device_scratch(hipStream_t st, void** out) {
  int dev = -1;
  if (int rc = hip_check(hipGetDevice(&dev), "hipGetDevice")) return rc;
  if (dev < 0 || dev >= kMaxDevices) return fail(FX_E_UNSUPPORTED, "device %d out of range", dev);
  std::lock_guard<std::mutex> g(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void* p = nullptr;
    if (int rc = hip_check(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)), "hipGetSymbolAddress"))
      return rc;
    const int64_t words = (int64_t)(kStaticScratchBytes / sizeof(uint32_t));
    hipLaunchKernelGGL((k_fill_zero<uint32_t>), dim3(1024), dim3(256), 0, st,
                       static_cast<uint32_t*>(p), words);
    if (int rc = hip_check(hipGetLastError(), "k_fill_zero launch")) return rc;
    g_scratch_ptr[dev] = p;
  }
  *out = g_scratch_ptr[dev];
  return FX_OK;
}

}  // namespace
}  // namespace fx

using namespace fx;

extern "C" {

int fx_tape_eval_static(const fx_tape* t, fx_dtype dt, const void* const* inputs, int32_t n_inputs,
                        fx_shape s, int kind, void* out, const fx_launch* cfg, void* stream) {
  if (!t) return fail(FX_E_ARG, "NULL tape");
  if (int rc = check_shape(s)) return rc;
  if (int rc = check_launch(cfg)) return rc;
  if (kind != 0) {
    const size_t need = fx_workspace_bytes(kind, dt, s, cfg);
    if (need > kStaticScratchBytes)
      return fail(FX_E_WORKSPACE,
                  "the reduction needs %zu bytes of workspace; the static scratch holds %zu",
                  need, kStaticScratchBytes);
  }
  void* ws = nullptr;
  if (int rc = device_scratch(S(stream), &ws)) return rc;
  return tape_eval_exact(t, dt, inputs, n_inputs, s, kind, out, ws, kStaticScratchBytes, cfg,
                         S(stream));
}

}  // extern "C"
