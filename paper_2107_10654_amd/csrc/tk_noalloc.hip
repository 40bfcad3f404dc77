// The sampled core update for callers that cannot allocate device memory
// (code under HIP graph capture, tight serving loops, harnesses that forbid
// hipMalloc).  Its workspace is a file-scope device array instead of a caller
// buffer; every kernel is the one tucker_core_update_sketched launches.
#include <mutex>

#include "tk_internal.h"

namespace {

constexpr size_t kScratchBytes = TK_NOALLOC_SCRATCH_BYTES;

// One copy per GPU, held until the process ends.  In host code `scratch` is
// only a stand-in for the symbol: its device address comes from
// hipGetSymbolAddress, once per device, and only that address is used.
static __device__ __align__(256) unsigned char scratch[kScratchBytes];

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxDevices];

// Device address of the current device's copy of `scratch` (looked up on the
// first call made with that device current).
tk_status scratch_address(void** out) {
  int dev = -1;
  if (hipGetDevice(&dev) != hipSuccess) return TK_E_HIP;
  if (dev < 0 || dev >= kMaxDevices) return TK_E_HIP;
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void* ptr = nullptr;
    if (hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)) != hipSuccess || !ptr) return TK_E_HIP;
    g_scratch_ptr[dev] = ptr;
  }
  *out = g_scratch_ptr[dev];
  return TK_OK;
}

}  // namespace

extern "C" {

tk_status tucker_core_update_sketched_noalloc(const tk_problem* p, const tk_sketch_opts* opts,
                                              const int32_t* idx_in, const double* weight_in,
                                              int32_t* idx_out, double* weight_out,
                                              void* core_out, int32_t* dev_status,
                                              double* dev_info, void* stream) {
  if (!p || !opts) return TK_E_ARG;
  // 0 means the problem or the options are invalid: the full entry point
  // below returns the precise code before it enqueues anything.
  const size_t need = tucker_workspace_bytes(p, opts, TK_CALL_SKETCHED);
  if (need > kScratchBytes) return TK_E_WORKSPACE;
  void* ws = nullptr;
  const tk_status stt = scratch_address(&ws);
  if (stt != TK_OK) return stt;
  return tucker_core_update_sketched(p, opts, idx_in, weight_in, idx_out, weight_out, core_out,
                                     dev_status, dev_info, ws, kScratchBytes, stream);
}

}  // extern "C"
