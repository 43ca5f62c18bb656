// Entry points that allocate nothing: their scratch memory is a file-scope
// device array instead of a caller workspace, for callers that cannot call
// hipMalloc (code under stream capture, serving loops that must not
// allocate).  The array is loaded with the library's code object, once per
// device, and stays allocated until the process ends.
#include <stdio.h>

#include <mutex>

#include "../../include/nadmm.h"
#include "kernels.h"

namespace nadmm {
// Sets the calling thread's nadmm_last_error() message and returns s
// (defined in capi.hip, where that message lives).
nadmm_status set_last_error(nadmm_status s, const char* msg);
}  // namespace nadmm

using namespace nadmm;

// Partials of the Jacobian reduction: 4 doubles (min, max, sum, count) for
// each of the at most kJacBlocks blocks of its first launch (32 KB).
constexpr size_t kScratchDoubles = 4 * (size_t)kJacBlocks;
static __device__ __align__(256) double scratch[kScratchDoubles];

namespace {

// In host code `scratch` names a host-side stand-in, not device memory: the
// device address of each GPU's copy comes from hipGetSymbolAddress, taken
// once per device with that device current, and only that address is used.
constexpr int kMaxDevices = 64;
std::mutex g_mu;
bool g_have[kMaxDevices] = {};
void* g_ptr[kMaxDevices] = {};

hipError_t scratch_ptr(void** out) {
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return e;
  if (dev < 0 || dev >= kMaxDevices) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lock(g_mu);
  if (!g_have[dev]) {
    void* p = nullptr;
    e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    if (!p) return hipErrorInvalidSymbol;
    g_ptr[dev] = p;
    g_have[dev] = true;
  }
  *out = g_ptr[dev];
  return hipSuccess;
}

nadmm_status fail_msg(nadmm_status s, const char* msg, const char* detail) {
  char buf[256];
  snprintf(buf, sizeof(buf), "%s%s", msg, detail ? detail : "");
  return set_last_error(s, buf);
}

bool aligned16(const void* p) { return (reinterpret_cast<uintptr_t>(p) & 15) == 0; }

}  // namespace

extern "C" {

nadmm_status nadmm_jacobian_noalloc(nadmm_dims d, const float* disp, float* det, double* stats,
                                    int64_t* n_nonpos, void* stream) {
  // the same argument checks as nadmm_jacobian (dims through the workspace
  // query, which validates them and allocates nothing)
  size_t ws_bytes = 0;
  const nadmm_status sd = nadmm_workspace_size(d, nullptr, &ws_bytes);
  if (sd != NADMM_OK) return sd;  // nadmm_last_error() holds the reason
  if (!disp || !stats || !n_nonpos)
    return fail_msg(NADMM_ERR_INVALID_ARG, "disp, stats and n_nonpos must not be NULL", nullptr);
  if (!aligned16(disp) || !aligned16(det) || !aligned16(stats) || !aligned16(n_nonpos))
    return fail_msg(NADMM_ERR_INVALID_ARG, "every array pointer must be 16-byte aligned", nullptr);
  const Geo g{d.nx, d.ny, d.nz, d.nx * d.ny * d.nz};
  const size_t need = 4 * sizeof(double) * (size_t)jacobian_blocks(g);
  if (need > sizeof(scratch))
    return fail_msg(NADMM_ERR_UNSUPPORTED_SIZE, "nadmm_jacobian_noalloc: partials exceed the "
                    "32 KB scratch array", nullptr);
  void* p = nullptr;
  hipError_t e = scratch_ptr(&p);
  if (e != hipSuccess)
    return fail_msg(NADMM_ERR_HIP, "hipGetSymbolAddress(scratch): ", hipGetErrorString(e));
  e = launch_jacobian(g, disp, det, static_cast<double*>(p), stats, n_nonpos,
                      static_cast<hipStream_t>(stream));
  if (e != hipSuccess) return fail_msg(NADMM_ERR_HIP, "launch_jacobian: ", hipGetErrorString(e));
  return NADMM_OK;
}

}  // extern "C"
