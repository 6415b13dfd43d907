// sar_reconstruct_noalloc: the per-scan pipeline of sar_reconstruct (the same
// kernels, launched the same way) with its workspace in a file-scope device
// array instead of a caller-provided buffer, for callers that cannot allocate
// device memory (code under HIP graph capture, tight serving loops).
//
// The array `scratch` exists once per device the library runs on and stays
// until the process ends.  In host code its name only stands in for the
// symbol: its device address (one per device) comes from hipGetSymbolAddress,
// looked up on the first call on each device with that device current, and
// only that address is handed to the kernels.  Every call on a device uses the
// same array; the pipeline clears what it needs zeroed (the per-cell counts)
// with a fill kernel and overwrites everything else, so a call never depends
// on what an earlier one left.  Calls that overlap on one device (different
// streams or host threads) race on the array.
#include <hip/hip_runtime.h>

#include <mutex>
#include <string>

#include "sar_internal.hpp"

namespace sar {
namespace {

__device__ __align__(256) char scratch[SAR_NOALLOC_SCRATCH_BYTES];

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxDevices] = {};

// device address of `scratch` on device `dev` (which must be current)
sar_status scratch_address(int dev, void** out) {
  if (dev < 0 || dev >= kMaxDevices) return fail(SAR_ERR_INVALID, "device index out of range");
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void* ptr = nullptr;
    const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !ptr) return check_hip(e != hipSuccess ? e : hipErrorInvalidSymbol, "scratch address");
    g_scratch_ptr[dev] = ptr;
  }
  *out = g_scratch_ptr[dev];
  return SAR_OK;
}

}  // namespace
}  // namespace sar

using namespace sar;

extern "C" sar_status sar_reconstruct_noalloc(sar_plan plan, const double* d_pos, int64_t n_pos, const void* d_echo,
                                              float echo_scale, void* d_image, sar_stream_t stream) {
  sar_status st = check_reconstruct_args(plan, n_pos, d_pos, d_echo, d_image);
  if (st != SAR_OK) return st;
  const Plan& p = plan->p;
  const size_t need = workspace_bytes(p, n_pos, nullptr, nullptr);
  if (need > (size_t)SAR_NOALLOC_SCRATCH_BYTES)
    return fail(SAR_ERR_UNSUPPORTED, "the scan needs " + std::to_string(need) +
                                         " bytes of workspace; the fixed scratch of sar_reconstruct_noalloc holds " +
                                         std::to_string((size_t)SAR_NOALLOC_SCRATCH_BYTES));
  int old = -1;
  if (hipGetDevice(&old) != hipSuccess) old = -1;
  const bool switched = old != p.device;
  if (switched && (st = check_hip(hipSetDevice(p.device), "hipSetDevice")) != SAR_OK) return st;
  void* ws = nullptr;
  st = scratch_address(p.device, &ws);
  if (st == SAR_OK) st = reconstruct_on(p, d_pos, n_pos, d_echo, echo_scale, d_image, ws, (hipStream_t)stream);
  if (switched && old >= 0) (void)hipSetDevice(old);
  return st;
}
