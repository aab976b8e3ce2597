// Allocation-free execution (fbst_execute_static): the path of
// fbst_execute_batched with its workspace in a fixed device array of this
// library instead of caller or plan memory, for callers that cannot allocate
// device memory at execution time (code under graph capture, tight serving
// loops, harnesses that forbid hipMalloc).
//
// The array `scratch` below is a device-side object.  In host code its name
// is only a host stand-in, so host code never passes it to a kernel: the
// device address is looked up once per device with hipGetSymbolAddress (with
// that device current) and kept in g_scratch, and only that address reaches
// the kernels.  Each device holds its own copy of the array until the process
// ends.
#include <hip/hip_runtime.h>

#include <mutex>
#include <string>

#include "kernels.h"
#include "plan.h"

__device__ __align__(256) unsigned char scratch[FBST_STATIC_SCRATCH_BYTES];

namespace {

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch[kMaxDevices] = {};

fbst_status fail(fbst_status st, const std::string& msg) {
  fbst::set_last_error(msg);
  return st;
}

// Device address of `scratch` on the current device (looked up on first use).
fbst_status scratch_address(int device, void** out) {
  if (device < 0 || device >= kMaxDevices)
    return fail(FBST_E_UNSUPPORTED, "device index beyond the static scratch table");
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (!g_scratch[device]) {
    void* ptr = nullptr;
    const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !ptr)
      return fail(FBST_E_DEVICE, std::string("hipGetSymbolAddress of the static scratch: ") +
                                     hipGetErrorString(e));
    g_scratch[device] = ptr;
  }
  *out = g_scratch[device];
  return FBST_OK;
}

}  // namespace

extern "C" {

size_t fbst_static_scratch_bytes(void) { return FBST_STATIC_SCRATCH_BYTES; }

fbst_status fbst_execute_static(const fbst_plan* plan, int nblocks, const void* x, void* beams,
                                void* hip_stream) {
  if (!plan) return fail(FBST_E_INVALID, "plan is NULL");
  if (plan->host_only) return fail(FBST_E_INVALID, "plan was created host-only");
  if (nblocks < 0) return fail(FBST_E_INVALID, "nblocks must be >= 0");
  if (nblocks == 0) return FBST_OK;
  if (!x || !beams) return fail(FBST_E_INVALID, "x and beams must not be NULL");
  const size_t per_block = plan->ws_bytes_per_block, fixed = plan->ws_fixed_bytes;
  if (per_block + fixed > FBST_STATIC_SCRATCH_BYTES)
    return fail(FBST_E_UNSUPPORTED,
                "one block of this plan needs " + std::to_string(per_block + fixed) +
                    " bytes of workspace, more than the " +
                    std::to_string(static_cast<size_t>(FBST_STATIC_SCRATCH_BYTES)) +
                    "-byte static scratch; use fbst_execute_batched with a workspace");
  int device = -1;
  hipError_t e = hipGetDevice(&device);
  if (e != hipSuccess) return fail(FBST_E_DEVICE, std::string("hipGetDevice: ") + hipGetErrorString(e));
  if (device != plan->device)
    return fail(FBST_E_INVALID, "the plan's device must be the current device");
  void* ws = nullptr;
  fbst_status s = scratch_address(device, &ws);
  if (s != FBST_OK) return s;
  int chunk = static_cast<int>((FBST_STATIC_SCRATCH_BYTES - fixed) / per_block);
  if (chunk > fbst::MAX_LAUNCH_BLOCKS) chunk = fbst::MAX_LAUNCH_BLOCKS;
  if (chunk > nblocks) chunk = nblocks;
  e = fbst::run_contiguous(plan, nblocks, chunk, x, beams, ws, static_cast<hipStream_t>(hip_stream));
  if (e != hipSuccess)
    return fail(FBST_E_DEVICE, std::string("fbst_execute_static launch: ") + hipGetErrorString(e));
  return FBST_OK;
}

}  // extern "C"
