// fmm_evaluate_noalloc: the forward evaluation with every device buffer of
// the evaluation (multipoles, locals, FP64 top levels, P2P partial sums)
// taken from one fixed array of device memory that the code object holds, so
// the call allocates nothing.  For callers that cannot allocate (code under
// stream capture, tight serving loops, harnesses that forbid allocation).
#include <hip/hip_runtime.h>

#include <mutex>

#include "fmm.h"
#include "fmm_internal.h"

namespace {

constexpr size_t kScratchBytes = size_t(FMM_NOALLOC_SCRATCH_BYTES);
constexpr int kMaxDevices = 64;

// One copy per GPU, held from the library's load until the process ends.
static __device__ __align__(256) unsigned char scratch[kScratchBytes];

std::mutex g_scratch_mutex;
void *g_scratch_ptr[kMaxDevices] = {};

// Device address of `scratch` on the current device, looked up once per
// device.  (In host code `scratch` itself is only a stand-in for the symbol,
// never a device address.)
int scratch_address(void **out) {
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) {
    fmmlib::set_last_error(hipGetErrorString(e));
    return FMM_EDEVICE;
  }
  if (dev < 0 || dev >= kMaxDevices) {
    fmmlib::set_last_error("fmm_evaluate_noalloc: device ordinal out of range");
    return FMM_EDEVICE;
  }
  std::lock_guard<std::mutex> lock(g_scratch_mutex);
  if (!g_scratch_ptr[dev]) {
    void *ptr = nullptr;
    e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !ptr) {
      fmmlib::set_last_error(e != hipSuccess ? hipGetErrorString(e)
                                             : "hipGetSymbolAddress returned NULL");
      return FMM_EDEVICE;
    }
    g_scratch_ptr[dev] = ptr;
  }
  *out = g_scratch_ptr[dev];
  return FMM_OK;
}

}  // namespace

extern "C" int fmm_evaluate_noalloc(const fmm_tree *t, const fmm_lists *l,
                                    const fmm_eval_opts *o, const void *q_dev, void *phi_dev,
                                    void *grad_dev, void *stream) {
  return fmmlib::evaluate_fixed_scratch(t, l, o, q_dev, phi_dev, grad_dev, stream,
                                        scratch_address, kScratchBytes);
}

extern "C" size_t fmm_noalloc_scratch_bytes(void) { return kScratchBytes; }
