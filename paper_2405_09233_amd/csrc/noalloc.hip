// Allocation-free form of tsylv_apply for callers that cannot allocate
// device memory (code under HIP graph capture, tight serving loops): every
// intermediate buffer of Algorithm 1 (Fourier planes, transform matrices,
// low-precision copies) lives in one file-scope device array, `scratch`,
// that each GPU holds from the library's load until the process ends.
//
// In host code `scratch` names a host-side stand-in, not the device
// address: the address is taken once per device with hipGetSymbolAddress
// (that device current) and kept, and only that pointer is handed to
// kernels.  Every call on a GPU shares that GPU's array, and the kernels of
// one call overwrite what the previous call left there; calls that overlap
// on one GPU (different streams, or threads without ordering) race.
// Nothing in the scratch has to start at zero: every buffer is written in
// full before it is read.
#include <mutex>

#include "runtime.hpp"
#include "solvers.hpp"

namespace {

constexpr size_t kScratchBytes = size_t(256) << 20;
constexpr int kMaxDevices = 64;

static __device__ __align__(256) char scratch[kScratchBytes];

std::mutex g_mu;
void* g_scratch[kMaxDevices] = {};

// The device address of this GPU's scratch (taken on first use).
void* device_scratch(int dev) {
  std::lock_guard<std::mutex> g(g_mu);
  if (!g_scratch[dev]) {
    void* ptr = nullptr;
    const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (e != hipSuccess || ptr == nullptr)
      throw tsylv::Error(TSYLV_EHIP, std::string("hipGetSymbolAddress(scratch): ") +
                                         hipGetErrorString(e));
    g_scratch[dev] = ptr;
  }
  return g_scratch[dev];
}

}  // namespace

extern "C" {

size_t tsylv_noalloc_scratch_bytes(void) { return kScratchBytes; }

int tsylv_apply_noalloc(void* hip_stream, int64_t n, int64_t s, int64_t p, const double* A,
                        const double* B, const double* X, double* Y, int prec) {
  if (!A || !B || !X || !Y || n <= 0 || s <= 0 || p <= 0 || n > (int64_t(1) << 20) ||
      s > (int64_t(1) << 20) || p > 4096)
    return TSYLV_EINVAL;
  if (prec != TSYLV_FP64 && prec != TSYLV_FP32 && prec != TSYLV_BF16) return TSYLV_EINVAL;
  if (tsylv::apply_workspace_bytes(n, s, p) > kScratchBytes) return TSYLV_ESCRATCH;
  try {
    int dev = 0;
    TSYLV_HIP(hipGetDevice(&dev));
    if (dev < 0 || dev >= kMaxDevices) return TSYLV_EINVAL;
    char* buf = static_cast<char*>(device_scratch(dev));
    tsylv::apply_spatial_into(buf, kScratchBytes, static_cast<hipStream_t>(hip_stream), n, s, p,
                              A, B, X, Y, prec);
    return TSYLV_OK;
  } catch (const tsylv::Error& e) {
    return e.status;
  } catch (...) {
    return TSYLV_EHIP;
  }
}

}  // extern "C"
