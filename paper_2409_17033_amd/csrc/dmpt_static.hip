// dmpt_response_static: the responses Tr[chi_k H1_p] (Eq. dual) with no
// workspace argument and no allocation, for callers that cannot allocate
// device memory.  The FP64 partial sums and the reduced results live in a
// file-scope device array of kStaticScratchBytes on each device; its device
// address is looked up once per device (hipGetSymbolAddress with that
// device current) and passed to the same kernels dmpt_response launches.
// Every call on a device uses that device's array: calls that overlap on one
// device race on it.  Nothing in it needs clearing: every partial is written
// before it is read, and every result before it is copied out.
#include <hip/hip_runtime.h>

#include <mutex>

#include "dmpt_internal.h"

namespace dmpt {
namespace {

constexpr size_t kStaticScratchBytes = (size_t)4 << 20;   // 4 MiB per device
constexpr int kMaxDevices = 64;

static __device__ __align__(256) char scratch[kStaticScratchBytes];

std::mutex g_mu;
void* g_ptr[kMaxDevices] = {};

// Device address of this device's scratch array (nullptr on failure, with
// the HIP error in *err).
void* scratch_ptr(int dev, hipError_t* err) {
  std::lock_guard<std::mutex> lk(g_mu);
  if (!g_ptr[dev]) {
    void* p = nullptr;
    *err = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (*err != hipSuccess) return nullptr;
    g_ptr[dev] = p;
  }
  *err = hipSuccess;
  return g_ptr[dev];
}

}  // namespace
}  // namespace dmpt

extern "C" dmpt_status dmpt_response_static(const float* chi, int32_t nobs, const float* H1, int32_t npert,
                                            int32_t n, double* out, void* stream) {
  using namespace dmpt;
  if (!chi || !H1 || !out) return report_error(DMPT_ERR_ARG, "chi, H1 and out must not be NULL");
  const size_t need = response_workspace_bytes(nobs, npert, n);
  if (need == 0) return DMPT_ERR_ARG;   // message set by response_workspace_bytes
  if (need > kStaticScratchBytes)
    return report_error(DMPT_ERR_WORKSPACE,
                        "dmpt_response_static: these sizes need more than its 4 MiB device scratch "
                        "(use dmpt_response with a workspace of dmpt_response_workspace_bytes)");
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kMaxDevices)
    return report_error(DMPT_ERR_DEVICE, "dmpt_response_static: no current HIP device");
  hipError_t e = hipSuccess;
  void* p = scratch_ptr(dev, &e);
  if (!p) return report_error(DMPT_ERR_DEVICE, hipGetErrorString(e));
  return response_run(chi, nobs, H1, npert, n, out, stream, p, kStaticScratchBytes);
}
