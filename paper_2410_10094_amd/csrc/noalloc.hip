// sptc_contract_noalloc: one contraction with no device allocation, for
// callers that cannot allocate.  Its workspace is a static device array of
// SPTC_NOALLOC_SCRATCH_BYTES, one per device, that the library holds until
// the process ends.
#include <hip/hip_runtime.h>

#include <mutex>

#include "../../include/sptc.h"

namespace sptc {
sptc_status contract_in_scratch(void* base, size_t bytes, const sptc_coo* X, const sptc_coo* Y, int32_t ncontract,
                                const int32_t* cx, const int32_t* cy, const sptc_options* opt, int32_t* out_idx,
                                double* out_val, int64_t out_cap, int64_t* out_nnz, void* stream);
sptc_status report_hip_error(hipError_t e, const char* what);
}  // namespace sptc

namespace {

// In host code the name `scratch` stands for the array but is not its
// device address: every host use goes through the address that
// hipGetSymbolAddress gives for the current device.
static __device__ __align__(256) unsigned char scratch[SPTC_NOALLOC_SCRATCH_BYTES];

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_addr[kMaxDevices] = {};  // device address of `scratch`, per device

// The array's address on `dev` (current), looked up once per device.
hipError_t scratch_address(int dev, void** out) {
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_addr[dev]) {
    void* p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    if (!p) return hipErrorInvalidSymbol;
    g_scratch_addr[dev] = p;
  }
  *out = g_scratch_addr[dev];
  return hipSuccess;
}

}  // namespace

extern "C" SPTC_API sptc_status sptc_contract_noalloc(const sptc_coo* X, const sptc_coo* Y, int32_t ncontract,
                                                      const int32_t* cx, const int32_t* cy, const sptc_options* opt,
                                                      int32_t* out_idx, double* out_val, int64_t out_cap,
                                                      int64_t* out_nnz, void* stream) {
  int dev = -1;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return sptc::report_hip_error(e, "hipGetDevice");
  if (dev < 0 || dev >= kMaxDevices) return sptc::report_hip_error(hipErrorInvalidDevice, "device index");
  void* base = nullptr;
  e = scratch_address(dev, &base);
  if (e != hipSuccess) return sptc::report_hip_error(e, "hipGetSymbolAddress(scratch)");
  return sptc::contract_in_scratch(base, SPTC_NOALLOC_SCRATCH_BYTES, X, Y, ncontract, cx, cy, opt, out_idx, out_val,
                                   out_cap, out_nnz, stream);
}
