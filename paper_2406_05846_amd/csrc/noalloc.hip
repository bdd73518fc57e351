// noalloc.hip -- the entry point that allocates no device memory: the certificate's dual bound
// with its work memory in a static device array instead of a per-call hipMalloc.
//
// The array is a device-side object: in host code its name is only a stand-in, so its device
// address is looked up once per device with hipGetSymbolAddress (at context creation, with
// the device current) and only that address is used from then on.  Every call on a device
// shares that device's array: calls that overlap on one device race (the library serializes
// its own calls; independent processes or threads driving the device around it must not).
#include <hip/hip_runtime.h>

#include <mutex>
#include <string>

#include "../../include/strom.h"
#include "strom_internal.h"

namespace {
constexpr size_t kScratchBytes = size_t(32) << 20;  // 32 MiB per device
constexpr int kMaxDevices = 64;

static __device__ __align__(256) unsigned char scratch[kScratchBytes];

std::mutex g_mu;
void *g_ptr[kMaxDevices] = {};
}  // namespace

namespace strom {
strom_status scratch_init(int device) {
  if (device < 0 || device >= kMaxDevices) return set_error(STROM_E_INVAL, "device index beyond the scratch table");
  std::lock_guard<std::mutex> lk(g_mu);
  if (g_ptr[device]) return STROM_OK;
  void *p = nullptr;
  const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
  if (e != hipSuccess || !p)
    return set_error(STROM_E_HIP, std::string("hipGetSymbolAddress of the scratch buffer: ") + hipGetErrorString(e));
  g_ptr[device] = p;
  return STROM_OK;
}
}  // namespace strom

extern "C" strom_status strom_dual_bound_noalloc(strom_sdp *s, const double *R_beta, double *lb, double *lam_min) {
  if (!s) return strom::set_error(STROM_E_INVAL, "sdp is NULL");
  const int dev = strom::sdp_device(s);
  void *p = nullptr;
  {
    std::lock_guard<std::mutex> lk(g_mu);
    if (dev >= 0 && dev < kMaxDevices) p = g_ptr[dev];
  }
  if (!p) return strom::set_error(STROM_E_STATE, "no scratch address for this device (context not created)");
  strom::DeviceBuf work{static_cast<unsigned char *>(p), kScratchBytes};
  return strom::dual_bound_impl(s, R_beta, lb, lam_min, &work);
}

extern "C" size_t strom_scratch_bytes(void) { return kScratchBytes; }
