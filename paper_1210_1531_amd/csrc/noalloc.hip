// Fixed device scratch of the allocation-free entry point (mag_sk_vjp_noalloc).
//
// The scratch is a file-scope device array, so each GPU the library runs on
// holds its own copy, at its own address, from module load until the process
// ends.  In host code the array's name is only a stand-in: its device
// address is looked up once per device with hipGetSymbolAddress (called from
// mag_create with that device current) and kept here; every kernel argument
// and copy uses that address.
#include <mutex>

#include "mag_internal.h"

namespace mag {

// per pattern block: three doubles of the pair's force part (3 * MAX
// doubles), then one int32 per block for the index of its transposed block
static __device__ __align__(256) double scratch[NOALLOC_DOUBLES];

namespace {
constexpr int MAX_DEVICES = 64;
struct DeviceScratch {
  bool looked_up = false;
  void* ptr = nullptr;
  hipError_t err = hipSuccess;
};
std::mutex g_lock;
DeviceScratch g_scratch[MAX_DEVICES];
}  // namespace

void noalloc_init(int device) {
  if (device < 0 || device >= MAX_DEVICES) return;
  std::lock_guard<std::mutex> guard(g_lock);
  DeviceScratch& d = g_scratch[device];
  if (d.looked_up) return;
  d.looked_up = true;
  void* p = nullptr;
  d.err = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
  if (d.err == hipSuccess) {
    d.ptr = p;
  } else {
    (void)hipGetLastError();
  }
}

hipError_t noalloc_scratch(int device, void** ptr) {
  *ptr = nullptr;
  if (device < 0 || device >= MAX_DEVICES) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> guard(g_lock);
  const DeviceScratch& d = g_scratch[device];
  if (!d.looked_up) return hipErrorNotInitialized;
  if (d.err != hipSuccess) return d.err;
  *ptr = d.ptr;
  return hipSuccess;
}

}  // namespace mag
