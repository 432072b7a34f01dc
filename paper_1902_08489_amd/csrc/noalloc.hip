// Fixed device scratch of the no-allocation entry point (tdmps_heff_apply_noalloc).
//
// The array lives in the code object: every GPU the library runs on holds its own copy, at its
// own address, until the process ends.  Host code never takes the array's name as a device
// address: the per-device address is read once with hipGetSymbolAddress (at context creation,
// with the device current) and only that pointer is handed to copies and kernels.
#include <hip/hip_runtime.h>

#include <mutex>
#include <string>

#include "common.h"
#include "kernels.h"

namespace tdmps {
namespace {

static __device__ __align__(256) unsigned char scratch[TDMPS_NOALLOC_SCRATCH_BYTES];

constexpr int MAX_DEVICES = 64;
std::mutex g_mu;
void* g_ptr[MAX_DEVICES] = {};

}  // namespace

void noalloc_init(int device) {
  TDMPS_REQUIRE(device >= 0 && device < MAX_DEVICES, TDMPS_ERR_ARG, "device index out of range");
  std::lock_guard<std::mutex> lk(g_mu);
  if (g_ptr[device]) return;
  int cur = -1;
  hipError_t e = hipGetDevice(&cur);
  TDMPS_REQUIRE(e == hipSuccess && cur == device, TDMPS_ERR_HIP, "noalloc_init: device is not current");
  void* p = nullptr;
  e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
  TDMPS_REQUIRE(e == hipSuccess && p != nullptr, TDMPS_ERR_HIP,
                std::string("hipGetSymbolAddress of the no-allocation scratch: ") + hipGetErrorString(e));
  g_ptr[device] = p;
}

void* noalloc_scratch(int device, size_t* cap) {
  *cap = TDMPS_NOALLOC_SCRATCH_BYTES;
  if (device < 0 || device >= MAX_DEVICES) return nullptr;
  std::lock_guard<std::mutex> lk(g_mu);
  return g_ptr[device];
}

}  // namespace tdmps
