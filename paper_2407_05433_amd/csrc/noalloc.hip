// eclqr_solve_noalloc: eclqr_solve with the workspace in a static device
// array of the library instead of caller memory, for callers that cannot
// allocate (code under stream capture, serving loops that forbid it).
//
// The array `scratch` exists once per GPU the library runs on and lives until
// the process ends.  Its device address is looked up once per device
// (hipGetSymbolAddress, with that device current) and only that address is
// used from the host: the name itself is a host-side stand-in.
#include <hip/hip_runtime.h>

#include <mutex>
#include <string>

#include "eclqr.h"
#include "plan.hpp"

namespace eclqr {
eclqr_status report_error(eclqr_status st, const char* msg);
eclqr_status solve_in_shared(eclqr_plan* plan, const eclqr_problem* prob, eclqr_solution* sol, void* buf,
                             size_t bytes, void* stream, uint64_t* owner);
}

namespace {

constexpr size_t kScratchBytes = (size_t)64 << 20;  // the largest plan workspace this entry point serves
constexpr int kMaxDevices = 64;

static __device__ __align__(256) unsigned char scratch[kScratchBytes];

struct DeviceScratch {
  void* ptr = nullptr;   // device address of `scratch` on this device
  uint64_t owner = 0;    // plan whose tables the array holds (0: none)
};
DeviceScratch g_dev[kMaxDevices];
std::mutex g_mu;

}  // namespace

extern "C" eclqr_status eclqr_solve_noalloc(eclqr_plan* plan, const eclqr_problem* prob, eclqr_solution* sol,
                                            void* stream) {
  int dev = -1;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kMaxDevices)
    return eclqr::report_error(ECLQR_HIP_ERROR, "hipGetDevice failed or device index beyond 63");
  std::lock_guard<std::mutex> lock(g_mu);
  DeviceScratch& d = g_dev[dev];
  if (!d.ptr) {
    void* ptr = nullptr;
    const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !ptr)
      return eclqr::report_error(ECLQR_HIP_ERROR, "hipGetSymbolAddress of the static scratch array failed");
    d.ptr = ptr;
  }
  return eclqr::solve_in_shared(plan, prob, sol, d.ptr, kScratchBytes, stream, &d.owner);
}
