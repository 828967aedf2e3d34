// The device area of the entry point that allocates nothing
// (hca_cluster_noalloc, in hca_api.cpp): hca_cluster with its device
// workspace in a fixed array of this library, for callers that cannot call
// hipMalloc (graph capture, tight serving loops).
//
// The array is a file-scope __device__ object, so every device the library's
// code is loaded on holds its own copy until the process ends.  Host code
// never passes the array's name to a kernel or a copy: that name is a host
// stand-in, not a device address.  hca_create looks the real address up once
// per device with that device current, and every call uses the address.
// All calls on one device share the area and it keeps the last call's
// contents: each call re-initialises what must start at zero (its counters,
// histograms, look-back words and tables, with kernels), and calls that
// overlap in time on one device race.
#include <hip/hip_runtime.h>

#include <mutex>

#include "hca.h"
#include "hca_internal.h"

namespace {

constexpr size_t kScratchBytes = (size_t)HCA_NOALLOC_BYTES;
constexpr int kMaxDevices = 64;

__device__ __align__(256) unsigned char scratch[kScratchBytes];

std::mutex g_mu;
void *g_area[kMaxDevices];

}  // namespace

namespace hca {

hipError_t scratch_setup(int device)
{
    if (device < 0 || device >= kMaxDevices) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lk(g_mu);
    if (g_area[device]) return hipSuccess;
    void *p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    g_area[device] = p;
    return hipSuccess;
}

void *scratch_area(int device, size_t *bytes)
{
    *bytes = kScratchBytes;
    if (device < 0 || device >= kMaxDevices) return nullptr;
    std::lock_guard<std::mutex> lk(g_mu);
    return g_area[device];
}

}  // namespace hca
