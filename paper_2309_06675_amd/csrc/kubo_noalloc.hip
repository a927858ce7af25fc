// kubo_noalloc.hip -- kubo_ahc_noalloc: the forward on a workspace that lives
// in a static device array of the library, for callers that cannot allocate
// device memory themselves.
//
// The array is `scratch` below.  In host code its name stands for a host-side
// shadow, not for device memory, so it is never passed to a kernel or a copy:
// on the first call on a device (with that device current) the device address
// of that device's copy is looked up once with hipGetSymbolAddress and kept;
// every later use goes through the kept address.
#include <hip/hip_runtime.h>

#include <cstdint>
#include <mutex>

#include "../../include/kubo.h"
#include "kubo_launch.h"

namespace kubo {
namespace {

constexpr size_t kNoAllocBytes = KUBO_NOALLOC_MAX_BYTES;
static_assert(kNoAllocBytes % 256 == 0, "scratch size");

// One copy per GPU, held until the process ends.  Shared by every call on
// that GPU; it keeps the last call's contents.
static __device__ __align__(256) unsigned char scratch[kNoAllocBytes];

constexpr int kMaxDevices = 64;
std::mutex g_mu;
void* g_ptr[kMaxDevices] = {nullptr};

// Device address of the current device's copy of `scratch` (nullptr on error).
void* scratch_ptr() {
    int dev = -1;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kMaxDevices) return nullptr;
    std::lock_guard<std::mutex> lock(g_mu);
    if (!g_ptr[dev]) {
        void* p = nullptr;
        if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess || !p) return nullptr;
        g_ptr[dev] = p;
    }
    return g_ptr[dev];
}

}  // namespace
}  // namespace kubo

extern "C" kubo_status kubo_ahc_noalloc(kubo_plan_t plan, const double* t, const double* e_fermi,
                                        double eta, double kT, double* sigma,
                                        uint32_t* device_status, void* stream) {
    if (!plan || !t || !e_fermi || !sigma) return KUBO_E_INVALID;
    void* ws = kubo::scratch_ptr();
    if (!ws) return KUBO_E_HIP;
    // ahc_enqueue rejects a plan whose workspace exceeds the array (KUBO_E_WORKSPACE)
    kubo_status st = kubo::ahc_enqueue(plan, t, e_fermi, eta, kT, sigma, ws, kubo::kNoAllocBytes,
                                       stream, false);
    if (st != KUBO_OK || !device_status) return st;
    // the status word sits at the start of the workspace
    if (hipMemcpyAsync(device_status, ws, sizeof(uint32_t), hipMemcpyDeviceToDevice,
                       static_cast<hipStream_t>(stream)) != hipSuccess)
        return KUBO_E_HIP;
    return KUBO_OK;
}
