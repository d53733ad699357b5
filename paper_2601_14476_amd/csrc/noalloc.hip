// noalloc.hip -- the static device scratch behind psa_anneal_noalloc.
//
// A whole anneal needs device memory beyond its inputs and outputs: the
// schedule and per-p-bit factors as the kernels read them, the spin state,
// the task order, SpSA held inputs or TApSA windows, and the partial sums of
// the energy reduction.  psa_anneal allocates these per call; the
// no-allocation variant carves them from this file-scope array instead.
// Every GPU the library runs on holds its own copy of the array (at its own
// address) from the first context on that device until the process ends.
//
// In host code `scratch` names a host-side stand-in, not device memory: the
// device address is looked up once per device with hipGetSymbolAddress and
// only that address is ever handed to copies and kernels.
#include <hip/hip_runtime.h>

#include <mutex>
#include <string>

#include "engine.hpp"

static __device__ __align__(256) unsigned char scratch[PSA_NOALLOC_SCRATCH_BYTES];

namespace psa {

namespace {
constexpr int32_t kMaxDevices = 64;
std::mutex g_scratch_mu;
void *g_scratch_ptr[kMaxDevices] = {};
}  // namespace

psa_status noalloc_scratch_init(int32_t device) {
    if (device < 0 || device >= kMaxDevices) {
        set_error("static scratch: device index " + std::to_string(device) + " out of range");
        return PSA_EINVAL;
    }
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (g_scratch_ptr[device]) return PSA_OK;
    void *ptr = nullptr;
    PSA_HIP(hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)), "hipGetSymbolAddress(scratch)");
    if (!ptr) {
        set_error("static scratch: hipGetSymbolAddress returned no address");
        return PSA_EHIP;
    }
    g_scratch_ptr[device] = ptr;
    return PSA_OK;
}

void *noalloc_scratch(int32_t device) {
    if (device < 0 || device >= kMaxDevices) return nullptr;
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    return g_scratch_ptr[device];
}

}  // namespace psa
