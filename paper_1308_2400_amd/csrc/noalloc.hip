// Strict product for callers that cannot allocate (afmm_multiply_noalloc):
// the workspace lives in a fixed device array of this library, one copy per
// device, instead of coming from the caller or the stream-ordered allocator.
#include <mutex>
#include <vector>

#include "afmm.h"
#include "common.hpp"

namespace afmm {

// Declared in api.cpp: argument checks, configuration choice and the strict
// launch sequence with the given workspace; AFMM_ERR_WORKSPACE when the
// product needs more than ws_bytes.
afmm_status strict_product_in(afmm_case c, int64_t n, const void* X, const void* Y, float* Z,
                              void* ws, size_t ws_bytes, hipStream_t s);

namespace {

// Each device that runs this code holds its own copy until the process ends.
// In host code `scratch` is only a handle: its device address comes from
// hipGetSymbolAddress, once per device, and only that address is used.
static __device__ __align__(256) uint8_t scratch[AFMM_NOALLOC_SCRATCH_BYTES];

std::mutex g_mu;
std::vector<void*> g_ptr;  // device address of `scratch`, per device (nullptr: not looked up)

// Address of this device's array; looked up with the device current.
hipError_t scratch_on(int dev, void** out) {
    std::lock_guard<std::mutex> lk(g_mu);
    if ((int)g_ptr.size() <= dev) g_ptr.resize(dev + 1, nullptr);
    if (!g_ptr[dev]) {
        void* p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return e;
        if (!p) return hipErrorInvalidSymbol;
        g_ptr[dev] = p;
    }
    *out = g_ptr[dev];
    return hipSuccess;
}

}  // namespace
}  // namespace afmm

extern "C" afmm_status afmm_multiply_noalloc(afmm_case c, int64_t n, const void* X, const void* Y,
                                             float* Z, hipStream_t stream) {
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) return AFMM_ERR_NO_DEVICE;
    void* ws = nullptr;
    const hipError_t e = afmm::scratch_on(dev, &ws);
    if (e != hipSuccess) {
        afmm::set_last_hip_error((int)e);
        return AFMM_ERR_HIP;
    }
    return afmm::strict_product_in(c, n, X, Y, Z, ws, AFMM_NOALLOC_SCRATCH_BYTES, stream);
}
