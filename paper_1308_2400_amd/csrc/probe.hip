// Binary32 add-rate probe: long straight-line runs of v_add_f32 with VGPR
// operands, one block per compute unit.  It measures the denominator of the
// strict kernels' roofline on the device at hand; it computes nothing of the
// method.
#include "afmm.h"
#include "common.hpp"

namespace afmm {
namespace {

constexpr int kProbeAcc = 16;  // independent accumulators per lane
constexpr int kProbeRep = 8;   // additions per accumulator per loop trip

// 96 KB of LDS keeps a second block off the compute unit, so the waves per SIMD
// are exactly W / 4.
template <int W>
__global__ __launch_bounds__(W * 64) void add_rate_probe_kernel(float* __restrict__ out, int trips,
                                                               float seed) {
    __shared__ float hold[24576];
    float acc[kProbeAcc], b[kProbeAcc];
#pragma unroll
    for (int i = 0; i < kProbeAcc; ++i) {
        acc[i] = seed * (float)(threadIdx.x + i);
        b[i] = seed + (float)i;
    }
    if (trips < 0) hold[threadIdx.x] = acc[0];  // never true: keeps the LDS allocation
    for (int t = 0; t < trips; ++t) {
#pragma unroll
        for (int r = 0; r < kProbeRep; ++r)
#pragma unroll
            for (int i = 0; i < kProbeAcc; ++i) acc[i] = acc[i] + b[i];
    }
    float s = 0.0f;
#pragma unroll
    for (int i = 0; i < kProbeAcc; ++i) s = s + acc[i];
    out[threadIdx.x] = s + (trips < 0 ? hold[threadIdx.x] : 0.0f);
}

}  // namespace
}  // namespace afmm

extern "C" afmm_status afmm_probe_add_rate(int32_t waves_per_simd, int32_t trips, float* d_out,
                                           uint64_t* adds, hipStream_t stream) {
    if (!d_out || !adds || trips < 1 || (waves_per_simd != 1 && waves_per_simd != 2 &&
                                         waves_per_simd != 4))
        return AFMM_ERR_INVALID_ARG;
    int dev = 0;
    hipDeviceProp_t prop;
    if (hipGetDevice(&dev) != hipSuccess || hipGetDeviceProperties(&prop, dev) != hipSuccess)
        return AFMM_ERR_NO_DEVICE;
    const int blocks = prop.multiProcessorCount, W = 4 * waves_per_simd;
    const float seed = 1.0f / 1024.0f;
    if (W == 4)
        hipLaunchKernelGGL(afmm::add_rate_probe_kernel<4>, dim3(blocks), dim3(256), 0, stream, d_out,
                           trips, seed);
    else if (W == 8)
        hipLaunchKernelGGL(afmm::add_rate_probe_kernel<8>, dim3(blocks), dim3(512), 0, stream, d_out,
                           trips, seed);
    else
        hipLaunchKernelGGL(afmm::add_rate_probe_kernel<16>, dim3(blocks), dim3(1024), 0, stream,
                           d_out, trips, seed);
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) {
        afmm::set_last_hip_error((int)e);
        return AFMM_ERR_HIP;
    }
    *adds = (uint64_t)blocks * W * 64 * (uint64_t)trips * afmm::kProbeAcc * afmm::kProbeRep;
    return AFMM_OK;
}
