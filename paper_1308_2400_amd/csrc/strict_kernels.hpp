// Strict AFMM kernel templates (bit-exact binary32 repeated addition, Section 2);
// instantiated over several translation units so that they compile in parallel.
#pragma once

#include "strict_body.hpp"

namespace afmm {



template <int R, int C, int W, int U, int KP, bool VEC, bool TRANS_OUT, bool BUF>
__global__ __launch_bounds__(W * kWave) void rep_uniform_kernel(
    int n_r, int n_c, int n_k, const uint8_t* __restrict__ P8, int64_t ldp,
    const int32_t* __restrict__ P32, int64_t p32_sr, int64_t p32_sk,
    const float* __restrict__ Q, int64_t ldq, float* __restrict__ Z, int64_t z_sr, int64_t z_sc,
    const uint32_t* __restrict__ esc, int n_row_blocks, int n_tiles,
    const uint32_t* __restrict__ gate) {
    using T = RepTile<R, C, W, KP>;
    __shared__ float lds[T::LDS_FLOATS];
    AFMM_GATE(gate);
    const int t = xcd_remap(blockIdx.x, n_tiles);
    const int band = t / n_row_blocks, rb = t - band * n_row_blocks;
    if (*esc)
        rep_uniform_tile<R, C, W, KP, VEC, TRANS_OUT, true, BUF, U>(
            n_r, n_c, n_k, P8, ldp, P32, p32_sr, p32_sk, Q, ldq, Z, z_sr, z_sc, rb * T::TM,
            band * T::TN, lds);
    else
        rep_uniform_tile<R, C, W, KP, VEC, TRANS_OUT, false, BUF, U>(
            n_r, n_c, n_k, P8, ldp, P32, p32_sr, p32_sk, Q, ldq, Z, z_sr, z_sc, rb * T::TM,
            band * T::TN, lds);
}

template <int R, int C, int W, int U, int KP>
inline hipError_t launch_rep(const StrictArgs& a, hipStream_t s) {
    using T = RepTile<R, C, W, KP>;
    const int n_row_blocks = (a.n_r + T::TM - 1) / T::TM;
    const int n_bands = (a.n_c + T::TN - 1) / T::TN;
    const int n_tiles = n_row_blocks * n_bands;
    const bool trans = a.trans_out;
    const bool vec = (a.ldq % 4 == 0) && (a.n_c % 4 == 0 || a.q_padded) &&
                     (reinterpret_cast<uintptr_t>(a.Q) % 16 == 0);
    // buffer-resource loads: byte offsets of the whole base matrix fit in 31 bits
    const bool buf = vec && (int64_t)a.n_k * a.ldq * 4 < ((int64_t)1 << 31);
    dim3 grid(n_tiles), block(W * kWave);
#define AFMM_LAUNCH(VEC, TR, BUF)                                                              \
    hipLaunchKernelGGL((rep_uniform_kernel<R, C, W, U, KP, VEC, TR, BUF>), grid, block, 0, s, a.n_r, \
                       a.n_c, a.n_k, a.P8, a.ldp, a.P32, a.p32_sr, a.p32_sk, a.Q, a.ldq, a.Z,    \
                       a.z_sr, a.z_sc, a.esc, n_row_blocks, n_tiles, a.gate)
    if (trans) {
        if (!vec) return hipErrorInvalidValue;  // case A's base is always the padded transpose
        if (buf) AFMM_LAUNCH(true, true, true);
        else AFMM_LAUNCH(true, true, false);
    } else if (buf) {
        AFMM_LAUNCH(true, false, true);
    } else if (vec) {
        AFMM_LAUNCH(true, false, false);
    } else {
        AFMM_LAUNCH(false, false, false);
    }
#undef AFMM_LAUNCH
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Direct-load variant (no LDS panel; waves meet every kSyncK rows of k).
constexpr int kSyncK = 64;

template <int R, int C, int W, bool TRANS_OUT>
__global__ __launch_bounds__(W * kWave) void rep_direct_kernel(
    int n_r, int n_c, int n_k, const uint8_t* __restrict__ P8, int64_t ldp,
    const int32_t* __restrict__ P32, int64_t p32_sr, int64_t p32_sk,
    const float* __restrict__ Q, int64_t ldq, float* __restrict__ Z, int64_t z_sr, int64_t z_sc,
    const uint32_t* __restrict__ esc, int n_row_blocks, int n_tiles,
    const uint32_t* __restrict__ gate) {
    constexpr int TM = W * R, TN = kWave * C;
    AFMM_GATE(gate);
    const int t = xcd_remap(blockIdx.x, n_tiles);
    const int band = t / n_row_blocks, rb = t - band * n_row_blocks;
    if (*esc)
        rep_direct_tile<R, C, W, kSyncK, TRANS_OUT, true>(n_r, n_c, n_k, P8, ldp, P32, p32_sr,
                                                          p32_sk, Q, ldq, Z, z_sr, z_sc, rb * TM,
                                                          band * TN);
    else
        rep_direct_tile<R, C, W, kSyncK, TRANS_OUT, false>(n_r, n_c, n_k, P8, ldp, P32, p32_sr,
                                                           p32_sk, Q, ldq, Z, z_sr, z_sc, rb * TM,
                                                           band * TN);
}

template <int R, int C, int W>
inline hipError_t launch_direct(const StrictArgs& a, hipStream_t s) {
    constexpr int TM = W * R, TN = kWave * C;
    static_assert(TM <= kRowPad, "row padding must cover a tile");
    const int n_row_blocks = (a.n_r + TM - 1) / TM;
    const int n_tiles = n_row_blocks * ((a.n_c + TN - 1) / TN);
    const bool vec = (a.ldq % 4 == 0) && (a.n_c % 4 == 0 || a.q_padded) &&
                     (reinterpret_cast<uintptr_t>(a.Q) % 16 == 0);
    if (!vec) return hipErrorInvalidValue;
    dim3 grid(n_tiles), block(W * kWave);
    if (a.trans_out)
        hipLaunchKernelGGL((rep_direct_kernel<R, C, W, true>), grid, block, 0, s, a.n_r, a.n_c,
                           a.n_k, a.P8, a.ldp, a.P32, a.p32_sr, a.p32_sk, a.Q, a.ldq, a.Z, a.z_sr,
                           a.z_sc, a.esc, n_row_blocks, n_tiles, a.gate);
    else
        hipLaunchKernelGGL((rep_direct_kernel<R, C, W, false>), grid, block, 0, s, a.n_r, a.n_c,
                           a.n_k, a.P8, a.ldp, a.P32, a.p32_sr, a.p32_sk, a.Q, a.ldq, a.Z, a.z_sr,
                           a.z_sc, a.esc, n_row_blocks, n_tiles, a.gate);
    return hipGetLastError();
}

}  // namespace afmm

