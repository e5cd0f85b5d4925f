// Strict AFMM kernels: bit-exact binary32 repeated addition (Section 2).
#include "strict_body.hpp"

namespace afmm {



template <int R, int C, int W, int U, int KP, bool VEC, bool TRANS_OUT, bool BUF>
__global__ __launch_bounds__(W * kWave) void rep_uniform_kernel(
    int n_r, int n_c, int n_k, const uint8_t* __restrict__ P8, int64_t ldp,
    const int32_t* __restrict__ P32, int64_t p32_sr, int64_t p32_sk,
    const float* __restrict__ Q, int64_t ldq, float* __restrict__ Z, int64_t z_sr, int64_t z_sc,
    const uint32_t* __restrict__ esc, int n_row_blocks, int n_tiles) {
    using T = RepTile<R, C, W, KP>;
    __shared__ float lds[T::LDS_FLOATS];
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
static hipError_t launch_rep(const StrictArgs& a, hipStream_t s) {
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
                       a.z_sr, a.z_sc, a.esc, n_row_blocks, n_tiles)
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

// Compiled (R, C, W, U, KP) combinations of the LDS-panel kernel (U: repetition
// loop unroll, KP: base rows per LDS panel).
#define AFMM_REP_CONFIGS(X) \
    X(8, 8, 8, 1, 16)       \
    X(8, 8, 8, 2, 16)       \
    X(4, 8, 8, 1, 16)       \
    X(8, 4, 8, 1, 16)       \
    X(8, 4, 8, 2, 16)       \
    X(4, 4, 8, 1, 16)       \
    X(8, 8, 4, 1, 16)       \
    X(8, 4, 4, 1, 16)       \
    X(8, 4, 4, 2, 16)       \
    X(4, 4, 4, 1, 16)       \
    X(4, 2, 4, 1, 16)       \
    X(4, 2, 4, 2, 16)       \
    X(2, 1, 4, 1, 16)       \
    X(4, 16, 8, 1, 8)       \
    X(4, 16, 8, 2, 8)       \
    X(6, 16, 4, 1, 8)       \
    X(8, 8, 8, 2, 8)        \
    X(4, 16, 16, 1, 16)

bool rep_uniform_supported(int R, int C, int W, int U, int KP) {
#define AFMM_CASE(r, c, w, u, kp) \
    if (R == r && C == c && W == w && U == u && KP == kp) return true;
    AFMM_REP_CONFIGS(AFMM_CASE)
#undef AFMM_CASE
    return false;
}

hipError_t launch_rep_uniform(const StrictArgs& a, int R, int C, int W, int U, int KP,
                              hipStream_t s) {
#define AFMM_CASE(r, c, w, u, kp) \
    if (R == r && C == c && W == w && U == u && KP == kp) return launch_rep<r, c, w, u, kp>(a, s);
    AFMM_REP_CONFIGS(AFMM_CASE)
#undef AFMM_CASE
    return hipErrorInvalidValue;
}

// ---------------------------------------------------------------------------
// Direct-load variant (no LDS panel; waves meet every kSyncK rows of k).
constexpr int kSyncK = 64;

template <int R, int C, int W, bool TRANS_OUT>
__global__ __launch_bounds__(W * kWave) void rep_direct_kernel(
    int n_r, int n_c, int n_k, const uint8_t* __restrict__ P8, int64_t ldp,
    const int32_t* __restrict__ P32, int64_t p32_sr, int64_t p32_sk,
    const float* __restrict__ Q, int64_t ldq, float* __restrict__ Z, int64_t z_sr, int64_t z_sc,
    const uint32_t* __restrict__ esc, int n_row_blocks, int n_tiles) {
    constexpr int TM = W * R, TN = kWave * C;
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
static hipError_t launch_direct(const StrictArgs& a, hipStream_t s) {
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
                           a.z_sc, a.esc, n_row_blocks, n_tiles);
    else
        hipLaunchKernelGGL((rep_direct_kernel<R, C, W, false>), grid, block, 0, s, a.n_r, a.n_c,
                           a.n_k, a.P8, a.ldp, a.P32, a.p32_sr, a.p32_sk, a.Q, a.ldq, a.Z, a.z_sr,
                           a.z_sc, a.esc, n_row_blocks, n_tiles);
    return hipGetLastError();
}

#define AFMM_DIRECT_CONFIGS(X) \
    X(8, 8, 4)                 \
    X(8, 8, 8)                 \
    X(6, 8, 4)                 \
    X(4, 8, 8)                 \
    X(8, 4, 4)                 \
    X(16, 4, 4)                \
    X(4, 4, 4)

bool rep_direct_supported(int R, int C, int W) {
#define AFMM_CASE(r, c, w) \
    if (R == r && C == c && W == w) return true;
    AFMM_DIRECT_CONFIGS(AFMM_CASE)
#undef AFMM_CASE
    return false;
}

bool rep_direct_usable(const StrictArgs& a) {
    return (a.ldq % 4 == 0) && (a.n_c % 4 == 0 || a.q_padded) &&
           (reinterpret_cast<uintptr_t>(a.Q) % 16 == 0);
}

hipError_t launch_rep_direct(const StrictArgs& a, int R, int C, int W, hipStream_t s) {
#define AFMM_CASE(r, c, w) \
    if (R == r && C == c && W == w) return launch_direct<r, c, w>(a, s);
    AFMM_DIRECT_CONFIGS(AFMM_CASE)
#undef AFMM_CASE
    return hipErrorInvalidValue;
}

bool base_uniform_supported(int, int, int) { return false; }

hipError_t launch_base_uniform(const BaseUniformArgs&, int, int, int, hipStream_t) {
    return hipErrorInvalidValue;
}

}  // namespace afmm
