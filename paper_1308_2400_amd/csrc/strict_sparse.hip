// Strict AFMM kernel, sparse-k form (Section 2, bit-exact binary32 repeated
// addition): eight waves per SIMD, base panels loaded straight into LDS, and
// only the k with a non-zero count visited.  Instantiations and launcher.
#include "sparse_body.hpp"

namespace afmm {

template <int R, int C, int W, int U, int KP, bool TRANS_OUT>
__global__ __launch_bounds__(W * kWave) __attribute__((amdgpu_waves_per_eu(8, 8))) void
rep_sparse_kernel(int n_r, int n_c, int n_k, const uint8_t* __restrict__ P8, int64_t ldp,
                  const int32_t* __restrict__ P32, int64_t p32_sr, int64_t p32_sk,
                  const float* __restrict__ Q, int64_t ldq, float* __restrict__ Z, int64_t z_sr,
                  int64_t z_sc, const uint32_t* __restrict__ esc, int n_row_blocks,
                  int n_tiles, const uint32_t* __restrict__ gate) {
    using T = SparseTile<R, C, W, KP>;
    __shared__ __attribute__((aligned(16))) float lds[T::LDS_FLOATS];
    AFMM_GATE(gate);
    const int t = xcd_remap(blockIdx.x, n_tiles);
    const int band = t / n_row_blocks, rb = t - band * n_row_blocks;
    if (*esc)
        rep_sparse_tile<R, C, W, KP, TRANS_OUT, true, U>(n_r, n_c, n_k, P8, ldp, P32, p32_sr,
                                                         p32_sk, Q, ldq, Z, z_sr, z_sc,
                                                         rb * T::TM, band * T::TN, lds);
    else
        rep_sparse_tile<R, C, W, KP, TRANS_OUT, false, U>(n_r, n_c, n_k, P8, ldp, P32, p32_sr,
                                                          p32_sk, Q, ldq, Z, z_sr, z_sc,
                                                          rb * T::TM, band * T::TN, lds);
}

template <int R, int C, int W, int U, int KP>
hipError_t launch_sparse(const StrictArgs& a, hipStream_t s) {
    using T = SparseTile<R, C, W, KP>;
    if (!rep_sparse_usable(a)) return hipErrorInvalidValue;
    const int n_row_blocks = (a.n_r + T::TM - 1) / T::TM;
    const int n_tiles = n_row_blocks * ((a.n_c + T::TN - 1) / T::TN);
    dim3 grid(n_tiles), block(W * kWave);
    if (a.trans_out)
        hipLaunchKernelGGL((rep_sparse_kernel<R, C, W, U, KP, true>), grid, block, 0, s, a.n_r,
                           a.n_c, a.n_k, a.P8, a.ldp, a.P32, a.p32_sr, a.p32_sk, a.Q, a.ldq, a.Z,
                           a.z_sr, a.z_sc, a.esc, n_row_blocks, n_tiles, a.gate);
    else
        hipLaunchKernelGGL((rep_sparse_kernel<R, C, W, U, KP, false>), grid, block, 0, s, a.n_r,
                           a.n_c, a.n_k, a.P8, a.ldp, a.P32, a.p32_sr, a.p32_sk, a.Q, a.ldq, a.Z,
                           a.z_sr, a.z_sc, a.esc, n_row_blocks, n_tiles, a.gate);
    return hipGetLastError();
}

// (R, C, W, U, KP); LDS per block 2*KP*64*C floats; 32 waves per compute unit
#define AFMM_SPARSE_CONFIGS(X) \
    X(2, 16, 16, 1, 8)         \
    X(2, 16, 16, 2, 8)         \
    X(4, 8, 16, 1, 16)         \
    X(4, 8, 16, 2, 16)         \
    X(2, 8, 16, 2, 16)         \
    X(2, 16, 8, 1, 4)          \
    X(2, 16, 8, 2, 4)          \
    X(1, 16, 16, 1, 8)

bool rep_sparse_usable(const StrictArgs& a) {
    // float4-readable base rows, byte offsets of the whole base matrix in 31 bits
    return (a.ldq % 4 == 0) && (a.n_c % 4 == 0 || a.q_padded) &&
           (reinterpret_cast<uintptr_t>(a.Q) % 16 == 0) &&
           (int64_t)a.n_k * a.ldq * 4 < ((int64_t)1 << 31);
}

bool rep_sparse_supported(int R, int C, int W, int U, int KP) {
#define AFMM_CASE(r, c, w, u, kp) \
    if (R == r && C == c && W == w && U == u && KP == kp) return true;
    AFMM_SPARSE_CONFIGS(AFMM_CASE)
#undef AFMM_CASE
    return false;
}

hipError_t launch_rep_sparse(const StrictArgs& a, int R, int C, int W, int U, int KP,
                             hipStream_t s) {
#define AFMM_CASE(r, c, w, u, kp) \
    if (R == r && C == c && W == w && U == u && KP == kp) return launch_sparse<r, c, w, u, kp>(a, s);
    AFMM_SPARSE_CONFIGS(AFMM_CASE)
#undef AFMM_CASE
    return hipErrorInvalidValue;
}

}  // namespace afmm
