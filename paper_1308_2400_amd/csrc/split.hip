// Split-precision form of the AFMM product on the matrix cores (gfx950 MFMA).
//
// The real factor x is written as three bfloat16 terms, each the
// round-to-nearest-even bfloat16 of what the previous ones leave:
//     hi = bf16(x), mid = bf16(x - hi), lo = bf16(x - hi - mid)
// (both differences are exact in binary32, so hi + mid + lo == x for
// 2^-100 <= |x| < 2^127).  The integer factor (0..256) is exact in bfloat16.
// Z = sum over the three terms of (term . integer factor), contracted with
// v_mfma_f32_32x32x16_bf16 into binary32 accumulators.  The hi products go to
// one accumulator set and the mid/lo products to a second one; Z = hi + rest
// at the end.  The hi products carry at most 16 significant bits, so their
// running sum is nearly exact, and the rounding of the small mid/lo sum is
// 2^-8 times smaller than it would be in a shared accumulator.
//
// Operand layout: both operands K-contiguous, "A" rows = rows of Z (m),
// "B" rows = columns of Z (n), zero padded to the tile sizes so the GEMM has
// no bounds checks inside the K loop.
#include "common.hpp"

namespace afmm {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x16 __attribute__((ext_vector_type(16)));

constexpr int kGM = 128;   // tile rows (m)
constexpr int kGN = 128;   // tile cols (n)
constexpr int kGK = 32;    // K per LDS stage
constexpr int kLdsRow = kGK + 8;  // bf16 per LDS row (80 B: spreads rows over banks)

int split_rows_pad(int n) { return (int)round_up(n, kGM); }

// ---------------------------------------------------------------------------
// Conversions (binary32 -> bfloat16, round to nearest even).
__device__ __forceinline__ uint16_t bf16_bits_rne(float x) {
    uint32_t b = __float_as_uint(x);
    if ((b & 0x7F800000u) == 0x7F800000u && (b & 0x007FFFFFu)) return (uint16_t)((b >> 16) | 0x40u);
    b += 0x7FFFu + ((b >> 16) & 1u);
    return (uint16_t)(b >> 16);
}

__device__ __forceinline__ float bf16_bits_to_f32(uint16_t h) {
    return __uint_as_float((uint32_t)h << 16);
}

// out planes [rows_pad x ld] (bf16 bits).  Tile 64 x 64 through LDS, block (64, 4).
// TRANS: out[c][r] = f(in[r][c]); else out[r][c] = f(in[r][c]).
template <bool TRANS>
__global__ __launch_bounds__(256) void split_real_kernel(const float* __restrict__ in, int n,
                                                        uint16_t* __restrict__ hi,
                                                        uint16_t* __restrict__ mid,
                                                        uint16_t* __restrict__ lo, int64_t ld) {
    __shared__ float tile[64][65];
    const int o0 = blockIdx.x * 64;  // output row block
    const int c0 = blockIdx.y * 64;  // output column (K) block
    const int tx = threadIdx.x, ty = threadIdx.y;
    for (int t = ty; t < 64; t += 4) {
        // TRANS: read in[c0 + t][o0 + tx] (coalesced), keep at tile[tx][t]
        const int r = TRANS ? c0 + t : o0 + t;
        const int c = TRANS ? o0 + tx : c0 + tx;
        const float v = (r < n && c < n) ? in[(int64_t)r * n + c] : 0.0f;
        if (TRANS) tile[tx][t] = v; else tile[t][tx] = v;
    }
    __syncthreads();
    for (int t = ty; t < 64; t += 4) {
        const float x = tile[t][tx];
        const uint16_t h = bf16_bits_rne(x);
        const float r1 = x - bf16_bits_to_f32(h);
        const uint16_t m = bf16_bits_rne(r1);
        const float r2 = r1 - bf16_bits_to_f32(m);
        const int64_t o = (int64_t)(o0 + t) * ld + c0 + tx;
        hi[o] = h;
        mid[o] = m;
        lo[o] = bf16_bits_rne(r2);
    }
}

template <bool TRANS>
__global__ __launch_bounds__(256) void int_bf16_kernel(const int32_t* __restrict__ in, int n,
                                                      uint16_t* __restrict__ out, int64_t ld) {
    __shared__ int32_t tile[64][65];
    const int o0 = blockIdx.x * 64, c0 = blockIdx.y * 64;
    const int tx = threadIdx.x, ty = threadIdx.y;
    for (int t = ty; t < 64; t += 4) {
        const int r = TRANS ? c0 + t : o0 + t;
        const int c = TRANS ? o0 + tx : c0 + tx;
        const int32_t v = (r < n && c < n) ? in[(int64_t)r * n + c] : 0;
        if (TRANS) tile[tx][t] = v; else tile[t][tx] = v;
    }
    __syncthreads();
    for (int t = ty; t < 64; t += 4) {
        const int32_t v = tile[t][tx];
        // a count <= 0 adds nothing; 1..256 are exact in bfloat16
        out[(int64_t)(o0 + t) * ld + c0 + tx] = v <= 0 ? (uint16_t)0 : bf16_bits_rne((float)v);
    }
}

hipError_t launch_split_real(const float* R, int n, bool transpose, uint16_t* hi, uint16_t* mid,
                             uint16_t* lo, int64_t ld, int rows_pad, hipStream_t s) {
    dim3 grid(rows_pad / 64, (unsigned)(ld / 64));
    if (transpose)
        hipLaunchKernelGGL(split_real_kernel<true>, grid, dim3(64, 4), 0, s, R, n, hi, mid, lo, ld);
    else
        hipLaunchKernelGGL(split_real_kernel<false>, grid, dim3(64, 4), 0, s, R, n, hi, mid, lo, ld);
    return hipGetLastError();
}

hipError_t launch_int_to_bf16(const int32_t* I, int n, bool transpose, uint16_t* out, int64_t ld,
                              int rows_pad, hipStream_t s) {
    dim3 grid(rows_pad / 64, (unsigned)(ld / 64));
    if (transpose)
        hipLaunchKernelGGL(int_bf16_kernel<true>, grid, dim3(64, 4), 0, s, I, n, out, ld);
    else
        hipLaunchKernelGGL(int_bf16_kernel<false>, grid, dim3(64, 4), 0, s, I, n, out, ld);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// GEMM: Z[m][c] = sum_k sum_s A_s[m][k] * B_s[c][k].  TRIPLE_A: three A
// planes and one B plane (case A: the real pre-factor is split); otherwise
// one A plane and three B planes (case B).  256 threads = 2 x 2 waves, each
// wave a 64 x 64 block of Z = 2 x 2 MFMA 32 x 32 blocks.
//
// MFMA 32x32x16 operand layout: lane l supplies row (l % 32) of A (column
// (l % 32) of B) and the eight K values 8*(l / 32) .. +7 of the 16; result
// register v of lane l holds row 8*(v / 4) + 4*(l / 32) + v % 4, column l % 32.
template <bool TRIPLE_A>
__global__ __launch_bounds__(256) void gemm_bf16x3_kernel(
    int n, const uint16_t* __restrict__ A0, const uint16_t* __restrict__ A1,
    const uint16_t* __restrict__ A2, const uint16_t* __restrict__ B0,
    const uint16_t* __restrict__ B1, const uint16_t* __restrict__ B2, int64_t ld,
    float* __restrict__ Z, int tiles_m, int n_tiles) {
    constexpr int NA = TRIPLE_A ? 3 : 1, NB = TRIPLE_A ? 1 : 3;
    constexpr int PLANE = kGM * kLdsRow;              // bf16 per plane tile
    constexpr int STAGE = (NA + NB) * PLANE;
    __shared__ __attribute__((aligned(16))) uint16_t lds[2 * STAGE];

    const int t = xcd_remap(blockIdx.x, n_tiles);
    const int tn = t / tiles_m, tm = t - tn * tiles_m;
    const int m0 = tm * kGM, c0 = tn * kGN;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int wm = (wave & 1) * 64, wc = (wave >> 1) * 64;

    const uint16_t* ap[3] = {A0, A1, A2};
    const uint16_t* bp[3] = {B0, B1, B2};

    // Global -> LDS staging: each plane tile is 128 rows x 32 K = 512 chunks of
    // 8 bf16; thread tid moves chunks tid and tid + 256 of every plane.
    uint4 stg[(NA + NB) * 2];
    auto load_stage = [&](int k0) {
#pragma unroll
        for (int p = 0; p < NA + NB; ++p)
#pragma unroll
            for (int h = 0; h < 2; ++h) {
                const int ch = tid + h * 256, row = ch >> 2, kc = (ch & 3) * 8;
                const uint16_t* base = p < NA ? ap[p] + (int64_t)(m0 + row) * ld
                                              : bp[p - NA] + (int64_t)(c0 + row) * ld;
                stg[p * 2 + h] = *reinterpret_cast<const uint4*>(base + k0 + kc);
            }
    };
    auto store_stage = [&](uint16_t* dst) {
#pragma unroll
        for (int p = 0; p < NA + NB; ++p)
#pragma unroll
            for (int h = 0; h < 2; ++h) {
                const int ch = tid + h * 256, row = ch >> 2, kc = (ch & 3) * 8;
                *reinterpret_cast<uint4*>(dst + p * PLANE + row * kLdsRow + kc) = stg[p * 2 + h];
            }
    };

    f32x16 acc_hi[2][2], acc_lo[2][2];
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j)
#pragma unroll
            for (int v = 0; v < 16; ++v) {
                acc_hi[i][j][v] = 0.0f;
                acc_lo[i][j][v] = 0.0f;
            }

    const int n_k = (int)(ld / kGK);
    load_stage(0);
    store_stage(lds);
    __syncthreads();
    const int fr = lane & 31, fk = (lane >> 5) * 8;
    for (int ks = 0; ks < n_k; ++ks) {
        const uint16_t* cur = lds + (ks & 1) * STAGE;
        const bool more = ks + 1 < n_k;
        if (more) load_stage((ks + 1) * kGK);
#pragma unroll
        for (int kk = 0; kk < kGK; kk += 16) {
            bf16x8 a[NA][2], b[NB][2];
#pragma unroll
            for (int p = 0; p < NA; ++p)
#pragma unroll
                for (int i = 0; i < 2; ++i)
                    a[p][i] = *reinterpret_cast<const bf16x8*>(
                        cur + p * PLANE + (wm + i * 32 + fr) * kLdsRow + kk + fk);
#pragma unroll
            for (int p = 0; p < NB; ++p)
#pragma unroll
                for (int j = 0; j < 2; ++j)
                    b[p][j] = *reinterpret_cast<const bf16x8*>(
                        cur + (NA + p) * PLANE + (wc + j * 32 + fr) * kLdsRow + kk + fk);
#pragma unroll
            for (int i = 0; i < 2; ++i)
#pragma unroll
                for (int j = 0; j < 2; ++j) {
                    // term 0 (hi) alone; terms 2 (lo) then 1 (mid) into the second set
                    acc_hi[i][j] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(
                        a[0][i], b[0][j], acc_hi[i][j], 0, 0, 0);
                    acc_lo[i][j] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(
                        a[TRIPLE_A ? 2 : 0][i], b[TRIPLE_A ? 0 : 2][j], acc_lo[i][j], 0, 0, 0);
                    acc_lo[i][j] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(
                        a[TRIPLE_A ? 1 : 0][i], b[TRIPLE_A ? 0 : 1][j], acc_lo[i][j], 0, 0, 0);
                }
        }
        if (more) store_stage(lds + ((ks + 1) & 1) * STAGE);
        __syncthreads();
    }

#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j)
#pragma unroll
            for (int v = 0; v < 16; ++v) {
                const int row = m0 + wm + i * 32 + 8 * (v / 4) + 4 * (lane >> 5) + (v & 3);
                const int col = c0 + wc + j * 32 + (lane & 31);
                if (row < n && col < n) Z[(int64_t)row * n + col] = acc_hi[i][j][v] + acc_lo[i][j][v];
            }
}

hipError_t launch_gemm_bf16x3(int n, const uint16_t* A0, const uint16_t* A1, const uint16_t* A2,
                              const uint16_t* B0, const uint16_t* B1, const uint16_t* B2,
                              int64_t ld, float* Z, hipStream_t s) {
    const int tiles_m = (n + kGM - 1) / kGM, tiles_n = (n + kGN - 1) / kGN;
    const int n_tiles = tiles_m * tiles_n;
    const bool triple_a = A0 != A1;
    if (triple_a)
        hipLaunchKernelGGL(gemm_bf16x3_kernel<true>, dim3(n_tiles), dim3(256), 0, s, n, A0, A1, A2,
                           B0, B1, B2, ld, Z, tiles_m, n_tiles);
    else
        hipLaunchKernelGGL(gemm_bf16x3_kernel<false>, dim3(n_tiles), dim3(256), 0, s, n, A0, A1,
                           A2, B0, B1, B2, ld, Z, tiles_m, n_tiles);
    return hipGetLastError();
}

}  // namespace afmm
