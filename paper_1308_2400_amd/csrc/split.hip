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

// out planes [rows_pad x ld] (bf16 bits) from in: rows x cols with leading
// dimension ldi (zero outside).  Tile 64 x 64 through LDS, block (64, 4).
// TRANS: out[c][r] = f(in[r][c]); else out[r][c] = f(in[r][c]).
template <bool TRANS>
__global__ __launch_bounds__(256) void split_real_kernel(const float* __restrict__ in, int rows,
                                                        int cols, int64_t ldi,
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
        const float v = (r < rows && c < cols) ? in[(int64_t)r * ldi + c] : 0.0f;
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
__global__ __launch_bounds__(256) void int_bf16_kernel(const int32_t* __restrict__ in, int rows,
                                                      int cols, int64_t ldi,
                                                      uint16_t* __restrict__ out, int64_t ld) {
    __shared__ int32_t tile[64][65];
    const int o0 = blockIdx.x * 64, c0 = blockIdx.y * 64;
    const int tx = threadIdx.x, ty = threadIdx.y;
    for (int t = ty; t < 64; t += 4) {
        const int r = TRANS ? c0 + t : o0 + t;
        const int c = TRANS ? o0 + tx : c0 + tx;
        const int32_t v = (r < rows && c < cols) ? in[(int64_t)r * ldi + c] : 0;
        if (TRANS) tile[tx][t] = v; else tile[t][tx] = v;
    }
    __syncthreads();
    for (int t = ty; t < 64; t += 4) {
        const int32_t v = tile[t][tx];
        // a count <= 0 adds nothing; 1..256 are exact in bfloat16
        out[(int64_t)(o0 + t) * ld + c0 + tx] = v <= 0 ? (uint16_t)0 : bf16_bits_rne((float)v);
    }
}

hipError_t launch_split_real(const float* R, int rows, int cols, int64_t ldr, bool transpose,
                             uint16_t* hi, uint16_t* mid, uint16_t* lo, int64_t ld, int rows_pad,
                             hipStream_t s) {
    dim3 grid(rows_pad / 64, (unsigned)(ld / 64));
    if (transpose)
        hipLaunchKernelGGL(split_real_kernel<true>, grid, dim3(64, 4), 0, s, R, rows, cols, ldr, hi,
                           mid, lo, ld);
    else
        hipLaunchKernelGGL(split_real_kernel<false>, grid, dim3(64, 4), 0, s, R, rows, cols, ldr,
                           hi, mid, lo, ld);
    return hipGetLastError();
}

hipError_t launch_int_to_bf16(const int32_t* I, int rows, int cols, int64_t ldi, bool transpose,
                              uint16_t* out, int64_t ld, int rows_pad, hipStream_t s) {
    dim3 grid(rows_pad / 64, (unsigned)(ld / 64));
    if (transpose)
        hipLaunchKernelGGL(int_bf16_kernel<true>, grid, dim3(64, 4), 0, s, I, rows, cols, ldi, out,
                           ld);
    else
        hipLaunchKernelGGL(int_bf16_kernel<false>, grid, dim3(64, 4), 0, s, I, rows, cols, ldi, out,
                           ld);
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
constexpr int kPlane = kGM * kLdsRow;  // bf16 per plane tile in LDS

// Tile order: each XCD gets a contiguous run of tiles (xcd_remap), and inside
// it tiles go column-band-major in groups of kGroupM row tiles so that blocks
// running together share both operand panels in that XCD's L2.
constexpr int kGroupM = 8;

__device__ __forceinline__ void gemm_tile_coords(int t, int tiles_m, int tiles_n, int& tm, int& tn) {
    const int per_group = kGroupM * tiles_n;
    const int g = t / per_group, first_m = g * kGroupM;
    const int gm = min(tiles_m - first_m, kGroupM);
    const int r = t - g * per_group;
    tm = first_m + r % gm;
    tn = r / gm;
}

template <bool TRIPLE_A>
__global__ __launch_bounds__(256, 2) void gemm_bf16x3_kernel(
    int M, int N, const uint16_t* __restrict__ A0, const uint16_t* __restrict__ A1,
    const uint16_t* __restrict__ A2, const uint16_t* __restrict__ B0,
    const uint16_t* __restrict__ B1, const uint16_t* __restrict__ B2, int64_t ld,
    float* __restrict__ Z, int64_t ldz, int tiles_m, int tiles_n) {
    // LDS stage: planes 0..2 = the split side (hi, mid, lo), plane 3 = the other side
    constexpr int STAGE = 4 * kPlane;
    __shared__ __attribute__((aligned(16))) uint16_t lds[2 * STAGE];

    int tm, tn;
    gemm_tile_coords(xcd_remap(blockIdx.x, tiles_m * tiles_n), tiles_m, tiles_n, tm, tn);
    const int m0 = tm * kGM, c0 = tn * kGN;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int wm = (wave & 1) * 64, wc = (wave >> 1) * 64;

    // split side rows start at s0 (m0 for TRIPLE_A, c0 otherwise); the other side at o0
    const int s0 = TRIPLE_A ? m0 : c0, o0 = TRIPLE_A ? c0 : m0;
    const uint16_t* S0 = TRIPLE_A ? A0 : B0;
    const uint16_t* S1 = TRIPLE_A ? A1 : B1;
    const uint16_t* S2 = TRIPLE_A ? A2 : B2;
    const uint16_t* O = TRIPLE_A ? B0 : A0;

    // Global -> LDS staging: a plane tile is 128 rows x 32 K = 512 chunks of 8 bf16;
    // thread tid moves chunks tid and tid + 256 of each of the four planes.
    const int row_a = tid >> 2, row_b = row_a + 64, kc = (tid & 3) * 8;
    const int64_t sa = (int64_t)(s0 + row_a) * ld + kc, sb = (int64_t)(s0 + row_b) * ld + kc;
    const int64_t oa = (int64_t)(o0 + row_a) * ld + kc, ob = (int64_t)(o0 + row_b) * ld + kc;
    const int la = row_a * kLdsRow + kc, lb = row_b * kLdsRow + kc;
    uint4 g0a, g0b, g1a, g1b, g2a, g2b, goa, gob;
#define AFMM_GLOAD(k0)                                                     \
    g0a = *reinterpret_cast<const uint4*>(S0 + sa + (k0));                 \
    g0b = *reinterpret_cast<const uint4*>(S0 + sb + (k0));                 \
    g1a = *reinterpret_cast<const uint4*>(S1 + sa + (k0));                 \
    g1b = *reinterpret_cast<const uint4*>(S1 + sb + (k0));                 \
    g2a = *reinterpret_cast<const uint4*>(S2 + sa + (k0));                 \
    g2b = *reinterpret_cast<const uint4*>(S2 + sb + (k0));                 \
    goa = *reinterpret_cast<const uint4*>(O + oa + (k0));                  \
    gob = *reinterpret_cast<const uint4*>(O + ob + (k0));
#define AFMM_LSTORE(dst)                                                   \
    *reinterpret_cast<uint4*>((dst) + 0 * kPlane + la) = g0a;              \
    *reinterpret_cast<uint4*>((dst) + 0 * kPlane + lb) = g0b;              \
    *reinterpret_cast<uint4*>((dst) + 1 * kPlane + la) = g1a;              \
    *reinterpret_cast<uint4*>((dst) + 1 * kPlane + lb) = g1b;              \
    *reinterpret_cast<uint4*>((dst) + 2 * kPlane + la) = g2a;              \
    *reinterpret_cast<uint4*>((dst) + 2 * kPlane + lb) = g2b;              \
    *reinterpret_cast<uint4*>((dst) + 3 * kPlane + la) = goa;              \
    *reinterpret_cast<uint4*>((dst) + 3 * kPlane + lb) = gob;

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
    AFMM_GLOAD(0)
    AFMM_LSTORE(lds)
    __syncthreads();
    const int fr = lane & 31, fk = (lane >> 5) * 8;
    // fragment rows inside the stage: A rows (wm + 32 i + fr), B rows (wc + 32 j + fr)
    const int ra0 = (wm + fr) * kLdsRow + fk, ra1 = ra0 + 32 * kLdsRow;
    const int rb0 = (wc + fr) * kLdsRow + fk, rb1 = rb0 + 32 * kLdsRow;
    // plane of the A operand for term s, and of the B operand
    constexpr int PA0 = TRIPLE_A ? 0 : 3, PA1 = TRIPLE_A ? 1 : 3, PA2 = TRIPLE_A ? 2 : 3;
    constexpr int PB0 = TRIPLE_A ? 3 : 0, PB1 = TRIPLE_A ? 3 : 1, PB2 = TRIPLE_A ? 3 : 2;
    for (int ks = 0; ks < n_k; ++ks) {
        const uint16_t* cur = lds + (ks & 1) * STAGE;
        const bool more = ks + 1 < n_k;
        if (more) {
            AFMM_GLOAD((ks + 1) * kGK)
        }
#pragma unroll
        for (int kk = 0; kk < kGK; kk += 16) {
#define AFMM_FRAG(plane, off) (*reinterpret_cast<const bf16x8*>(cur + (plane) * kPlane + (off) + kk))
            const bf16x8 a00 = AFMM_FRAG(PA0, ra0), a01 = AFMM_FRAG(PA0, ra1);
            const bf16x8 b00 = AFMM_FRAG(PB0, rb0), b01 = AFMM_FRAG(PB0, rb1);
            // term 0 (hi) into its own accumulators
            acc_hi[0][0] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a00, b00, acc_hi[0][0], 0, 0, 0);
            acc_hi[0][1] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a00, b01, acc_hi[0][1], 0, 0, 0);
            acc_hi[1][0] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a01, b00, acc_hi[1][0], 0, 0, 0);
            acc_hi[1][1] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a01, b01, acc_hi[1][1], 0, 0, 0);
            // terms 2 (lo) then 1 (mid) into the second set
            const bf16x8 a20 = AFMM_FRAG(PA2, ra0), a21 = AFMM_FRAG(PA2, ra1);
            const bf16x8 b20 = AFMM_FRAG(PB2, rb0), b21 = AFMM_FRAG(PB2, rb1);
            acc_lo[0][0] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a20, b20, acc_lo[0][0], 0, 0, 0);
            acc_lo[0][1] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a20, b21, acc_lo[0][1], 0, 0, 0);
            acc_lo[1][0] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a21, b20, acc_lo[1][0], 0, 0, 0);
            acc_lo[1][1] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a21, b21, acc_lo[1][1], 0, 0, 0);
            const bf16x8 a10 = AFMM_FRAG(PA1, ra0), a11 = AFMM_FRAG(PA1, ra1);
            const bf16x8 b10 = AFMM_FRAG(PB1, rb0), b11 = AFMM_FRAG(PB1, rb1);
            acc_lo[0][0] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a10, b10, acc_lo[0][0], 0, 0, 0);
            acc_lo[0][1] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a10, b11, acc_lo[0][1], 0, 0, 0);
            acc_lo[1][0] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a11, b10, acc_lo[1][0], 0, 0, 0);
            acc_lo[1][1] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a11, b11, acc_lo[1][1], 0, 0, 0);
#undef AFMM_FRAG
        }
        if (more) {
            uint16_t* nxt = lds + ((ks + 1) & 1) * STAGE;
            AFMM_LSTORE(nxt)
        }
        __syncthreads();
    }
#undef AFMM_GLOAD
#undef AFMM_LSTORE

#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j)
#pragma unroll
            for (int v = 0; v < 16; ++v) {
                const int row = m0 + wm + i * 32 + 8 * (v / 4) + 4 * (lane >> 5) + (v & 3);
                const int col = c0 + wc + j * 32 + (lane & 31);
                if (row < M && col < N) Z[(int64_t)row * ldz + col] = acc_hi[i][j][v] + acc_lo[i][j][v];
            }
}

hipError_t launch_gemm_bf16x3(int M, int N, const uint16_t* A0, const uint16_t* A1,
                              const uint16_t* A2, const uint16_t* B0, const uint16_t* B1,
                              const uint16_t* B2, int64_t ld, float* Z, int64_t ldz,
                              hipStream_t s) {
    // A planes: split_rows_pad(M) rows, B planes: split_rows_pad(N) rows, K pitch ld
    const int tiles_m = (M + kGM - 1) / kGM, tiles_n = (N + kGN - 1) / kGN;
    const int n_tiles = tiles_m * tiles_n;
    const bool triple_a = A0 != A1;
    if (triple_a)
        hipLaunchKernelGGL(gemm_bf16x3_kernel<true>, dim3(n_tiles), dim3(256), 0, s, M, N, A0, A1,
                           A2, B0, B1, B2, ld, Z, ldz, tiles_m, tiles_n);
    else
        hipLaunchKernelGGL(gemm_bf16x3_kernel<false>, dim3(n_tiles), dim3(256), 0, s, M, N, A0,
                           A1, A2, B0, B1, B2, ld, Z, ldz, tiles_m, tiles_n);
    return hipGetLastError();
}

}  // namespace afmm
