// Split-precision form of the AFMM product on the matrix cores (gfx950 MFMA).
//
// The real factor x is written as three bfloat16 terms, each the
// round-to-nearest-even bfloat16 of what the previous ones leave:
//     hi = bf16(x), mid = bf16(x - hi), lo = bf16(x - hi - mid)
// (both differences are exact in binary32, so hi + mid + lo == x for
// 2^-100 <= |x| < 2^127).  The integer factor (0..256) is exact in bfloat16.
// Z = sum over the three terms of (term . integer factor), contracted with
// v_mfma_f32_32x32x16_bf16 into binary32 accumulators.  The hi products go to
// one accumulator set and the mid/lo products (lo first) to a second; Z = hi +
// rest at the end.  The hi products carry at most 16 significant bits, so their
// running sum is nearly exact, and the rounding of the small mid/lo sum is 2^-8
// times smaller than it would be in a shared accumulator (one shared set would
// round every mid/lo addition at the scale of Z: about 10x the error at n=4096,
// growing with the square root of K).
//
// Operand layout: every plane is K-contiguous with one row per row of Z (the
// factor on the left) or per column of Z (the factor on the right), zero padded
// to the block tile so the GEMM has no bounds checks inside the K loop.
#include "split.hpp"

namespace afmm {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x16 __attribute__((ext_vector_type(16)));

constexpr int kTI = 256;  // block rows on the integer side
constexpr int kTS = 128;  // block rows on the split (three-term) side

int split_real_rows_pad(int n) { return (int)round_up(n, kTS); }
int split_int_rows_pad(int n) { return (int)round_up(n, kTI); }

// ---------------------------------------------------------------------------
// Conversions (binary32 -> bfloat16, round to nearest even).
__device__ __forceinline__ uint32_t bf16_bits_rne(float x) {
    uint32_t b = __float_as_uint(x);
    if ((b & 0x7F800000u) == 0x7F800000u && (b & 0x007FFFFFu)) return ((b >> 16) | 0x40u) & 0xFFFFu;
    b += 0x7FFFu + ((b >> 16) & 1u);
    return b >> 16;
}

__device__ __forceinline__ float bf16_bits_to_f32(uint32_t h) { return __uint_as_float(h << 16); }

// A 64 x 64 block of the input goes through LDS as tile[output row][k]; the
// write phase gives each lane eight consecutive k of one output row, so every
// plane is written in 16-byte pieces, eight lanes to a 128-byte row segment.
// TRANS: output row o, column k come from in[k][o]; else from in[o][k].
// Outputs are [rows_pad x ld] with zeros outside rows x cols.
// vec: every input row starts 16-byte aligned.  Turned round, a lane reads four
// consecutive output rows of one input row with one 16-byte load (16 lanes to a
// 256-byte row segment) and scatters them down a tile column.
template <bool TRANS, typename T>
__device__ __forceinline__ void load_block(const T* __restrict__ in, int rows, int cols, int64_t ldi,
                                           bool vec, int o0, int c0, T (*tile)[65]) {
    if (TRANS) {
        const int j4 = (threadIdx.x & 15) * 4, tt = threadIdx.x >> 4;
#pragma unroll
        for (int it = 0; it < 4; ++it) {
            const int t = tt + 16 * it, r = c0 + t, c = o0 + j4;  // input row r, columns c..c+3
            const T* src = in + (int64_t)r * ldi + c;
            T v[4];
            if (r < rows && vec && c + 4 <= cols) {
                const uint4 w = *reinterpret_cast<const uint4*>(src);
                v[0] = __builtin_bit_cast(T, w.x);
                v[1] = __builtin_bit_cast(T, w.y);
                v[2] = __builtin_bit_cast(T, w.z);
                v[3] = __builtin_bit_cast(T, w.w);
            } else {
#pragma unroll
                for (int q = 0; q < 4; ++q) v[q] = (r < rows && c + q < cols) ? src[q] : T(0);
            }
#pragma unroll
            for (int q = 0; q < 4; ++q) tile[j4 + q][t] = v[q];
        }
    } else {
        const int lx = threadIdx.x & 63, ly = threadIdx.x >> 6;
        for (int t = ly; t < 64; t += 4) {
            const int r = o0 + t, c = c0 + lx;
            tile[t][lx] = (r < rows && c < cols) ? in[(int64_t)r * ldi + c] : T(0);
        }
    }
}

template <bool TRANS>
__device__ __forceinline__ void split_real_block(const float* __restrict__ in, int rows, int cols,
                                                 int64_t ldi, uint16_t* __restrict__ hi,
                                                 uint16_t* __restrict__ mid,
                                                 uint16_t* __restrict__ lo, int64_t ld, int o0,
                                                 int c0, bool vec, float (*tile)[65]) {
    load_block<TRANS>(in, rows, cols, ldi, vec, o0, c0, tile);
    __syncthreads();
    for (int h = 0; h < 2; ++h) {
        const int c = threadIdx.x + 256 * h, o = c >> 3, kq = (c & 7) * 8;
        uint32_t ph[4], pm[4], pl[4];
#pragma unroll
        for (int e = 0; e < 8; ++e) {
            const float x = tile[o][kq + e];
            const uint32_t bh = bf16_bits_rne(x);
            const float r1 = x - bf16_bits_to_f32(bh);
            const uint32_t bm = bf16_bits_rne(r1);
            const uint32_t bl = bf16_bits_rne(r1 - bf16_bits_to_f32(bm));
            const int w = e >> 1, sh = (e & 1) * 16;
            ph[w] = (e & 1) ? ph[w] | (bh << sh) : bh;
            pm[w] = (e & 1) ? pm[w] | (bm << sh) : bm;
            pl[w] = (e & 1) ? pl[w] | (bl << sh) : bl;
        }
        const int64_t off = (int64_t)(o0 + o) * ld + c0 + kq;
        *reinterpret_cast<uint4*>(hi + off) = make_uint4(ph[0], ph[1], ph[2], ph[3]);
        *reinterpret_cast<uint4*>(mid + off) = make_uint4(pm[0], pm[1], pm[2], pm[3]);
        *reinterpret_cast<uint4*>(lo + off) = make_uint4(pl[0], pl[1], pl[2], pl[3]);
    }
}

template <bool TRANS>
__device__ __forceinline__ void int_bf16_block(const int32_t* __restrict__ in, int rows, int cols,
                                               int64_t ldi, uint16_t* __restrict__ out, int64_t ld,
                                               int o0, int c0, bool vec, int32_t (*tile)[65]) {
    load_block<TRANS>(in, rows, cols, ldi, vec, o0, c0, tile);
    __syncthreads();
    for (int h = 0; h < 2; ++h) {
        const int c = threadIdx.x + 256 * h, o = c >> 3, kq = (c & 7) * 8;
        uint32_t p[4];
#pragma unroll
        for (int e = 0; e < 8; ++e) {
            const int32_t v = tile[o][kq + e];
            // a count <= 0 adds nothing; 1..256 are exact in bfloat16
            const uint32_t b = v <= 0 ? 0u : bf16_bits_rne((float)v);
            const int w = e >> 1;
            p[w] = (e & 1) ? p[w] | (b << 16) : b;
        }
        *reinterpret_cast<uint4*>(out + (int64_t)(o0 + o) * ld + c0 + kq) =
            make_uint4(p[0], p[1], p[2], p[3]);
    }
}

// The same conversions for a factor that is not turned round (output row o,
// column k from in[o][k]): no LDS, each lane reads the eight k it writes, with
// two 16-byte loads where the row allows them (vec: every row starts 16-byte
// aligned).
__device__ __forceinline__ void load8(const uint32_t* __restrict__ in, int rows, int cols,
                                      int64_t ldi, bool vec, int o, int k, uint32_t (&v)[8]) {
    const uint32_t* src = in + (int64_t)o * ldi + k;
    if (o < rows && vec && k + 8 <= cols) {
        const uint4 a = reinterpret_cast<const uint4*>(src)[0];
        const uint4 b = reinterpret_cast<const uint4*>(src)[1];
        v[0] = a.x; v[1] = a.y; v[2] = a.z; v[3] = a.w;
        v[4] = b.x; v[5] = b.y; v[6] = b.z; v[7] = b.w;
    } else {
#pragma unroll
        for (int e = 0; e < 8; ++e) v[e] = (o < rows && k + e < cols) ? src[e] : 0u;
    }
}

__device__ __forceinline__ void split_real_direct(const float* __restrict__ in, int rows,
                                                  int cols, int64_t ldi, bool vec,
                                                  uint16_t* __restrict__ hi,
                                                  uint16_t* __restrict__ mid,
                                                  uint16_t* __restrict__ lo, int64_t ld, int o0,
                                                  int c0) {
    for (int h = 0; h < 2; ++h) {
        const int c = threadIdx.x + 256 * h, o = c >> 3, kq = (c & 7) * 8;
        uint32_t v[8];
        load8(reinterpret_cast<const uint32_t*>(in), rows, cols, ldi, vec, o0 + o, c0 + kq, v);
        uint32_t ph[4], pm[4], pl[4];
#pragma unroll
        for (int e = 0; e < 8; ++e) {
            const float x = __uint_as_float(v[e]);
            const uint32_t bh = bf16_bits_rne(x);
            const float r1 = x - bf16_bits_to_f32(bh);
            const uint32_t bm = bf16_bits_rne(r1);
            const uint32_t bl = bf16_bits_rne(r1 - bf16_bits_to_f32(bm));
            const int w = e >> 1, sh = (e & 1) * 16;
            ph[w] = (e & 1) ? ph[w] | (bh << sh) : bh;
            pm[w] = (e & 1) ? pm[w] | (bm << sh) : bm;
            pl[w] = (e & 1) ? pl[w] | (bl << sh) : bl;
        }
        const int64_t off = (int64_t)(o0 + o) * ld + c0 + kq;
        *reinterpret_cast<uint4*>(hi + off) = make_uint4(ph[0], ph[1], ph[2], ph[3]);
        *reinterpret_cast<uint4*>(mid + off) = make_uint4(pm[0], pm[1], pm[2], pm[3]);
        *reinterpret_cast<uint4*>(lo + off) = make_uint4(pl[0], pl[1], pl[2], pl[3]);
    }
}

__device__ __forceinline__ void int_bf16_direct(const int32_t* __restrict__ in, int rows, int cols,
                                                int64_t ldi, bool vec, uint16_t* __restrict__ out,
                                                int64_t ld, int o0, int c0) {
    for (int h = 0; h < 2; ++h) {
        const int c = threadIdx.x + 256 * h, o = c >> 3, kq = (c & 7) * 8;
        uint32_t v[8];
        load8(reinterpret_cast<const uint32_t*>(in), rows, cols, ldi, vec, o0 + o, c0 + kq, v);
        uint32_t p[4];
#pragma unroll
        for (int e = 0; e < 8; ++e) {
            const int32_t x = (int32_t)v[e];
            // a count <= 0 adds nothing; 1..256 are exact in bfloat16
            const uint32_t b = x <= 0 ? 0u : bf16_bits_rne((float)x);
            const int w = e >> 1;
            p[w] = (e & 1) ? p[w] | (b << 16) : b;
        }
        *reinterpret_cast<uint4*>(out + (int64_t)(o0 + o) * ld + c0 + kq) =
            make_uint4(p[0], p[1], p[2], p[3]);
    }
}

// Both conversions in one launch: blocks [0, int_blocks) fill the integer
// plane, the rest the three term planes; block b of a plane covers K columns
// 64 (b % (ld / 64)) and output rows 64 (b / (ld / 64)), so blocks running
// together write whole output rows.  The integer factor is the one turned round in case A
// (Y[k][j] -> [j][k]), the real factor in case B (Y[k][j] -> [j][k]).
template <bool CASE_A>
__global__ __launch_bounds__(256) void split_prep_kernel(SplitPrepArgs a) {
    __shared__ uint32_t tile[64][65];
    const int k_tiles = (int)(a.ld / 64);
    int b = blockIdx.x;
    if (b < a.int_blocks) {
        const int o0 = (b / k_tiles) * 64, c0 = (b % k_tiles) * 64;
        if (CASE_A)
            int_bf16_block<true>(a.I, a.i_rows, a.i_cols, a.ldi, a.ip, a.ld, o0, c0, a.i_vec,
                                 reinterpret_cast<int32_t(*)[65]>(tile));
        else
            int_bf16_direct(a.I, a.i_rows, a.i_cols, a.ldi, a.i_vec, a.ip, a.ld, o0, c0);
    } else {
        b -= a.int_blocks;
        const int o0 = (b / k_tiles) * 64, c0 = (b % k_tiles) * 64;
        if (CASE_A)
            split_real_direct(a.R, a.r_rows, a.r_cols, a.ldr, a.r_vec, a.hi, a.mid, a.lo, a.ld,
                              o0, c0);
        else
            split_real_block<true>(a.R, a.r_rows, a.r_cols, a.ldr, a.hi, a.mid, a.lo, a.ld, o0,
                                   c0, a.r_vec, reinterpret_cast<float(*)[65]>(tile));
    }
}

hipError_t launch_split_prep(bool case_a, const SplitPrepArgs& a, hipStream_t s) {
    const int64_t k_tiles = a.ld / 64;
    const int64_t blocks = (int64_t)(a.int_blocks + a.r_tiles_o * k_tiles);
    if (a.int_blocks != (int64_t)a.i_tiles_o * k_tiles || blocks > INT32_MAX)
        return hipErrorInvalidValue;
    if (case_a)
        hipLaunchKernelGGL(split_prep_kernel<true>, dim3((unsigned)blocks), dim3(256), 0, s, a);
    else
        hipLaunchKernelGGL(split_prep_kernel<false>, dim3((unsigned)blocks), dim3(256), 0, s, a);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// GEMM over one 256 x 128 block of Z: 256 rows of the integer plane (the I
// side) against 128 rows of each of the three term planes (the S side); for
// the case-B product the I side runs along the rows of Z, for case A along its
// columns.  One block of 8 waves per compute unit (two waves per SIMD, so one
// wave's MFMAs run while the other waits): wave w owns I rows 128 (w & 1) ..
// +127 and S rows 32 (w >> 1) .. +31, i.e. 4 MFMA 32 x 32 blocks, each with a
// hi and a mid/lo accumulator (128 binary32 accumulators per lane).  Per
// 16-wide K step a wave reads 4 integer and 3 term fragments for 12 MFMAs.
//
// MFMA 32x32x16 operand layout: lane l supplies row (l % 32) of A (column
// (l % 32) of B) and the eight K values 8*(l / 32) .. +7 of the 16; result
// register v of lane l holds row 8*(v / 4) + 4*(l / 32) + v % 4, column l % 32.
//
// LDS: three stages of 32 K (120 KB), each the I tile (256 rows) then the
// three S tiles (128 rows), each row 32 bf16 = four 16-byte chunks with chunk q
// of row r kept at slot q ^ swz(r).  Fragment reads (32 consecutive rows, one
// chunk) touch every bank once per 16 lanes.  Global loads go straight into
// LDS (buffer loads with an LDS destination, 1 KB = 16 rows per instruction;
// lane L fills slot L % 4 of row L / 4 of the group, so it fetches the chunk
// that belongs there), two stages ahead of the MFMAs, with one barrier per
// stage.
constexpr int kGemmWaves = 8;

// Stage geometry for GK K values per LDS stage (32: four 16-byte chunks per
// row, three stages in flight; 64: eight chunks, two stages).  A 1 KB direct
// load fills RPG rows of one plane (a row group).
template <int GK>
struct GemmStage {
    static constexpr int CH = GK / 8;                     // 16-byte chunks per row
    static constexpr int PLANE_I = kTI * GK;              // bf16 per I tile
    static constexpr int PLANE_S = kTS * GK;              // bf16 per S tile
    static constexpr int STAGE = PLANE_I + 3 * PLANE_S;   // bf16 per stage
    static constexpr int STAGES = GK == 32 ? 3 : 2;       // stages in LDS
    static constexpr int RPG = 512 / GK;                  // rows per 1 KB group
    static constexpr int IG = kTI / RPG / kGemmWaves;     // I groups per wave
    static constexpr int SG = kTS / RPG / kGemmWaves;     // S groups per wave and plane
    static constexpr int GPW = IG + 3 * SG;               // loads per wave and stage
    static_assert(STAGES * STAGE * 2 <= 160 * 1024, "stages must fit in LDS");
    static_assert(IG >= 1 && SG >= 1, "every wave loads whole groups");
    // chunk slot of chunk q in row r: any 16 consecutive rows read one chunk
    // each from 16 different 16-byte bank groups
    __device__ __forceinline__ static int swz(int r) {
        if constexpr (GK == 32) return ((r >> 1) ^ (r >> 3)) & 3;
        else return (r >> 1) & 7;
    }
};
static_assert(kTI == 2 * 128 && kTS == 4 * 32, "wave grid 2 x 4");

// s_waitcnt immediate: vector memory count <= v (bits 3:0 and 15:14), LDS and
// scalar memory count not waited for (bits 11:8), export count not waited for
// (bits 6:4).
constexpr int wait_vm(int v) { return (v & 15) | ((v >> 4) << 14) | (7 << 4) | (15 << 8); }

// Tile order: each XCD gets a contiguous run of tiles (xcd_remap), and inside
// it tiles go S-band-major in groups of kGroupI I tiles so that blocks running
// together share both operand panels in that XCD's L2.
constexpr int kGroupI = 8;

__device__ __forceinline__ void gemm_tile_coords(int t, int tiles_i, int tiles_s, int& ti, int& ts) {
    const int per_group = kGroupI * tiles_s;
    const int g = t / per_group, first = g * kGroupI;
    const int gi = min(tiles_i - first, kGroupI);
    const int r = t - g * per_group;
    ti = first + r % gi;
    ts = r / gi;
}

// 16 bytes per lane from buffer offset voff + koff straight into LDS at gd
// (lane order).  A plain device function: inside the kernel template the host
// pass would not instantiate the builtin, and the launch would find no kernel.
__device__ __forceinline__ void load_lds16(__amdgpu_buffer_rsrc_t rs, uint16_t* gd, uint32_t voff,
                                           uint32_t koff) {
    __builtin_amdgcn_raw_ptr_buffer_load_lds(rs, (__attribute__((address_space(3))) void*)gd, 16,
                                             voff, koff, 0, 0);
}

template <bool CASE_A, int GK>
__global__ __launch_bounds__(kGemmWaves * 64, 1) void gemm_bf16x3_kernel(
    int M, int N, const uint16_t* __restrict__ I, const uint16_t* __restrict__ S0,
    const uint16_t* __restrict__ S1, const uint16_t* __restrict__ S2, int64_t ld,
    float* __restrict__ Z, int64_t ldz, int tiles_i, int tiles_s) {
    using G = GemmStage<GK>;
    __shared__ __attribute__((aligned(1024))) uint16_t lds[G::STAGES * G::STAGE];

    int ti, ts;
    gemm_tile_coords(xcd_remap(blockIdx.x, tiles_i * tiles_s), tiles_i, tiles_s, ti, ts);
    const int i0 = ti * kTI, s0 = ts * kTS;
    const int lane = threadIdx.x & 63;
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int wi = (wave & 1) * 128, ws = (wave >> 1) * 32;

    // Buffer resources over the block's rows of each plane (every plane is
    // padded to whole block tiles, so these rows exist); one covering nothing
    // for the loads past the last stage.
    const uint32_t row_bytes = (uint32_t)(ld * 2);
    const __amdgpu_buffer_rsrc_t rI = __builtin_amdgcn_make_buffer_rsrc(
        const_cast<uint16_t*>(I + (int64_t)i0 * ld), (short)0, (int)(kTI * row_bytes), 0x00020000);
    const __amdgpu_buffer_rsrc_t rS[3] = {
        __builtin_amdgcn_make_buffer_rsrc(const_cast<uint16_t*>(S0 + (int64_t)s0 * ld), (short)0,
                                          (int)(kTS * row_bytes), 0x00020000),
        __builtin_amdgcn_make_buffer_rsrc(const_cast<uint16_t*>(S1 + (int64_t)s0 * ld), (short)0,
                                          (int)(kTS * row_bytes), 0x00020000),
        __builtin_amdgcn_make_buffer_rsrc(const_cast<uint16_t*>(S2 + (int64_t)s0 * ld), (short)0,
                                          (int)(kTS * row_bytes), 0x00020000)};
    const __amdgpu_buffer_rsrc_t rZero =
        __builtin_amdgcn_make_buffer_rsrc(const_cast<uint16_t*>(I), (short)0, 0, 0x00020000);
    const int n_st = (int)(ld / GK);  // ld is a multiple of 64

    // This wave's row groups of a stage: the I tile's groups 8 j + wave
    // (j < IG), then of each S tile the groups 8 j + wave (j < SG).  Lane L
    // fetches row RPG group + L / CH, chunk (L % CH) ^ swz(row), which the
    // direct load puts at slot L % CH.
    uint32_t voff[G::GPW];
#pragma unroll
    for (int j = 0; j < G::GPW; ++j) {
        const int grp = (j < G::IG ? j : (j - G::IG) % G::SG) * kGemmWaves + wave;
        const int row = grp * G::RPG + lane / G::CH;
        const int chunk = (lane % G::CH) ^ G::swz(row);
        voff[j] = (uint32_t)row * row_bytes + (uint32_t)chunk * 16u;
    }
    // Stage st (K GK st .. +GK-1) into buffer st % STAGES.  Past the last stage
    // the resource covers no bytes: the loads return zeros into a buffer nobody
    // reads any more, which keeps the loop free of branches.
    auto issue = [&](int st) {
        uint16_t* dst = lds + (st % G::STAGES) * G::STAGE;
        const uint32_t koff = (uint32_t)st * (GK * 2);
        const bool live = st < n_st;
#pragma unroll
        for (int j = 0; j < G::GPW; ++j) {
            const int plane = j < G::IG ? -1 : (j - G::IG) / G::SG;
            const int grp = (j < G::IG ? j : (j - G::IG) % G::SG) * kGemmWaves + wave;
            __amdgpu_buffer_rsrc_t rs = plane < 0 ? rI : rS[plane];
            if (!live) rs = rZero;
            uint16_t* gd = dst + (plane < 0 ? 0 : G::PLANE_I + plane * G::PLANE_S) +
                           grp * G::RPG * GK;
            load_lds16(rs, gd, voff[j], koff);
        }
    };

    f32x16 acc_hi[4], acc_lo[4];
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int v = 0; v < 16; ++v) {
            acc_hi[i][v] = 0.0f;
            acc_lo[i][v] = 0.0f;
        }

    // Fragment rows are a multiple of 32 plus fr, and swz(32 a + fr) == swz(fr):
    // one swizzled chunk offset per lane and K step (chunks 2 s and 2 s + 1).
    const int fr = lane & 31, fq = lane >> 5;
    int fo[GK / 16];
#pragma unroll
    for (int k = 0; k < GK / 16; ++k) fo[k] = fr * GK + (((2 * k + fq) ^ G::swz(fr)) * 8);
#define AFMM_FRAG(cur, off) (*reinterpret_cast<const bf16x8*>((cur) + (off)))
#define AFMM_MFMA(acc, a, b) acc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a, b, acc, 0, 0, 0);
    // The fragments of one 16-wide K step from the stage at cur, and its MFMAs:
    // hi into its own set, lo then mid into the second.
#define AFMM_READ(fi, fs, cur, fo)                                                        \
    _Pragma("unroll") for (int i = 0; i < 4; ++i)                                         \
        fi[i] = AFMM_FRAG(cur, (wi + 32 * i) * GK + (fo));                                \
    _Pragma("unroll") for (int t = 0; t < 3; ++t)                                         \
        fs[t] = AFMM_FRAG(cur, G::PLANE_I + t * G::PLANE_S + ws * GK + (fo));
#define AFMM_STEP(fi, fs)                                                                 \
    _Pragma("unroll") for (int i = 0; i < 4; ++i) {                                       \
        if (CASE_A) { AFMM_MFMA(acc_hi[i], fs[0], fi[i]) }                                \
        else { AFMM_MFMA(acc_hi[i], fi[i], fs[0]) }                                       \
    }                                                                                     \
    _Pragma("unroll") for (int t = 2; t >= 1; --t)                                        \
    _Pragma("unroll") for (int i = 0; i < 4; ++i) {                                       \
        if (CASE_A) { AFMM_MFMA(acc_lo[i], fs[t], fi[i]) }                                \
        else { AFMM_MFMA(acc_lo[i], fi[i], fs[t]) }                                       \
    }

    // STAGES - 1 stages are in flight while one is computed.  At the top of
    // each stage a wave waits for its own loads of the stage, then the barrier:
    // every wave's loads of it have landed, and every wave is done with the
    // buffer the next issue overwrites.  (A plain barrier: the compiler's
    // workgroup barrier would also wait for the loads still in flight.)
#pragma unroll
    for (int st = 0; st < G::STAGES - 1; ++st) issue(st);
    for (int st = 0; st < n_st; ++st) {
        // loads issued after this stage's: those of the STAGES - 2 later stages
        __builtin_amdgcn_s_waitcnt(wait_vm(G::GPW * (G::STAGES - 2)));
        asm volatile("" ::: "memory");
        __builtin_amdgcn_s_barrier();
        asm volatile("" ::: "memory");
        const uint16_t* cur = lds + (st % G::STAGES) * G::STAGE;
        // the compiler spreads the reads between the MFMAs (reading both steps'
        // fragments at once queues the LDS up behind eight waves: slower)
#pragma unroll
        for (int h = 0; h < GK / 32; ++h) {
            bf16x8 fi0[4], fs0[3], fi1[4], fs1[3];
            AFMM_READ(fi0, fs0, cur, fo[2 * h])
            if (h == 0) issue(st + G::STAGES - 1);
            AFMM_READ(fi1, fs1, cur, fo[2 * h + 1])
            AFMM_STEP(fi0, fs0)
            AFMM_STEP(fi1, fs1)
        }
    }
    // the zero loads past the last stage must land before the block's LDS goes
    __builtin_amdgcn_s_waitcnt(wait_vm(0));
#undef AFMM_FRAG
#undef AFMM_MFMA
#undef AFMM_READ
#undef AFMM_STEP

    // block i covers I rows wi + 32 i .. +31 and S rows ws .. ws + 31; the
    // MFMA's A operand (its result rows) is the I side for case B and the S
    // side for case A.
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int v = 0; v < 16; ++v) {
            const int a = 8 * (v / 4) + 4 * (lane >> 5) + (v & 3), b = lane & 31;
            const int row = CASE_A ? s0 + ws + a : i0 + wi + 32 * i + a;
            const int col = CASE_A ? i0 + wi + 32 * i + b : s0 + ws + b;
            if (row < M && col < N) Z[(int64_t)row * ldz + col] = acc_hi[i][v] + acc_lo[i][v];
        }
}

// K per stage of the GEMM the launcher runs
constexpr int kGemmGK = 64;

hipError_t launch_gemm_bf16x3(bool case_a, int M, int N, const uint16_t* I, const uint16_t* S0,
                              const uint16_t* S1, const uint16_t* S2, int64_t ld, float* Z,
                              int64_t ldz, hipStream_t s) {
    // I plane: split_int_rows_pad(rows) rows, S planes: split_real_rows_pad(rows)
    // rows, K pitch ld (a multiple of 64)
    const int rows_i = case_a ? N : M, rows_s = case_a ? M : N;
    const int tiles_i = (rows_i + kTI - 1) / kTI, tiles_s = (rows_s + kTS - 1) / kTS;
    const int n_tiles = tiles_i * tiles_s;
    if (case_a)
        hipLaunchKernelGGL((gemm_bf16x3_kernel<true, kGemmGK>), dim3(n_tiles), dim3(kGemmWaves * 64),
                           0, s, M, N, I, S0, S1, S2, ld, Z, ldz, tiles_i, tiles_s);
    else
        hipLaunchKernelGGL((gemm_bf16x3_kernel<false, kGemmGK>), dim3(n_tiles), dim3(kGemmWaves * 64),
                           0, s, M, N, I, S0, S1, S2, ld, Z, ldz, tiles_i, tiles_s);
    return hipGetLastError();
}

}  // namespace afmm

namespace afmm {

// ---------------------------------------------------------------------------
// Read-back of a converted plane in the factor's own orientation (for the
// conversion's parity check): out[r][c] = plane[c][r] (TRANS) or plane[r][c].
__global__ __launch_bounds__(256) void plane_unpack_kernel(const uint16_t* __restrict__ plane,
                                                           int64_t ld, bool trans, int rows,
                                                           int cols, uint16_t* __restrict__ out) {
    const int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (e >= (int64_t)rows * cols) return;
    const int64_t r = e / cols, c = e - r * cols;
    out[e] = trans ? plane[c * ld + r] : plane[r * ld + c];
}

hipError_t launch_plane_unpack(const uint16_t* plane, int64_t ld, bool trans, int rows, int cols,
                               uint16_t* out, hipStream_t s) {
    const int64_t total = (int64_t)rows * cols;
    const int64_t blocks = (total + 255) / 256;
    if (blocks > INT32_MAX) return hipErrorInvalidValue;
    hipLaunchKernelGGL(plane_unpack_kernel, dim3((unsigned)blocks), dim3(256), 0, s, plane, ld,
                       trans, rows, cols, out);
    return hipGetLastError();
}

}  // namespace afmm

namespace afmm {

SplitLayout split_planes_layout(bool case_a, int m, int k, int n) {
    SplitLayout L;
    L.rows_real = split_real_rows_pad(case_a ? m : n);
    L.rows_int = split_int_rows_pad(case_a ? n : m);
    L.ld = round_up(k, 64);
    size_t off = 0;
    auto take = [&](size_t bytes) {
        const size_t at = off;
        off = (off + bytes + 255) / 256 * 256;
        return at;
    };
    for (int q = 0; q < 3; ++q) L.planes[q] = take((size_t)L.rows_real * L.ld * 2);
    L.planes[3] = take((size_t)L.rows_int * L.ld * 2);
    L.total = off;
    return L;
}

hipError_t launch_split_prepare(bool case_a, int m, int k, int n, const void* X, int64_t ldx,
                                const void* Y, int64_t ldy, const SplitLayout& L, uint8_t* base,
                                hipStream_t s) {
    // case A: X's three terms [i][k], Y as bf16 turned to [j][k];
    // case B: X as bf16 [i][k], Y's three terms turned to [j][k]
    SplitPrepArgs a;
    a.I = static_cast<const int32_t*>(case_a ? Y : X);
    a.i_rows = case_a ? k : m;
    a.i_cols = case_a ? n : k;
    a.ldi = case_a ? ldy : ldx;
    a.ip = reinterpret_cast<uint16_t*>(base + L.planes[3]);
    a.i_tiles_o = L.rows_int / 64;
    a.R = static_cast<const float*>(case_a ? X : Y);
    a.r_rows = case_a ? m : k;
    a.r_cols = case_a ? k : n;
    a.ldr = case_a ? ldx : ldy;
    a.hi = reinterpret_cast<uint16_t*>(base + L.planes[0]);
    a.mid = reinterpret_cast<uint16_t*>(base + L.planes[1]);
    a.lo = reinterpret_cast<uint16_t*>(base + L.planes[2]);
    a.r_tiles_o = L.rows_real / 64;
    a.ld = L.ld;
    a.int_blocks = (int)((int64_t)a.i_tiles_o * (L.ld / 64));
    a.i_vec = a.ldi % 4 == 0 && reinterpret_cast<uintptr_t>(a.I) % 16 == 0;
    a.r_vec = a.ldr % 4 == 0 && reinterpret_cast<uintptr_t>(a.R) % 16 == 0;
    return launch_split_prep(case_a, a, s);
}

hipError_t launch_split_gemm(bool case_a, int m, int n, const SplitLayout& L, const uint8_t* base,
                             float* Z, int64_t ldz, hipStream_t s) {
    auto plane = [&](int q) { return reinterpret_cast<const uint16_t*>(base + L.planes[q]); };
    return launch_gemm_bf16x3(case_a, m, n, plane(3), plane(0), plane(1), plane(2), L.ld, Z, ldz,
                              s);
}

}  // namespace afmm
