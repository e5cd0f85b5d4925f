// Strict repeated-addition tile, sparse-k form: the same count-uniform mapping
// and the same order of additions as rep_uniform_tile (each output row takes
// its k in ascending order, each k its count of repetitions, straight into the
// accumulator), organised for eight waves per SIMD:
//  - base panels go from global memory straight into LDS (buffer loads with
//    an LDS destination), so no staging registers and no LDS store pass;
//  - a wave visits only the k of a panel where at least one of its R rows has
//    a non-zero count: the zero tests of the other k and their LDS reads are
//    skipped as a whole (one scalar bit scan per visited k);
//  - no LDS read is issued ahead of use: the other waves of the SIMD cover
//    its latency, which keeps the register budget at 64.
// A k is visited in ascending order (lowest set bit first), so every
// accumulator still receives its additions in the order of the Case-A /
// Case-B loops of Section 2 and the bits equal the sequential result.
#pragma once

#include "strict_body.hpp"

namespace afmm {

// Bit i of the result is set when byte i of `w` is non-zero (i = 0..3).
__device__ __forceinline__ uint32_t nonzero_bytes(uint32_t w) {
    uint32_t t = w | (w >> 4);
    t |= t >> 2;
    t |= t >> 1;
    t &= 0x01010101u;
    // the four flags sit at bits 0, 8, 16, 24; the product gathers them at
    // bits 24..27 without carries
    return (t * 0x01020408u) >> 24;
}

// The count bytes of one row for one panel, little-endian in 64-bit words:
// count of k0 + kk is byte kk % 8 of word kk / 8.  Kept as plain scalars so
// that picking a byte at a run-time kk is a shift, not an indexed access.
template <int KP>
struct SparseCounts;
template <>
struct SparseCounts<4> {
    uint32_t lo;
    __device__ __forceinline__ void load(const uint8_t* p) { lo = *reinterpret_cast<const uint32_t*>(p); }
    __device__ __forceinline__ uint32_t byte(int kk) const { return (lo >> (8 * kk)) & 0xFFu; }
    __device__ __forceinline__ uint32_t nonzero_mask() const { return nonzero_bytes(lo); }
    __device__ __forceinline__ void or_into(SparseCounts& a) const { a.lo |= lo; }
    __device__ __forceinline__ void clear() { lo = 0; }
};
template <>
struct SparseCounts<8> {
    uint64_t lo;
    __device__ __forceinline__ void load(const uint8_t* p) { lo = *reinterpret_cast<const uint64_t*>(p); }
    __device__ __forceinline__ uint32_t byte(int kk) const { return (uint32_t)(lo >> (8 * kk)) & 0xFFu; }
    __device__ __forceinline__ uint32_t nonzero_mask() const {
        return nonzero_bytes((uint32_t)lo) | (nonzero_bytes((uint32_t)(lo >> 32)) << 4);
    }
    __device__ __forceinline__ void or_into(SparseCounts& a) const { a.lo |= lo; }
    __device__ __forceinline__ void clear() { lo = 0; }
};
template <>
struct SparseCounts<16> {
    uint64_t lo, hi;
    __device__ __forceinline__ void load(const uint8_t* p) {
        lo = *reinterpret_cast<const uint64_t*>(p);
        hi = *reinterpret_cast<const uint64_t*>(p + 8);
    }
    __device__ __forceinline__ uint32_t byte(int kk) const {
        // shift both words, then pick: a pick between the two words themselves
        // would become an indexed access to the (then unpromotable) array
        const uint32_t a = (uint32_t)(lo >> (8 * (kk & 7))), b = (uint32_t)(hi >> (8 * (kk & 7)));
        return ((kk & 8) ? b : a) & 0xFFu;
    }
    __device__ __forceinline__ uint32_t nonzero_mask() const {
        return nonzero_bytes((uint32_t)lo) | (nonzero_bytes((uint32_t)(lo >> 32)) << 4) |
               (nonzero_bytes((uint32_t)hi) << 8) | (nonzero_bytes((uint32_t)(hi >> 32)) << 12);
    }
    __device__ __forceinline__ void or_into(SparseCounts& a) const { a.lo |= lo; a.hi |= hi; }
    __device__ __forceinline__ void clear() { lo = hi = 0; }
};

// The next panel's count bytes of one row, fetched through the vector memory
// path (its own wait counter, so the LDS waits of the current panel do not
// wait for them too) and moved to scalar registers once they have landed.
// readfirstlane yields a signed int: widen through uint32_t, never sign-extend
// (a count byte >= 128 in the top byte would otherwise spill 0xFF bytes into
// the upper word)
__device__ __forceinline__ uint32_t uniform_u32(uint32_t v) {
    return (uint32_t)__builtin_amdgcn_readfirstlane(v);
}
__device__ __forceinline__ uint64_t join(uint32_t lo, uint32_t hi) {
    return ((uint64_t)uniform_u32(hi) << 32) | (uint64_t)uniform_u32(lo);
}
typedef unsigned int u32x2_t __attribute__((ext_vector_type(2)));
typedef unsigned int u32x4_t __attribute__((ext_vector_type(4)));
template <int KP>
struct CountFetch;
template <>
struct CountFetch<4> {
    uint32_t v;
    __device__ __forceinline__ void fetch(__amdgpu_buffer_rsrc_t rs, uint32_t off) {
        v = __builtin_amdgcn_raw_buffer_load_b32(rs, off, 0, 0);
    }
    __device__ __forceinline__ void to(SparseCounts<4>& c) const { c.lo = uniform_u32(v); }
};
template <>
struct CountFetch<8> {
    u32x2_t v;
    __device__ __forceinline__ void fetch(__amdgpu_buffer_rsrc_t rs, uint32_t off) {
        v = __builtin_amdgcn_raw_buffer_load_b64(rs, off, 0, 0);
    }
    __device__ __forceinline__ void to(SparseCounts<8>& c) const { c.lo = join(v[0], v[1]); }
};
template <>
struct CountFetch<16> {
    u32x4_t v;
    __device__ __forceinline__ void fetch(__amdgpu_buffer_rsrc_t rs, uint32_t off) {
        v = __builtin_amdgcn_raw_buffer_load_b128(rs, off, 0, 0);
    }
    __device__ __forceinline__ void to(SparseCounts<16>& c) const {
        c.lo = join(v[0], v[1]);
        c.hi = join(v[2], v[3]);
    }
};

// s_waitcnt operand: LDS/scalar-memory counter 0, the others left at their maxima
constexpr int kWaitLgkm0 = 0xC07F;

template <int R, int C, int W, int KP>
struct SparseTile {
    static constexpr int G = C / 4;                   // 16-byte LDS reads per k
    static constexpr int TN = kWave * C;              // columns per tile
    static constexpr int TM = W * R;                  // rows per tile
    static constexpr int CHUNKS = KP * G;             // 1 KB LDS chunks per panel
    static constexpr int CPW = CHUNKS / W;            // chunks each wave loads
    static constexpr int LDS_FLOATS = 2 * KP * TN;
    static_assert(C % 4 == 0, "16-byte base reads");
    static_assert(CHUNKS % W == 0, "the panel splits evenly over the waves");
    static_assert(kKPad % KP == 0, "KP must divide the k padding");
    static_assert(TM <= kRowPad, "row padding must cover a tile");
};

// Requirements (checked by the launcher): Q rows readable in float4 units and
// the whole base matrix addressable with 31-bit byte offsets.
template <int R, int C, int W, int KP, bool TRANS_OUT, bool ESC, int UNR>
__device__ __forceinline__ void rep_sparse_tile(
    int n_r, int n_c, int n_k, const uint8_t* __restrict__ P8, int64_t ldp,
    const int32_t* __restrict__ P32, int64_t p32_sr, int64_t p32_sk,
    const float* __restrict__ Q, int64_t ldq, float* __restrict__ Z, int64_t z_sr, int64_t z_sc,
    int r0, int c0, float* lds) {
    using T = SparseTile<R, C, W, KP>;
    constexpr int G = T::G, TN = T::TN, CPW = T::CPW;
    const int lane = threadIdx.x & (kWave - 1);
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x / kWave);
    const int rw0 = r0 + wave * R;
    const uint8_t* __restrict__ prow = P8 + (int64_t)rw0 * ldp;

    float acc[R][C];
#pragma unroll
    for (int r = 0; r < R; ++r)
#pragma unroll
        for (int c = 0; c < C; ++c) acc[r][c] = 0.0f;  // Z starts at +0.0

    // Chunk q = wave + W*s of a panel is base row kk = q / G, columns
    // c0 + 256*(q % G) + [0, 256): lane l moves its 16 bytes to LDS float
    // kk*TN + 256*(q % G) + 4*l, the layout the additions read back.
    uint32_t voff[CPW];
    int ldsoff[CPW];
#pragma unroll
    for (int s = 0; s < CPW; ++s) {
        const int q = wave + W * s, kk = q / G, g = q - kk * G;
        voff[s] = (uint32_t)((kk * ldq + c0 + g * 256 + 4 * lane) * 4);
        ldsoff[s] = kk * TN + g * 256;
    }
    const int n_panels = (n_k + KP - 1) / KP;
    // panel p -> LDS buffer p & 1
#define AFMM_SPARSE_ISSUE(p)                                                                  \
    do {                                                                                      \
        const int k0_ = (p) * KP; /* < n_k for every issued panel */                          \
        const __amdgpu_buffer_rsrc_t rsrc_ = __builtin_amdgcn_make_buffer_rsrc(               \
            const_cast<float*>(Q + (int64_t)k0_ * ldq), (short)0,                             \
            base_records(n_k, k0_, ldq, n_c), 0x00020000);                                    \
        float* dst_ = lds + ((p) & 1) * (KP * TN);                                            \
        _Pragma("unroll") for (int s = 0; s < CPW; ++s)                                       \
            __builtin_amdgcn_raw_ptr_buffer_load_lds(                                         \
                rsrc_, (__attribute__((address_space(3))) void*)(dst_ + ldsoff[s]), 16,       \
                voff[s], 0, 0, 0);                                                            \
    } while (0)

    // count bytes: rows [0, round_up(n_r, TM)) x ldp of P8 (the padding is zero)
    const int rows_bound = (n_r + T::TM - 1) / T::TM * T::TM;
    const __amdgpu_buffer_rsrc_t crs = __builtin_amdgcn_make_buffer_rsrc(
        const_cast<uint8_t*>(P8), (short)0, (int)(rows_bound * ldp), 0x00020000);

    AFMM_SPARSE_ISSUE(0);
    SparseCounts<KP> cw[R];
    CountFetch<KP> nx[R];
#pragma unroll
    for (int r = 0; r < R; ++r) cw[r].load(prow + (int64_t)r * ldp);
    __builtin_amdgcn_s_waitcnt(0);
    __syncthreads();

    const float* lane_base = lds + lane * 4;
    for (int p = 0; p < n_panels; ++p) {
        const int k0 = p * KP;
        const bool more = p + 1 < n_panels;
        // the other buffer was last read before the previous barrier
        if (more) {
            AFMM_SPARSE_ISSUE(p + 1);
#pragma unroll
            for (int r = 0; r < R; ++r)
                nx[r].fetch(crs, (uint32_t)((rw0 + r) * ldp + k0 + KP));
        }

        // k of this panel with a non-zero count in any of the wave's rows
        SparseCounts<KP> any;
        any.clear();
#pragma unroll
        for (int r = 0; r < R; ++r) cw[r].or_into(any);
        uint32_t mask = any.nonzero_mask();
        mask = __builtin_amdgcn_readfirstlane(mask);

        const float* pan = lane_base + (p & 1) * (KP * TN);
        while (mask != 0) {
            const int kk = __builtin_ctz(mask);  // ascending k
            mask &= mask - 1;
            float b[C];
            const float* brow = pan + kk * TN;
#pragma unroll
            for (int g = 0; g < G; ++g) {
                const float4 t = *reinterpret_cast<const float4*>(brow + g * 256);
                b[4 * g + 0] = t.x;
                b[4 * g + 1] = t.y;
                b[4 * g + 2] = t.z;
                b[4 * g + 3] = t.w;
            }
            // wait for the base here, once, rather than inside every repetition loop
            __builtin_amdgcn_s_waitcnt(kWaitLgkm0);
#pragma unroll
            for (int r = 0; r < R; ++r) {
                uint32_t rep = cw[r].byte(kk);
                if (rep == 0) continue;  // a zero Rep-factor adds nothing
                if (ESC && rep == 0xFFu) {
                    const int32_t full = __builtin_amdgcn_readfirstlane(
                        P32[(int64_t)(rw0 + r) * p32_sr + (int64_t)(k0 + kk) * p32_sk]);
                    // >= 255 by construction of the packed bytes; a value changed
                    // under a running call must still end the repetition loop
                    if (full <= 0) continue;
                    rep = (uint32_t)full;
                }
                if (UNR == 2) {
                    // the same base added rep times: an odd one first, then pairs
                    if (rep & 1u) {
#pragma unroll
                        for (int c = 0; c < C; ++c) acc[r][c] = acc[r][c] + b[c];
                    }
                    for (rep >>= 1; rep != 0; --rep) {
#pragma unroll
                        for (int c = 0; c < C; ++c) acc[r][c] = acc[r][c] + b[c];
#pragma unroll
                        for (int c = 0; c < C; ++c) acc[r][c] = acc[r][c] + b[c];
                    }
                } else {
                    do {
#pragma unroll
                        for (int c = 0; c < C; ++c) acc[r][c] = acc[r][c] + b[c];
                    } while (--rep != 0);
                }
            }
        }

        // this wave's part of the next panel (and its counts) have landed;
        // then all waves are done reading the current one
        __builtin_amdgcn_s_waitcnt(0);
        __syncthreads();
        if (more) {
#pragma unroll
            for (int r = 0; r < R; ++r) nx[r].to(cw[r]);
        }
    }

    rep_store<R, C, TRANS_OUT>(acc, n_r, n_c, Z, z_sr, z_sc, rw0, c0, lane);
}
#undef AFMM_SPARSE_ISSUE

}  // namespace afmm
