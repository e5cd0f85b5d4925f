// Strict AFMM kernel, compacted-base form (Section 2, bit-exact binary32
// repeated addition) for a real factor with few non-zeros.
//
// The count-uniform mapping puts lanes over the real factor's columns, so a
// lane whose base is zero idles through the repetitions of its row.  Here a
// block keeps a TM x CT tile of Z in LDS instead of registers; for each k the
// lanes take the compacted non-zero bases of the block's CT columns, and each
// wave walks its R rows with the count uniform per row: read Z from LDS, add
// the base `rep` times, write it back.  Every element still receives its
// additions in ascending k, a k's repetitions consecutively, so the result is
// bit-identical to the other forms.  A wave owns its rows, so no two waves
// touch one element and the k loop has no barrier.
#include "sparse_body.hpp"
#include "strict_acc.hpp"

namespace afmm {

constexpr int kAccKP = 16;  // k padding of the segment table (covers panels of 8 and 16 k)
constexpr int kAccWaitVm0 = 0x0F70;  // s_waitcnt vmcnt(0), other counters at their maxima

size_t acc_lists_bytes(int n_c, int n_k, int C) {
    const int64_t ct = (int64_t)kWave * C;
    const int64_t bands = (n_c + ct - 1) / ct, kp = round_up(n_k, kAccKP);
    return (size_t)round_up(bands * kp * ct * 8, 256) + (size_t)round_up(bands * kp * 4, 256);
}

AccLists acc_lists_at(uint8_t* p, int n_c, int n_k, int C) {
    const int64_t ct = (int64_t)kWave * C;
    const int64_t bands = (n_c + ct - 1) / ct, kp = round_up(n_k, kAccKP);
    AccLists L;
    L.ent = reinterpret_cast<uint2*>(p);
    L.lens = reinterpret_cast<int32_t*>(p + round_up(bands * kp * ct * 8, 256));
    L.n_k_pad = kp;
    return L;
}

// One wave per segment (band, k): ballot the non-zero bases of 64 columns at
// a time and write them at their rank.  Segments with k >= n_k get length 0.
__global__ __launch_bounds__(256) void compact_base_kernel(const float* __restrict__ Q,
                                                           int64_t ldq, int n_k, int n_c, int ct,
                                                           int64_t n_k_pad, int64_t n_segs,
                                                           uint2* __restrict__ ent,
                                                           int32_t* __restrict__ lens,
                                                           const uint32_t* __restrict__ gate) {
    AFMM_GATE(gate);
    const int lane = threadIdx.x & (kWave - 1);
    const int64_t seg = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
    if (seg >= n_segs) return;  // whole waves
    const int band = (int)(seg / n_k_pad);
    const int k = (int)(seg - (int64_t)band * n_k_pad);
    int count = 0;
    if (k < n_k) {
        const float* __restrict__ q = Q + (int64_t)k * ldq + (int64_t)band * ct;
        const int cols = min(ct, n_c - band * ct);
        uint2* __restrict__ out = ent + seg * ct;
        for (int ch = 0; ch < cols; ch += kWave) {
            const int c = ch + lane;
            const float v = c < cols ? q[c] : 0.0f;
            const bool nz = v != 0.0f;  // IEEE: -0 is zero, NaN is not
            const uint64_t m = __ballot(nz);
            if (nz) {
                const uint32_t below = __builtin_amdgcn_mbcnt_hi(
                    (uint32_t)(m >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)m, 0u));
                out[count + (int)below] = make_uint2(__float_as_uint(v), (uint32_t)c);
            }
            count += __popcll(m);
        }
    }
    if (lane == 0) lens[seg] = count;
}

hipError_t launch_compact_base(const float* Q, int64_t ldq, int n_k, int n_c, int C,
                               const AccLists& L, hipStream_t s, const uint32_t* gate) {
    const int ct = kWave * C;
    const int64_t bands = (n_c + ct - 1) / ct;
    const int64_t n_segs = bands * L.n_k_pad;
    const int64_t blocks = (n_segs + 3) / 4;
    hipLaunchKernelGGL(compact_base_kernel, dim3((unsigned)blocks), dim3(256), 0, s, Q, ldq, n_k,
                       n_c, ct, L.n_k_pad, n_segs, L.ent, L.lens, gate);
    return hipGetLastError();
}

template <int R, int C, int W, int KP>
struct AccTile {
    static constexpr int CT = kWave * C;        // columns per block (one band)
    static constexpr int E = C >= 16 ? C / 16 : 1;  // entries per lane per k
    static constexpr int TM = W * R;            // rows per block
    // LDS row: the band's CT columns, then one sink column per lane (a lane
    // without an entry adds +0.0 there), then one float that keeps rows on
    // different banks
    static constexpr int STRIDE = CT + kWave + 1;
    static constexpr int LDS_FLOATS = TM * STRIDE;
    static_assert(TM <= kRowPad, "row padding must cover a tile");
    static_assert(TM % 4 == 0, "the tile is cleared in float4 units");
    static_assert(LDS_FLOATS * 4 <= 160 * 1024, "the Z tile must fit in LDS");
    static_assert(KP == 8 || KP == 16, "count words of 8 or 16 k");
    static_assert(kKPad % KP == 0, "KP must divide the k padding");
};

// One chunk of up to 64*E entries of the segment of k0 + kk, slot q of lane l
// holding entry ch_ + 64 q + l: a slot past the segment's end turns into a +0.0
// base on the lane's sink column, so every lane runs every slot.  Each of the
// wave's rows with a non-zero count reads its E Z elements from LDS, adds each
// slot's base `rep` times (the E chains side by side) and writes them back; the
// reads of all rows go out before the first addition.
#define AFMM_ACC_CHUNK(ev_, ch_)                                                               \
    {                                                                                          \
        int col_[T::E];                                                                        \
        float b_[T::E];                                                                        \
        _Pragma("unroll") for (int q = 0; q < T::E; ++q) {                                     \
            const bool ok_ = (ch_) + q * kWave + lane < len_;                                  \
            col_[q] = ok_ ? (int)(ev_)[q][1] : T::CT + lane;                                   \
            b_[q] = ok_ ? __uint_as_float((ev_)[q][0]) : 0.0f;                                 \
        }                                                                                      \
        float z_[R][T::E];                                                                     \
        _Pragma("unroll") for (int r = 0; r < R; ++r) {                                        \
            if (rep_[r] == 0) continue;                                                        \
            _Pragma("unroll") for (int q = 0; q < T::E; ++q) z_[r][q] =                        \
                arow[r * T::STRIDE + col_[q]];                                                 \
        }                                                                                      \
        __builtin_amdgcn_s_waitcnt(kWaitLgkm0);                                                \
        _Pragma("unroll") for (int r = 0; r < R; ++r) {                                        \
            uint32_t n_ = rep_[r];                                                             \
            if (n_ == 0) continue;                                                             \
            float zz_[T::E];                                                                   \
            _Pragma("unroll") for (int q = 0; q < T::E; ++q) zz_[q] = z_[r][q];                \
            if (U == 4) {                                                                      \
                /* bits of the count: 1, 2 and 4 additions under scalar bit */                 \
                /* tests, then runs of 8 */                                                    \
                if (n_ & 1u) AFMM_ACC_ADD(1);                                                  \
                if (n_ & 2u) AFMM_ACC_ADD(2);                                                  \
                if (n_ & 4u) AFMM_ACC_ADD(4);                                                  \
                for (n_ >>= 3; n_ != 0; --n_) AFMM_ACC_ADD(8);                                 \
            } else if (U == 2) {                                                               \
                if (n_ & 1u) AFMM_ACC_ADD(1);                                                  \
                for (n_ >>= 1; n_ != 0; --n_) AFMM_ACC_ADD(2);                                 \
            } else {                                                                           \
                do {                                                                           \
                    AFMM_ACC_ADD(1);                                                           \
                } while (--n_ != 0);                                                           \
            }                                                                                  \
            _Pragma("unroll") for (int q = 0; q < T::E; ++q) arow[r * T::STRIDE + col_[q]] =   \
                zz_[q];                                                                        \
        }                                                                                      \
    }

// `times` more repetitions of every slot's base (slots interleaved, each
// slot's own additions in order)
#define AFMM_ACC_ADD(times)                                                                    \
    {                                                                                          \
        _Pragma("unroll") for (int t_ = 0; t_ < (times); ++t_)                                 \
            _Pragma("unroll") for (int q = 0; q < T::E; ++q) zz_[q] = zz_[q] + b_[q];          \
    }

// The additions of k0 + kk for the wave's R rows: the prefetched first 64*E
// entries, then (longer segments) the rest, 64*E at a time.
#define AFMM_ACC_K(kk)                                                                         \
    do {                                                                                       \
        const int len_ = Lc[kk];                                                               \
        if (len_ == 0) break;                                                                  \
        uint32_t rep_[R];                                                                      \
        uint32_t any_ = 0;                                                                     \
        _Pragma("unroll") for (int r = 0; r < R; ++r) {                                        \
            uint32_t v_ = cw[r].byte(kk);                                                      \
            if (ESC && v_ == 0xFFu) {                                                          \
                const int32_t full_ = __builtin_amdgcn_readfirstlane(                          \
                    P32[(int64_t)(rw0 + r) * p32_sr + (int64_t)(k0 + (kk)) * p32_sk]);         \
                /* >= 255 by construction; a value changed under a running call */             \
                /* must still end the repetition loop */                                       \
                v_ = full_ > 0 ? (uint32_t)full_ : 0u;                                         \
            }                                                                                  \
            rep_[r] = v_;                                                                      \
            any_ |= v_;                                                                        \
        }                                                                                      \
        if (any_ == 0) break;                                                                  \
        AFMM_ACC_CHUNK(ec[kk], 0)                                                              \
        for (int ch2_ = kWave * T::E; ch2_ < len_; ch2_ += kWave * T::E) {                     \
            u32x2_t e2_[T::E];                                                                 \
            _Pragma("unroll") for (int q = 0; q < T::E; ++q) e2_[q] =                          \
                __builtin_amdgcn_raw_buffer_load_b64(                                          \
                    ers, (uint32_t)(((k0 + (kk)) * T::CT + ch2_ + q * kWave + lane) * 8), 0,   \
                    0); /* ch2_ + q * 64 + lane < CT */                                        \
            AFMM_ACC_CHUNK(e2_, ch2_)                                                          \
        }                                                                                      \
    } while (0)

template <int R, int C, int W, int U, int KP, bool TRANS_OUT, bool ESC>
__device__ __forceinline__ void rep_acc_tile(int n_r, int n_c, int n_k,
                                             const uint8_t* __restrict__ P8, int64_t ldp,
                                             const int32_t* __restrict__ P32, int64_t p32_sr,
                                             int64_t p32_sk, const uint2* __restrict__ ent,
                                             const int32_t* __restrict__ lens, int64_t n_k_pad,
                                             float* __restrict__ Z, int64_t z_sr, int64_t z_sc,
                                             int r0, int band, float* lds) {
    using T = AccTile<R, C, W, KP>;
    constexpr int NT = W * kWave;
    const int lane = threadIdx.x & (kWave - 1);
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x / kWave);
    const int rw0 = r0 + wave * R;
    const int c0 = band * T::CT;
    float* arow = lds + wave * R * T::STRIDE;

    // Z starts at +0.0 (the sink columns too: they only ever receive +0.0)
    float4* l4 = reinterpret_cast<float4*>(lds);
    for (int i = threadIdx.x; i < T::LDS_FLOATS / 4; i += NT) l4[i] = make_float4(0.f, 0.f, 0.f, 0.f);
    __syncthreads();

    // The band's segments, their lengths and the count bytes go through buffer
    // resources (byte offsets in 31 bits, checked by the launcher), so the next
    // panel's loads run on the vector memory counter while this panel's LDS
    // traffic waits on its own.
    const __amdgpu_buffer_rsrc_t ers = __builtin_amdgcn_make_buffer_rsrc(
        const_cast<uint2*>(ent + (int64_t)band * n_k_pad * T::CT), (short)0,
        (int)(n_k_pad * T::CT * 8), 0x00020000);
    const __amdgpu_buffer_rsrc_t lrs = __builtin_amdgcn_make_buffer_rsrc(
        const_cast<int32_t*>(lens + (int64_t)band * n_k_pad), (short)0, (int)(n_k_pad * 4),
        0x00020000);
    const int rows_bound = (n_r + T::TM - 1) / T::TM * T::TM;
    const __amdgpu_buffer_rsrc_t crs = __builtin_amdgcn_make_buffer_rsrc(
        const_cast<uint8_t*>(P8), (short)0, (int)((int64_t)rows_bound * ldp), 0x00020000);

    const int n_panels = (n_k + KP - 1) / KP;
    int32_t Lc[KP];
    u32x2_t ec[KP][T::E];
    SparseCounts<KP> cw[R];
    {
        u32x4_t lv[KP / 4];
        CountFetch<KP> cf[R];
#pragma unroll
        for (int q = 0; q < KP / 4; ++q)
            lv[q] = __builtin_amdgcn_raw_buffer_load_b128(lrs, (uint32_t)(q * 16), 0, 0);
#pragma unroll
        for (int kk = 0; kk < KP; ++kk)
#pragma unroll
            for (int q = 0; q < T::E; ++q)
                ec[kk][q] = __builtin_amdgcn_raw_buffer_load_b64(
                    ers, (uint32_t)((kk * T::CT + q * kWave + lane) * 8), 0, 0);
#pragma unroll
        for (int r = 0; r < R; ++r) cf[r].fetch(crs, (uint32_t)((rw0 + r) * ldp));
#pragma unroll
        for (int kk = 0; kk < KP; ++kk) Lc[kk] = (int32_t)uniform_u32(lv[kk / 4][kk % 4]);
#pragma unroll
        for (int r = 0; r < R; ++r) cf[r].to(cw[r]);
        // both ways into the loop arrive with nothing pending (see the end of
        // the loop body): an empty statement that reads the entries keeps
        // their loads above it and makes the compiler wait for them here
#pragma unroll
        for (int kk = 0; kk < KP; ++kk)
#pragma unroll
            for (int q = 0; q < T::E; ++q) asm volatile("" ::"v"(ec[kk][q]));
    }

    for (int p = 0; p < n_panels; ++p) {
        const int k0 = p * KP;
        const bool more = p + 1 < n_panels;
        u32x4_t lv[KP / 4];
        u32x2_t en[KP][T::E];
        CountFetch<KP> cf[R];
        if (more) {
            const int k1 = k0 + KP;
#pragma unroll
            for (int q = 0; q < KP / 4; ++q)
                lv[q] = __builtin_amdgcn_raw_buffer_load_b128(lrs, (uint32_t)((k1 + 4 * q) * 4), 0, 0);
#pragma unroll
            for (int kk = 0; kk < KP; ++kk)
#pragma unroll
                for (int q = 0; q < T::E; ++q)
                    en[kk][q] = __builtin_amdgcn_raw_buffer_load_b64(
                        ers, (uint32_t)(((k1 + kk) * T::CT + q * kWave + lane) * 8), 0, 0);
#pragma unroll
            for (int r = 0; r < R; ++r) cf[r].fetch(crs, (uint32_t)((rw0 + r) * ldp + k1));
        }
#pragma unroll
        for (int kk = 0; kk < KP; ++kk) AFMM_ACC_K(kk);
        // the next panel's loads have had this whole panel to land; waiting for
        // them here leaves nothing pending at the top of the loop, so the uses
        // of the entries there need no wait of their own
        __builtin_amdgcn_s_waitcnt(kAccWaitVm0);
        if (more) {
#pragma unroll
            for (int kk = 0; kk < KP; ++kk) {
                Lc[kk] = (int32_t)uniform_u32(lv[kk / 4][kk % 4]);
#pragma unroll
                for (int q = 0; q < T::E; ++q) ec[kk][q] = en[kk][q];
            }
#pragma unroll
            for (int r = 0; r < R; ++r) cf[r].to(cw[r]);
        }
    }
    __syncthreads();

    if (TRANS_OUT) {
        // element (r, c) at Z[(c0 + c) * z_sc + r0 + r]: runs of TM rows per column
        for (int i = threadIdx.x; i < T::TM * T::CT; i += NT) {
            const int r = i % T::TM, c = i / T::TM;
            if (r0 + r < n_r && c0 + c < n_c)
                Z[(int64_t)(c0 + c) * z_sc + r0 + r] = lds[r * T::STRIDE + c];
        }
    } else {
        for (int i = threadIdx.x; i < T::TM * T::CT; i += NT) {
            const int c = i % T::CT, r = i / T::CT;
            if (r0 + r < n_r && c0 + c < n_c)
                Z[(int64_t)(r0 + r) * z_sr + c0 + c] = lds[r * T::STRIDE + c];
        }
    }
}
#undef AFMM_ACC_K
#undef AFMM_ACC_ADD
#undef AFMM_ACC_CHUNK

template <int R, int C, int W, int U, int KP, bool TRANS_OUT>
__global__ __launch_bounds__(W * kWave) void rep_acc_kernel(
    int n_r, int n_c, int n_k, const uint8_t* __restrict__ P8, int64_t ldp,
    const int32_t* __restrict__ P32, int64_t p32_sr, int64_t p32_sk, const uint2* __restrict__ ent,
    const int32_t* __restrict__ lens, int64_t n_k_pad, float* __restrict__ Z, int64_t z_sr,
    int64_t z_sc, const uint32_t* __restrict__ esc, int n_row_blocks, int n_tiles,
    const uint32_t* __restrict__ gate) {
    using T = AccTile<R, C, W, KP>;
    __shared__ __attribute__((aligned(16))) float lds[T::LDS_FLOATS];
    AFMM_GATE(gate);
    const int t = xcd_remap(blockIdx.x, n_tiles);
    const int band = t / n_row_blocks, rb = t - band * n_row_blocks;
    if (*esc)
        rep_acc_tile<R, C, W, U, KP, TRANS_OUT, true>(n_r, n_c, n_k, P8, ldp, P32, p32_sr, p32_sk,
                                                      ent, lens, n_k_pad, Z, z_sr, z_sc,
                                                      rb * T::TM, band, lds);
    else
        rep_acc_tile<R, C, W, U, KP, TRANS_OUT, false>(n_r, n_c, n_k, P8, ldp, P32, p32_sr,
                                                       p32_sk, ent, lens, n_k_pad, Z, z_sr, z_sc,
                                                       rb * T::TM, band, lds);
}

template <int R, int C, int W, int U, int KP>
hipError_t launch_acc(const StrictArgs& a, const AccLists& L, hipStream_t s) {
    using T = AccTile<R, C, W, KP>;
    if (!rep_acc_usable(a, C)) return hipErrorInvalidValue;
    const int n_row_blocks = (a.n_r + T::TM - 1) / T::TM;
    const int n_tiles = n_row_blocks * ((a.n_c + T::CT - 1) / T::CT);
    dim3 grid(n_tiles), block(W * kWave);
    if (a.trans_out)
        hipLaunchKernelGGL((rep_acc_kernel<R, C, W, U, KP, true>), grid, block, 0, s, a.n_r,
                           a.n_c, a.n_k, a.P8, a.ldp, a.P32, a.p32_sr, a.p32_sk, L.ent, L.lens,
                           L.n_k_pad, a.Z, a.z_sr, a.z_sc, a.esc, n_row_blocks, n_tiles, a.gate);
    else
        hipLaunchKernelGGL((rep_acc_kernel<R, C, W, U, KP, false>), grid, block, 0, s, a.n_r,
                           a.n_c, a.n_k, a.P8, a.ldp, a.P32, a.p32_sr, a.p32_sk, L.ent, L.lens,
                           L.n_k_pad, a.Z, a.z_sr, a.z_sc, a.esc, n_row_blocks, n_tiles, a.gate);
    return hipGetLastError();
}

// (R, C, W, U, KP): TM = W*R rows x CT = 64*C columns of Z in LDS per block;
// each lane takes max(1, C/16) entries of a k's segment
#define AFMM_ACC_CONFIGS(X) \
    X(4, 16, 8, 1, 16)      \
    X(4, 16, 8, 2, 16)      \
    X(4, 16, 8, 4, 16)      \
    X(2, 16, 16, 1, 16)     \
    X(2, 16, 16, 2, 16)     \
    X(2, 16, 16, 4, 16)     \
    X(4, 8, 16, 1, 16)      \
    X(8, 8, 8, 1, 16)       \
    X(4, 4, 8, 1, 16)       \
    X(2, 32, 8, 2, 8)       \
    X(1, 32, 16, 2, 8)      \
    X(1, 64, 8, 2, 8)       \
    X(1, 64, 8, 1, 8)

bool rep_acc_usable(const StrictArgs& a, int C) {
    // buffer-resource byte offsets of one band's segments and of the count
    // bytes in 31 bits
    const int64_t lim = (int64_t)1 << 31;
    return round_up(a.n_k, kAccKP) * kWave * C * 8 < lim &&
           round_up(a.n_r, kRowPad) * a.ldp < lim;
}

bool rep_acc_supported(int R, int C, int W, int U, int KP) {
#define AFMM_CASE(r, c, w, u, kp) \
    if (R == r && C == c && W == w && U == u && KP == kp) return true;
    AFMM_ACC_CONFIGS(AFMM_CASE)
#undef AFMM_CASE
    return false;
}

hipError_t launch_rep_acc(const StrictArgs& a, const AccLists& L, int R, int C, int W, int U,
                          int KP, hipStream_t s) {
#define AFMM_CASE(r, c, w, u, kp) \
    if (R == r && C == c && W == w && U == u && KP == kp) return launch_acc<r, c, w, u, kp>(a, L, s);
    AFMM_ACC_CONFIGS(AFMM_CASE)
#undef AFMM_CASE
    return hipErrorInvalidValue;
}

}  // namespace afmm
