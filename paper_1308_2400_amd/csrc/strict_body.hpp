// The strict repeated-addition tile (count-uniform mapping), shared by the
// single-product kernel and the batched persistent kernel.
//
// Orientation.  Rows r carry the integer factor (the Rep-factor), columns c
// the real factor (the Base):  out(r, c) = sum over k ascending of
// count(r, k) repetitions of Z += base(k, c).
//   case B:  r = i, c = j, count = X[i,k], base = Y[k,j]   (Section 2, Case-B)
//   case A:  r = j, c = i, count = Y[k,j], base = X[i,k]   (Case-A on the
//            transposed problem: the additions into Z[i,j] and their order
//            are the same, so the bits are too)
//
// Mapping.  A wave owns R rows and 64*C columns; lane l keeps its C columns
// of each of the R rows in binary32 registers.  The count of (r, k) is the
// same for every lane, so it lives in a scalar register and the repetition
// loop is a scalar loop: no lane divergence.  A zero count skips the k for
// that row wave-wide.  A zero base adds +-0 to a Z that is never -0, which
// leaves Z unchanged bit for bit: that lane slot is spent but the result is
// the one the skip gives.  Base rows are staged per k-panel in LDS (double
// buffered, one barrier per panel) and read back as 16-byte vectors.
#pragma once

#include "common.hpp"

namespace afmm {

template <int R, int C, int W, int KP>
struct RepTile {
    static constexpr int V = C >= 4 ? 4 : C;          // floats per LDS read
    static constexpr int G = C / V;                   // LDS reads per k
    static constexpr int TN = kWave * C;              // columns per tile
    static constexpr int TM = W * R;                  // rows per tile
    static constexpr int F4 = KP * TN / 4;            // float4 per panel
    static constexpr int F4T = (F4 + W * kWave - 1) / (W * kWave);  // per thread
    static constexpr int LDS_FLOATS = 2 * KP * TN;
    static_assert(C == 1 || C == 2 || C % 4 == 0, "C must be 1, 2 or a multiple of 4");
    static_assert(kKPad % KP == 0 && KP % 4 == 0, "KP must divide the k padding");
    static_assert(TM <= kRowPad, "row padding must cover a tile");
};

// The count bytes of one row for one panel: KP bytes, one scalar load.
template <int KP>
struct PanelCounts;
template <>
struct PanelCounts<16> {
    uint4 v;
    __device__ __forceinline__ void load(const uint8_t* p) { v = *reinterpret_cast<const uint4*>(p); }
    __device__ __forceinline__ uint32_t get(int i) const {
        return i == 0 ? v.x : i == 1 ? v.y : i == 2 ? v.z : v.w;
    }
};
template <>
struct PanelCounts<8> {
    uint2 v;
    __device__ __forceinline__ void load(const uint8_t* p) { v = *reinterpret_cast<const uint2*>(p); }
    __device__ __forceinline__ uint32_t get(int i) const { return i == 0 ? v.x : v.y; }
};

// Stage panel rows [k0, k0 + KP) x columns [c0, c0 + TN) of the base into
// registers (float4 units; out-of-range entries read as zero).
template <int R, int C, int W, int KP, bool VEC>
__device__ __forceinline__ void panel_load(float4* buf,
                                           const float* __restrict__ Q, int64_t ldq, int n_k,
                                           int n_c, int k0, int c0) {
    using T = RepTile<R, C, W, KP>;
    constexpr int ROWF4 = T::TN / 4;
#pragma unroll
    for (int s = 0; s < T::F4T; ++s) {
        const int e = threadIdx.x + s * W * kWave;
        float4 v = make_float4(0.f, 0.f, 0.f, 0.f);
        if (T::F4 % (W * kWave) == 0 || e < T::F4) {
            const int kr = e / ROWF4, cv = e % ROWF4;
            const int k = k0 + kr, c = c0 + cv * 4;
            if (k < n_k) {
                const float* src = Q + (int64_t)k * ldq + c;
                if (VEC) {
                    if (c < n_c) v = *reinterpret_cast<const float4*>(src);
                } else {
                    if (c < n_c) v.x = src[0];
                    if (c + 1 < n_c) v.y = src[1];
                    if (c + 2 < n_c) v.z = src[2];
                    if (c + 3 < n_c) v.w = src[3];
                }
            }
        }
        buf[s] = v;
    }
}

// Bytes of the base rows [k0, n_k) a buffer resource may cover: whole rows of
// pitch ldq, except that the last row ends at its n_c-th element (the caller
// may own no more than that).
__device__ __forceinline__ int base_records(int n_k, int k0, int64_t ldq, int n_c) {
    const int rows = n_k - k0;
    return rows > 0 ? (int)(((int64_t)(rows - 1) * ldq + n_c) * 4) : 0;
}

// Same with a buffer resource covering the base rows from k0 on: the
// per-thread offsets are fixed, the panel start moves in scalar registers, and
// reads past the resource's end read as zero instead of faulting.  Columns
// past n_c read neighbouring data (or zero); those lanes are never stored, and
// rows past n_k have zero counts, so neither value is used.
template <int R, int C, int W, int KP>
__device__ __forceinline__ void panel_load_buf(float4* buf, const float* __restrict__ Q,
                                               int64_t ldq, int n_k, int n_c, int k0,
                                               const uint32_t* voff) {
    using T = RepTile<R, C, W, KP>;
    const __amdgpu_buffer_rsrc_t rsrc = __builtin_amdgcn_make_buffer_rsrc(
        const_cast<float*>(Q + (int64_t)k0 * ldq), (short)0, base_records(n_k, k0, ldq, n_c),
        0x00020000);
#pragma unroll
    for (int s = 0; s < T::F4T; ++s) {
        const int e = threadIdx.x + s * W * kWave;
        if (T::F4 % (W * kWave) == 0 || e < T::F4)
            buf[s] = __builtin_bit_cast(float4, __builtin_amdgcn_raw_buffer_load_b128(rsrc, voff[s], 0, 0));
        else
            buf[s] = make_float4(0.f, 0.f, 0.f, 0.f);
    }
}

template <int R, int C, int W, int KP>
__device__ __forceinline__ void panel_store(const float4* buf,
                                            float* lds) {
    using T = RepTile<R, C, W, KP>;
#pragma unroll
    for (int s = 0; s < T::F4T; ++s) {
        const int e = threadIdx.x + s * W * kWave;
        if (T::F4 % (W * kWave) == 0 || e < T::F4) reinterpret_cast<float4*>(lds)[e] = buf[s];
    }
}

// Store a wave's R x C accumulators: column of acc[r][g*V + v] is
// c0 + g*64*V + lane*V + v, row rw0 + r; out-of-range rows and columns are
// not written.
template <int R, int C, bool TRANS_OUT>
__device__ __forceinline__ void rep_store(const float (&acc)[R][C], int n_r, int n_c,
                                          float* __restrict__ Z, int64_t z_sr, int64_t z_sc,
                                          int rw0, int c0, int lane) {
    constexpr int V = C >= 4 ? 4 : C, G = C / V;
    if (TRANS_OUT) {
        // the R rows of one column are consecutive in Z (z_sr == 1)
#pragma unroll
        for (int g = 0; g < G; ++g)
#pragma unroll
            for (int v = 0; v < V; ++v) {
                const int col = c0 + g * kWave * V + lane * V + v;
                if (col < n_c) {
                    float* zp = Z + (int64_t)col * z_sc + rw0;
#pragma unroll
                    for (int r = 0; r < R; ++r)
                        if (rw0 + r < n_r) zp[r] = acc[r][g * V + v];
                }
            }
    } else {
#pragma unroll
        for (int r = 0; r < R; ++r) {
            const int row = rw0 + r;
            if (row >= n_r) break;
#pragma unroll
            for (int g = 0; g < G; ++g)
#pragma unroll
                for (int v = 0; v < V; ++v) {
                    const int col = c0 + g * kWave * V + lane * V + v;
                    if (col < n_c) Z[(int64_t)row * z_sr + col] = acc[r][g * V + v];
                }
        }
    }
}

// One tile: rows [r0, r0 + TM) x columns [c0, c0 + TN).  `lds` holds
// LDS_FLOATS floats.  All threads of the block must call it (barriers).
// ESC: some count byte may be 255, meaning "re-read the full int32 count";
// without it the byte is the count (the packing pass reports which holds).
// VEC: float4 loads allowed; BUF (with VEC): buffer-resource loads (the base
// matrix is below 2^31 bytes).  UNR: repetition loop unrolled by two.
template <int R, int C, int W, int KP, bool VEC, bool TRANS_OUT, bool ESC, bool BUF = false,
          int UNR = 1>
__device__ __forceinline__ void rep_uniform_tile(
    int n_r, int n_c, int n_k, const uint8_t* __restrict__ P8, int64_t ldp,
    const int32_t* __restrict__ P32, int64_t p32_sr, int64_t p32_sk,
    const float* __restrict__ Q, int64_t ldq, float* __restrict__ Z, int64_t z_sr, int64_t z_sc,
    int r0, int c0, float* lds) {
    using T = RepTile<R, C, W, KP>;
    constexpr int V = T::V, G = T::G, TN = T::TN;
    const int lane = threadIdx.x & (kWave - 1);
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x / kWave);
    const int rw0 = r0 + wave * R;
    const uint8_t* __restrict__ prow = P8 + (int64_t)rw0 * ldp;

    float acc[R][C];
#pragma unroll
    for (int r = 0; r < R; ++r)
#pragma unroll
        for (int c = 0; c < C; ++c) acc[r][c] = 0.0f;  // Z starts at +0.0

    static_assert(KP == 16 || KP == 8, "the count words of a panel are one dwordx4 / dwordx2 per row");
    const int n_panels = (n_k + KP - 1) / KP;
    float4 stage[T::F4T];
    uint32_t voff[T::F4T];
#pragma unroll
    for (int s = 0; s < T::F4T; ++s) {
        const int e = threadIdx.x + s * W * kWave;
        voff[s] = (uint32_t)(((e / (TN / 4)) * ldq + c0 + (e % (TN / 4)) * 4) * 4);
    }
    if (BUF) panel_load_buf<R, C, W, KP>(stage, Q, ldq, n_k, n_c, 0, voff);
    else panel_load<R, C, W, KP, VEC>(stage, Q, ldq, n_k, n_c, 0, c0);
    panel_store<R, C, W, KP>(stage, lds);
    // counts of the first panel: 16 bytes per row (scalar loads)
    PanelCounts<KP> cw[R];
#pragma unroll
    for (int r = 0; r < R; ++r) cw[r].load(prow + (int64_t)r * ldp);
    __syncthreads();

    for (int p = 0; p < n_panels; ++p) {
        const int k0 = p * KP;
        const float* pan = lds + (p & 1) * (KP * TN);
        const bool more = p + 1 < n_panels;
        if (more) {
            if (BUF) panel_load_buf<R, C, W, KP>(stage, Q, ldq, n_k, n_c, k0 + KP, voff);
            else panel_load<R, C, W, KP, VEC>(stage, Q, ldq, n_k, n_c, k0 + KP, c0);
        }

        // base rows ping-pong through two register sets: row kk + 1 is read from
        // LDS while the additions of row kk run
        float bA[C], bB[C];
        auto lds_row = [&](float* b, int kk) {
            const float* brow = pan + kk * TN + lane * V;
#pragma unroll
            for (int g = 0; g < G; ++g) {
                if constexpr (V == 4) {
                    const float4 t = *reinterpret_cast<const float4*>(brow + g * kWave * V);
                    b[g * 4 + 0] = t.x;
                    b[g * 4 + 1] = t.y;
                    b[g * 4 + 2] = t.z;
                    b[g * 4 + 3] = t.w;
                } else if constexpr (V == 2) {
                    const float2 t = *reinterpret_cast<const float2*>(brow + g * kWave * V);
                    b[g * 2 + 0] = t.x;
                    b[g * 2 + 1] = t.y;
                } else {
                    b[g] = brow[g * kWave];
                }
            }
        };
        lds_row(bA, 0);
#pragma unroll
        for (int kk = 0; kk < KP; ++kk) {
            float* b = (kk & 1) ? bB : bA;
            // row kk's reads are done once no more than row kk + 1's G reads are
            // outstanding (LDS reads return in order): one wait per k, where the
            // compiler would otherwise wait inside every repetition loop
            static_assert(G <= 15, "lgkmcnt holds 4 bits");
            if (kk + 1 < KP) {
                lds_row((kk & 1) ? bA : bB, kk + 1);
                __builtin_amdgcn_s_waitcnt(0xC07F | (G << 8));  // lgkmcnt(G)
            } else {
                __builtin_amdgcn_s_waitcnt(0xC07F);  // lgkmcnt(0)
            }
#pragma unroll
            for (int r = 0; r < R; ++r) {
                const uint32_t word = __builtin_amdgcn_readfirstlane(cw[r].get(kk >> 2));
                const uint32_t field = word & (0xFFu << (8 * (kk & 3)));
                if (field != 0) {  // a zero Rep-factor adds nothing
                    uint32_t rep = field >> (8 * (kk & 3));
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
        }

        if (more) {
            // counts of the next panel (the current ones are spent), then its base rows
#pragma unroll
            for (int r = 0; r < R; ++r)
                cw[r].load(prow + (int64_t)r * ldp + k0 + KP);
            panel_store<R, C, W, KP>(stage, lds + ((p + 1) & 1) * (KP * TN));
        }
        __syncthreads();
    }

    rep_store<R, C, TRANS_OUT>(acc, n_r, n_c, Z, z_sr, z_sc, rw0, c0, lane);
}

}  // namespace afmm

namespace afmm {

// ---------------------------------------------------------------------------
// Direct-load variant of the count-uniform tile: no LDS panel and no
// per-panel barrier.  The W waves of a block own different rows but the same
// 64*C columns, so each base row they read is shared through the compute
// unit's L1; each wave streams its base rows straight into registers, four k
// ahead (two register sets, ping-pong, no copies), and the waves only meet at
// a barrier every SYNC_K rows of k, which bounds how far apart they drift.
// Requires C % 4 == 0 and rows of Q readable in float4 units.
template <int C>
struct DirectBuf {
    float4 v[4][C / 4];
};

template <int C>
__device__ __forceinline__ void direct_load(DirectBuf<C>& d, const float* __restrict__ Q,
                                            int64_t ldq, int n_k, int k0, const int* colo,
                                            const bool* cok) {
#pragma unroll
    for (int kk = 0; kk < 4; ++kk) {
        const int k = k0 + kk;
#pragma unroll
        for (int g = 0; g < C / 4; ++g) {
            float4 v = make_float4(0.f, 0.f, 0.f, 0.f);
            if (k < n_k && cok[g]) v = *reinterpret_cast<const float4*>(Q + (int64_t)k * ldq + colo[g]);
            d.v[kk][g] = v;
        }
    }
}

template <int R, int C, bool ESC>
__device__ __forceinline__ void direct_group(float (&acc)[R][C], const DirectBuf<C>& d,
                                             const uint8_t* __restrict__ prow, int64_t ldp,
                                             const int32_t* __restrict__ P32, int64_t p32_sr,
                                             int64_t p32_sk, int rw0, int k0) {
    uint32_t cw[R];
#pragma unroll
    for (int r = 0; r < R; ++r)
        cw[r] = __builtin_amdgcn_readfirstlane(
            *reinterpret_cast<const uint32_t*>(prow + (int64_t)r * ldp + k0));
#pragma unroll
    for (int kk = 0; kk < 4; ++kk) {
        float b[C];
#pragma unroll
        for (int g = 0; g < C / 4; ++g) {
            b[4 * g + 0] = d.v[kk][g].x;
            b[4 * g + 1] = d.v[kk][g].y;
            b[4 * g + 2] = d.v[kk][g].z;
            b[4 * g + 3] = d.v[kk][g].w;
        }
#pragma unroll
        for (int r = 0; r < R; ++r) {
            uint32_t rep = (cw[r] >> (8 * kk)) & 0xFFu;
            if (rep != 0) {
                if (ESC && rep == 0xFFu) {
                    const int32_t full = __builtin_amdgcn_readfirstlane(
                        P32[(int64_t)(rw0 + r) * p32_sr + (int64_t)(k0 + kk) * p32_sk]);
                    if (full <= 0) continue;  // >= 255 unless changed under the call
                    rep = (uint32_t)full;
                }
                do {
#pragma unroll
                    for (int c = 0; c < C; ++c) acc[r][c] = acc[r][c] + b[c];
                } while (--rep != 0);
            }
        }
    }
}

template <int R, int C, int W, int SYNC_K, bool TRANS_OUT, bool ESC>
__device__ __forceinline__ void rep_direct_tile(
    int n_r, int n_c, int n_k, const uint8_t* __restrict__ P8, int64_t ldp,
    const int32_t* __restrict__ P32, int64_t p32_sr, int64_t p32_sk,
    const float* __restrict__ Q, int64_t ldq, float* __restrict__ Z, int64_t z_sr, int64_t z_sc,
    int r0, int c0) {
    static_assert(C % 4 == 0, "direct tiles read float4 columns");
    static_assert(SYNC_K % 8 == 0, "barrier spacing is a multiple of two groups");
    constexpr int G = C / 4;
    const int lane = threadIdx.x & (kWave - 1);
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x / kWave);
    const int rw0 = r0 + wave * R;
    const uint8_t* __restrict__ prow = P8 + (int64_t)rw0 * ldp;
    int colo[G];
    bool cok[G];
#pragma unroll
    for (int g = 0; g < G; ++g) {
        colo[g] = c0 + g * kWave * 4 + lane * 4;
        cok[g] = colo[g] < n_c;
    }
    float acc[R][C];
#pragma unroll
    for (int r = 0; r < R; ++r)
#pragma unroll
        for (int c = 0; c < C; ++c) acc[r][c] = 0.0f;  // Z starts at +0.0

    DirectBuf<C> ba, bb;
    direct_load<C>(ba, Q, ldq, n_k, 0, colo, cok);
    for (int k0 = 0; k0 < n_k; k0 += 8) {
        direct_load<C>(bb, Q, ldq, n_k, k0 + 4, colo, cok);
        direct_group<R, C, ESC>(acc, ba, prow, ldp, P32, p32_sr, p32_sk, rw0, k0);
        if (k0 + 8 < n_k) direct_load<C>(ba, Q, ldq, n_k, k0 + 8, colo, cok);
        if (k0 + 4 < n_k) direct_group<R, C, ESC>(acc, bb, prow, ldp, P32, p32_sr, p32_sk, rw0, k0 + 4);
        if ((k0 + 8) % SYNC_K == 0) __syncthreads();
    }

#pragma unroll
    for (int r = 0; r < R; ++r) {
        const int row = rw0 + r;
        if (row >= n_r) break;
#pragma unroll
        for (int g = 0; g < G; ++g)
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                const int col = colo[g] + v;
                if (col < n_c) {
                    if (TRANS_OUT)
                        Z[(int64_t)col * z_sc + row] = acc[r][4 * g + v];
                    else
                        Z[(int64_t)row * z_sr + col] = acc[r][4 * g + v];
                }
            }
    }
}

}  // namespace afmm
