// Shared device helpers and host launcher declarations of libafmm (gfx950).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace afmm {

constexpr int kWave = 64;        // CDNA wavefront width
constexpr int kXcds = 8;         // MI355X: 8 accelerator complex dies, own L2 each
constexpr int kRowPad = 64;      // packed-count rows are padded to this multiple
constexpr int kKPad = 64;        // and the reduction axis too

static inline int64_t round_up(int64_t v, int64_t m) { return (v + m - 1) / m * m; }

// Workgroups of a 1-D grid are dealt to the XCDs round-robin (block b runs on
// XCD b % 8).  Renumber so that each XCD receives one contiguous run of the
// logical tile order; tiles that share operand panels then share an L2.
__device__ __forceinline__ int xcd_remap(int bid, int n_tiles) {
    const int per = n_tiles / kXcds, rem = n_tiles % kXcds;
    const int xcd = bid % kXcds, local = bid / kXcds;
    return xcd < rem ? xcd * (per + 1) + local : rem * (per + 1) + (xcd - rem) * per + local;
}

// A launch queued for a choice made on the device: the kernel leaves at once
// unless its gate word is non-zero (a null gate: it always runs).
#define AFMM_GATE(g)                           \
    do {                                       \
        if ((g) != nullptr && *(g) == 0u) return; \
    } while (0)

// Saturating byte of a repetition count: <= 0 -> 0 (no additions), 1..254 as
// is, >= 255 -> 255, which tells the kernel to re-read the full int32 count.
__device__ __forceinline__ uint32_t count_byte(int32_t v) {
    return v <= 0 ? 0u : (v >= 255 ? 255u : (uint32_t)v);
}

// Counting helpers.  Flag bits as in afmm.h.
constexpr uint32_t kNeg = 1u, kAbove255 = 2u, kAbove256 = 4u, kOverflow = 8u;

__device__ __forceinline__ uint32_t int_flags(int32_t v) {
    return (v < 0 ? kNeg : 0u) | (v > 255 ? kAbove255 : 0u) | (v > 256 ? kAbove256 : 0u);
}

__device__ __forceinline__ uint64_t sat_add(uint64_t a, uint64_t b, uint32_t& fl) {
    uint64_t r;
    if (__builtin_add_overflow(a, b, &r)) {
        fl |= kOverflow;
        return ~0ull;
    }
    return r;
}

__device__ __forceinline__ uint64_t sat_mul(uint64_t a, uint64_t b, uint32_t& fl) {
    uint64_t r;
    if (__builtin_mul_overflow(a, b, &r)) {
        fl |= kOverflow;
        return ~0ull;
    }
    return r;
}

// ---------------------------------------------------------------------------
// Host side.  HIP error code reported by afmm_last_hip_error() (thread-local).
void set_last_hip_error(int e);

// Host launchers (each returns the hipError_t of its launch).

// prep.hip
// Both clear *esc first and set it when some count byte is 255.
// I / X: rows x cols with leading dimension ldi / ldx.
// gate: see AFMM_GATE (nullable).
hipError_t launch_pack_rows(const int32_t* I, int rows, int cols, int64_t ldi, uint8_t* P8,
                            int64_t ldp, int rows_pad, uint32_t* esc, hipStream_t s,
                            const uint32_t* gate = nullptr);
hipError_t launch_pack_transpose(const int32_t* I, int rows, int cols, int64_t ldi, uint8_t* P8,
                                 int64_t ldp, int rows_pad, uint32_t* esc, hipStream_t s,
                                 const uint32_t* gate = nullptr);
hipError_t launch_transpose_f32(const float* X, int rows, int cols, int64_t ldx, float* Xt,
                                int64_t ldq, int rows_pad, hipStream_t s,
                                const uint32_t* gate = nullptr);
// X: m x kd (ldx), Y: kd x n (ldy); wk: kd entries, rows: m entries.
hipError_t launch_count(int case_id, int m, int kd, int n, const void* X, int64_t ldx,
                        const void* Y, int64_t ldy, uint64_t* wk, uint64_t* rows, uint64_t* total,
                        uint32_t* flags, hipStream_t s);

// strict.hip
struct StrictArgs {
    int n_r, n_c, n_k;                       // rows (count-uniform), lanes, reduction
    const uint8_t* P8; int64_t ldp;          // packed counts [rows_pad x ldp]
    const int32_t* P32; int64_t p32_sr, p32_sk;  // original counts (escape 255)
    const float* Q; int64_t ldq;             // base rows k, contiguous over lanes
    float* Z; int64_t z_sr, z_sc;            // output (r, c) at r*z_sr + c*z_sc
    const uint32_t* esc;                     // device word: non-zero if a byte is 255
    bool trans_out;                          // z_sr == 1: output (r, c) at c*z_sc + r
    bool q_padded;                           // Q rows readable up to round_up(n_c, 4)
    const uint32_t* gate = nullptr;          // see AFMM_GATE
};
hipError_t launch_rep_uniform(const StrictArgs& a, int R, int C, int W, int U, int KP,
                              hipStream_t s);
bool rep_uniform_supported(int R, int C, int W, int U, int KP);
hipError_t launch_rep_direct(const StrictArgs& a, int R, int C, int W, hipStream_t s);
bool rep_direct_supported(int R, int C, int W);
bool rep_direct_usable(const StrictArgs& a);  // Q readable in float4 units
// strict_sparse.hip
hipError_t launch_rep_sparse(const StrictArgs& a, int R, int C, int W, int U, int KP,
                             hipStream_t s);
bool rep_sparse_supported(int R, int C, int W, int U, int KP);
bool rep_sparse_usable(const StrictArgs& a);  // float4 rows, 31-bit byte offsets


}  // namespace afmm
