// Host declarations of the compacted-base strict form (mapping 4).
#pragma once

#include "common.hpp"

namespace afmm {

// Band of CT = 64 * C lane columns.  The compacted base of band b holds, per k
// in [0, n_k_pad), a segment of CT entries {bits of Q[k][c], c - b*CT} for the
// columns c of the band with a non-zero base, in ascending c, and its length.
constexpr int kAccKPad = 16;  // k padding of the segment table (covers panels of 8 and 16 k)
struct AccLists {
    uint2* ent;       // [n_bands][n_k_pad][CT]
    int32_t* lens;    // [n_bands][n_k_pad]
    int64_t n_k_pad;  // round_up(n_k, 16)
};
size_t acc_lists_bytes(int n_c, int n_k, int C);  // both arrays, each 256-byte aligned
AccLists acc_lists_at(uint8_t* p, int n_c, int n_k, int C);

// gate: see AFMM_GATE (nullable).
hipError_t launch_compact_base(const float* Q, int64_t ldq, int n_k, int n_c, int C,
                               const AccLists& L, hipStream_t s, const uint32_t* gate = nullptr);
hipError_t launch_rep_acc(const StrictArgs& a, const AccLists& L, int R, int C, int W, int U,
                          int KP, hipStream_t s);
bool rep_acc_supported(int R, int C, int W, int U, int KP);
bool rep_acc_usable(const StrictArgs& a, int C);  // 31-bit buffer offsets

}  // namespace afmm
