// Host declarations of the split-BF16x3 form (split.hip).
#pragma once

#include "common.hpp"

namespace afmm {

// split.hip.  The integer factor I (i_rows x i_cols, pitch ldi) becomes the
// bfloat16 plane ip, the real factor R (r_rows x r_cols, pitch ldr) the term
// planes hi, mid, lo; planes are [64 * tiles_o x ld] bfloat16, K-contiguous,
// zero outside the factor.  int_blocks = i_tiles_o * (ld / 64).
struct SplitPrepArgs {
    const int32_t* I;
    int i_rows, i_cols;
    int64_t ldi;
    uint16_t* ip;
    int i_tiles_o;
    const float* R;
    int r_rows, r_cols;
    int64_t ldr;
    uint16_t *hi, *mid, *lo;
    int r_tiles_o;
    int64_t ld;
    int int_blocks;
};
hipError_t launch_split_prep(bool case_a, const SplitPrepArgs& a, hipStream_t s);
// Z (M x N, pitch ldz) from the integer plane I and the term planes S0..S2
// (hi, mid, lo), all with K pitch ld; I has one row per column of Z in case A
// and per row of Z in case B, the term planes the other.
hipError_t launch_gemm_bf16x3(bool case_a, int M, int N, const uint16_t* I, const uint16_t* S0,
                              const uint16_t* S1, const uint16_t* S2, int64_t ld, float* Z,
                              int64_t ldz, hipStream_t s);
int split_real_rows_pad(int n);  // rows of a term plane
int split_int_rows_pad(int n);   // rows of the integer plane

}  // namespace afmm
