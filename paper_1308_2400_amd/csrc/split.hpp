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
    // every row of I (of R) starts 16-byte aligned: 16-byte loads allowed
    bool i_vec = false, r_vec = false;
};
hipError_t launch_split_prep(bool case_a, const SplitPrepArgs& a, hipStream_t s);
// Z (M x N, pitch ldz) from the integer plane I and the term planes S0..S2
// (hi, mid, lo), all with K pitch ld; I has one row per column of Z in case A
// and per row of Z in case B, the term planes the other.
hipError_t launch_gemm_bf16x3(bool case_a, int M, int N, const uint16_t* I, const uint16_t* S0,
                              const uint16_t* S1, const uint16_t* S2, int64_t ld, float* Z,
                              int64_t ldz, hipStream_t s);
// out (rows x cols, row-major) = the plane read back: out[r][c] = plane[c][r]
// (trans) or plane[r][c], plane pitch ld.
hipError_t launch_plane_unpack(const uint16_t* plane, int64_t ld, bool trans, int rows, int cols,
                               uint16_t* out, hipStream_t s);
int split_real_rows_pad(int n);  // rows of a term plane
int split_int_rows_pad(int n);   // rows of the integer plane

// Workspace layout of a split product of an m x k real-or-integer pre-factor
// and a k x n post-factor: K-contiguous bfloat16 planes; the real factor's three
// terms have one row per i (case A) or per j (case B), the integer plane the other.
struct SplitLayout {
    int rows_real, rows_int;  // padded rows of the real-term planes and the integer plane
    int64_t ld;               // K pitch
    size_t planes[4], total;  // byte offsets: hi, mid, lo, then the integer plane
};
SplitLayout split_planes_layout(bool case_a, int m, int k, int n);
// Conversion of X (m x k, pitch ldx) and Y (k x n, pitch ldy) into the planes at base.
hipError_t launch_split_prepare(bool case_a, int m, int k, int n, const void* X, int64_t ldx,
                                const void* Y, int64_t ldy, const SplitLayout& L, uint8_t* base,
                                hipStream_t s);
// Z (m x n, pitch ldz) from the planes at base.
hipError_t launch_split_gemm(bool case_a, int m, int n, const SplitLayout& L, const uint8_t* base,
                             float* Z, int64_t ldz, hipStream_t s);

}  // namespace afmm
