// Host declarations of the strict form over the non-zeros of both factors
// (mapping 7).
#pragma once

#include "common.hpp"

namespace afmm {

// Row lists of X ({value bits, k}, capacity xcap = round_up(kd, 64) per row) and
// band lists of Y ({value bits, column in the band}, capacity 64*C per (band, k)).
struct RowsLists {
    uint2* xent;      // [m][xcap]
    int32_t* xlen;    // [m]
    uint2* yent;      // [bands][kd][64*C]
    int32_t* ylen;    // [bands][kd]
    int64_t xcap;
};
size_t rows_lists_bytes(int m, int kd, int n, int C);
RowsLists rows_lists_at(uint8_t* p, int m, int kd, int n, int C);

// case_id 0 (A: X real, Y counts) or 1 (B: X counts, Y real); X m x kd (ldx),
// Y kd x n (ldy), in elements.
hipError_t launch_compact_rows(int case_id, const void* X, int64_t ldx, const void* Y,
                               int64_t ldy, int m, int kd, int n, int C, const RowsLists& L,
                               hipStream_t s);
hipError_t launch_rep_rows(int case_id, int m, int kd, int n, const RowsLists& L, float* Z,
                           int64_t ldz, int C, int W, hipStream_t s);
bool rep_rows_supported(int R, int C, int W, int U, int KP);

// Adds to *out (device) the number of entries of M (rows x cols, ld) that take part
// in an addition: is_int, count > 0; otherwise base != 0.
hipError_t launch_count_nonzero(bool is_int, const void* M, int64_t ld, int rows, int cols,
                                uint64_t* out, hipStream_t s);

}  // namespace afmm
