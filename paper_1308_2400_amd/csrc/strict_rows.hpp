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
// gate: see AFMM_GATE (nullable).
hipError_t launch_compact_rows(int case_id, const void* X, int64_t ldx, const void* Y,
                               int64_t ldy, int m, int kd, int n, int C, const RowsLists& L,
                               hipStream_t s, const uint32_t* gate = nullptr);
// One list per (band, row) of M (rows x cols, ld; bands of ct columns): the
// entries taking part in an addition, ascending column (the pass both lists
// above are built with).  ent [bands][rows][ct], lens [bands][rows].
hipError_t launch_compact_lists(bool is_int, const void* M, int64_t ld, int rows, int cols,
                                int ct, uint2* ent, int32_t* lens, hipStream_t s);
hipError_t launch_rep_rows(int case_id, int m, int kd, int n, const RowsLists& L, float* Z,
                           int64_t ldz, int C, int W, hipStream_t s,
                           const uint32_t* gate = nullptr);
bool rep_rows_supported(int R, int C, int W, int U, int KP);

// Adds to *out (device) the number of entries of M (rows x cols, ld) that take part
// in an addition: is_int, count > 0; otherwise base != 0.
hipError_t launch_count_nonzero(bool is_int, const void* M, int64_t ld, int rows, int cols,
                                uint64_t* out, hipStream_t s);

// The plain strict call's choice of form on the device, from the density of
// kChooseRows evenly spaced rows of each factor: one block per sampled row
// writes its count of participating entries to part[], then one block turns
// the two sampled densities into four gate words (see AFMM_GATE):
//   gates[0]  the size-keyed form's kernels
//   gates[1]  the count bytes (both count-uniform forms read them)
//   gates[2]  the compacted-base form (mapping 4)
//   gates[3]  the row-list form (mapping 7)
// Exactly one of gates[0], gates[2], gates[3] is set.  Nothing needs clearing
// beforehand.
constexpr int kChooseRows = 128;
constexpr size_t kChooseCtlBytes = 2 * kChooseRows * 8 + 256;  // part[], then gates[]
struct ChooseArgs {
    const void* R;  // real factor, r_rows x r_cols, ld ldr
    int r_rows, r_cols;
    int64_t ldr;
    const void* I;  // integer factor, i_rows x i_cols, ld ldi
    int i_rows, i_cols;
    int64_t ldi;
    double size;              // the size the thresholds are keyed by
    double row_list_max;      // row-list form while d_real * d_int * size <= this
    double sparse_real_max;   // else compacted base while d_real <= this ...
    int allow_sparse_real;    // ... and this is non-zero
    int default_mapping;      // the size-keyed form's mapping
    int32_t* chosen;          // nullable: receives the chosen form's mapping
};
// ctl: kChooseCtlBytes of workspace, 256-byte aligned; the gates sit at
// ctl + 2 * kChooseRows * 8.
hipError_t launch_choose_form(const ChooseArgs& a, uint8_t* ctl, hipStream_t s);
inline uint32_t* choose_gates(uint8_t* ctl) {
    return reinterpret_cast<uint32_t*>(ctl + 2 * kChooseRows * 8);
}

}  // namespace afmm
