// Strict AFMM kernel over the non-zeros of both factors (mapping 7; Section 2,
// bit-exact binary32 repeated addition), for the low-density regime of Section
// 2.2 where d1 * d2 ~ 1/n and the additions grow as n^2.
//
// Two compaction passes list, for every row i of X, its entries with a non-zero
// base or a positive count ({value bits, k}, ascending k), and for every row k
// of Y and band of 64*C columns, its entries likewise ({value bits, column in
// the band}).  A workgroup keeps W rows x 64*C columns of Z in LDS; wave w owns
// row i and walks X's list for i in ascending k; for each k its lanes take Y's
// list for (k, band), 64 entries at a time, read Z[i][j] from LDS, add the base
// the count's number of times and write it back.  Case B: the count X[i,k] is
// the same for the whole wave and the base Y[k,j] differs per lane; case A: the
// base X[i,k] is the wave's and the count Y[k,j] the lane's (a lane loops its own
// count).  Every element receives its additions in ascending k, a k's
// repetitions consecutively, so the bits are those of the sequential loops; the
// work is proportional to the number of (i,k,j) with both entries non-zero.
#include "strict_rows.hpp"

#include <algorithm>

namespace afmm {

size_t rows_lists_bytes(int m, int kd, int n, int C) {
    const int64_t ct = (int64_t)kWave * C;
    const int64_t xcap = round_up(kd, kWave), bands = (n + ct - 1) / ct;
    return (size_t)round_up((int64_t)m * xcap * 8, 256) + (size_t)round_up((int64_t)m * 4, 256) +
           (size_t)round_up(bands * kd * ct * 8, 256) + (size_t)round_up(bands * kd * 4, 256);
}

RowsLists rows_lists_at(uint8_t* p, int m, int kd, int n, int C) {
    const int64_t ct = (int64_t)kWave * C;
    const int64_t xcap = round_up(kd, kWave), bands = (n + ct - 1) / ct;
    RowsLists L;
    L.xcap = xcap;
    L.xent = reinterpret_cast<uint2*>(p);
    p += round_up((int64_t)m * xcap * 8, 256);
    L.xlen = reinterpret_cast<int32_t*>(p);
    p += round_up((int64_t)m * 4, 256);
    L.yent = reinterpret_cast<uint2*>(p);
    p += round_up(bands * kd * ct * 8, 256);
    L.ylen = reinterpret_cast<int32_t*>(p);
    return L;
}

// One wave per segment (band, row): the entries of M[row][band*ct, band*ct + ct)
// that take part in an addition (INT: count > 0; otherwise base != 0, so -0.0
// is dropped and NaN kept), ascending column, at their rank.
template <bool INT>
__global__ __launch_bounds__(256) void compact_rows_kernel(const uint32_t* __restrict__ M,
                                                           int64_t ld, int rows, int cols, int ct,
                                                           int64_t n_segs, uint2* __restrict__ ent,
                                                           int32_t* __restrict__ lens,
                                                           const uint32_t* __restrict__ gate) {
    AFMM_GATE(gate);
    const int lane = threadIdx.x & (kWave - 1);
    const int64_t seg = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
    if (seg >= n_segs) return;  // whole waves
    const int band = (int)(seg / rows);
    const int row = (int)(seg - (int64_t)band * rows);
    const uint32_t* __restrict__ src = M + (int64_t)row * ld + (int64_t)band * ct;
    const int width = min(ct, cols - band * ct);
    uint2* __restrict__ out = ent + seg * ct;
    int count = 0;
    // four chunks of 64 columns per step: their loads go out together, then
    // the chunks are ranked in column order
    for (int ch = 0; ch < width; ch += 4 * kWave) {
        uint32_t v[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            const int c = ch + u * kWave + lane;
            v[u] = c < width ? src[c] : 0u;
        }
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            const int c = ch + u * kWave + lane;
            const bool take = c < width && (INT ? (int32_t)v[u] > 0 : __uint_as_float(v[u]) != 0.0f);
            const uint64_t mk = __ballot(take);
            if (take) {
                const uint32_t below = __builtin_amdgcn_mbcnt_hi(
                    (uint32_t)(mk >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)mk, 0u));
                out[count + (int)below] = make_uint2(v[u], (uint32_t)c);
            }
            count += __popcll(mk);
        }
    }
    if (lane == 0) lens[seg] = count;
}

template <bool INT>
hipError_t launch_compact(const void* M, int64_t ld, int rows, int cols, int ct, uint2* ent,
                          int32_t* lens, hipStream_t s, const uint32_t* gate) {
    const int64_t bands = (cols + ct - 1) / ct;
    const int64_t n_segs = bands * rows;
    hipLaunchKernelGGL(compact_rows_kernel<INT>, dim3((unsigned)((n_segs + 3) / 4)), dim3(256), 0,
                       s, static_cast<const uint32_t*>(M), ld, rows, cols, ct, n_segs, ent, lens,
                       gate);
    return hipGetLastError();
}

hipError_t launch_compact_lists(bool is_int, const void* M, int64_t ld, int rows, int cols,
                                int ct, uint2* ent, int32_t* lens, hipStream_t s) {
    return is_int ? launch_compact<true>(M, ld, rows, cols, ct, ent, lens, s, nullptr)
                  : launch_compact<false>(M, ld, rows, cols, ct, ent, lens, s, nullptr);
}

hipError_t launch_compact_rows(int case_id, const void* X, int64_t ldx, const void* Y,
                               int64_t ldy, int m, int kd, int n, int C, const RowsLists& L,
                               hipStream_t s, const uint32_t* gate) {
    const bool x_int = case_id == 1;  // case B: X holds the counts
    // X: one band as wide as its row (capacity xcap)
    hipError_t e = x_int ? launch_compact<true>(X, ldx, m, kd, (int)L.xcap, L.xent, L.xlen, s, gate)
                         : launch_compact<false>(X, ldx, m, kd, (int)L.xcap, L.xent, L.xlen, s, gate);
    if (e != hipSuccess) return e;
    return x_int ? launch_compact<false>(Y, ldy, kd, n, kWave * C, L.yent, L.ylen, s, gate)
                 : launch_compact<true>(Y, ldy, kd, n, kWave * C, L.yent, L.ylen, s, gate);
}

template <int C, int W>
struct RowsTile {
    static constexpr int CT = kWave * C;   // columns per block (one band)
    static constexpr int STRIDE = CT + 1;  // LDS row pitch in floats
    static constexpr int LDS_FLOATS = W * STRIDE;
    static_assert(LDS_FLOATS * 4 <= 160 * 1024, "the Z rows must fit in LDS");
};

template <int C, int W, bool CASE_A>
__global__ __launch_bounds__(W * kWave) void rep_rows_kernel(
    int m, int kd, int n, const uint2* __restrict__ xent, const int32_t* __restrict__ xlen,
    int64_t xcap, const uint2* __restrict__ yent, const int32_t* __restrict__ ylen,
    float* __restrict__ Z, int64_t ldz, int n_row_blocks, int n_tiles,
    const uint32_t* __restrict__ gate) {
    using T = RowsTile<C, W>;
    __shared__ __attribute__((aligned(16))) float lds[T::LDS_FLOATS];
    AFMM_GATE(gate);
    const int t = xcd_remap(blockIdx.x, n_tiles);
    const int band = t / n_row_blocks, rb = t - band * n_row_blocks;
    const int lane = threadIdx.x & (kWave - 1);
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x / kWave);
    const int i = rb * W + wave;
    const int c0 = band * T::CT;
    float* zrow = lds + wave * T::STRIDE;

    for (int q = threadIdx.x; q < T::LDS_FLOATS; q += W * kWave) lds[q] = 0.0f;  // Z = +0.0
    __syncthreads();

    if (i < m) {
        const uint2* __restrict__ xl = xent + (int64_t)i * xcap;
        const int nx = xlen[i];
        const uint2* __restrict__ yb = yent + (int64_t)band * kd * T::CT;
        const int32_t* __restrict__ yl = ylen + (int64_t)band * kd;
        for (int xc = 0; xc < nx; xc += kWave) {
            // 64 of row i's entries, one per lane, taken one at a time below;
            // each lane also fetches the length of its entry's Y list
            const bool xin = xc + lane < nx;
            const uint2 xe = xin ? xl[xc + lane] : make_uint2(0u, 0u);
            const int lenv = xin ? yl[(int)xe.y] : 0;
            const int cnt = min(kWave, nx - xc);
            // The first 64 entries of entry e's Y list are requested while
            // the three entries before it are processed: the loop takes
            // entries four at a time, each with a register of its own that is
            // refilled for entry e + 4 as soon as entry e is done, so no load
            // result is moved while in flight.  The requests are unconditional
            // (an index past the last entry reads the last entry's list again)
            // so the wait counts stay exact.
#define AFMM_YFETCH(e)                                                                    \
    yb[(int64_t)__builtin_amdgcn_readlane((int)xe.y, min((e), cnt - 1)) * T::CT + lane]
#define AFMM_ADD(yv)                                                                      \
    {                                                                                     \
        const int j = (int)(yv).y;                                                         \
        float z = zrow[j];                                                                \
        /* CASE_A: base X[i,k] for the wave, count Y[k,j] for the lane; else   */    \
        /* count X[i,k] for the wave, base Y[k,j] for the lane.  Two additions */    \
        /* per trip, the same sequence of additions.                           */    \
        const float base = __uint_as_float(CASE_A ? xv : (yv).x);                         \
        int32_t r = (int32_t)(CASE_A ? (yv).x : xv);                                      \
        for (; r >= 2; r -= 2) {                                                          \
            z = z + base;                                                                 \
            z = z + base;                                                                 \
        }                                                                                 \
        if (r > 0) z = z + base;                                                          \
        zrow[j] = z;                                                                      \
    }
#define AFMM_ENTRY(e, yreg)                                                               \
    {                                                                                     \
        if ((e) < cnt) {                                                                  \
            const uint32_t xv = (uint32_t)__builtin_amdgcn_readlane((int)xe.x, (e));      \
            const int len_cur = __builtin_amdgcn_readlane(lenv, (e));                     \
            if (lane < len_cur) AFMM_ADD(yreg)                                            \
            if (len_cur > kWave) {                                                        \
                const int k_cur = __builtin_amdgcn_readlane((int)xe.y, (e));              \
                for (int yc = kWave; yc < len_cur; yc += kWave) {                         \
                    const uint2 y = yb[(int64_t)k_cur * T::CT + yc + lane];               \
                    if (lane < len_cur - yc) AFMM_ADD(y)                                  \
                }                                                                         \
            }                                                                             \
        }                                                                                 \
        yreg = AFMM_YFETCH((e) + 4);                                                      \
    }
            uint2 y0 = AFMM_YFETCH(0), y1 = AFMM_YFETCH(1), y2 = AFMM_YFETCH(2), y3 = AFMM_YFETCH(3);
            for (int e = 0; e < cnt; e += 4) {
                AFMM_ENTRY(e, y0)
                AFMM_ENTRY(e + 1, y1)
                AFMM_ENTRY(e + 2, y2)
                AFMM_ENTRY(e + 3, y3)
            }
#undef AFMM_ENTRY
#undef AFMM_ADD
#undef AFMM_YFETCH
        }
    }
    __syncthreads();
    for (int q = threadIdx.x; q < W * T::CT; q += W * kWave) {
        const int r = q / T::CT, c = q - r * T::CT;
        const int row = rb * W + r;
        if (row < m && c0 + c < n) Z[(int64_t)row * ldz + c0 + c] = lds[r * T::STRIDE + c];
    }
}

template <int C, int W>
hipError_t launch_rows(int case_id, int m, int kd, int n, const RowsLists& L, float* Z,
                       int64_t ldz, hipStream_t s, const uint32_t* gate) {
    using T = RowsTile<C, W>;
    const int n_row_blocks = (m + W - 1) / W;
    const int n_tiles = n_row_blocks * ((n + T::CT - 1) / T::CT);
    dim3 grid(n_tiles), block(W * kWave);
    if (case_id == 0)
        hipLaunchKernelGGL((rep_rows_kernel<C, W, true>), grid, block, 0, s, m, kd, n, L.xent,
                           L.xlen, L.xcap, L.yent, L.ylen, Z, ldz, n_row_blocks, n_tiles, gate);
    else
        hipLaunchKernelGGL((rep_rows_kernel<C, W, false>), grid, block, 0, s, m, kd, n, L.xent,
                           L.xlen, L.xcap, L.yent, L.ylen, Z, ldz, n_row_blocks, n_tiles, gate);
    return hipGetLastError();
}

// (C, W): W rows x 64*C columns of Z in LDS per workgroup
#define AFMM_ROWS_CONFIGS(X) \
    X(64, 8)                 \
    X(32, 16)                \
    X(16, 16)                \
    X(16, 8)

bool rep_rows_supported(int R, int C, int W, int U, int KP) {
    if (R != 1 || U != 1 || KP != 16) return false;
#define AFMM_CASE(c, w) \
    if (C == c && W == w) return true;
    AFMM_ROWS_CONFIGS(AFMM_CASE)
#undef AFMM_CASE
    return false;
}

hipError_t launch_rep_rows(int case_id, int m, int kd, int n, const RowsLists& L, float* Z,
                           int64_t ldz, int C, int W, hipStream_t s, const uint32_t* gate) {
#define AFMM_CASE(c, w) \
    if (C == c && W == w) return launch_rows<c, w>(case_id, m, kd, n, L, Z, ldz, s, gate);
    AFMM_ROWS_CONFIGS(AFMM_CASE)
#undef AFMM_CASE
    return hipErrorInvalidValue;
}

// Entries of a rows x cols matrix (leading dimension ld) that take part in an
// addition (INT: count > 0; otherwise base != 0), summed into *out (cleared by
// the caller).
template <bool INT>
__global__ __launch_bounds__(256) void count_nonzero_kernel(const uint32_t* __restrict__ M,
                                                            int64_t ld, int rows, int cols,
                                                            unsigned long long* __restrict__ out) {
    __shared__ unsigned long long part[4];
    unsigned long long c = 0;
    const int64_t total = (int64_t)rows * cols;
    for (int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x; e < total;
         e += (int64_t)gridDim.x * 256) {
        const int64_t r = e / cols, col = e - r * cols;
        const uint32_t v = M[r * ld + col];
        c += (INT ? (int32_t)v > 0 : __uint_as_float(v) != 0.0f) ? 1u : 0u;
    }
    const int lane = threadIdx.x & (kWave - 1), wave = threadIdx.x >> 6;
    for (int off = kWave / 2; off > 0; off >>= 1) c += __shfl_down(c, off);
    if (lane == 0) part[wave] = c;
    __syncthreads();
    if (threadIdx.x == 0) atomicAdd(out, part[0] + part[1] + part[2] + part[3]);
}

hipError_t launch_count_nonzero(bool is_int, const void* M, int64_t ld, int rows, int cols,
                                uint64_t* out, hipStream_t s) {
    const int64_t total = (int64_t)rows * cols;
    const int blocks = (int)std::min<int64_t>(2048, std::max<int64_t>(1, (total + 255) / 256));
    auto* o = reinterpret_cast<unsigned long long*>(out);
    if (is_int)
        hipLaunchKernelGGL(count_nonzero_kernel<true>, dim3(blocks), dim3(256), 0, s,
                           static_cast<const uint32_t*>(M), ld, rows, cols, o);
    else
        hipLaunchKernelGGL(count_nonzero_kernel<false>, dim3(blocks), dim3(256), 0, s,
                           static_cast<const uint32_t*>(M), ld, rows, cols, o);
    return hipGetLastError();
}

// Block b < kChooseRows counts row b of the real factor's sample, the next
// kChooseRows blocks the integer factor's; a sample row is the middle of its
// stratum of rows / s_eff rows.
__global__ __launch_bounds__(256) void choose_count_kernel(ChooseArgs a,
                                                           unsigned long long* __restrict__ part) {
    __shared__ unsigned long long wsum[4];
    const bool is_int = blockIdx.x >= (unsigned)kChooseRows;
    const int t = (int)blockIdx.x - (is_int ? kChooseRows : 0);
    const int rows = is_int ? a.i_rows : a.r_rows, cols = is_int ? a.i_cols : a.r_cols;
    const int s_eff = rows < kChooseRows ? rows : kChooseRows;
    unsigned long long c = 0;
    if (t < s_eff) {
        const int64_t r = ((int64_t)(2 * t + 1) * rows) / (2 * s_eff);
        const uint32_t* row = static_cast<const uint32_t*>(is_int ? a.I : a.R) +
                              r * (is_int ? a.ldi : a.ldr);
        for (int col = threadIdx.x; col < cols; col += 256) {
            const uint32_t v = row[col];
            c += (is_int ? (int32_t)v > 0 : __uint_as_float(v) != 0.0f) ? 1u : 0u;
        }
    }
    for (int off = kWave / 2; off > 0; off >>= 1) c += __shfl_down(c, off);
    if ((threadIdx.x & (kWave - 1)) == 0) wsum[threadIdx.x >> 6] = c;
    __syncthreads();
    if (threadIdx.x == 0) part[blockIdx.x] = wsum[0] + wsum[1] + wsum[2] + wsum[3];
}

__global__ __launch_bounds__(64) void choose_decide_kernel(ChooseArgs a,
                                                           const unsigned long long* __restrict__ part,
                                                           uint32_t* __restrict__ gates) {
    const int lane = threadIdx.x;
    unsigned long long cr = part[lane] + part[lane + 64];
    unsigned long long ci = part[kChooseRows + lane] + part[kChooseRows + lane + 64];
    for (int off = kWave / 2; off > 0; off >>= 1) {
        cr += __shfl_down(cr, off);
        ci += __shfl_down(ci, off);
    }
    if (lane != 0) return;
    const int sr = a.r_rows < kChooseRows ? a.r_rows : kChooseRows;
    const int si = a.i_rows < kChooseRows ? a.i_rows : kChooseRows;
    const double d_real = (double)cr / ((double)sr * (double)a.r_cols);
    const double d_int = (double)ci / ((double)si * (double)a.i_cols);
    int sel = 0;
    if (d_real * d_int * a.size <= a.row_list_max)
        sel = 7;
    else if (a.allow_sparse_real && d_real <= a.sparse_real_max)
        sel = 4;
    gates[0] = sel == 0;
    gates[1] = sel != 7;
    gates[2] = sel == 4;
    gates[3] = sel == 7;
    if (a.chosen) *a.chosen = sel == 0 ? a.default_mapping : sel;
}

hipError_t launch_choose_form(const ChooseArgs& a, uint8_t* ctl, hipStream_t s) {
    static_assert(kChooseRows == 128, "the decision sums two sample rows per lane");
    auto* part = reinterpret_cast<unsigned long long*>(ctl);
    hipLaunchKernelGGL(choose_count_kernel, dim3(2 * kChooseRows), dim3(256), 0, s, a, part);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(choose_decide_kernel, dim3(1), dim3(64), 0, s, a, part, choose_gates(ctl));
    return hipGetLastError();
}

}  // namespace afmm
