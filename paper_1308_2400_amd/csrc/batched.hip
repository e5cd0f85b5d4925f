// Batched persistent AFMM: many independent strict products of uneven size,
// density and integer range in one persistent launch.  (Split-mode plans run
// the counting kernels and then each product's split conversion and matrix-core
// product; see afmm_batched_plan_create.)
//
// Per launch (captured once into a HIP graph, then replayed):
//   1. reset      per-problem counters and the work-queue head
//   2. prep       count bytes (and the real factor laid out for the lanes) of
//                 every problem, 64 x 64 chunks over a flattened chunk space
//   3. kstat/rows the exact addition count of every problem (Section 2.2) and
//                 the sum of its counts (what the count-uniform mapping issues)
//   4. schedule   one block sorts the problems by cost per tile, largest first,
//                 and lays out the tile queue (longest-processing-time order)
//   5. persistent eight 4-wave blocks per compute unit pull tiles from the
//                 queue with one atomic each and run a strict tile body (the
//                 sparse-k or LDS-panel code of the single-product kernels);
//                 every block leaves when the queue is empty.
#include <algorithm>
#include <cstring>
#include <mutex>
#include <vector>

#include "afmm.h"
#include "sparse_body.hpp"
#include "split.hpp"

namespace afmm {
namespace {

constexpr int kBW = 4;          // waves per persistent block
constexpr int kBKP = 16;        // reduction rows per LDS panel
constexpr int kMaxBatch = 4096; // problems per plan (sort in LDS)

struct BatchProblem {
    int case_id, n;
    const void* X;
    const void* Y;
    float* Z;
    uint8_t* P8;  // count bytes [rows_pad x ldp]
    int64_t ldp;
    float* Q;     // base rows k: case A X^T, case B a padded copy of Y
    int64_t ldq;
    int shape;    // 0: sparse-k R2 C8, 1: sparse-k R2 C4, 2: LDS panel R2 C1 (4 waves)
    int tiles_r, tiles_c;
    int64_t row_start;    // first global row in the counting kernels
    int64_t chunk_start;  // first 64 x 64 chunk in the prep kernel
    int64_t wk_off;       // first per-k weight
};

// Tile shapes: the sparse-k body (16-byte base reads, only the k with a
// non-zero count visited) for the larger problems, the LDS-panel body with one
// column per lane for the small ones (a 256-column tile would be mostly empty).
__host__ __device__ inline int shape_R(int) { return 2; }
__host__ __device__ inline int shape_C(int s) { return s == 0 ? 8 : (s == 1 ? 4 : 1); }
// Size thresholds of the shapes (afmm_set_batch_shapes; the autotuner's
// table): n >= g_n_wide takes shape 0, n >= g_n_mid shape 1, the rest shape 2.
std::mutex g_shape_mu;
int64_t g_n_wide = 512, g_n_mid = 128;
inline int shape_for(int n) {
    std::lock_guard<std::mutex> lk(g_shape_mu);
    return n >= g_n_wide ? 0 : (n >= g_n_mid ? 1 : 2);
}
constexpr int kKP0 = 4, kKP1 = 8;  // k-panel rows of the two sparse-k shapes

// Largest t with start[t] <= v (start ascending, start[0] == 0).
template <typename T>
__device__ __forceinline__ int find_slot(const T* start, int count, int64_t v) {
    int lo = 0, hi = count - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if ((int64_t)start[mid] <= v) lo = mid; else hi = mid - 1;
    }
    return lo;
}

__device__ __forceinline__ int find_problem_chunk(const BatchProblem* P, int count, int64_t v) {
    int lo = 0, hi = count - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (P[mid].chunk_start <= v) lo = mid; else hi = mid - 1;
    }
    return lo;
}

__device__ __forceinline__ int find_problem_row(const BatchProblem* P, int count, int64_t v) {
    int lo = 0, hi = count - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (P[mid].row_start <= v) lo = mid; else hi = mid - 1;
    }
    return lo;
}

// ---------------------------------------------------------------------------
__global__ void batch_reset_kernel(int count, uint64_t* adds, uint64_t* isum, uint32_t* esc,
                                   uint32_t* head, uint32_t* flags) {
    for (int p = blockIdx.x * blockDim.x + threadIdx.x; p < count; p += gridDim.x * blockDim.x) {
        adds[p] = 0;
        isum[p] = 0;
        esc[p] = 0;
    }
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        *head = 0;
        *flags = 0;
    }
}

// One block (64 x 4 threads) per 64 x 64 chunk.
__global__ __launch_bounds__(256) void batch_prep_kernel(const BatchProblem* __restrict__ P,
                                                        int count, int64_t total_chunks,
                                                        uint32_t* __restrict__ esc) {
    __shared__ int32_t ti[64][65];
    __shared__ float tf[64][65];
    const int tx = threadIdx.x, ty = threadIdx.y, tid = ty * 64 + tx;
    for (int64_t ch = blockIdx.x; ch < total_chunks; ch += gridDim.x) {
        const int p = find_problem_chunk(P, count, ch);
        const BatchProblem& b = P[p];
        const int n = b.n, nb = (int)((b.ldp) / 64);
        const int64_t local = ch - b.chunk_start;
        const int a0 = (int)(local / nb) * 64, b0 = (int)(local % nb) * 64;
        bool hit = false;
        if (b.case_id == 1) {
            // counts: rows i = a0.., k = b0..;  base copy: rows k = a0.., columns j = b0..
            const int32_t* X = (const int32_t*)b.X;
            const float* Y = (const float*)b.Y;
            for (int e = tid; e < 64 * 16; e += 256) {
                const int r = a0 + e / 16, k = b0 + (e % 16) * 4;
                uint32_t word = 0;
                if (r < n)
                    for (int t = 0; t < 4; ++t)
                        if (k + t < n) {
                            const uint32_t c = count_byte(X[(int64_t)r * n + k + t]);
                            hit |= c == 255u;
                            word |= c << (8 * t);
                        }
                *reinterpret_cast<uint32_t*>(b.P8 + (int64_t)r * b.ldp + k) = word;
            }
            for (int e = tid; e < 64 * 64; e += 256) {
                const int k = a0 + e / 64, j = b0 + e % 64;
                b.Q[(int64_t)k * b.ldq + j] = (k < n && j < n) ? Y[(int64_t)k * n + j] : 0.0f;
            }
        } else {
            // counts turned: P8[j][k] = Y[k][j] for j = a0.., k = b0..
            const float* X = (const float*)b.X;
            const int32_t* Y = (const int32_t*)b.Y;
            for (int kr = ty; kr < 64; kr += 4) {
                const int k = b0 + kr, j = a0 + tx;
                ti[kr][tx] = (k < n && j < n) ? Y[(int64_t)k * n + j] : 0;
            }
            // base turned: Q[k][i] = X[i][k] for k = a0.., i = b0..
            for (int ir = ty; ir < 64; ir += 4) {
                const int i = b0 + ir, k = a0 + tx;
                tf[ir][tx] = (i < n && k < n) ? X[(int64_t)i * n + k] : 0.0f;
            }
            __syncthreads();
            for (int e = tid; e < 64 * 16; e += 256) {
                const int jr = e / 16, q = e % 16;
                uint32_t word = 0;
                for (int t = 0; t < 4; ++t) {
                    const uint32_t c = count_byte(ti[4 * q + t][jr]);
                    hit |= c == 255u;
                    word |= c << (8 * t);
                }
                *reinterpret_cast<uint32_t*>(b.P8 + (int64_t)(a0 + jr) * b.ldp + b0 + 4 * q) = word;
            }
            for (int kr = ty; kr < 64; kr += 4)
                b.Q[(int64_t)(a0 + kr) * b.ldq + b0 + tx] = tf[tx][kr];
            __syncthreads();
        }
        if (hit) atomicOr(&esc[p], 1u);
    }
}

__device__ __forceinline__ uint64_t wave_sum_sat(uint64_t v, uint32_t& fl) {
    for (int off = 32; off > 0; off >>= 1) {
        const uint64_t o = __shfl_xor(v, off, 64);
        v = sat_add(v, o, fl);
    }
    return v;
}

// One wave per row k of a post-factor: wk = positive sum (case A) or non-zero
// count (case B); case A also adds the row's counts to isum.
__global__ __launch_bounds__(256) void batch_kstat_kernel(const BatchProblem* __restrict__ P,
                                                         int count, int64_t total_rows,
                                                         uint64_t* __restrict__ wk,
                                                         uint64_t* __restrict__ isum,
                                                         uint32_t* __restrict__ flags) {
    const int lane = threadIdx.x & 63;
    const int64_t g = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
    if (g >= total_rows) return;
    const int p = find_problem_row(P, count, g);
    const BatchProblem& b = P[p];
    const int n = b.n;
    const int64_t k = g - b.row_start;
    uint64_t s = 0;
    uint32_t fl = 0;
    if (b.case_id == 0) {
        const int32_t* y = (const int32_t*)b.Y + k * n;
        for (int j = lane; j < n; j += 64) {
            const int32_t v = y[j];
            fl |= int_flags(v);
            if (v > 0) s += (uint64_t)v;
        }
    } else {
        const float* y = (const float*)b.Y + k * n;
        for (int j = lane; j < n; j += 64) s += y[j] != 0.0f ? 1u : 0u;
    }
    s = wave_sum_sat(s, fl);
    for (int off = 32; off > 0; off >>= 1) fl |= __shfl_xor(fl, off, 64);
    if (lane == 0) {
        wk[b.wk_off + k] = s;
        if (b.case_id == 0) atomicAdd((unsigned long long*)&isum[p], (unsigned long long)s);
        if (fl) atomicOr(flags, fl);
    }
}

// One wave per row i of a pre-factor: the row's addition count goes to adds[p].
__global__ __launch_bounds__(256) void batch_rows_kernel(const BatchProblem* __restrict__ P,
                                                        int count, int64_t total_rows,
                                                        const uint64_t* __restrict__ wk,
                                                        uint64_t* __restrict__ adds,
                                                        uint64_t* __restrict__ isum,
                                                        uint32_t* __restrict__ flags) {
    const int lane = threadIdx.x & 63;
    const int64_t g = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
    if (g >= total_rows) return;
    const int p = find_problem_row(P, count, g);
    const BatchProblem& b = P[p];
    const int n = b.n;
    const int64_t i = g - b.row_start;
    const uint64_t* w = wk + b.wk_off;
    uint64_t s = 0, cs = 0;
    uint32_t fl = 0;
    if (b.case_id == 0) {
        const float* x = (const float*)b.X + i * n;
        for (int k = lane; k < n; k += 64)
            if (x[k] != 0.0f) s = sat_add(s, w[k], fl);
    } else {
        const int32_t* x = (const int32_t*)b.X + i * n;
        for (int k = lane; k < n; k += 64) {
            const int32_t v = x[k];
            fl |= int_flags(v);
            if (v > 0) {
                s = sat_add(s, sat_mul((uint64_t)v, w[k], fl), fl);
                cs += (uint64_t)v;
            }
        }
    }
    s = wave_sum_sat(s, fl);
    cs = wave_sum_sat(cs, fl);
    for (int off = 32; off > 0; off >>= 1) fl |= __shfl_xor(fl, off, 64);
    if (lane == 0) {
        const unsigned long long old = atomicAdd((unsigned long long*)&adds[p], (unsigned long long)s);
        if (old + s < old) fl |= kOverflow;
        if (b.case_id == 1) atomicAdd((unsigned long long*)&isum[p], (unsigned long long)cs);
        if (fl) atomicOr(flags, fl);
    }
}

// One block: order problems by estimated cost per tile (largest first) and
// lay out the tile queue.  Cost per tile = the lane additions the count-
// uniform mapping issues for the tile (sum of counts * tile width / row
// tiles) plus a per-(row, k) overhead.
__global__ __launch_bounds__(1024) void batch_schedule_kernel(const BatchProblem* __restrict__ P,
                                                             int count,
                                                             const uint64_t* __restrict__ isum,
                                                             int* __restrict__ order,
                                                             int64_t* __restrict__ tile_start,
                                                             uint32_t* __restrict__ head) {
    __shared__ uint64_t key[kMaxBatch];
    __shared__ int idx[kMaxBatch];
    int n2 = 1;
    while (n2 < count) n2 <<= 1;
    for (int i = threadIdx.x; i < n2; i += blockDim.x) {
        uint64_t k = 0;
        if (i < count) {
            const BatchProblem& b = P[i];
            const int TM = shape_R(b.shape) * kBW, TN = 64 * shape_C(b.shape);
            const double c = (double)isum[i] * TN / b.tiles_r + (double)b.n * TM * 32.0 + 1.0;
            k = c < 1.8e19 ? (uint64_t)c : ~0ull;
        }
        key[i] = k;
        idx[i] = i;
    }
    __syncthreads();
    // bitonic sort, descending by key, ties by ascending index
    for (int size = 2; size <= n2; size <<= 1) {
        for (int stride = size >> 1; stride > 0; stride >>= 1) {
            for (int i = threadIdx.x; i < n2; i += blockDim.x) {
                const int j = i ^ stride;
                if (j > i) {
                    const bool desc = (i & size) == 0;
                    const bool i_first = key[i] > key[j] || (key[i] == key[j] && idx[i] < idx[j]);
                    if (desc != i_first) {
                        const uint64_t tk = key[i];
                        key[i] = key[j];
                        key[j] = tk;
                        const int t = idx[i];
                        idx[i] = idx[j];
                        idx[j] = t;
                    }
                }
            }
            __syncthreads();
        }
    }
    if (threadIdx.x == 0) {
        int64_t acc = 0;
        for (int s = 0; s < count; ++s) {
            const int p = idx[s];
            order[s] = p;
            tile_start[s] = acc;
            acc += (int64_t)P[p].tiles_r * P[p].tiles_c;
        }
        tile_start[count] = acc;
        *head = 0;
    }
}

// KP > 0: the sparse-k body with that k-panel; KP == 0: the LDS-panel body.
// Case A runs as the transposed problem (counts Y[k,j] on rows j, Zᵀ written).
template <int R, int C, int KP, bool TRANS, bool ESC>
__device__ __forceinline__ void run_tile(const BatchProblem& b, int r0, int c0, float* lds) {
    const int n = b.n;
    const int32_t* P32 = (const int32_t*)(TRANS ? b.Y : b.X);
    const int64_t p_sr = TRANS ? 1 : n, p_sk = TRANS ? n : 1;
    const int64_t z_sr = TRANS ? 1 : n, z_sc = TRANS ? n : 1;
    if constexpr (KP > 0)
        rep_sparse_tile<R, C, kBW, KP, TRANS, ESC, 2>(n, n, n, b.P8, b.ldp, P32, p_sr, p_sk, b.Q,
                                                      b.ldq, b.Z, z_sr, z_sc, r0, c0, lds);
    else
        rep_uniform_tile<R, C, kBW, kBKP, true, TRANS, ESC>(n, n, n, b.P8, b.ldp, P32, p_sr, p_sk,
                                                            b.Q, b.ldq, b.Z, z_sr, z_sc, r0, c0,
                                                            lds);
}

template <int R, int C, int KP>
__device__ __forceinline__ void run_shape(const BatchProblem& b, bool esc, int r0, int c0,
                                          float* lds) {
    if (b.case_id == 0) {
        if (esc) run_tile<R, C, KP, true, true>(b, r0, c0, lds);
        else run_tile<R, C, KP, true, false>(b, r0, c0, lds);
    } else {
        if (esc) run_tile<R, C, KP, false, true>(b, r0, c0, lds);
        else run_tile<R, C, KP, false, false>(b, r0, c0, lds);
    }
}

constexpr int kBatchLds =
    std::max(std::max(SparseTile<2, 8, kBW, kKP0>::LDS_FLOATS, SparseTile<2, 4, kBW, kKP1>::LDS_FLOATS),
             RepTile<2, 1, kBW, kBKP>::LDS_FLOATS);

// eight blocks (waves) per compute unit (SIMD): 64 VGPRs, 16 KB of LDS each
__global__ __launch_bounds__(kBW * 64) __attribute__((amdgpu_waves_per_eu(8, 8))) void
batch_persistent_kernel(const BatchProblem* __restrict__ P, int count, const int* __restrict__ order,
                        const int64_t* __restrict__ tile_start, uint32_t* __restrict__ head,
                        const uint32_t* __restrict__ esc) {
    __shared__ __attribute__((aligned(16))) float lds[kBatchLds];
    __shared__ int64_t item_sh;
    const int64_t total = tile_start[count];
    for (;;) {
        if (threadIdx.x == 0) item_sh = (int64_t)atomicAdd(head, 1u);
        __syncthreads();
        const int64_t item = item_sh;
        __syncthreads();
        if (item >= total) break;  // the queue is empty: every block ends here
        const int s = find_slot(tile_start, count, item);
        const int p = order[s];
        const BatchProblem& b = P[p];
        const int64_t local = item - tile_start[s];
        const int tr = (int)(local % b.tiles_r), tc = (int)(local / b.tiles_r);
        const bool e = esc[p] != 0;
        switch (b.shape) {
        case 0: run_shape<2, 8, kKP0>(b, e, tr * 2 * kBW, tc * 512, lds); break;
        case 1: run_shape<2, 4, kKP1>(b, e, tr * 2 * kBW, tc * 256, lds); break;
        default: run_shape<2, 1, 0>(b, e, tr * 2 * kBW, tc * 64, lds); break;
        }
    }
}

}  // namespace
}  // namespace afmm

using namespace afmm;

struct afmm_plan {
    int count = 0;
    afmm_mode mode = AFMM_MODE_STRICT;
    // split mode: each product's operands, plane layout and plane offset in mem
    std::vector<afmm_problem> probs;
    std::vector<SplitLayout> split_layouts;
    std::vector<size_t> split_off;
    int device = 0;
    int64_t total_chunks = 0, total_rows = 0, total_tiles = 0;
    int persist_grid = 0;
    void* mem = nullptr;  // one device allocation for tables and scratch
    BatchProblem* d_probs = nullptr;
    uint64_t *d_adds = nullptr, *d_isum = nullptr, *d_wk = nullptr;
    uint32_t *d_esc = nullptr, *d_head = nullptr, *d_flags = nullptr;
    int* d_order = nullptr;
    int64_t* d_tile_start = nullptr;
    hipStream_t cap = nullptr;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    std::mutex mu;
};

namespace {

afmm_status enqueue(afmm_plan* pl, hipStream_t s) {
    const int count = pl->count;
    hipLaunchKernelGGL(batch_reset_kernel, dim3((count + 255) / 256), dim3(256), 0, s, count,
                       pl->d_adds, pl->d_isum, pl->d_esc, pl->d_head, pl->d_flags);
    if (pl->mode == AFMM_MODE_STRICT) {
        const int prep_grid = (int)std::min<int64_t>(pl->total_chunks, 65536);
        hipLaunchKernelGGL(batch_prep_kernel, dim3(prep_grid), dim3(64, 4), 0, s, pl->d_probs,
                           count, pl->total_chunks, pl->d_esc);
    }
    const int row_blocks = (int)((pl->total_rows + 3) / 4);
    hipLaunchKernelGGL(batch_kstat_kernel, dim3(row_blocks), dim3(256), 0, s, pl->d_probs, count,
                       pl->total_rows, pl->d_wk, pl->d_isum, pl->d_flags);
    hipLaunchKernelGGL(batch_rows_kernel, dim3(row_blocks), dim3(256), 0, s, pl->d_probs, count,
                       pl->total_rows, pl->d_wk, pl->d_adds, pl->d_isum, pl->d_flags);
    if (pl->mode == AFMM_MODE_SPLIT_BF16X3) {
        // the counts above serve afmm_batched_plan_problem_adds; the products
        // are the single-product split form, one conversion and one matrix-core
        // launch each
        uint8_t* m = static_cast<uint8_t*>(pl->mem);
        for (int p = 0; p < count; ++p) {
            const afmm_problem& q = pl->probs[p];
            const bool case_a = q.case_id == AFMM_CASE_A;
            const SplitLayout& L = pl->split_layouts[p];
            uint8_t* base = m + pl->split_off[p];
            hipError_t e = launch_split_prepare(case_a, q.n, q.n, q.n, q.X, q.n, q.Y, q.n, L, base, s);
            if (e == hipSuccess) e = launch_split_gemm(case_a, q.n, q.n, L, base, q.Z, q.n, s);
            if (e != hipSuccess) {
                set_last_hip_error((int)e);
                return AFMM_ERR_HIP;
            }
        }
        const hipError_t e = hipGetLastError();
        if (e != hipSuccess) {
            set_last_hip_error((int)e);
            return AFMM_ERR_HIP;
        }
        return AFMM_OK;
    }
    hipLaunchKernelGGL(batch_schedule_kernel, dim3(1), dim3(1024), 0, s, pl->d_probs, count,
                       pl->d_isum, pl->d_order, pl->d_tile_start, pl->d_head);
    hipLaunchKernelGGL(batch_persistent_kernel, dim3(pl->persist_grid), dim3(kBW * 64), 0, s,
                       pl->d_probs, count, pl->d_order, pl->d_tile_start, pl->d_head, pl->d_esc);
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) {
        set_last_hip_error((int)e);
        return AFMM_ERR_HIP;
    }
    return AFMM_OK;
}

// True when some output Z of the batch overlaps any X, Y or another Z of the
// batch (inputs may share memory with each other).  Sort the address ranges by
// start; a range overlaps an earlier one exactly when it starts below the
// largest end seen so far, so track that end over all ranges and over the Z
// ranges alone.
bool batch_aliases(const afmm_problem* problems, int32_t count) {
    struct Range {
        uintptr_t lo, hi;
        bool z;
    };
    std::vector<Range> r;
    r.reserve(3 * (size_t)count);
    for (int32_t p = 0; p < count; ++p) {
        const size_t bytes = (size_t)problems[p].n * problems[p].n * 4;
        r.push_back({reinterpret_cast<uintptr_t>(problems[p].X),
                     reinterpret_cast<uintptr_t>(problems[p].X) + bytes, false});
        r.push_back({reinterpret_cast<uintptr_t>(problems[p].Y),
                     reinterpret_cast<uintptr_t>(problems[p].Y) + bytes, false});
        r.push_back({reinterpret_cast<uintptr_t>(problems[p].Z),
                     reinterpret_cast<uintptr_t>(problems[p].Z) + bytes, true});
    }
    std::sort(r.begin(), r.end(), [](const Range& a, const Range& b) { return a.lo < b.lo; });
    uintptr_t end_all = 0, end_z = 0;
    for (const Range& x : r) {
        if (x.z ? x.lo < end_all : x.lo < end_z) return true;
        end_all = std::max(end_all, x.hi);
        if (x.z) end_z = std::max(end_z, x.hi);
    }
    return false;
}

}  // namespace

extern "C" {

afmm_status afmm_batched_plan_create(const afmm_problem* problems, int32_t count, afmm_mode mode,
                             afmm_plan** out) {
    if (!out || !problems || count < 1 || count > kMaxBatch) return AFMM_ERR_INVALID_ARG;
    *out = nullptr;
    if (mode != AFMM_MODE_STRICT && mode != AFMM_MODE_SPLIT_BF16X3) return AFMM_ERR_INVALID_ARG;
    for (int32_t p = 0; p < count; ++p) {
        const afmm_problem& q = problems[p];
        if ((q.case_id != AFMM_CASE_A && q.case_id != AFMM_CASE_B) || q.n < 1 ||
            q.n > AFMM_MAX_BATCH_N || !q.X || !q.Y || !q.Z)
            return AFMM_ERR_INVALID_ARG;
        if ((reinterpret_cast<uintptr_t>(q.X) | reinterpret_cast<uintptr_t>(q.Y) |
             reinterpret_cast<uintptr_t>(q.Z)) & 3)
            return AFMM_ERR_INVALID_ARG;
    }
    if (batch_aliases(problems, count)) return AFMM_ERR_ALIAS;
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) return AFMM_ERR_NO_DEVICE;
    hipDeviceProp_t prop;
    if (hipGetDeviceProperties(&prop, dev) != hipSuccess ||
        std::strncmp(prop.gcnArchName, "gfx950", 6) != 0)
        return AFMM_ERR_NO_DEVICE;

    // host-side table and memory layout
    std::vector<BatchProblem> hp(count);
    size_t off = 0;
    auto take = [&](size_t bytes) {
        const size_t at = off;
        off = (off + bytes + 255) / 256 * 256;
        return at;
    };
    const size_t o_probs = take(sizeof(BatchProblem) * count);
    const size_t o_adds = take(8 * (size_t)count), o_isum = take(8 * (size_t)count);
    const size_t o_esc = take(4 * (size_t)count), o_order = take(4 * (size_t)count);
    const size_t o_ts = take(8 * ((size_t)count + 1));
    const size_t o_head = take(4), o_flags = take(4);
    int64_t chunks = 0, rows = 0, tiles = 0;
    std::vector<size_t> o_p8(count), o_q(count);
    for (int32_t p = 0; p < count; ++p) {
        const int n = problems[p].n;
        BatchProblem& b = hp[p];
        b.case_id = problems[p].case_id;
        b.n = n;
        b.X = problems[p].X;
        b.Y = problems[p].Y;
        b.Z = problems[p].Z;
        b.ldp = round_up(n, 64);
        b.ldq = round_up(n, 64);
        b.shape = shape_for(n);
        const int TM = shape_R(b.shape) * kBW, TN = 64 * shape_C(b.shape);
        b.tiles_r = (n + TM - 1) / TM;
        b.tiles_c = (n + TN - 1) / TN;
        b.row_start = rows;
        b.chunk_start = chunks;
        b.wk_off = rows;
        rows += n;
        chunks += (b.ldp / 64) * (b.ldp / 64);
        tiles += (int64_t)b.tiles_r * b.tiles_c;
        if (mode == AFMM_MODE_STRICT) {
            o_p8[p] = take((size_t)b.ldp * b.ldp);
            o_q[p] = take((size_t)b.ldp * b.ldq * 4);
        }
    }
    const size_t o_wk = take(8 * (size_t)rows);

    afmm_plan* pl = new afmm_plan();
    pl->count = count;
    pl->mode = mode;
    if (mode == AFMM_MODE_SPLIT_BF16X3) {
        pl->probs.assign(problems, problems + count);
        pl->split_layouts.resize(count);
        pl->split_off.resize(count);
        for (int32_t p = 0; p < count; ++p) {
            const int n = problems[p].n;
            pl->split_layouts[p] = split_planes_layout(problems[p].case_id == AFMM_CASE_A, n, n, n);
            pl->split_off[p] = take(pl->split_layouts[p].total);
        }
    }
    pl->device = dev;
    pl->total_chunks = chunks;
    pl->total_rows = rows;
    pl->total_tiles = tiles;
    pl->persist_grid = (int)std::min<int64_t>(tiles, (int64_t)prop.multiProcessorCount * 8);
    hipError_t e = hipMalloc(&pl->mem, off);
    if (e != hipSuccess) {
        set_last_hip_error((int)e);
        delete pl;
        return AFMM_ERR_HIP;
    }
    uint8_t* m = static_cast<uint8_t*>(pl->mem);
    for (int32_t p = 0; p < count && mode == AFMM_MODE_STRICT; ++p) {
        hp[p].P8 = m + o_p8[p];
        hp[p].Q = reinterpret_cast<float*>(m + o_q[p]);
    }
    pl->d_probs = reinterpret_cast<BatchProblem*>(m + o_probs);
    pl->d_adds = reinterpret_cast<uint64_t*>(m + o_adds);
    pl->d_isum = reinterpret_cast<uint64_t*>(m + o_isum);
    pl->d_esc = reinterpret_cast<uint32_t*>(m + o_esc);
    pl->d_order = reinterpret_cast<int*>(m + o_order);
    pl->d_tile_start = reinterpret_cast<int64_t*>(m + o_ts);
    pl->d_head = reinterpret_cast<uint32_t*>(m + o_head);
    pl->d_flags = reinterpret_cast<uint32_t*>(m + o_flags);
    pl->d_wk = reinterpret_cast<uint64_t*>(m + o_wk);
    e = hipMemcpy(pl->d_probs, hp.data(), sizeof(BatchProblem) * count, hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipStreamCreateWithFlags(&pl->cap, hipStreamNonBlocking);
    if (e != hipSuccess) {
        set_last_hip_error((int)e);
        (void)hipFree(pl->mem);
        delete pl;
        return AFMM_ERR_HIP;
    }
    *out = pl;
    return AFMM_OK;
}

afmm_status afmm_batched_plan_launch(afmm_plan* pl, hipStream_t stream) {
    if (!pl) return AFMM_ERR_INVALID_ARG;
    std::lock_guard<std::mutex> lk(pl->mu);
    if (!pl->exec) {
        // capture the launch sequence once on the plan's own stream
        hipError_t e = hipStreamBeginCapture(pl->cap, hipStreamCaptureModeRelaxed);
        if (e != hipSuccess) {
            set_last_hip_error((int)e);
            return AFMM_ERR_HIP;
        }
        const afmm_status st = enqueue(pl, pl->cap);
        hipGraph_t g = nullptr;
        e = hipStreamEndCapture(pl->cap, &g);
        if (st != AFMM_OK) {
            if (g) (void)hipGraphDestroy(g);
            return st;
        }
        if (e == hipSuccess) e = hipGraphInstantiate(&pl->exec, g, nullptr, nullptr, 0);
        if (e != hipSuccess) {
            if (g) (void)hipGraphDestroy(g);
            pl->exec = nullptr;
            set_last_hip_error((int)e);
            return AFMM_ERR_HIP;
        }
        pl->graph = g;
    }
    const hipError_t e = hipGraphLaunch(pl->exec, stream);
    if (e != hipSuccess) {
        set_last_hip_error((int)e);
        return AFMM_ERR_HIP;
    }
    return AFMM_OK;
}

afmm_status afmm_batched_plan_problem_adds(const afmm_plan* pl, uint64_t* d_out, hipStream_t stream) {
    if (!pl || !d_out) return AFMM_ERR_INVALID_ARG;
    const hipError_t e = hipMemcpyAsync(d_out, pl->d_adds, 8 * (size_t)pl->count,
                                        hipMemcpyDeviceToDevice, stream);
    if (e != hipSuccess) {
        set_last_hip_error((int)e);
        return AFMM_ERR_HIP;
    }
    return AFMM_OK;
}

afmm_status afmm_batched_plan_destroy(afmm_plan* pl) {
    if (!pl) return AFMM_ERR_INVALID_ARG;
    (void)hipDeviceSynchronize();
    if (pl->exec) (void)hipGraphExecDestroy(pl->exec);
    if (pl->graph) (void)hipGraphDestroy(pl->graph);
    if (pl->cap) (void)hipStreamDestroy(pl->cap);
    if (pl->mem) (void)hipFree(pl->mem);
    delete pl;
    return AFMM_OK;
}

afmm_status afmm_set_batch_shapes(int64_t n_wide, int64_t n_mid) {
    if (n_mid < 1 || n_wide < n_mid) return AFMM_ERR_INVALID_ARG;
    std::lock_guard<std::mutex> lk(g_shape_mu);
    g_n_wide = n_wide;
    g_n_mid = n_mid;
    return AFMM_OK;
}

afmm_status afmm_multiply_batched(const afmm_problem* problems, int32_t count, afmm_mode mode,
                                  hipStream_t stream) {
    afmm_plan* pl = nullptr;
    afmm_status st = afmm_batched_plan_create(problems, count, mode, &pl);
    if (st != AFMM_OK) return st;
    // one-shot: launch the sequence directly on the caller's stream (no graph)
    st = enqueue(pl, stream);
    if (st == AFMM_OK) {
        const hipError_t e = hipStreamSynchronize(stream);
        if (e != hipSuccess) {
            set_last_hip_error((int)e);
            st = AFMM_ERR_HIP;
        }
    }
    afmm_batched_plan_destroy(pl);
    return st;
}

}  // extern "C"
