// C ABI of libafmm (include/afmm.h): argument checks, workspace layout,
// kernel choice and launch order.  No arithmetic of the method happens here.
#include "afmm.h"

#include <algorithm>
#include <cmath>
#include <cstring>
#include <mutex>
#include <string>
#include <vector>

#include "common.hpp"
#include "split.hpp"
#include "strict_acc.hpp"
#include "strict_rows.hpp"

static int& g_last_hip_error_slot() {
    static thread_local int e = 0;
    return e;
}

using namespace afmm;

namespace afmm {
void set_last_hip_error(int e) { g_last_hip_error_slot() = e; }
}  // namespace afmm

namespace {

afmm_status hip_fail(hipError_t e) {
    set_last_hip_error((int)e);
    return AFMM_ERR_HIP;
}

#define AFMM_HIP(call)                                   \
    do {                                                 \
        const hipError_t e_ = (call);                    \
        if (e_ != hipSuccess) return hip_fail(e_);       \
    } while (0)

// ---- device check (once per device) ----------------------------------------
std::mutex g_dev_mu;
std::vector<int> g_dev_ok;  // -1 unknown, 0 bad, 1 gfx950

afmm_status check_device() {
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) return AFMM_ERR_NO_DEVICE;
    std::lock_guard<std::mutex> lk(g_dev_mu);
    if ((int)g_dev_ok.size() <= dev) g_dev_ok.resize(dev + 1, -1);
    if (g_dev_ok[dev] < 0) {
        hipDeviceProp_t prop;
        if (hipGetDeviceProperties(&prop, dev) != hipSuccess) return AFMM_ERR_NO_DEVICE;
        g_dev_ok[dev] = std::strncmp(prop.gcnArchName, "gfx950", 6) == 0 ? 1 : 0;
    }
    return g_dev_ok[dev] ? AFMM_OK : AFMM_ERR_NO_DEVICE;
}

bool overlaps(const void* a, size_t na, const void* b, size_t nb) {
    const uintptr_t x = reinterpret_cast<uintptr_t>(a), y = reinterpret_cast<uintptr_t>(b);
    return x < y + nb && y < x + na;
}

// Problem shape: X is m x k with leading dimension ldx, Y k x n (ldy), Z m x n
// (ldz), all row-major.  The square entry points are m = k = n = every ld.
struct Shape {
    int64_t m, k, n, ldx, ldy, ldz;
};
Shape square(int64_t n) { return Shape{n, n, n, n, n, n}; }

constexpr int64_t kMaxLd = (int64_t)1 << 28;  // element pitch limit (byte offsets in 64 bits)

bool shape_ok(const Shape& p) {
    return p.m >= 1 && p.k >= 1 && p.n >= 1 && p.m <= AFMM_MAX_N && p.k <= AFMM_MAX_N &&
           p.n <= AFMM_MAX_N && p.ldx >= p.k && p.ldy >= p.n && p.ldz >= p.n &&
           p.ldx <= kMaxLd && p.ldy <= kMaxLd && p.ldz <= kMaxLd;
}

// Size the tuning table and the built-in rule are keyed by: the cube root of
// the product of the three extents (n for a square problem).
int64_t shape_size(const Shape& p) {
    if (p.m == p.k && p.k == p.n) return p.n;
    return std::max<int64_t>(1, std::llround(std::cbrt((double)p.m * (double)p.k * (double)p.n)));
}

// Bytes from the first to one past the last element of a rows x cols matrix.
size_t extent(int64_t rows, int64_t cols, int64_t ld) { return (size_t)((rows - 1) * ld + cols) * 4; }

afmm_status check_args(const Shape& p, const void* X, const void* Y, const void* Z) {
    if (!shape_ok(p) || !X || !Y || !Z) return AFMM_ERR_INVALID_ARG;
    const size_t zb = extent(p.m, p.n, p.ldz);
    if (overlaps(Z, zb, X, extent(p.m, p.k, p.ldx)) || overlaps(Z, zb, Y, extent(p.k, p.n, p.ldy)))
        return AFMM_ERR_ALIAS;
    if ((reinterpret_cast<uintptr_t>(X) | reinterpret_cast<uintptr_t>(Y) |
         reinterpret_cast<uintptr_t>(Z)) & 3)
        return AFMM_ERR_INVALID_ARG;
    return AFMM_OK;
}

// ---- workspace layout -------------------------------------------------------
struct Carve {
    size_t off = 0;
    size_t take(size_t bytes) {
        const size_t at = off;
        off = (off + bytes + 255) / 256 * 256;
        return at;
    }
};

struct StrictLayout {
    int rows_pad;
    int64_t ldp, ldq;
    size_t p8, xt, esc, acc, total;
};

// Strict path: count bytes P8 [rows_pad x ldp] of the integer factor, rows
// being the count-uniform side (case B: i < m; case A: j < n) and columns k;
// case A also keeps its real factor transposed, Xt [round_up(k) x ldq], ldq
// covering i < m.  The compacted-base form (mapping 4) adds its lists of
// non-zero bases.
StrictLayout strict_layout(afmm_case c, const Shape& p, const afmm_config& cfg) {
    StrictLayout L;
    if (cfg.mapping == 7) {
        // only the row lists of both factors
        L.rows_pad = 0;
        L.ldp = L.ldq = 0;
        L.p8 = L.xt = L.esc = L.acc = 0;
        L.total = rows_lists_bytes((int)p.m, (int)p.k, (int)p.n, cfg.cols_per_lane);
        return L;
    }
    L.rows_pad = (int)round_up(c == AFMM_CASE_B ? p.m : p.n, kRowPad);
    L.ldp = round_up(p.k, kKPad);
    L.ldq = round_up(p.m, 64);
    Carve cv;
    L.p8 = cv.take((size_t)L.rows_pad * L.ldp);
    L.xt = c == AFMM_CASE_A ? cv.take((size_t)round_up(p.k, kKPad) * L.ldq * 4) : 0;
    L.esc = cv.take(4);
    L.acc = cfg.mapping == 4 ? cv.take(acc_lists_bytes((int)(c == AFMM_CASE_B ? p.n : p.m),
                                                       (int)p.k, cfg.cols_per_lane))
                             : 0;
    L.total = cv.off;
    return L;
}

// count scratch: per-k weights, per-row counts (when the caller passes none),
// flags and total
size_t count_ws(const Shape& p) {
    return (size_t)round_up(p.k * 8, 256) + (size_t)round_up(p.m * 8, 256) + 256 + 256;
}

// Workspace from the caller or from the stream-ordered allocator.
struct Scratch {
    void* ptr = nullptr;
    bool owned = false;
    hipStream_t s = nullptr;
    afmm_status get(void* ws, size_t ws_bytes, size_t need, hipStream_t stream) {
        s = stream;
        if (ws) {
            if (ws_bytes < need) return AFMM_ERR_WORKSPACE;
            ptr = ws;
            return AFMM_OK;
        }
        const hipError_t e = hipMallocAsync(&ptr, need, stream);
        if (e != hipSuccess) return hip_fail(e);
        owned = true;
        return AFMM_OK;
    }
    ~Scratch() {
        if (owned) (void)hipFreeAsync(ptr, s);
    }
    uint8_t* at(size_t off) const { return static_cast<uint8_t*>(ptr) + off; }
};

// ---- strict configurations --------------------------------------------------
struct TuneEntry {
    int32_t c;
    int64_t lo, hi;
    afmm_config cfg;
};
std::mutex g_tune_mu;
std::vector<TuneEntry> g_tune;

bool config_ok(afmm_case c, const afmm_config& g) {
    const int u = g.unroll == 0 ? 1 : g.unroll;
    const int kp = g.k_panel == 0 ? 16 : g.k_panel;
    if (g.mapping == 0)
        return rep_uniform_supported(g.rows_per_wave, g.cols_per_lane, g.waves, u, kp);
    if (g.mapping == 3)
        return rep_sparse_supported(g.rows_per_wave, g.cols_per_lane, g.waves, u, kp);
    if (g.mapping == 4)
        return rep_acc_supported(g.rows_per_wave, g.cols_per_lane, g.waves, u, kp);
    if (g.mapping == 7) return rep_rows_supported(g.rows_per_wave, g.cols_per_lane, g.waves, u, kp);
    if (kp != 16) return false;
    if (u != 1) return false;
    if (g.mapping == 2) return rep_direct_supported(g.rows_per_wave, g.cols_per_lane, g.waves);
    return false;
}

// LDS-panel configurations by size: 16-column lanes once a tile row of 1024
// columns is well filled, smaller tiles below.  Also the fallback of the
// variants whose layout requirements a problem does not meet.
afmm_config lds_config(int64_t n) {
    if (n > 2896) return afmm_config{0, 4, 16, 16, 1, 16};
    if (n > 1448) return afmm_config{0, 4, 4, 8, 1, 16};
    if (n > 512) return afmm_config{0, 4, 2, 4, 2, 16};
    return afmm_config{0, 2, 1, 4, 1, 16};
}

// Built-in rule, used when no tuning table is loaded: what the autotuner picked
// on MI355X.  The sparse-k variant at n = 2048, where its 16-row tiles fill the
// chip, and for case A above 5792 (even with the LDS-panel variant there); the
// LDS-panel variant with 16-column lanes elsewhere above 2896.  The compacted-base
// variant is never picked by size: it wins only on a sparse real factor.
afmm_config builtin_config(afmm_case c, int64_t n) {
    if (c == AFMM_CASE_A && n > 5792) return afmm_config{3, 2, 16, 16, 2, 8};
    if (c == AFMM_CASE_A && n > 2896) return afmm_config{0, 4, 16, 8, 2, 8};
    if (n > 2896) return afmm_config{0, 4, 16, 16, 2, 16};
    if (n > 1448) return afmm_config{3, 1, 16, 16, 1, 8};
    return lds_config(n);
}

// Count bytes (and case A's transposed real factor) into the workspace at
// base, laid out by L, and the kernel arguments over them.  gate: see AFMM_GATE.
afmm_status strict_prepare(afmm_case c, const Shape& p, const void* X, const void* Y, float* Z,
                           const StrictLayout& L, uint8_t* base, const uint32_t* gate,
                           StrictArgs& a, hipStream_t s) {
    uint8_t* P8 = base + L.p8;
    uint32_t* esc = reinterpret_cast<uint32_t*>(base + L.esc);
    a = StrictArgs{};
    a.n_k = (int)p.k;
    a.P8 = P8;
    a.ldp = L.ldp;
    a.Z = Z;
    a.esc = esc;
    if (c == AFMM_CASE_B) {
        // rows i carry the counts X[i,k]; lanes over j read Y[k,j]
        AFMM_HIP(launch_pack_rows(static_cast<const int32_t*>(X), (int)p.m, (int)p.k, p.ldx, P8,
                                  L.ldp, L.rows_pad, esc, s, gate));
        a.n_r = (int)p.m;
        a.n_c = (int)p.n;
        a.P32 = static_cast<const int32_t*>(X);
        a.p32_sr = p.ldx;
        a.p32_sk = 1;
        a.Q = static_cast<const float*>(Y);
        a.ldq = p.ldy;
        a.z_sr = p.ldz;
        a.z_sc = 1;
        a.trans_out = false;
        a.q_padded = false;
    } else {
        // transposed problem: rows j carry the counts Y[k,j]; lanes over i read X[i,k]
        float* Xt = reinterpret_cast<float*>(base + L.xt);
        AFMM_HIP(launch_pack_transpose(static_cast<const int32_t*>(Y), (int)p.k, (int)p.n, p.ldy,
                                       P8, L.ldp, L.rows_pad, esc, s, gate));
        AFMM_HIP(launch_transpose_f32(static_cast<const float*>(X), (int)p.m, (int)p.k, p.ldx, Xt,
                                      L.ldq, (int)round_up(p.k, kKPad), s, gate));
        a.n_r = (int)p.n;
        a.n_c = (int)p.m;
        a.P32 = static_cast<const int32_t*>(Y);
        a.p32_sr = 1;
        a.p32_sk = p.ldy;
        a.Q = Xt;
        a.ldq = L.ldq;
        a.z_sr = 1;
        a.z_sc = p.ldz;
        a.trans_out = true;
        a.q_padded = true;
    }
    return AFMM_OK;
}

// The kernels of a count-uniform configuration (mappings 0, 2, 3, 4) over the
// prepared arguments; lists: the compacted-base lists (mapping 4).
afmm_status strict_launch(const afmm_config& cfg, const Shape& p, const StrictArgs& a,
                          uint8_t* lists, hipStream_t s) {
    if (cfg.mapping == 4 && rep_acc_usable(a, cfg.cols_per_lane)) {
        const AccLists L = acc_lists_at(lists, a.n_c, a.n_k, cfg.cols_per_lane);
        AFMM_HIP(launch_compact_base(a.Q, a.ldq, a.n_k, a.n_c, cfg.cols_per_lane, L, s, a.gate));
        AFMM_HIP(launch_rep_acc(a, L, cfg.rows_per_wave, cfg.cols_per_lane, cfg.waves,
                                cfg.unroll == 0 ? 1 : cfg.unroll,
                                cfg.k_panel == 0 ? 16 : cfg.k_panel, s));
    } else if (cfg.mapping == 2 && rep_direct_usable(a)) {
        AFMM_HIP(launch_rep_direct(a, cfg.rows_per_wave, cfg.cols_per_lane, cfg.waves, s));
    } else if (cfg.mapping == 3 && rep_sparse_usable(a)) {
        AFMM_HIP(launch_rep_sparse(a, cfg.rows_per_wave, cfg.cols_per_lane, cfg.waves,
                                   cfg.unroll == 0 ? 1 : cfg.unroll,
                                   cfg.k_panel == 0 ? 16 : cfg.k_panel, s));
    } else if (cfg.mapping == 2 || cfg.mapping == 3 || cfg.mapping == 4 || cfg.mapping == 0) {
        // the direct and sparse-k variants need float4-readable base rows, the
        // sparse-k and compacted-base ones 31-bit offsets; the LDS-panel variant
        // takes the rest
        const afmm_config d = cfg.mapping == 0 ? cfg : lds_config(shape_size(p));
        AFMM_HIP(launch_rep_uniform(a, d.rows_per_wave, d.cols_per_lane, d.waves,
                                    d.unroll == 0 ? 1 : d.unroll,
                                    d.k_panel == 0 ? 16 : d.k_panel, s));
    } else {
        return AFMM_ERR_UNSUPPORTED;  // config_ok admits no other mapping
    }
    return AFMM_OK;
}

// The row-list form (mapping 7): lists of both factors at base, then the kernel.
afmm_status rows_launch(afmm_case c, const Shape& p, const void* X, const void* Y, float* Z,
                        const afmm_config& cfg, uint8_t* base, const uint32_t* gate,
                        hipStream_t s) {
    const int cid = c == AFMM_CASE_A ? 0 : 1;
    const RowsLists lists = rows_lists_at(base, (int)p.m, (int)p.k, (int)p.n, cfg.cols_per_lane);
    AFMM_HIP(launch_compact_rows(cid, X, p.ldx, Y, p.ldy, (int)p.m, (int)p.k, (int)p.n,
                                 cfg.cols_per_lane, lists, s, gate));
    AFMM_HIP(launch_rep_rows(cid, (int)p.m, (int)p.k, (int)p.n, lists, Z, p.ldz,
                             cfg.cols_per_lane, cfg.waves, s, gate));
    return AFMM_OK;
}

afmm_status strict_run(afmm_case c, const Shape& p, const void* X, const void* Y, float* Z,
                       const afmm_config& cfg, void* ws, size_t ws_bytes, hipStream_t s) {
    const StrictLayout L = strict_layout(c, p, cfg);
    Scratch sc;
    afmm_status st = sc.get(ws, ws_bytes, L.total, s);
    if (st != AFMM_OK) return st;
    if (cfg.mapping == 7) return rows_launch(c, p, X, Y, Z, cfg, sc.at(0), nullptr, s);
    StrictArgs a;
    if ((st = strict_prepare(c, p, X, Y, Z, L, sc.at(0), nullptr, a, s)) != AFMM_OK) return st;
    return strict_launch(cfg, p, a, sc.at(L.acc), s);
}

// ---- the plain strict call's choice of form, made on the device -------------
// Below this size the size-keyed configuration is right for any density.
constexpr int64_t kAdaptMin = 1024;

// The two forms for sparse factors the plain call may choose instead of the
// size-keyed one (what afmm_suggest_config returns).
afmm_config sparse_real_config(int64_t size) {
    (void)size;  // the best compacted-base shape at n = 2048 .. 16384
    return afmm_config{4, 2, 16, 8, 1, 16};
}
afmm_config row_list_config(int64_t size) {
    return afmm_config{7, 1, size <= 2896 ? 16 : 32, 16, 1, 16};
}
// d_real * d_int * size at or below which the row-list form wins
double row_list_threshold(afmm_case c) { return c == AFMM_CASE_A ? 32.0 : 64.0; }
constexpr double kSparseRealMax = 0.06;  // d_real at or below which the compacted base wins

// Above this size the lists of the two sparse forms (up to 24 bytes per entry
// of a factor) would cost more memory than the choice is worth.
constexpr int64_t kAdaptMax = 16384;

bool adaptive(afmm_case c, const Shape& p, const afmm_config& d) {
    (void)c;
    const int64_t size = shape_size(p);
    return size >= kAdaptMin && size <= kAdaptMax &&
           std::max({p.m, p.k, p.n}) <= kAdaptMax &&
           (d.mapping == 0 || d.mapping == 2 || d.mapping == 3);
}

// Workspace of the adaptive strict call: the choice's control words, then the
// count bytes and transposed factor of the count-uniform forms, then one region
// holding either form's lists (only the chosen form writes there).
struct AdaptiveLayout {
    StrictLayout L;  // offsets relative to base = workspace + kCtlBytes
    size_t lists, total;
};
constexpr size_t kCtlBytes = (kChooseCtlBytes + 255) / 256 * 256;
static_assert(kCtlBytes <= 4096, "afmm_plain_form documents 4096 bytes of workspace");

AdaptiveLayout adaptive_layout(afmm_case c, const Shape& p) {
    AdaptiveLayout A;
    const int64_t size = shape_size(p);
    const afmm_config c4 = sparse_real_config(size), c7 = row_list_config(size);
    A.L = strict_layout(c, p, c4);
    const size_t acc = acc_lists_bytes((int)(c == AFMM_CASE_B ? p.n : p.m), (int)p.k,
                                       c4.cols_per_lane);
    const size_t rows = rows_lists_bytes((int)p.m, (int)p.k, (int)p.n, c7.cols_per_lane);
    A.lists = A.L.acc;
    A.total = kCtlBytes + A.L.acc + std::max(acc, rows);
    return A;
}

// Launches the choice of form over the control words at ctl (kChooseCtlBytes).
// adapt false: the choice is the size-keyed form whatever the density.
hipError_t choose_form(afmm_case c, const Shape& p, const void* X, const void* Y,
                       const afmm_config& d, bool adapt, uint8_t* ctl, int32_t* chosen,
                       hipStream_t s) {
    const int64_t size = shape_size(p);
    const bool case_a = c == AFMM_CASE_A;
    // the real factor: X (m x k) in case A, Y (k x n) in case B; the counts the other
    ChooseArgs ch;
    ch.R = case_a ? X : Y;
    ch.r_rows = (int)(case_a ? p.m : p.k);
    ch.r_cols = (int)(case_a ? p.k : p.n);
    ch.ldr = case_a ? p.ldx : p.ldy;
    ch.I = case_a ? Y : X;
    ch.i_rows = (int)(case_a ? p.k : p.m);
    ch.i_cols = (int)(case_a ? p.n : p.k);
    ch.ldi = case_a ? p.ldy : p.ldx;
    ch.size = (double)size;
    ch.row_list_max = row_list_threshold(c);
    ch.sparse_real_max = kSparseRealMax;
    // the compacted-base form needs 31-bit offsets over its lists and count bytes
    StrictArgs probe{};
    probe.n_r = (int)(case_a ? p.n : p.m);
    probe.n_c = (int)(case_a ? p.m : p.n);
    probe.n_k = (int)p.k;
    probe.ldp = round_up(p.k, kKPad);
    ch.allow_sparse_real = rep_acc_usable(probe, sparse_real_config(size).cols_per_lane) ? 1 : 0;
    if (!adapt) {
        ch.row_list_max = -1.0;
        ch.allow_sparse_real = 0;
    }
    ch.default_mapping = d.mapping;
    ch.chosen = chosen;
    return launch_choose_form(ch, ctl, s);
}

afmm_status strict_adaptive(afmm_case c, const Shape& p, const void* X, const void* Y, float* Z,
                            const afmm_config& d, void* ws, size_t ws_bytes, hipStream_t s) {
    const int64_t size = shape_size(p);
    const afmm_config c4 = sparse_real_config(size), c7 = row_list_config(size);
    const AdaptiveLayout A = adaptive_layout(c, p);
    Scratch sc;
    afmm_status st = sc.get(ws, ws_bytes, A.total, s);
    if (st != AFMM_OK) return st;
    uint8_t* ctl = sc.at(0);
    uint8_t* base = sc.at(kCtlBytes);
    AFMM_HIP(choose_form(c, p, X, Y, d, true, ctl, nullptr, s));
    const uint32_t* gates = choose_gates(ctl);
    const uint32_t* g_default = gates + 0;  // the size-keyed form's kernels
    const uint32_t* g_counts = gates + 1;   // count bytes (either count-uniform form)
    const uint32_t* g_sparse_real = gates + 2;
    const uint32_t* g_row_list = gates + 3;
    StrictArgs a;
    if ((st = strict_prepare(c, p, X, Y, Z, A.L, base, g_counts, a, s)) != AFMM_OK) return st;
    a.gate = g_default;
    if ((st = strict_launch(d, p, a, base + A.lists, s)) != AFMM_OK) return st;
    a.gate = g_sparse_real;
    if ((st = strict_launch(c4, p, a, base + A.lists, s)) != AFMM_OK) return st;
    return rows_launch(c, p, X, Y, Z, c7, base + A.lists, g_row_list, s);
}

SplitLayout split_layout(afmm_case c, const Shape& p) {
    return split_planes_layout(c == AFMM_CASE_A, (int)p.m, (int)p.k, (int)p.n);
}

afmm_status split_run(afmm_case c, const Shape& p, const void* X, const void* Y, float* Z,
                      void* ws, size_t ws_bytes, hipStream_t s) {
    const SplitLayout L = split_layout(c, p);
    Scratch sc;
    const afmm_status st = sc.get(ws, ws_bytes, L.total, s);
    if (st != AFMM_OK) return st;
    const bool case_a = c == AFMM_CASE_A;
    AFMM_HIP(launch_split_prepare(case_a, (int)p.m, (int)p.k, (int)p.n, X, p.ldx, Y, p.ldy, L,
                                  sc.at(0), s));
    AFMM_HIP(launch_split_gemm(case_a, (int)p.m, (int)p.n, L, sc.at(0), Z, p.ldz, s));
    return AFMM_OK;
}

size_t workspace_for(afmm_case c, const Shape& p, afmm_mode mode) {
    if (mode == AFMM_MODE_SPLIT_BF16X3) return split_layout(c, p).total;
    const afmm_config cfg = afmm_default_config(c, shape_size(p));
    const size_t strict = adaptive(c, p, cfg) ? adaptive_layout(c, p).total
                                              : strict_layout(c, p, cfg).total;
    return std::max(strict, count_ws(p));
}

afmm_status multiply(afmm_case c, const Shape& p, const void* X, const void* Y, float* Z,
                     afmm_mode mode, void* ws, size_t ws_bytes, hipStream_t s) {
    afmm_status st = check_args(p, X, Y, Z);
    if (st != AFMM_OK) return st;
    if (mode != AFMM_MODE_STRICT && mode != AFMM_MODE_SPLIT_BF16X3) return AFMM_ERR_INVALID_ARG;
    if ((st = check_device()) != AFMM_OK) return st;
    if (mode == AFMM_MODE_STRICT) {
        const afmm_config d = afmm_default_config(c, shape_size(p));
        if (adaptive(c, p, d)) return strict_adaptive(c, p, X, Y, Z, d, ws, ws_bytes, s);
        return strict_run(c, p, X, Y, Z, d, ws, ws_bytes, s);
    }
    return split_run(c, p, X, Y, Z, ws, ws_bytes, s);
}

afmm_status count_adds(afmm_case c, const Shape& p, const void* X, const void* Y,
                       uint64_t* d_total, uint64_t* d_row_counts, uint32_t* d_flags, void* ws,
                       size_t ws_bytes, hipStream_t stream) {
    if (!shape_ok(p) || !X || !Y || !d_total || (c != AFMM_CASE_A && c != AFMM_CASE_B))
        return AFMM_ERR_INVALID_ARG;
    afmm_status st = check_device();
    if (st != AFMM_OK) return st;
    Scratch sc;
    if ((st = sc.get(ws, ws_bytes, count_ws(p), stream)) != AFMM_OK) return st;
    const size_t wk_bytes = (size_t)round_up(p.k * 8, 256);
    uint64_t* wk = reinterpret_cast<uint64_t*>(sc.at(0));
    uint64_t* rows = d_row_counts ? d_row_counts : reinterpret_cast<uint64_t*>(sc.at(wk_bytes));
    uint32_t* flags = d_flags ? d_flags
                              : reinterpret_cast<uint32_t*>(
                                    sc.at(wk_bytes + (size_t)round_up(p.m * 8, 256)));
    AFMM_HIP(launch_count((int)c, (int)p.m, (int)p.k, (int)p.n, X, p.ldx, Y, p.ldy, wk, rows,
                          d_total, flags, stream));
    return AFMM_OK;
}

}  // namespace

namespace afmm {

afmm_status strict_product_in(afmm_case c, int64_t n, const void* X, const void* Y, float* Z,
                              void* ws, size_t ws_bytes, hipStream_t s) {
    if (c != AFMM_CASE_A && c != AFMM_CASE_B) return AFMM_ERR_INVALID_ARG;
    afmm_status st = check_args(square(n), X, Y, Z);
    if (st != AFMM_OK) return st;
    if ((st = check_device()) != AFMM_OK) return st;
    const afmm_config cfg = afmm_default_config(c, n);
    if (strict_layout(c, square(n), cfg).total > ws_bytes) return AFMM_ERR_WORKSPACE;
    return strict_run(c, square(n), X, Y, Z, cfg, ws, ws_bytes, s);
}

}  // namespace afmm

extern "C" {

size_t afmm_workspace_size(afmm_case c, int64_t n, afmm_mode mode) {
    if (n < 1 || n > AFMM_MAX_N || (c != AFMM_CASE_A && c != AFMM_CASE_B)) return 0;
    return workspace_for(c, square(n), mode);
}

size_t afmm_workspace_size_config(afmm_case c, int64_t n, const afmm_config* cfg) {
    if (n < 1 || n > AFMM_MAX_N || (c != AFMM_CASE_A && c != AFMM_CASE_B) || !cfg ||
        !config_ok(c, *cfg))
        return 0;
    return std::max(strict_layout(c, square(n), *cfg).total, count_ws(square(n)));
}

size_t afmm_workspace_size_ex(afmm_case c, int64_t m, int64_t k, int64_t n, afmm_mode mode) {
    const Shape p{m, k, n, k, n, n};
    if (!shape_ok(p) || (c != AFMM_CASE_A && c != AFMM_CASE_B)) return 0;
    return workspace_for(c, p, mode);
}

afmm_status afmm_multiply_caseA(int64_t n, const float* X, const int32_t* Y, float* Z,
                                afmm_mode mode, void* workspace, size_t workspace_bytes,
                                hipStream_t stream) {
    return multiply(AFMM_CASE_A, square(n), X, Y, Z, mode, workspace, workspace_bytes, stream);
}

afmm_status afmm_multiply_caseB(int64_t n, const int32_t* X, const float* Y, float* Z,
                                afmm_mode mode, void* workspace, size_t workspace_bytes,
                                hipStream_t stream) {
    return multiply(AFMM_CASE_B, square(n), X, Y, Z, mode, workspace, workspace_bytes, stream);
}

afmm_status afmm_multiply_caseA_ex(int64_t m, int64_t k, int64_t n, const float* X, int64_t ldx,
                                   const int32_t* Y, int64_t ldy, float* Z, int64_t ldz,
                                   afmm_mode mode, void* workspace, size_t workspace_bytes,
                                   hipStream_t stream) {
    return multiply(AFMM_CASE_A, Shape{m, k, n, ldx, ldy, ldz}, X, Y, Z, mode, workspace,
                    workspace_bytes, stream);
}

afmm_status afmm_multiply_caseB_ex(int64_t m, int64_t k, int64_t n, const int32_t* X, int64_t ldx,
                                   const float* Y, int64_t ldy, float* Z, int64_t ldz,
                                   afmm_mode mode, void* workspace, size_t workspace_bytes,
                                   hipStream_t stream) {
    return multiply(AFMM_CASE_B, Shape{m, k, n, ldx, ldy, ldz}, X, Y, Z, mode, workspace,
                    workspace_bytes, stream);
}

afmm_status afmm_count_adds(afmm_case c, int64_t n, const void* X, const void* Y,
                            uint64_t* d_total, uint64_t* d_row_counts, uint32_t* d_flags,
                            void* workspace, size_t workspace_bytes, hipStream_t stream) {
    if (n < 1 || n > AFMM_MAX_N) return AFMM_ERR_INVALID_ARG;
    return count_adds(c, square(n), X, Y, d_total, d_row_counts, d_flags, workspace,
                      workspace_bytes, stream);
}

afmm_status afmm_count_adds_ex(afmm_case c, int64_t m, int64_t k, int64_t n, const void* X,
                               int64_t ldx, const void* Y, int64_t ldy, uint64_t* d_total,
                               uint64_t* d_row_counts, uint32_t* d_flags, void* workspace,
                               size_t workspace_bytes, hipStream_t stream) {
    return count_adds(c, Shape{m, k, n, ldx, ldy, n}, X, Y, d_total, d_row_counts, d_flags,
                      workspace, workspace_bytes, stream);
}

afmm_status afmm_split_terms(afmm_case c, int64_t n, const void* X, const void* Y,
                             uint16_t* d_terms, uint16_t* d_ints, void* workspace,
                             size_t workspace_bytes, hipStream_t stream) {
    if (n < 1 || n > AFMM_MAX_N || !X || !Y || !d_terms || !d_ints ||
        (c != AFMM_CASE_A && c != AFMM_CASE_B))
        return AFMM_ERR_INVALID_ARG;
    afmm_status st = check_device();
    if (st != AFMM_OK) return st;
    const Shape p = square(n);
    const SplitLayout L = split_layout(c, p);
    Scratch sc;
    if ((st = sc.get(workspace, workspace_bytes, L.total, stream)) != AFMM_OK) return st;
    const bool case_a = c == AFMM_CASE_A;
    AFMM_HIP(launch_split_prepare(case_a, (int)n, (int)n, (int)n, X, n, Y, n, L, sc.at(0),
                                  stream));
    const uint16_t* P[4];
    for (int q = 0; q < 4; ++q) P[q] = reinterpret_cast<const uint16_t*>(sc.at(L.planes[q]));
    // the real factor's planes are [i][k] in case A (its own orientation) and
    // [j][k] in case B (turned); the integer plane the other way round
    const size_t nn = (size_t)n * (size_t)n;
    for (int q = 0; q < 3; ++q)
        AFMM_HIP(launch_plane_unpack(P[q], L.ld, !case_a, (int)n, (int)n, d_terms + q * nn, stream));
    AFMM_HIP(launch_plane_unpack(P[3], L.ld, case_a, (int)n, (int)n, d_ints, stream));
    return AFMM_OK;
}

afmm_status afmm_base_lists(const float* Q, int64_t k, int64_t n_c, int64_t ldq, int32_t C,
                            uint32_t* d_entries, int32_t* d_lens, hipStream_t stream) {
    if (!Q || !d_entries || !d_lens || k < 1 || k > AFMM_MAX_N || n_c < 1 || n_c > AFMM_MAX_N ||
        ldq < n_c || ldq > kMaxLd || C < 1 || C > 64)
        return AFMM_ERR_INVALID_ARG;
    afmm_status st = check_device();
    if (st != AFMM_OK) return st;
    AccLists L;
    L.ent = reinterpret_cast<uint2*>(d_entries);
    L.lens = d_lens;
    L.n_k_pad = round_up(k, kAccKPad);
    AFMM_HIP(launch_compact_base(Q, ldq, (int)k, (int)n_c, C, L, stream));
    return AFMM_OK;
}

afmm_status afmm_row_lists(int32_t is_int, const void* M, int64_t rows, int64_t cols, int64_t ld,
                           int64_t band, uint32_t* d_entries, int32_t* d_lens,
                           hipStream_t stream) {
    if (!M || !d_entries || !d_lens || (is_int != 0 && is_int != 1) || rows < 1 ||
        rows > AFMM_MAX_N || cols < 1 || cols > AFMM_MAX_N || ld < cols || ld > kMaxLd ||
        band < 1 || band > AFMM_MAX_N)
        return AFMM_ERR_INVALID_ARG;
    const int64_t segs = (cols + band - 1) / band * rows;
    if (segs > ((int64_t)1 << 31)) return AFMM_ERR_INVALID_ARG;  // grid of segs / 4 blocks
    afmm_status st = check_device();
    if (st != AFMM_OK) return st;
    AFMM_HIP(launch_compact_lists(is_int != 0, M, ld, (int)rows, (int)cols, (int)band,
                                  reinterpret_cast<uint2*>(d_entries), d_lens, stream));
    return AFMM_OK;
}

afmm_status afmm_validate(afmm_case c, int64_t n, const void* X, const void* Y, afmm_mode mode,
                          hipStream_t stream) {
    if (mode != AFMM_MODE_STRICT && mode != AFMM_MODE_SPLIT_BF16X3) return AFMM_ERR_INVALID_ARG;
    if (n < 1 || n > AFMM_MAX_N || !X || !Y || (c != AFMM_CASE_A && c != AFMM_CASE_B))
        return AFMM_ERR_INVALID_ARG;
    afmm_status st = check_device();
    if (st != AFMM_OK) return st;
    void* buf = nullptr;
    const size_t cws = count_ws(square(n));
    AFMM_HIP(hipMallocAsync(&buf, cws + 256, stream));
    uint8_t* b = static_cast<uint8_t*>(buf);
    uint64_t* total = reinterpret_cast<uint64_t*>(b + cws);
    uint32_t* flags = reinterpret_cast<uint32_t*>(b + cws + 8);
    st = afmm_count_adds(c, n, X, Y, total, nullptr, flags, b, cws, stream);
    uint32_t hflags = 0;
    if (st == AFMM_OK) {
        hipError_t e = hipMemcpyAsync(&hflags, flags, 4, hipMemcpyDeviceToHost, stream);
        if (e == hipSuccess) e = hipStreamSynchronize(stream);
        if (e != hipSuccess) st = hip_fail(e);
    }
    (void)hipFreeAsync(buf, stream);
    if (st != AFMM_OK) return st;
    if (hflags & AFMM_FLAG_NEGATIVE) return AFMM_ERR_NEGATIVE_INT;
    if (mode == AFMM_MODE_SPLIT_BF16X3 && (hflags & AFMM_FLAG_ABOVE256)) return AFMM_ERR_INT_RANGE;
    if (hflags & AFMM_FLAG_OVERFLOW) return AFMM_ERR_COUNT_OVERFLOW;
    return AFMM_OK;
}

afmm_status afmm_suggest_config(afmm_case c, int64_t n, const void* X, const void* Y,
                                hipStream_t stream, afmm_config* out) {
    if (n < 1 || n > AFMM_MAX_N || !X || !Y || !out || (c != AFMM_CASE_A && c != AFMM_CASE_B))
        return AFMM_ERR_INVALID_ARG;
    afmm_status st = check_device();
    if (st != AFMM_OK) return st;
    *out = afmm_default_config(c, n);
    if (n < kAdaptMin) return AFMM_OK;  // below this the size-keyed choice holds for any density
    void* buf = nullptr;
    hipError_t e = hipMallocAsync(&buf, 16, stream);
    if (e != hipSuccess) return hip_fail(e);
    uint64_t* cnt = static_cast<uint64_t*>(buf);
    uint64_t h[2] = {0, 0};
    const void* real = c == AFMM_CASE_A ? X : Y;
    const void* ints = c == AFMM_CASE_A ? Y : X;
    e = hipMemsetAsync(cnt, 0, 16, stream);
    if (e == hipSuccess) e = launch_count_nonzero(false, real, n, (int)n, (int)n, cnt, stream);
    if (e == hipSuccess) e = launch_count_nonzero(true, ints, n, (int)n, (int)n, cnt + 1, stream);
    if (e == hipSuccess) e = hipMemcpyAsync(h, cnt, 16, hipMemcpyDeviceToHost, stream);
    if (e == hipSuccess) e = hipStreamSynchronize(stream);
    (void)hipFreeAsync(buf, stream);
    if (e != hipSuccess) return hip_fail(e);
    const double nn = (double)n * (double)n;
    const double d_real = (double)h[0] / nn, d_int = (double)h[1] / nn;
    // thresholds from measurements on MI355X (n = 2048..16384): the row-list form
    // while a row meets few non-zero pairs per k (d_real * d_int * n, its work per
    // k of a row, is at most 32 in case A, where a lane loops its own count, and
    // 64 in case B), the compacted-base form when the real factor alone is very
    // sparse, the size-keyed choice otherwise
    if (d_real * d_int * (double)n <= row_list_threshold(c))
        *out = row_list_config(n);
    else if (d_real <= kSparseRealMax)
        *out = sparse_real_config(n);
    return AFMM_OK;
}

afmm_status afmm_plain_form(afmm_case c, int64_t n, const void* X, const void* Y,
                            int32_t* d_mapping, void* workspace, size_t workspace_bytes,
                            hipStream_t stream) {
    if (n < 1 || n > AFMM_MAX_N || !X || !Y || !d_mapping ||
        (c != AFMM_CASE_A && c != AFMM_CASE_B))
        return AFMM_ERR_INVALID_ARG;
    afmm_status st = check_device();
    if (st != AFMM_OK) return st;
    const Shape p = square(n);
    const afmm_config d = afmm_default_config(c, n);
    Scratch sc;
    if ((st = sc.get(workspace, workspace_bytes, kCtlBytes, stream)) != AFMM_OK) return st;
    AFMM_HIP(choose_form(c, p, X, Y, d, adaptive(c, p, d), sc.at(0), d_mapping, stream));
    return AFMM_OK;
}

int afmm_config_supported(afmm_case c, const afmm_config* cfg) {
    if (!cfg || (c != AFMM_CASE_A && c != AFMM_CASE_B)) return 0;
    return config_ok(c, *cfg) ? 1 : 0;
}

afmm_config afmm_default_config(afmm_case c, int64_t n) {
    {
        std::lock_guard<std::mutex> lk(g_tune_mu);
        for (auto it = g_tune.rbegin(); it != g_tune.rend(); ++it)
            if (it->c == (int32_t)c && n >= it->lo && n <= it->hi) return it->cfg;
    }
    return builtin_config(c, n);
}

afmm_status afmm_multiply_strict_config(afmm_case c, int64_t n, const void* X, const void* Y,
                                        float* Z, const afmm_config* cfg, void* workspace,
                                        size_t workspace_bytes, hipStream_t stream) {
    if (c != AFMM_CASE_A && c != AFMM_CASE_B) return AFMM_ERR_INVALID_ARG;
    afmm_status st = check_args(square(n), X, Y, Z);
    if (st != AFMM_OK) return st;
    if (!cfg || !config_ok(c, *cfg)) return AFMM_ERR_INVALID_ARG;
    if ((st = check_device()) != AFMM_OK) return st;
    return strict_run(c, square(n), X, Y, Z, *cfg, workspace, workspace_bytes, stream);
}

afmm_status afmm_set_tuning(int32_t count, const int32_t* cases, const int64_t* n_lo,
                            const int64_t* n_hi, const afmm_config* cfgs) {
    if (count < 0 || (count > 0 && (!cases || !n_lo || !n_hi || !cfgs))) return AFMM_ERR_INVALID_ARG;
    std::vector<TuneEntry> t;
    for (int32_t i = 0; i < count; ++i) {
        if (cases[i] != AFMM_CASE_A && cases[i] != AFMM_CASE_B) return AFMM_ERR_INVALID_ARG;
        if (!config_ok((afmm_case)cases[i], cfgs[i]) || n_lo[i] > n_hi[i]) return AFMM_ERR_INVALID_ARG;
        t.push_back(TuneEntry{cases[i], n_lo[i], n_hi[i], cfgs[i]});
    }
    std::lock_guard<std::mutex> lk(g_tune_mu);
    g_tune.swap(t);
    return AFMM_OK;
}

const char* afmm_status_string(afmm_status s) {
    switch (s) {
    case AFMM_OK: return "ok";
    case AFMM_ERR_INVALID_ARG: return "invalid argument";
    case AFMM_ERR_ALIAS: return "output overlaps an input";
    case AFMM_ERR_NEGATIVE_INT: return "negative integer entry";
    case AFMM_ERR_INT_RANGE: return "integer entry out of range for the split form";
    case AFMM_ERR_COUNT_OVERFLOW: return "addition count exceeds 2^64-1";
    case AFMM_ERR_NO_DEVICE: return "no gfx950 device";
    case AFMM_ERR_HIP: return "HIP error";
    case AFMM_ERR_UNSUPPORTED: return "unsupported";
    case AFMM_ERR_WORKSPACE: return "workspace too small";
    }
    return "unknown status";
}

int afmm_last_hip_error(void) { return g_last_hip_error_slot(); }

const char* afmm_version(void) { return "0.1.0"; }

}  // extern "C"
