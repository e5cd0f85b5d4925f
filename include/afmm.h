/*
 * afmm.h -- C ABI of the MI355X (gfx950) AFMM library, libafmm.so.
 *
 * AFMM (Singh, Chakraborty, Mallick, arXiv 1308.2400, Section 2) forms the
 * product Z = X . Y of two dense n x n matrices, one of which holds
 * non-negative integers, without a single multiplication: every product
 * term X[i,k] * Y[k,j] is made by adding the real entry into Z[i,j] as many
 * times as the integer entry says.
 *   Case A (Section 2, Case-A loop): X real (binary32), Y integer (int32).
 *       For each non-zero X[i,k] and each j, X[i,k] is added into Z[i,j]
 *       Y[k,j] times.
 *   Case B (Section 2, Case-B loop): X integer, Y real.  For each j with a
 *       non-zero Y[k,j], Y[k,j] is added into Z[i,j] X[i,k] times.
 *
 * Conventions shared by every entry point
 *  - Matrices are dense, row-major, n x n, contiguous (element (r, c) at
 *    r * n + c), 4-byte aligned, in device memory owned by the caller.  The
 *    library keeps no pointer after a call returns (plans excepted: they keep
 *    theirs until destroyed).
 *  - Z is fully overwritten: it starts from zero (Section 2: "Z ... initialized
 *    with all zeroes"); there is no accumulate mode.  Z may not overlap X or Y.
 *  - Work is queued on `stream` (0 = the null stream) and the call returns
 *    without waiting, except afmm_validate.  Argument errors are detected on
 *    the host before anything is queued; a failed launch returns
 *    AFMM_ERR_HIP and afmm_last_hip_error() gives the HIP error code.
 *  - Integer entries are repetition counts (Section 2.1: the Rep-factor is an
 *    integer count).  An entry <= 0 performs no additions (the empty sum).
 *    Entries are not checked by the multiply calls; afmm_validate and
 *    afmm_count_adds report negative and out-of-range entries.
 *  - Non-finite reals are outside the contract (they propagate as IEEE says).
 *  - Calls are thread-safe; calls on different streams may overlap.
 *
 * Precision modes
 *  - AFMM_MODE_STRICT: the method itself.  Every addition is a binary32
 *    round-to-nearest-even addition performed in the paper's order (k
 *    ascending, then the Rep-factor repetitions, straight into Z[i,j]), so
 *    the result is bit-identical to a sequential CPU run of the Case-A or
 *    Case-B loop in binary32 with denormals kept.
 *  - AFMM_MODE_SPLIT_BF16X3: the same product on the matrix cores: the real
 *    factor is split into three bfloat16 terms (hi + mid + lo == x exactly
 *    for 2^-100 <= |x| < 2^127), the integer factor is held exactly in
 *    bfloat16 (requires 0 <= entry <= 256), and the terms are contracted with
 *    MFMA into binary32 accumulators.  Not bit-identical to STRICT; relative
 *    Frobenius error against the exact product stays near 1e-7 on the
 *    reference workloads.  Uses multiplications (on the matrix cores).
 */
#ifndef AFMM_H
#define AFMM_H

#include <stddef.h>
#include <stdint.h>

#include <hip/hip_runtime_api.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum { AFMM_CASE_A = 0, AFMM_CASE_B = 1 } afmm_case;

typedef enum { AFMM_MODE_STRICT = 0, AFMM_MODE_SPLIT_BF16X3 = 1 } afmm_mode;

typedef enum {
    AFMM_OK = 0,
    AFMM_ERR_INVALID_ARG = 1,    /* null pointer, n < 1, n > AFMM_MAX_N, bad enum      */
    AFMM_ERR_ALIAS = 2,          /* Z overlaps X or Y                                  */
    AFMM_ERR_NEGATIVE_INT = 3,   /* afmm_validate: an integer entry is negative        */
    AFMM_ERR_INT_RANGE = 4,      /* afmm_validate: entry > 256 in split mode           */
    AFMM_ERR_COUNT_OVERFLOW = 5, /* afmm_validate: the add count exceeds 2^64 - 1      */
    AFMM_ERR_NO_DEVICE = 6,      /* no usable gfx950 device                            */
    AFMM_ERR_HIP = 7,            /* a HIP call failed; see afmm_last_hip_error()       */
    AFMM_ERR_UNSUPPORTED = 8,    /* valid request the library does not implement       */
    AFMM_ERR_WORKSPACE = 9       /* workspace given but smaller than required          */
} afmm_status;

/* Largest supported n (element offsets stay below 2^31 per row stride). */
#define AFMM_MAX_N 65536

/* Flag bits written by afmm_count_adds into *d_flags. */
#define AFMM_FLAG_NEGATIVE 1u /* an integer entry is < 0                      */
#define AFMM_FLAG_ABOVE255 2u /* an integer entry is > 255                    */
#define AFMM_FLAG_ABOVE256 4u /* an integer entry is > 256 (split mode: bad)  */
#define AFMM_FLAG_OVERFLOW 8u /* the add count saturated at 2^64 - 1          */

/*
 * Bytes of device scratch a multiply of this case, size and mode needs.
 * Pass at least that much as `workspace` to the multiply calls, or pass
 * workspace = NULL to let the library take it from the stream-ordered HIP
 * allocator (hipMallocAsync / hipFreeAsync on `stream`).  For a strict
 * product that chooses its form on the device (see afmm_multiply_caseA) this
 * covers every form it may choose: about 17 n^2 bytes (case B) or 21 n^2
 * (case A), against n^2 (B) or 5 n^2 (A) for the size-keyed form alone
 * (afmm_workspace_size_config of afmm_default_config).
 */
size_t afmm_workspace_size(afmm_case c, int64_t n, afmm_mode mode);

/*
 * Case A product (Section 2, Case-A loop).  X: n x n binary32, Y: n x n
 * int32 (repetition counts), Z: n x n binary32 output.  See the mode notes
 * above.  workspace / workspace_bytes: caller scratch or NULL / 0.
 *
 * Strict mode picks its kernel form on the device, with no wait for the host,
 * when 1024 <= n <= 16384 and the size-keyed configuration (afmm_default_config)
 * is a dense one (mapping 0, 2 or 3): two small kernels count the participating
 * entries of 128 evenly spaced rows of each factor and apply the rule of
 * afmm_suggest_config to these sampled densities, and the kernels of the forms
 * not chosen return at once.  Every form gives the same bits, so the choice
 * changes only the time.  afmm_plain_form reports the choice.
 */
afmm_status afmm_multiply_caseA(int64_t n, const float *X, const int32_t *Y, float *Z,
                                afmm_mode mode, void *workspace, size_t workspace_bytes,
                                hipStream_t stream);

/* Case B product (Section 2, Case-B loop).  X: int32 counts, Y: binary32. */
afmm_status afmm_multiply_caseB(int64_t n, const int32_t *X, const float *Y, float *Z,
                                afmm_mode mode, void *workspace, size_t workspace_bytes,
                                hipStream_t stream);

/*
 * Number of additions the method performs on (X, Y) (Section 2.2, counted
 * exactly rather than estimated as mu' d1 d2 n^3):
 *   case A: sum over (i,k) with X[i,k] != 0 and over j of max(Y[k,j], 0)
 *   case B: sum over (i,k) and over j with Y[k,j] != 0 of max(X[i,k], 0)
 * Writes into device memory: *d_total (uint64, saturated at 2^64-1),
 * d_row_counts[i] = additions of row i of Z (nullable), *d_flags = the
 * AFMM_FLAG_* bits found (nullable).  Needs 16 * n + 512 bytes of workspace
 * rounded up (afmm_workspace_size(c, n, AFMM_MODE_STRICT) is enough), or NULL
 * (see afmm_workspace_size).  Asynchronous.
 */
afmm_status afmm_count_adds(afmm_case c, int64_t n, const void *X, const void *Y,
                            uint64_t *d_total, uint64_t *d_row_counts, uint32_t *d_flags,
                            void *workspace, size_t workspace_bytes, hipStream_t stream);

/* ---------------------------------------------------------------------------
 * Rectangular and strided forms.  The paper's matrices are n x n (Section 2);
 * its loops run unchanged with separate bounds for i, k and j, which is the
 * product of an m x k pre-factor and a k x n post-factor.  Matrices are
 * row-major with leading dimensions (element (r, c) of X at X[r * ldx + c]):
 * X is m x k (ldx >= k), Y is k x n (ldy >= n), Z is m x n (ldz >= n); 1 <=
 * m, k, n <= AFMM_MAX_N and every leading dimension <= 2^28.  Only the m x n
 * block of Z is written (its padding keeps its contents); padding in X and Y
 * is never read.  The address ranges of Z and of X, Y (first to last element)
 * may not overlap.  Everything else is as for the square calls, which are
 * these with m = k = n = ldx = ldy = ldz.
 */
size_t afmm_workspace_size_ex(afmm_case c, int64_t m, int64_t k, int64_t n, afmm_mode mode);

afmm_status afmm_multiply_caseA_ex(int64_t m, int64_t k, int64_t n, const float *X, int64_t ldx,
                                   const int32_t *Y, int64_t ldy, float *Z, int64_t ldz,
                                   afmm_mode mode, void *workspace, size_t workspace_bytes,
                                   hipStream_t stream);

afmm_status afmm_multiply_caseB_ex(int64_t m, int64_t k, int64_t n, const int32_t *X, int64_t ldx,
                                   const float *Y, int64_t ldy, float *Z, int64_t ldz,
                                   afmm_mode mode, void *workspace, size_t workspace_bytes,
                                   hipStream_t stream);

/* Addition count of the rectangular product: d_row_counts has m entries; the
 * workspace needs afmm_workspace_size_ex(c, m, k, n, AFMM_MODE_STRICT) bytes. */
afmm_status afmm_count_adds_ex(afmm_case c, int64_t m, int64_t k, int64_t n, const void *X,
                               int64_t ldx, const void *Y, int64_t ldy, uint64_t *d_total,
                               uint64_t *d_row_counts, uint32_t *d_flags, void *workspace,
                               size_t workspace_bytes, hipStream_t stream);

/*
 * The split form's operand conversion, read back (for checking it against an
 * independent split; not needed for computing products).  Runs the conversion
 * pass a split-mode multiply runs on (X, Y) and writes, in device memory:
 *   d_terms: three n x n bfloat16 bit patterns, hi then mid then lo, of the
 *            real factor in its own row-major layout (X[i][k] in case A,
 *            Y[k][j] in case B): hi = RNE_bf16(x), mid = RNE_bf16(x - hi),
 *            lo = RNE_bf16(x - hi - mid);
 *   d_ints:  the n x n integer factor as bfloat16 patterns, row-major in its
 *            own layout (a count <= 0 becomes +0; 1..256 are exact).
 * workspace: afmm_workspace_size(c, n, AFMM_MODE_SPLIT_BF16X3) bytes or NULL
 * (stream-ordered allocation).  Asynchronous on `stream`.
 */
afmm_status afmm_split_terms(afmm_case c, int64_t n, const void *X, const void *Y,
                             uint16_t *d_terms, uint16_t *d_ints, void *workspace,
                             size_t workspace_bytes, hipStream_t stream);

/*
 * The compacted-base form's lists of non-zero bases, read back (for checking
 * the list builder; not needed for computing products).  Q: a k x n_c
 * row-major binary32 matrix in device memory, leading dimension ldq >= n_c,
 * row t holding the bases of one k (case B: Y; case A: X transposed).  With
 * CT = 64*C columns per band (C in 1..64), bands = ceil(n_c / CT),
 * k_pad = round_up(k, 16) and E = max(1, C/16), writes in device memory:
 *   d_entries: [bands][k_pad][CT] pairs of uint32 {bits of Q[t][b*CT + c],
 *              4*c} (the byte offset of column c in a row of the band); slot
 *              q*64 + l of a segment is the q-th entry lane l adds.  Lane l
 *              owns the columns c = l (mod 64) and takes them first; a lane's
 *              surplus goes to lane l ^ 32 first, then alternately to free
 *              slots of the other and of its own half-wave; free slots hold
 *              {+0.0, 4*(CT + l)} (the lane's sink column);
 *   d_lens:    [bands][k_pad] int32, the slots in use: ceil(nnz / 64) rounded
 *              up to a multiple of E, times 64; 0 when the segment has no
 *              non-zero base (-0.0 counts as zero, NaN as non-zero).  Slots
 *              past the length are not written.
 * Asynchronous on `stream`.
 */
afmm_status afmm_base_lists(const float *Q, int64_t k, int64_t n_c, int64_t ldq, int32_t C,
                            uint32_t *d_entries, int32_t *d_lens, hipStream_t stream);

/*
 * The row-list form's lists, read back (for checking the list builder; not
 * needed for computing products).  M: a rows x cols row-major matrix in device
 * memory, leading dimension ld >= cols, of int32 counts (is_int = 1) or
 * binary32 bases (is_int = 0).  With bands of `band` columns
 * (bands = ceil(cols / band)), writes in device memory:
 *   d_entries: [bands][rows][band] pairs of uint32 {bits of M[r][b*band + c], c}
 *              for the entries of row r in band b that take part in an
 *              addition (a count > 0; a base != 0, so -0.0 is dropped and NaN
 *              kept), in ascending c; slots past the length are not written;
 *   d_lens:    [bands][rows] int32, the number of such entries.
 * The row-list form lists X with one band as wide as its rows (rounded up to
 * 64) and Y with bands of 64*C columns.  Asynchronous on `stream`.
 */
afmm_status afmm_row_lists(int32_t is_int, const void *M, int64_t rows, int64_t cols, int64_t ld,
                           int64_t band, uint32_t *d_entries, int32_t *d_lens,
                           hipStream_t stream);

/*
 * Synchronous data check: runs the counting pass on `stream`, waits for it,
 * and returns AFMM_ERR_NEGATIVE_INT, AFMM_ERR_INT_RANGE (split mode, an
 * entry > 256), AFMM_ERR_COUNT_OVERFLOW or AFMM_OK.
 */
afmm_status afmm_validate(afmm_case c, int64_t n, const void *X, const void *Y, afmm_mode mode,
                          hipStream_t stream);

/*
 * Kernel configuration of the strict path (the autotuner's knobs).
 *   mapping: 0 = rep-uniform (each wave walks R rows of the integer factor
 *            with the count in a scalar register; lanes over the real
 *            factor's columns; case A runs on the transposed problem),
 *            (1 is not used: a base-uniform mapping with per-lane counts,
 *            rejected for its SIMD efficiency),
 *            2 = rep-uniform with base rows streamed straight into
 *            registers (no LDS panel); falls back to 0 when the base rows
 *            are not readable in 16-byte units (case B with n % 4 != 0),
 *            3 = rep-uniform, sparse-k: eight waves per SIMD, base panels
 *            loaded straight into LDS, and each wave visits only the k where
 *            one of its R rows has a non-zero count; falls back to 0 when
 *            the base rows are not readable in 16-byte units or the base
 *            matrix exceeds 2^31 bytes,
 *            4 = rep-uniform, compacted base, for a real factor with few
 *            non-zeros: a pass lists the non-zero bases of every k in bands
 *            of 64*C lane columns; a workgroup keeps a (W*R) x (64*C) block
 *            of Z in LDS, and for each k its lanes take the listed bases
 *            (max(1, C/16) per lane, 64 lanes at a time) while each wave walks
 *            its R rows with the count uniform, reading, repeatedly adding to
 *            and writing back its Z elements.  Lanes never idle on a zero
 *            base; k_panel (8 or 16) is the number of k whose lists and
 *            counts are fetched ahead together.  The lists take
 *            8 * round_up(lane extent, 64*C) * round_up(k, 16) bytes of
 *            workspace (afmm_workspace_size_config); falls back to 0 when one
 *            band of them or the count bytes exceed 2^31 bytes,
 *            7 = over the non-zeros of both factors, for the low-density regime
 *            of Section 2.2 (d1 * d2 ~ 1/n, additions ~ n^2): passes list the
 *            non-zero entries of X's rows and of Y's rows (per band of 64*C
 *            columns); a workgroup keeps W rows x 64*C columns of Z in LDS,
 *            a wave walks its row's X list in ascending k and, for each k,
 *            its lanes take Y's list for that k (case B: the count is the
 *            wave's, the base the lane's; case A: the other way round, each
 *            lane looping its own count).  Work is proportional to the
 *            pairs of non-zero entries; R = 1, U = 1, k_panel 16 only.
 *            Lists: 8 * (m * round_up(k, 64) + k * round_up(n, 64*C)) bytes
 *            plus lengths (afmm_workspace_size_config).
 *   rows_per_wave R, cols_per_lane C, waves per workgroup W, unroll U (1
 *   or 2: the repetition loop does U additions per trip; 4, mapping 4
 *   only: one, two and four additions under tests of the count's low bits,
 *   then trips of eight; 0 means 1),
 *   k_panel (rows of the base staged per LDS panel, 4, 8 or 16; 0 means 16):
 *   one of the compiled combinations (afmm_config_supported tells which).
 *   Every configuration performs the same additions in the same order, so
 *   all give bit-identical results.
 */
typedef struct {
    int32_t mapping;
    int32_t rows_per_wave;
    int32_t cols_per_lane;
    int32_t waves;
    int32_t unroll;
    int32_t k_panel;
} afmm_config;

/* 1 when `cfg` names a compiled kernel for case c, else 0. */
int afmm_config_supported(afmm_case c, const afmm_config *cfg);

/* The configuration the library picks for a strict product of this case and
 * size (tuning table, else built-in rule). */
afmm_config afmm_default_config(afmm_case c, int64_t n);

/* Workspace bytes of a strict n x n product run with `cfg` (0 when cfg is not
 * compiled); afmm_workspace_size covers the configuration the library picks. */
size_t afmm_workspace_size_config(afmm_case c, int64_t n, const afmm_config *cfg);

/* A configuration for the strict n x n product of these operands, chosen from
 * the densities of the two factors, counted on the device (the call waits for
 * `stream`): with d_real the fraction of non-zero real entries and d_int that
 * of positive counts, the form over the non-zeros of both factors (mapping 7)
 * when d_real * d_int * n <= 32 (case A) or 64 (case B), else the
 * compacted-base form (mapping 4) when
 * d_real <= 0.06, otherwise afmm_default_config (also for n < 1024).  The
 * thresholds come from measurements on MI355X; every configuration gives the
 * same bits.  For callers that know nothing of their data's sparsity. */
afmm_status afmm_suggest_config(afmm_case c, int64_t n, const void *X, const void *Y,
                                hipStream_t stream, afmm_config *out);

/*
 * The mapping (afmm_config.mapping) a strict afmm_multiply_caseA / caseB call
 * on these operands runs, chosen exactly as that call chooses it (see
 * afmm_multiply_caseA): written as one int32 to *d_mapping (device) on
 * `stream`, asynchronously.  workspace: 4096 bytes or NULL.  A diagnostic for
 * callers that want to see which form their data gets.
 */
afmm_status afmm_plain_form(afmm_case c, int64_t n, const void *X, const void *Y,
                            int32_t *d_mapping, void *workspace, size_t workspace_bytes,
                            hipStream_t stream);

/* Strict product with an explicit configuration (for the autotuner). */
afmm_status afmm_multiply_strict_config(afmm_case c, int64_t n, const void *X, const void *Y,
                                        float *Z, const afmm_config *cfg, void *workspace,
                                        size_t workspace_bytes, hipStream_t stream);

/*
 * Tuning table: `count` entries, entry t applying to products of case
 * cases[t] with n in [n_lo[t], n_hi[t]].  Replaces the previous table; a
 * later entry wins over an earlier one.  Entries naming an unsupported
 * configuration are rejected (AFMM_ERR_INVALID_ARG, table unchanged).
 */
afmm_status afmm_set_tuning(int32_t count, const int32_t *cases, const int64_t *n_lo,
                            const int64_t *n_hi, const afmm_config *cfgs);

/* ---------------------------------------------------------------------------
 * Batched products: many independent AFMM products of uneven size, density
 * and integer range.  In strict mode they run in one persistent launch: work
 * is cut into tiles and handed out largest-first by each tile's cost, which is
 * data-dependent as Section 2.2 says: the lane additions the kernel issues for
 * the tile (the integer factor's counts summed over the tile's rows, times the
 * tile's width) plus a per-(row, k) term, measured on the device from the data
 * at every launch.
 */
typedef struct {
    int32_t case_id; /* AFMM_CASE_A or AFMM_CASE_B                             */
    int32_t n;       /* 1 .. AFMM_MAX_BATCH_N                                  */
    const void *X;   /* case A: const float*, case B: const int32_t*           */
    const void *Y;   /* case A: const int32_t*, case B: const float*           */
    float *Z;        /* output, must not overlap any X, Y or other Z of the batch */
} afmm_problem;

#define AFMM_MAX_BATCH_N 8192

typedef struct afmm_plan afmm_plan;

/*
 * Build a plan for `count` (1 .. 4096) problems (host array, copied).
 * Returns AFMM_ERR_ALIAS when some Z overlaps any X, Y or other Z of the
 * batch (X and Y may be shared between problems).  Allocates the plan's
 * device tables and scratch on the current device.  The plan records the
 * pointers; the data they point to may change between launches.
 * mode AFMM_MODE_STRICT: the persistent path above, bit-identical to single
 * strict products.  mode AFMM_MODE_SPLIT_BF16X3: each product is the
 * single-product split form (its conversion pass and matrix-core product,
 * queued one after another), with the same result as afmm_multiply_caseA/B in
 * split mode; the per-problem addition counts are still computed.
 */
afmm_status afmm_batched_plan_create(const afmm_problem *problems, int32_t count, afmm_mode mode,
                                     afmm_plan **out);

/*
 * Run the plan on `stream`: prepare operands, compute the per-problem addition
 * counts and per-tile costs, order the tiles largest-first, and run the
 * persistent kernel (split mode: the per-product conversions and products).
 * The first launch captures these steps into a HIP graph; later launches
 * replay it.  Launches of one plan must not overlap.
 */
afmm_status afmm_batched_plan_launch(afmm_plan *plan, hipStream_t stream);

/* Queue on `stream` a copy of the per-problem addition counts (Section 2.2)
 * computed by the plan's last launch into d_out (device, uint64[count]). */
afmm_status afmm_batched_plan_problem_adds(const afmm_plan *plan, uint64_t *d_out,
                                           hipStream_t stream);

/* Release the plan (synchronises the device first). */
afmm_status afmm_batched_plan_destroy(afmm_plan *plan);

/*
 * Tile shapes of the persistent strict kernel, by problem size: a problem with
 * n >= n_wide gets 8-row x 512-column tiles (the sparse-k body), n >= n_mid
 * 8 x 256, smaller ones 8 x 64 (the LDS-panel body).  Built in: 512 and 128;
 * the autotuner measures the batched workload over a grid of thresholds and
 * stores the fastest pair in its table.  Applies to plans created after the
 * call; every shape gives the same bits.  AFMM_ERR_INVALID_ARG unless
 * 1 <= n_mid <= n_wide.
 */
afmm_status afmm_set_batch_shapes(int64_t n_wide, int64_t n_mid);

/* One-shot convenience: create, launch on `stream`, wait, destroy. */
afmm_status afmm_multiply_batched(const afmm_problem *problems, int32_t count, afmm_mode mode,
                                  hipStream_t stream);

/* ---------------------------------------------------------------------------
 * For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid allocation): the strict
 * product of afmm_multiply_caseA / afmm_multiply_caseB (same kernels, same
 * bits), with its workspace in a fixed array of AFMM_NOALLOC_SCRATCH_BYTES
 * that the library keeps on every device it runs on, for the life of the
 * process.  The call performs no allocation.  X, Y, Z and their layout are as
 * for the square calls (case A: X binary32, Y int32; case B the other way).
 * The call runs the size-keyed form
 * (afmm_default_config; it does not choose a form from the data) and returns
 * AFMM_ERR_WORKSPACE when that form's workspace (afmm_workspace_size_config)
 * exceeds the array; with the built-in configurations that admits case B up
 * to n = 9984 and case A up to n = 4480.  All calls on one device share its array and every call rewrites
 * what it uses: calls that overlap in time on one device (different streams,
 * or host threads racing) race on it and are not allowed.
 */
#define AFMM_NOALLOC_SCRATCH_BYTES ((size_t)96 << 20)

afmm_status afmm_multiply_noalloc(afmm_case c, int64_t n, const void *X, const void *Y, float *Z,
                                  hipStream_t stream);

/* ---------------------------------------------------------------------------
 * Diagnostic: the device's binary32 add rate, the denominator of the strict
 * kernels' roofline.  Queues one launch of straight-line v_add_f32 runs (VGPR
 * operands, 16 independent accumulators per lane, 128 additions per loop trip,
 * `trips` trips), one block of 4 * waves_per_simd waves (1, 2 or 4) per compute
 * unit, so each SIMD runs waves_per_simd waves.  d_out: 1024 floats of device
 * memory (results, kept so the additions are not removed).  *adds (host) is
 * set to the number of binary32 additions the launch performs; time the
 * launch with events on `stream`.  Computes nothing of the method.
 */
afmm_status afmm_probe_add_rate(int32_t waves_per_simd, int32_t trips, float *d_out,
                                uint64_t *adds, hipStream_t stream);

/* ------------------------------------------------------------------------- */
const char *afmm_status_string(afmm_status s);

/* HIP error code of the last AFMM_ERR_HIP on this thread (0 if none). */
int afmm_last_hip_error(void);

/* Library version, "major.minor.patch". */
const char *afmm_version(void);

#ifdef __cplusplus
}
#endif

#endif
