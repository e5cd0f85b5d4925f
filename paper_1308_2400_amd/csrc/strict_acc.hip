// Strict AFMM kernel, compacted-base form (Section 2, bit-exact binary32
// repeated addition) for a real factor with few non-zeros.
//
// The count-uniform mapping puts lanes over the real factor's columns, so a
// lane whose base is zero idles through the repetitions of its row.  Here a
// block keeps a TM x CT tile of Z in LDS instead of registers; for each k the
// lanes take the compacted non-zero bases of the block's CT columns, and each
// wave walks its R rows with the count uniform per row: read Z from LDS, add
// the base `rep` times, write it back.  Every element still receives its
// additions in ascending k, a k's repetitions consecutively, so the result is
// bit-identical to the other forms.  A wave owns its rows, so no two waves
// touch one element and the k loop has no barrier.
#include <utility>

#include "sparse_body.hpp"
#include "strict_acc.hpp"

namespace afmm {

constexpr int kAccKP = kAccKPad;
constexpr int kAccWaitVm0 = 0x0F70;  // s_waitcnt vmcnt(0), other counters at their maxima

size_t acc_lists_bytes(int n_c, int n_k, int C) {
    const int64_t ct = (int64_t)kWave * C;
    const int64_t bands = (n_c + ct - 1) / ct, kp = round_up(n_k, kAccKP);
    return (size_t)round_up(bands * kp * ct * 8, 256) + (size_t)round_up(bands * kp * 4, 256);
}

AccLists acc_lists_at(uint8_t* p, int n_c, int n_k, int C) {
    const int64_t ct = (int64_t)kWave * C;
    const int64_t bands = (n_c + ct - 1) / ct, kp = round_up(n_k, kAccKP);
    AccLists L;
    L.ent = reinterpret_cast<uint2*>(p);
    L.lens = reinterpret_cast<int32_t*>(p + round_up(bands * kp * ct * 8, 256));
    L.n_k_pad = kp;
    return L;
}

// One wave per segment (band, k).  Lane l owns the band's columns l + 64 m
// (m < C), all of one residue modulo 64.  LDS serves a wave-wide 32-bit access
// as two half-waves (lanes 0-31, then 32-63), each over 32 banks of 4 bytes, and
// an element (row, column) of the Z tile sits in bank (row offset + column) mod
// 32: lanes l and l ^ 32 share a bank but are served in different half-waves,
// and every column a lane owns, its sink column CT + l included, is in that
// lane's bank.  With total non-zero bases in the band the segment gets
// nch = ceil(total / 64) chunks of 64 slots; slot (q, l) holds lane l's q-th
// non-zero column when it has one.  A lane with more than nch hands the rest
// on: first to the free slots of lane l ^ 32 (same bank, other half-wave, so
// still no conflict), then, once both lanes of its bank are full, to free
// slots of other lanes, alternating between the half-waves so that a bank
// takes one extra access per half-wave before it takes a second (each extra
// access costs its half-wave one conflict cycle).  Slots left over get the
// lane's sink column with a +0.0 base.  The chunks are padded to a multiple of
// E (the entries a lane takes per k).  An entry is {bits of the base, byte
// offset of its column in an LDS row}; the segment's length is the padded slot
// count, 0 when the band has no non-zero base at this k.  Which slot adds a
// base changes nothing in the sums: each column appears once per k.
__device__ __forceinline__ uint64_t shfl_u64(uint64_t v, int src) {
    const uint32_t lo = (uint32_t)__shfl((int)(uint32_t)v, src);
    const uint32_t hi = (uint32_t)__shfl((int)(uint32_t)(v >> 32), src);
    return ((uint64_t)hi << 32) | lo;
}

__global__ __launch_bounds__(256) void compact_base_kernel(const float* __restrict__ Q,
                                                           int64_t ldq, int n_k, int n_c, int C,
                                                           int E, int64_t n_k_pad, int64_t n_segs,
                                                           uint2* __restrict__ ent,
                                                           int32_t* __restrict__ lens,
                                                           const uint32_t* __restrict__ gate) {
    // per wave: the columns handed to lanes other than lane ^ 32, those bound
    // for the upper half-wave first (CT <= 4096 of them)
    __shared__ uint16_t handed[4][kWave * 64];
    AFMM_GATE(gate);
    const int lane = threadIdx.x & (kWave - 1), wv = threadIdx.x >> 6;
    const int64_t seg = (int64_t)blockIdx.x * 4 + wv;
    if (seg >= n_segs) return;  // whole waves
    const int ct = kWave * C;
    const int band = (int)(seg / n_k_pad);
    const int k = (int)(seg - (int64_t)band * n_k_pad);
    const int c0 = band * ct;
    uint64_t mine = 0;  // bit m: column lane + 64 m is non-zero
    const float* __restrict__ q = Q + (int64_t)k * ldq + c0;
    if (k < n_k) {
        for (int m = 0; m < C; ++m) {
            const int c = lane + kWave * m;
            const float v = c0 + c < n_c ? q[c] : 0.0f;
            if (v != 0.0f) mine |= (uint64_t)1 << m;  // IEEE: -0 is zero, NaN is not
        }
    }
    const int a = __popcll(mine);
    int total = a;
    for (int off = kWave / 2; off > 0; off >>= 1) total += __shfl_xor(total, off);
    if (total == 0) {
        if (lane == 0) lens[seg] = 0;
        return;
    }
    const int nch = (total + kWave - 1) / kWave;
    const int npad = (nch + E - 1) / E * E;
    uint2* __restrict__ out = ent + seg * ct;
    const uint2 sink = make_uint2(0u, (uint32_t)(ct + lane) * 4u);
    // the lane's own columns into its first min(a, nch) slots
    uint64_t rest = mine;
    const int own = a < nch ? a : nch;
    for (int s = 0; s < own; ++s) {
        const int m = __ffsll((unsigned long long)rest) - 1;
        rest &= rest - 1;
        const int c = lane + kWave * m;
        out[s * kWave + lane] = make_uint2(__float_as_uint(q[c]), (uint32_t)c * 4u);
    }
    // the partner's columns beyond its nch into this lane's free slots, and
    // this lane's beyond nch into the partner's
    const int partner = lane ^ (kWave / 2);
    const uint64_t mine_p = shfl_u64(mine, partner);
    const int a_p = __popcll(mine_p), own_p = a_p < nch ? a_p : nch;
    const int give = min(a - own, nch - own_p), recv = min(a_p - own_p, nch - own);
    {
        uint64_t rp = mine_p;
        for (int s = 0; s < own_p; ++s) rp &= rp - 1;
        for (int s = 0; s < recv; ++s) {
            const int m = __ffsll((unsigned long long)rp) - 1;
            rp &= rp - 1;
            const int c = partner + kWave * m;
            out[(own + s) * kWave + lane] = make_uint2(__float_as_uint(q[c]), (uint32_t)c * 4u);
        }
    }
    for (int u = 0; u < give; ++u) rest &= rest - 1;
    const int ov = a - own - give, holes = nch - own - recv;  // left after the pairing
    // the lane's j-th remaining column goes to the other half-wave for even j,
    // to its own for odd j
    const bool up = lane >= kWave / 2;
    const int n_up = up ? ov / 2 : (ov + 1) / 2, n_lo = ov - n_up;
    // exclusive scans over the lanes: entries bound up / down, free slots above / below
    int up_x = n_up, lo_x = n_lo, hu_x = up ? holes : 0, hl_x = up ? 0 : holes;
    for (int off = 1; off < kWave; off <<= 1) {
        const int t1 = __shfl_up(up_x, off), t2 = __shfl_up(lo_x, off);
        const int t3 = __shfl_up(hu_x, off), t4 = __shfl_up(hl_x, off);
        if (lane >= off) {
            up_x += t1;
            lo_x += t2;
            hu_x += t3;
            hl_x += t4;
        }
    }
    const int ue = __shfl(up_x, kWave - 1), le = __shfl(lo_x, kWave - 1);
    const int uh = __shfl(hu_x, kWave - 1), lh = __shfl(hl_x, kWave - 1);
    up_x -= n_up;
    lo_x -= n_lo;
    if (ue + le > 0) {
        // list: entries bound up at [0, ue), entries bound down at [ue, ue + le)
        int iu = 0, il = 0;
        for (int j = 0; j < ov; ++j) {
            const int m = __ffsll((unsigned long long)rest) - 1;
            rest &= rest - 1;
            const uint16_t c = (uint16_t)(lane + kWave * m);
            if ((j & 1) == (up ? 1 : 0))
                handed[wv][up_x + iu++] = c;
            else
                handed[wv][ue + lo_x + il++] = c;
        }
        // the wave's own LDS writes, read back by other lanes of the wave
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    }
    // free slots take the entries bound for their half-wave; a half-wave with
    // more entries than free slots passes the excess to the other one (the
    // slots suffice: 64 nch >= total)
    const int rank0 = up ? hu_x - holes : hl_x - holes;
    for (int s = own + recv; s < nch; ++s) {
        const int t = rank0 + (s - own - recv);
        int idx = -1;
        if (up) {
            const int fill = min(ue, uh);
            if (t < fill)
                idx = t;
            else if (le > lh && t - fill < le - lh)
                idx = ue + lh + (t - fill);
        } else {
            const int fill = min(le, lh);
            if (t < fill)
                idx = ue + t;
            else if (ue > uh && t - fill < ue - uh)
                idx = uh + (t - fill);
        }
        uint2 e = sink;
        if (idx >= 0) {
            const int c = handed[wv][idx];
            e = make_uint2(__float_as_uint(q[c]), (uint32_t)c * 4u);
        }
        out[s * kWave + lane] = e;
    }
    for (int s = nch; s < npad; ++s) out[s * kWave + lane] = sink;
    if (lane == 0) lens[seg] = npad * kWave;
}

hipError_t launch_compact_base(const float* Q, int64_t ldq, int n_k, int n_c, int C,
                               const AccLists& L, hipStream_t s, const uint32_t* gate) {
    const int ct = kWave * C;
    if (C < 1 || C > 64) return hipErrorInvalidValue;
    const int E = C >= 16 ? C / 16 : 1;  // entries a lane takes per k (AccTile::E)
    const int64_t bands = (n_c + ct - 1) / ct;
    const int64_t n_segs = bands * L.n_k_pad;
    const int64_t blocks = (n_segs + 3) / 4;
    hipLaunchKernelGGL(compact_base_kernel, dim3((unsigned)blocks), dim3(256), 0, s, Q, ldq, n_k,
                       n_c, C, E, L.n_k_pad, n_segs, L.ent, L.lens, gate);
    return hipGetLastError();
}

template <int R, int C, int W, int KP>
struct AccTile {
    static constexpr int CT = kWave * C;        // columns per block (one band)
    static constexpr int E = C >= 16 ? C / 16 : 1;  // entries per lane per k
    static constexpr int TM = W * R;            // rows per block
    // LDS row: the band's CT columns, then one sink column per lane (a lane
    // without an entry adds +0.0 there), then one float that keeps rows on
    // different banks
    static constexpr int STRIDE = CT + kWave + 1;
    static constexpr int LDS_FLOATS = TM * STRIDE;
    static_assert(TM <= kRowPad, "row padding must cover a tile");
    static_assert(TM % 4 == 0, "the tile is cleared in float4 units");
    static_assert(LDS_FLOATS * 4 <= 160 * 1024, "the Z tile must fit in LDS");
    static_assert(KP == 8 || KP == 16, "count words of 8 or 16 k");
    static_assert(kKPad % KP == 0, "KP must divide the k padding");
};

// 32-bit LDS addresses: of a pointer into a __shared__ array, and back.
typedef __attribute__((address_space(3))) float lds_float;
__device__ __forceinline__ uint32_t lds_address(float* p) {
    return (uint32_t)(uintptr_t)(lds_float*)p;
}
__device__ __forceinline__ lds_float* lds_at(uint32_t a) { return (lds_float*)(uintptr_t)a; }

// The per-row work of one chunk, for waves of one or two rows, as assembly:
// the compiler turns the skip of a row with a zero count into mask juggling on
// the vector unit, and its repetition loops into three scalar instructions a
// round.  acc_read issues the E reads of every row with a non-zero count and
// waits for them in the same block (no load is left in flight when it ends);
// acc_row adds each slot's base n times and writes the E elements back.  OFF
// is the row's byte offset in LDS.
#define AFMM_RD(z_, a_, o_) "ds_read_b32 %[" z_ "], %[" a_ "] offset:%[" o_ "]\n\t"
#define AFMM_WR(z_, a_) "ds_write_b32 %[" a_ "], %[" z_ "] offset:%[o]\n\t"
#define AFMM_ADD(z_, b_) "v_add_f32 %[" z_ "], %[" b_ "], %[" z_ "]\n\t"

template <int E, int R>
struct AccAsm;

template <>
struct AccAsm<1, 1> {
    template <int O>
    __device__ __forceinline__ static void read(float (&z)[2][1], const uint32_t (&n)[1],
                                                const uint32_t (&a)[1]) {
        asm volatile("s_cmp_eq_u32 %[n0], 0\n\ts_cbranch_scc1 1f\n\t" AFMM_RD("z0", "a0", "o0")
                     "1:\n\ts_waitcnt lgkmcnt(0)"
                     : [z0] "=&v"(z[0][0])
                     : [n0] "s"(n[0]), [a0] "v"(a[0]), [o0] "i"(0)
                     : "scc", "memory");
    }
};
template <>
struct AccAsm<1, 2> {
    template <int O>
    __device__ __forceinline__ static void read(float (&z)[2][1], const uint32_t (&n)[2],
                                                const uint32_t (&a)[1]) {
        asm volatile("s_cmp_eq_u32 %[n0], 0\n\ts_cbranch_scc1 1f\n\t" AFMM_RD("z0", "a0", "o0")
                     "1:\n\ts_cmp_eq_u32 %[n1], 0\n\ts_cbranch_scc1 2f\n\t"
                     AFMM_RD("z1", "a0", "o1") "2:\n\ts_waitcnt lgkmcnt(0)"
                     : [z0] "=&v"(z[0][0]), [z1] "=&v"(z[1][0])
                     : [n0] "s"(n[0]), [n1] "s"(n[1]), [a0] "v"(a[0]), [o0] "i"(0), [o1] "i"(O)
                     : "scc", "memory");
    }
};
template <>
struct AccAsm<2, 1> {
    template <int O>
    __device__ __forceinline__ static void read(float (&z)[2][2], const uint32_t (&n)[1],
                                                const uint32_t (&a)[2]) {
        asm volatile("s_cmp_eq_u32 %[n0], 0\n\ts_cbranch_scc1 1f\n\t" AFMM_RD("z00", "a0", "o0")
                     AFMM_RD("z01", "a1", "o0") "1:\n\ts_waitcnt lgkmcnt(0)"
                     : [z00] "=&v"(z[0][0]), [z01] "=&v"(z[0][1])
                     : [n0] "s"(n[0]), [a0] "v"(a[0]), [a1] "v"(a[1]), [o0] "i"(0)
                     : "scc", "memory");
    }
};
template <>
struct AccAsm<2, 2> {
    template <int O>
    __device__ __forceinline__ static void read(float (&z)[2][2], const uint32_t (&n)[2],
                                                const uint32_t (&a)[2]) {
        asm volatile("s_cmp_eq_u32 %[n0], 0\n\ts_cbranch_scc1 1f\n\t" AFMM_RD("z00", "a0", "o0")
                     AFMM_RD("z01", "a1", "o0") "1:\n\ts_cmp_eq_u32 %[n1], 0\n\t"
                     "s_cbranch_scc1 2f\n\t" AFMM_RD("z10", "a0", "o1") AFMM_RD("z11", "a1", "o1")
                     "2:\n\ts_waitcnt lgkmcnt(0)"
                     : [z00] "=&v"(z[0][0]), [z01] "=&v"(z[0][1]), [z10] "=&v"(z[1][0]),
                       [z11] "=&v"(z[1][1])
                     : [n0] "s"(n[0]), [n1] "s"(n[1]), [a0] "v"(a[0]), [a1] "v"(a[1]),
                       [o0] "i"(0), [o1] "i"(O)
                     : "scc", "memory");
    }
};
template <>
struct AccAsm<4, 1> {
    template <int O>
    __device__ __forceinline__ static void read(float (&z)[2][4], const uint32_t (&n)[1],
                                                const uint32_t (&a)[4]) {
        asm volatile("s_cmp_eq_u32 %[n0], 0\n\ts_cbranch_scc1 1f\n\t" AFMM_RD("z00", "a0", "o0")
                     AFMM_RD("z01", "a1", "o0") AFMM_RD("z02", "a2", "o0")
                     AFMM_RD("z03", "a3", "o0") "1:\n\ts_waitcnt lgkmcnt(0)"
                     : [z00] "=&v"(z[0][0]), [z01] "=&v"(z[0][1]), [z02] "=&v"(z[0][2]),
                       [z03] "=&v"(z[0][3])
                     : [n0] "s"(n[0]), [a0] "v"(a[0]), [a1] "v"(a[1]), [a2] "v"(a[2]),
                       [a3] "v"(a[3]), [o0] "i"(0)
                     : "scc", "memory");
    }
};
template <>
struct AccAsm<4, 2> {
    template <int O>
    __device__ __forceinline__ static void read(float (&z)[2][4], const uint32_t (&n)[2],
                                                const uint32_t (&a)[4]) {
        asm volatile("s_cmp_eq_u32 %[n0], 0\n\ts_cbranch_scc1 1f\n\t" AFMM_RD("z00", "a0", "o0")
                     AFMM_RD("z01", "a1", "o0") AFMM_RD("z02", "a2", "o0")
                     AFMM_RD("z03", "a3", "o0") "1:\n\ts_cmp_eq_u32 %[n1], 0\n\t"
                     "s_cbranch_scc1 2f\n\t" AFMM_RD("z10", "a0", "o1") AFMM_RD("z11", "a1", "o1")
                     AFMM_RD("z12", "a2", "o1") AFMM_RD("z13", "a3", "o1")
                     "2:\n\ts_waitcnt lgkmcnt(0)"
                     : [z00] "=&v"(z[0][0]), [z01] "=&v"(z[0][1]), [z02] "=&v"(z[0][2]),
                       [z03] "=&v"(z[0][3]), [z10] "=&v"(z[1][0]), [z11] "=&v"(z[1][1]),
                       [z12] "=&v"(z[1][2]), [z13] "=&v"(z[1][3])
                     : [n0] "s"(n[0]), [n1] "s"(n[1]), [a0] "v"(a[0]), [a1] "v"(a[1]),
                       [a2] "v"(a[2]), [a3] "v"(a[3]), [o0] "i"(0), [o1] "i"(O)
                     : "scc", "memory");
    }
};

// acc_row: n = 0 skips the row (no write); otherwise a scalar down-counter
// whose borrow ends the loop (two scalar instructions a round).  A binary
// decomposition (1, 2, 4 additions under forward skips, then rounds of 8)
// measured 3 % slower on the n=16384 case-A workload.
template <>
struct AccAsm<1, 4> {
    template <int O>
    __device__ __forceinline__ static void read(float (&z)[4][1], const uint32_t (&n)[4],
                                                const uint32_t (&a)[1]) {
        asm volatile("s_cmp_eq_u32 %[n0], 0\n\ts_cbranch_scc1 1f\n\t" AFMM_RD("z0", "a0", "o0")
                     "1:\n\ts_cmp_eq_u32 %[n1], 0\n\ts_cbranch_scc1 2f\n\t" AFMM_RD("z1", "a0", "o1")
                     "2:\n\ts_cmp_eq_u32 %[n2], 0\n\ts_cbranch_scc1 3f\n\t" AFMM_RD("z2", "a0", "o2")
                     "3:\n\ts_cmp_eq_u32 %[n3], 0\n\ts_cbranch_scc1 4f\n\t" AFMM_RD("z3", "a0", "o3")
                     "4:\n\ts_waitcnt lgkmcnt(0)"
                     : [z0] "=&v"(z[0][0]), [z1] "=&v"(z[1][0]), [z2] "=&v"(z[2][0]),
                       [z3] "=&v"(z[3][0])
                     : [n0] "s"(n[0]), [n1] "s"(n[1]), [n2] "s"(n[2]), [n3] "s"(n[3]),
                       [a0] "v"(a[0]), [o0] "i"(0), [o1] "i"(O), [o2] "i"(2 * O), [o3] "i"(3 * O)
                     : "scc", "memory");
    }
};
template <>
struct AccAsm<2, 4> {
    template <int O>
    __device__ __forceinline__ static void read(float (&z)[4][2], const uint32_t (&n)[4],
                                                const uint32_t (&a)[2]) {
        asm volatile("s_cmp_eq_u32 %[n0], 0\n\ts_cbranch_scc1 1f\n\t" AFMM_RD("z00", "a0", "o0")
                     AFMM_RD("z01", "a1", "o0")
                     "1:\n\ts_cmp_eq_u32 %[n1], 0\n\ts_cbranch_scc1 2f\n\t" AFMM_RD("z10", "a0", "o1")
                     AFMM_RD("z11", "a1", "o1")
                     "2:\n\ts_cmp_eq_u32 %[n2], 0\n\ts_cbranch_scc1 3f\n\t" AFMM_RD("z20", "a0", "o2")
                     AFMM_RD("z21", "a1", "o2")
                     "3:\n\ts_cmp_eq_u32 %[n3], 0\n\ts_cbranch_scc1 4f\n\t" AFMM_RD("z30", "a0", "o3")
                     AFMM_RD("z31", "a1", "o3") "4:\n\ts_waitcnt lgkmcnt(0)"
                     : [z00] "=&v"(z[0][0]), [z01] "=&v"(z[0][1]), [z10] "=&v"(z[1][0]),
                       [z11] "=&v"(z[1][1]), [z20] "=&v"(z[2][0]), [z21] "=&v"(z[2][1]),
                       [z30] "=&v"(z[3][0]), [z31] "=&v"(z[3][1])
                     : [n0] "s"(n[0]), [n1] "s"(n[1]), [n2] "s"(n[2]), [n3] "s"(n[3]),
                       [a0] "v"(a[0]), [a1] "v"(a[1]), [o0] "i"(0), [o1] "i"(O),
                       [o2] "i"(2 * O), [o3] "i"(3 * O)
                     : "scc", "memory");
    }
};

template <int E>
struct AccRow;
template <>
struct AccRow<1> {
    template <int O>
    __device__ __forceinline__ static void run(float (&z)[1], const float (&b)[1], uint32_t n,
                                               const uint32_t (&a)[1]) {
        uint32_t t;
        asm volatile("s_sub_u32 %[t], %[n], 1\n\ts_cbranch_scc1 2f\n"
                     "1:\n\t" AFMM_ADD("z0", "b0")
                     "s_sub_u32 %[t], %[t], 1\n\ts_cbranch_scc0 1b\n\t" AFMM_WR("z0", "a0") "2:"
                     : [z0] "+v"(z[0]), [t] "=&s"(t)
                     : [n] "s"(n), [b0] "v"(b[0]), [a0] "v"(a[0]), [o] "i"(O)
                     : "scc", "memory");
    }
};
template <>
struct AccRow<2> {
    template <int O>
    __device__ __forceinline__ static void run(float (&z)[2], const float (&b)[2], uint32_t n,
                                               const uint32_t (&a)[2]) {
        uint32_t t;
        asm volatile("s_sub_u32 %[t], %[n], 1\n\ts_cbranch_scc1 2f\n"
                     "1:\n\t" AFMM_ADD("z0", "b0") AFMM_ADD("z1", "b1")
                     "s_sub_u32 %[t], %[t], 1\n\ts_cbranch_scc0 1b\n\t" AFMM_WR("z0", "a0")
                     AFMM_WR("z1", "a1") "2:"
                     : [z0] "+v"(z[0]), [z1] "+v"(z[1]), [t] "=&s"(t)
                     : [n] "s"(n), [b0] "v"(b[0]), [b1] "v"(b[1]), [a0] "v"(a[0]),
                       [a1] "v"(a[1]), [o] "i"(O)
                     : "scc", "memory");
    }
};
template <>
struct AccRow<4> {
    template <int O>
    __device__ __forceinline__ static void run(float (&z)[4], const float (&b)[4], uint32_t n,
                                               const uint32_t (&a)[4]) {
        uint32_t t;
        asm volatile("s_sub_u32 %[t], %[n], 1\n\ts_cbranch_scc1 2f\n"
                     "1:\n\t" AFMM_ADD("z0", "b0") AFMM_ADD("z1", "b1") AFMM_ADD("z2", "b2")
                     AFMM_ADD("z3", "b3") "s_sub_u32 %[t], %[t], 1\n\ts_cbranch_scc0 1b\n\t"
                     AFMM_WR("z0", "a0") AFMM_WR("z1", "a1") AFMM_WR("z2", "a2")
                     AFMM_WR("z3", "a3") "2:"
                     : [z0] "+v"(z[0]), [z1] "+v"(z[1]), [z2] "+v"(z[2]), [z3] "+v"(z[3]),
                       [t] "=&s"(t)
                     : [n] "s"(n), [b0] "v"(b[0]), [b1] "v"(b[1]), [b2] "v"(b[2]),
                       [b3] "v"(b[3]), [a0] "v"(a[0]), [a1] "v"(a[1]), [a2] "v"(a[2]),
                       [a3] "v"(a[3]), [o] "i"(O)
                     : "scc", "memory");
    }
};
#undef AFMM_RD
#undef AFMM_WR
#undef AFMM_ADD

// z[q] += b[q], n times over (n >= 1), for waves of more than two rows
// (compiled loop).
template <int E>
__device__ __forceinline__ void add_times(float (&z)[E], const float (&b)[E], uint32_t n) {
    do {
#pragma unroll
        for (int q = 0; q < E; ++q) z[q] = z[q] + b[q];
    } while (--n != 0);
}

// The common k in one block of assembly, for waves of one or two rows and a
// segment of exactly one group of 64*E slots (no escaped counts): each row's
// count is cut from its count word with s_bfe, whose SCC (count != 0) drives
// the branch, so a row costs two scalar instructions before its loads; with
// two rows, four paths (both rows, either, none) avoid testing a count twice,
// and row 1's reads are in flight while row 0 adds.  No load is left in flight
// when the block ends (its writes may be).
template <int R, int E>
struct AccK;

#define AFMM_LOOP(L_, N_, ADD_, WR_)                                                           \
    "s_sub_u32 %[t], %[" N_ "], 1\n" L_ ":\n\t" ADD_                                          \
    "s_sub_u32 %[t], %[t], 1\n\ts_cbranch_scc0 " L_ "b\n\t" WR_
#define AFMM_ONE_ROW(RD0, AD0, WR0)                                                            \
    "s_bfe_u32 %[n0], %[w0], %[i0]\n\ts_cbranch_scc0 90f\n\t" RD0                              \
    "s_waitcnt lgkmcnt(0)\n\t" AFMM_LOOP("11", "n0", AD0, WR0) "90:"
#define AFMM_TWO_ROWS(EL, RD0, RD1, AD0, AD1, WR0, WR1)                                        \
    "s_bfe_u32 %[n0], %[w0], %[i0]\n\ts_cbranch_scc0 50f\n\t"                                  \
    "s_bfe_u32 %[n1], %[w1], %[i1]\n\ts_cbranch_scc0 30f\n\t" RD0 RD1                          \
    "s_waitcnt lgkmcnt(" EL ")\n\t" AFMM_LOOP("11", "n0", AD0, WR0)                            \
    "s_waitcnt lgkmcnt(" EL ")\n\t" AFMM_LOOP("12", "n1", AD1, WR1) "s_branch 90f\n"           \
    "30:\n\t" RD0 "s_waitcnt lgkmcnt(0)\n\t" AFMM_LOOP("13", "n0", AD0, WR0) "s_branch 90f\n"  \
    "50:\n\ts_bfe_u32 %[n1], %[w1], %[i1]\n\ts_cbranch_scc0 90f\n\t" RD1                       \
    "s_waitcnt lgkmcnt(0)\n\t" AFMM_LOOP("14", "n1", AD1, WR1) "90:"

#define AFMM_RD0(q) "ds_read_b32 %[z0" #q "], %[a" #q "]\n\t"
#define AFMM_RD1(q) "ds_read_b32 %[z1" #q "], %[a" #q "] offset:%[o1]\n\t"
#define AFMM_AD0(q) "v_add_f32 %[z0" #q "], %[b" #q "], %[z0" #q "]\n\t"
#define AFMM_AD1(q) "v_add_f32 %[z1" #q "], %[b" #q "], %[z1" #q "]\n\t"
#define AFMM_WR0(q) "ds_write_b32 %[a" #q "], %[z0" #q "]\n\t"
#define AFMM_WR1(q) "ds_write_b32 %[a" #q "], %[z1" #q "] offset:%[o1]\n\t"
#define AFMM_X1(M) M(0)
#define AFMM_X2(M) M(0) M(1)
#define AFMM_X4(M) M(0) M(1) M(2) M(3)

template <>
struct AccK<1, 1> {
    template <int I0, int O1>
    __device__ __forceinline__ static void run(const uint32_t (&w)[1], const uint32_t (&a)[1],
                                               const float (&b)[1]) {
        float z00;
        uint32_t n0, t;
        asm volatile(AFMM_ONE_ROW(AFMM_X1(AFMM_RD0), AFMM_X1(AFMM_AD0), AFMM_X1(AFMM_WR0))
                     : [z00] "=&v"(z00), [n0] "=&s"(n0), [t] "=&s"(t)
                     : [w0] "s"(w[0]), [i0] "i"(I0), [a0] "v"(a[0]), [b0] "v"(b[0])
                     : "scc", "memory");
    }
};
template <>
struct AccK<1, 2> {
    template <int I0, int O1>
    __device__ __forceinline__ static void run(const uint32_t (&w)[1], const uint32_t (&a)[2],
                                               const float (&b)[2]) {
        float z00, z01;
        uint32_t n0, t;
        asm volatile(AFMM_ONE_ROW(AFMM_X2(AFMM_RD0), AFMM_X2(AFMM_AD0), AFMM_X2(AFMM_WR0))
                     : [z00] "=&v"(z00), [z01] "=&v"(z01), [n0] "=&s"(n0), [t] "=&s"(t)
                     : [w0] "s"(w[0]), [i0] "i"(I0), [a0] "v"(a[0]), [a1] "v"(a[1]),
                       [b0] "v"(b[0]), [b1] "v"(b[1])
                     : "scc", "memory");
    }
};
template <>
struct AccK<1, 4> {
    template <int I0, int O1>
    __device__ __forceinline__ static void run(const uint32_t (&w)[1], const uint32_t (&a)[4],
                                               const float (&b)[4]) {
        float z00, z01, z02, z03;
        uint32_t n0, t;
        asm volatile(AFMM_ONE_ROW(AFMM_X4(AFMM_RD0), AFMM_X4(AFMM_AD0), AFMM_X4(AFMM_WR0))
                     : [z00] "=&v"(z00), [z01] "=&v"(z01), [z02] "=&v"(z02), [z03] "=&v"(z03),
                       [n0] "=&s"(n0), [t] "=&s"(t)
                     : [w0] "s"(w[0]), [i0] "i"(I0), [a0] "v"(a[0]), [a1] "v"(a[1]),
                       [a2] "v"(a[2]), [a3] "v"(a[3]), [b0] "v"(b[0]), [b1] "v"(b[1]),
                       [b2] "v"(b[2]), [b3] "v"(b[3])
                     : "scc", "memory");
    }
};
template <>
struct AccK<2, 1> {
    template <int I0, int O1>
    __device__ __forceinline__ static void run(const uint32_t (&w)[2], const uint32_t (&a)[1],
                                               const float (&b)[1]) {
        float z00, z10;
        uint32_t n0, n1, t;
        asm volatile(AFMM_TWO_ROWS("1", AFMM_X1(AFMM_RD0), AFMM_X1(AFMM_RD1), AFMM_X1(AFMM_AD0),
                                   AFMM_X1(AFMM_AD1), AFMM_X1(AFMM_WR0), AFMM_X1(AFMM_WR1))
                     : [z00] "=&v"(z00), [z10] "=&v"(z10), [n0] "=&s"(n0), [n1] "=&s"(n1),
                       [t] "=&s"(t)
                     : [w0] "s"(w[0]), [w1] "s"(w[1]), [i0] "i"(I0), [i1] "i"(I0), [o1] "i"(O1),
                       [a0] "v"(a[0]), [b0] "v"(b[0])
                     : "scc", "memory");
    }
};
template <>
struct AccK<2, 2> {
    template <int I0, int O1>
    __device__ __forceinline__ static void run(const uint32_t (&w)[2], const uint32_t (&a)[2],
                                               const float (&b)[2]) {
        float z00, z01, z10, z11;
        uint32_t n0, n1, t;
        asm volatile(AFMM_TWO_ROWS("2", AFMM_X2(AFMM_RD0), AFMM_X2(AFMM_RD1), AFMM_X2(AFMM_AD0),
                                   AFMM_X2(AFMM_AD1), AFMM_X2(AFMM_WR0), AFMM_X2(AFMM_WR1))
                     : [z00] "=&v"(z00), [z01] "=&v"(z01), [z10] "=&v"(z10), [z11] "=&v"(z11),
                       [n0] "=&s"(n0), [n1] "=&s"(n1), [t] "=&s"(t)
                     : [w0] "s"(w[0]), [w1] "s"(w[1]), [i0] "i"(I0), [i1] "i"(I0), [o1] "i"(O1),
                       [a0] "v"(a[0]), [a1] "v"(a[1]), [b0] "v"(b[0]), [b1] "v"(b[1])
                     : "scc", "memory");
    }
};
template <>
struct AccK<2, 4> {
    template <int I0, int O1>
    __device__ __forceinline__ static void run(const uint32_t (&w)[2], const uint32_t (&a)[4],
                                               const float (&b)[4]) {
        float z00, z01, z02, z03, z10, z11, z12, z13;
        uint32_t n0, n1, t;
        asm volatile(AFMM_TWO_ROWS("4", AFMM_X4(AFMM_RD0), AFMM_X4(AFMM_RD1), AFMM_X4(AFMM_AD0),
                                   AFMM_X4(AFMM_AD1), AFMM_X4(AFMM_WR0), AFMM_X4(AFMM_WR1))
                     : [z00] "=&v"(z00), [z01] "=&v"(z01), [z02] "=&v"(z02), [z03] "=&v"(z03),
                       [z10] "=&v"(z10), [z11] "=&v"(z11), [z12] "=&v"(z12), [z13] "=&v"(z13),
                       [n0] "=&s"(n0), [n1] "=&s"(n1), [t] "=&s"(t)
                     : [w0] "s"(w[0]), [w1] "s"(w[1]), [i0] "i"(I0), [i1] "i"(I0), [o1] "i"(O1),
                       [a0] "v"(a[0]), [a1] "v"(a[1]), [a2] "v"(a[2]), [a3] "v"(a[3]),
                       [b0] "v"(b[0]), [b1] "v"(b[1]), [b2] "v"(b[2]), [b3] "v"(b[3])
                     : "scc", "memory");
    }
};
#undef AFMM_LOOP
#undef AFMM_ONE_ROW
#undef AFMM_TWO_ROWS
#undef AFMM_RD0
#undef AFMM_RD1
#undef AFMM_AD0
#undef AFMM_AD1
#undef AFMM_WR0
#undef AFMM_WR1
#undef AFMM_X1
#undef AFMM_X2
#undef AFMM_X4

// The 32-bit word of a row's count bytes that holds byte kk.
template <int KP>
__device__ __forceinline__ uint32_t count_word(const SparseCounts<KP>& c, int kk) {
    if constexpr (KP == 4) {
        return c.lo;
    } else if constexpr (KP == 8) {
        return (uint32_t)(c.lo >> (32 * (kk >> 2)));
    } else {
        return (uint32_t)((kk < 8 ? c.lo : c.hi) >> (32 * ((kk >> 2) & 1)));
    }
}

// Calls f(std::integral_constant<int, i>) for i = 0 .. N-1, each inlined.
template <int N, typename F, int... I>
__device__ __forceinline__ void static_for_impl(F&& f, std::integer_sequence<int, I...>) {
    (f(std::integral_constant<int, I>{}), ...);
}
template <int N, typename F>
__device__ __forceinline__ void static_for(F&& f) {
    static_for_impl<N>(f, std::make_integer_sequence<int, N>{});
}

// One chunk of 64*E slots of the segment of k0 + kk, slot q of lane l being
// entry ch_ + 64 q + l ({base bits, byte offset of its column in an LDS row};
// a slot without a base holds +0.0 on the lane's sink column, so every lane
// runs every slot).  Each of the wave's rows with a non-zero count reads its
// E Z elements from LDS, adds each slot's base `rep` times (the E chains side
// by side) and writes them back; the reads of all rows go out before the
// first addition.
#define AFMM_ACC_CHUNK(ev_)                                                                    \
    {                                                                                          \
        uint32_t ad_[T::E];                                                                    \
        float b_[T::E];                                                                        \
        _Pragma("unroll") for (int q = 0; q < T::E; ++q) {                                     \
            ad_[q] = arow_a + (ev_)[q][1];                                                     \
            b_[q] = __uint_as_float((ev_)[q][0]);                                              \
        }                                                                                      \
        if constexpr (R <= 2 || (R == 4 && T::E <= 2)) {                                      \
            float z_[R < 2 ? 2 : R][T::E];                                                     \
            AccAsm<T::E, R>::template read<T::STRIDE * 4>(z_, rep_, ad_);                      \
            AccRow<T::E>::template run<0>(z_[0], b_, rep_[0], ad_);                            \
            if constexpr (R >= 2) AccRow<T::E>::template run<T::STRIDE * 4>(z_[1], b_, rep_[1], ad_); \
            if constexpr (R == 4) {                                                            \
                AccRow<T::E>::template run<2 * T::STRIDE * 4>(z_[2], b_, rep_[2], ad_);        \
                AccRow<T::E>::template run<3 * T::STRIDE * 4>(z_[3], b_, rep_[3], ad_);        \
            }                                                                                  \
        } else {                                                                               \
            float z_[R][T::E];                                                                 \
            _Pragma("unroll") for (int r = 0; r < R; ++r) {                                    \
                if (rep_[r] == 0) continue;                                                    \
                _Pragma("unroll") for (int q = 0; q < T::E; ++q) z_[r][q] =                    \
                    *lds_at(ad_[q] + r * T::STRIDE * 4);                                       \
            }                                                                                  \
            __builtin_amdgcn_s_waitcnt(kWaitLgkm0);                                            \
            _Pragma("unroll") for (int r = 0; r < R; ++r) {                                    \
                if (rep_[r] == 0) continue;                                                    \
                add_times<T::E>(z_[r], b_, rep_[r]);                                           \
                _Pragma("unroll") for (int q = 0; q < T::E; ++q)                               \
                    *lds_at(ad_[q] + r * T::STRIDE * 4) = z_[r][q];                            \
            }                                                                                  \
        }                                                                                      \
    }

// The additions of k0 + kk for the wave's R rows: the prefetched first 64*E
// slots, then (longer segments) the rest, 64*E at a time.  Segment lengths are
// 0 or multiples of 64*E.
#define AFMM_ACC_K(kk)                                                                         \
    if constexpr (!ESC && R <= 2) {                                                            \
        const int len_ = Lc[kk];                                                               \
        if (len_ != 0) {                                                                       \
            uint32_t w_[R], ad_[T::E];                                                         \
            float b_[T::E];                                                                    \
            _Pragma("unroll") for (int r = 0; r < R; ++r) w_[r] = count_word<KP>(cw[r], kk);   \
            _Pragma("unroll") for (int q = 0; q < T::E; ++q) {                                 \
                ad_[q] = arow_a + ec[kk][q][1];                                                \
                b_[q] = __uint_as_float(ec[kk][q][0]);                                         \
            }                                                                                  \
            AccK<R, T::E>::template run<((kk) % 4) * 8 | (8 << 16), T::STRIDE * 4>(w_, ad_, b_); \
            if (__builtin_expect(len_ > kWave * T::E, 0)) {                                    \
                uint32_t rep_[R];                                                              \
                _Pragma("unroll") for (int r = 0; r < R; ++r) rep_[r] = cw[r].byte(kk);        \
                AFMM_ACC_MORE(kk)                                                              \
            }                                                                                  \
        }                                                                                      \
    } else {                                                                                   \
        AFMM_ACC_K_ANY(kk);                                                                    \
    }

// The slots of k0 + kk past the first 64*E, 64*E at a time.
#define AFMM_ACC_MORE(kk)                                                                      \
    for (int ch2_ = kWave * T::E; ch2_ < len_; ch2_ += kWave * T::E) {                         \
        u32x2_t e2_[T::E];                                                                     \
        _Pragma("unroll") for (int q = 0; q < T::E; ++q) e2_[q] =                              \
            __builtin_amdgcn_raw_buffer_load_b64(                                              \
                ers, (uint32_t)(((k0 + (kk)) * T::CT + ch2_ + q * kWave + lane) * 8), 0,       \
                0); /* ch2_ + q * 64 + lane < CT */                                            \
        AFMM_ACC_CHUNK(e2_)                                                                    \
    }

// Any k: escaped counts, waves of more than two rows.
#define AFMM_ACC_K_ANY(kk)                                                                     \
    do {                                                                                       \
        const int len_ = Lc[kk];                                                               \
        if (len_ == 0) break;                                                                  \
        uint32_t rep_[R];                                                                      \
        uint32_t any_ = 0;                                                                     \
        _Pragma("unroll") for (int r = 0; r < R; ++r) {                                        \
            uint32_t v_ = cw[r].byte(kk);                                                      \
            if (ESC && v_ == 0xFFu) {                                                          \
                const int32_t full_ = __builtin_amdgcn_readfirstlane(                          \
                    P32[(int64_t)(rw0 + r) * p32_sr + (int64_t)(k0 + (kk)) * p32_sk]);         \
                /* >= 255 by construction; a value changed under a running call */             \
                /* must still end the repetition loop */                                       \
                v_ = full_ > 0 ? (uint32_t)full_ : 0u;                                         \
            }                                                                                  \
            rep_[r] = v_;                                                                      \
            any_ |= v_;                                                                        \
        }                                                                                      \
        if (any_ == 0) break;                                                                  \
        AFMM_ACC_CHUNK(ec[kk])                                                                 \
        AFMM_ACC_MORE(kk)                                                                      \
    } while (0)

template <int R, int C, int W, int KP, bool TRANS_OUT, bool ESC>
__device__ __forceinline__ void rep_acc_tile(int n_r, int n_c, int n_k,
                                             const uint8_t* __restrict__ P8, int64_t ldp,
                                             const int32_t* __restrict__ P32, int64_t p32_sr,
                                             int64_t p32_sk, const uint2* __restrict__ ent,
                                             const int32_t* __restrict__ lens, int64_t n_k_pad,
                                             float* __restrict__ Z, int64_t z_sr, int64_t z_sc,
                                             int r0, int band, float* lds) {
    using T = AccTile<R, C, W, KP>;
    constexpr int NT = W * kWave;
    const int lane = threadIdx.x & (kWave - 1);
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x / kWave);
    const int rw0 = r0 + wave * R;
    const int c0 = band * T::CT;
    // LDS byte address of the wave's first row (entries hold byte offsets in a row)
    const uint32_t arow_a = lds_address(lds + wave * R * T::STRIDE);

    // Z starts at +0.0 (the sink columns too: they only ever receive +0.0)
    float4* l4 = reinterpret_cast<float4*>(lds);
    for (int i = threadIdx.x; i < T::LDS_FLOATS / 4; i += NT) l4[i] = make_float4(0.f, 0.f, 0.f, 0.f);
    __syncthreads();

    // The band's segments, their lengths and the count bytes go through buffer
    // resources (byte offsets in 31 bits, checked by the launcher), so the next
    // panel's loads run on the vector memory counter while this panel's LDS
    // traffic waits on its own.
    const __amdgpu_buffer_rsrc_t ers = __builtin_amdgcn_make_buffer_rsrc(
        const_cast<uint2*>(ent + (int64_t)band * n_k_pad * T::CT), (short)0,
        (int)(n_k_pad * T::CT * 8), 0x00020000);
    const __amdgpu_buffer_rsrc_t lrs = __builtin_amdgcn_make_buffer_rsrc(
        const_cast<int32_t*>(lens + (int64_t)band * n_k_pad), (short)0, (int)(n_k_pad * 4),
        0x00020000);
    const int rows_bound = (n_r + T::TM - 1) / T::TM * T::TM;
    const __amdgpu_buffer_rsrc_t crs = __builtin_amdgcn_make_buffer_rsrc(
        const_cast<uint8_t*>(P8), (short)0, (int)((int64_t)rows_bound * ldp), 0x00020000);

    const int n_panels = (n_k + KP - 1) / KP;
    int32_t Lc[KP];
    u32x2_t ec[KP][T::E];
    SparseCounts<KP> cw[R];
    {
        u32x4_t lv[KP / 4];
        CountFetch<KP> cf[R];
#pragma unroll
        for (int q = 0; q < KP / 4; ++q)
            lv[q] = __builtin_amdgcn_raw_buffer_load_b128(lrs, (uint32_t)(q * 16), 0, 0);
#pragma unroll
        for (int kk = 0; kk < KP; ++kk)
#pragma unroll
            for (int q = 0; q < T::E; ++q)
                ec[kk][q] = __builtin_amdgcn_raw_buffer_load_b64(
                    ers, (uint32_t)((kk * T::CT + q * kWave + lane) * 8), 0, 0);
#pragma unroll
        for (int r = 0; r < R; ++r) cf[r].fetch(crs, (uint32_t)((rw0 + r) * ldp));
#pragma unroll
        for (int kk = 0; kk < KP; ++kk) Lc[kk] = (int32_t)uniform_u32(lv[kk / 4][kk % 4]);
#pragma unroll
        for (int r = 0; r < R; ++r) cf[r].to(cw[r]);
        // both ways into the loop arrive with nothing pending (see the end of
        // the loop body): an empty statement that reads the entries keeps
        // their loads above it and makes the compiler wait for them here
#pragma unroll
        for (int kk = 0; kk < KP; ++kk)
#pragma unroll
            for (int q = 0; q < T::E; ++q) asm volatile("" ::"v"(ec[kk][q]));
    }

    for (int p = 0; p < n_panels; ++p) {
        const int k0 = p * KP;
        const bool more = p + 1 < n_panels;
        u32x4_t lv[KP / 4];
        u32x2_t en[KP][T::E];
        CountFetch<KP> cf[R];
        if (more) {
            const int k1 = k0 + KP;
#pragma unroll
            for (int q = 0; q < KP / 4; ++q)
                lv[q] = __builtin_amdgcn_raw_buffer_load_b128(lrs, (uint32_t)((k1 + 4 * q) * 4), 0, 0);
#pragma unroll
            for (int kk = 0; kk < KP; ++kk)
#pragma unroll
                for (int q = 0; q < T::E; ++q)
                    en[kk][q] = __builtin_amdgcn_raw_buffer_load_b64(
                        ers, (uint32_t)(((k1 + kk) * T::CT + q * kWave + lane) * 8), 0, 0);
#pragma unroll
            for (int r = 0; r < R; ++r) cf[r].fetch(crs, (uint32_t)((rw0 + r) * ldp + k1));
        }
        static_for<KP>([&](auto kc) __attribute__((always_inline)) {
            constexpr int kk = decltype(kc)::value;
            AFMM_ACC_K(kk);
        });
        // the next panel's loads have had this whole panel to land; waiting for
        // them here leaves nothing pending at the top of the loop, so the uses
        // of the entries there need no wait of their own
        __builtin_amdgcn_s_waitcnt(kAccWaitVm0);
        if (more) {
#pragma unroll
            for (int kk = 0; kk < KP; ++kk) {
                Lc[kk] = (int32_t)uniform_u32(lv[kk / 4][kk % 4]);
#pragma unroll
                for (int q = 0; q < T::E; ++q) ec[kk][q] = en[kk][q];
            }
#pragma unroll
            for (int r = 0; r < R; ++r) cf[r].to(cw[r]);
        }
    }
    __syncthreads();

    if (TRANS_OUT) {
        // element (r, c) at Z[(c0 + c) * z_sc + r0 + r]: runs of TM rows per column
        for (int i = threadIdx.x; i < T::TM * T::CT; i += NT) {
            const int r = i % T::TM, c = i / T::TM;
            if (r0 + r < n_r && c0 + c < n_c)
                Z[(int64_t)(c0 + c) * z_sc + r0 + r] = lds[r * T::STRIDE + c];
        }
    } else {
        for (int i = threadIdx.x; i < T::TM * T::CT; i += NT) {
            const int c = i % T::CT, r = i / T::CT;
            if (r0 + r < n_r && c0 + c < n_c)
                Z[(int64_t)(r0 + r) * z_sr + c0 + c] = lds[r * T::STRIDE + c];
        }
    }
}
#undef AFMM_ACC_K
#undef AFMM_ACC_K_ANY
#undef AFMM_ACC_MORE
#undef AFMM_ACC_CHUNK

template <int R, int C, int W, int KP, bool TRANS_OUT>
__global__ __launch_bounds__(W * kWave) void rep_acc_kernel(
    int n_r, int n_c, int n_k, const uint8_t* __restrict__ P8, int64_t ldp,
    const int32_t* __restrict__ P32, int64_t p32_sr, int64_t p32_sk, const uint2* __restrict__ ent,
    const int32_t* __restrict__ lens, int64_t n_k_pad, float* __restrict__ Z, int64_t z_sr,
    int64_t z_sc, const uint32_t* __restrict__ esc, int n_row_blocks, int n_tiles,
    const uint32_t* __restrict__ gate) {
    using T = AccTile<R, C, W, KP>;
    __shared__ __attribute__((aligned(16))) float lds[T::LDS_FLOATS];
    AFMM_GATE(gate);
    const int t = xcd_remap(blockIdx.x, n_tiles);
    const int band = t / n_row_blocks, rb = t - band * n_row_blocks;
    if (*esc)
        rep_acc_tile<R, C, W, KP, TRANS_OUT, true>(n_r, n_c, n_k, P8, ldp, P32, p32_sr, p32_sk,
                                                      ent, lens, n_k_pad, Z, z_sr, z_sc,
                                                      rb * T::TM, band, lds);
    else
        rep_acc_tile<R, C, W, KP, TRANS_OUT, false>(n_r, n_c, n_k, P8, ldp, P32, p32_sr,
                                                       p32_sk, ent, lens, n_k_pad, Z, z_sr, z_sc,
                                                       rb * T::TM, band, lds);
}

template <int R, int C, int W, int KP>
hipError_t launch_acc(const StrictArgs& a, const AccLists& L, hipStream_t s) {
    using T = AccTile<R, C, W, KP>;
    if (!rep_acc_usable(a, C)) return hipErrorInvalidValue;
    const int n_row_blocks = (a.n_r + T::TM - 1) / T::TM;
    const int n_tiles = n_row_blocks * ((a.n_c + T::CT - 1) / T::CT);
    dim3 grid(n_tiles), block(W * kWave);
    if (a.trans_out)
        hipLaunchKernelGGL((rep_acc_kernel<R, C, W, KP, true>), grid, block, 0, s, a.n_r,
                           a.n_c, a.n_k, a.P8, a.ldp, a.P32, a.p32_sr, a.p32_sk, L.ent, L.lens,
                           L.n_k_pad, a.Z, a.z_sr, a.z_sc, a.esc, n_row_blocks, n_tiles, a.gate);
    else
        hipLaunchKernelGGL((rep_acc_kernel<R, C, W, KP, false>), grid, block, 0, s, a.n_r,
                           a.n_c, a.n_k, a.P8, a.ldp, a.P32, a.p32_sr, a.p32_sk, L.ent, L.lens,
                           L.n_k_pad, a.Z, a.z_sr, a.z_sc, a.esc, n_row_blocks, n_tiles, a.gate);
    return hipGetLastError();
}

// (R, C, W, U, KP): TM = W*R rows x CT = 64*C columns of Z in LDS per block;
// each lane takes max(1, C/16) entries of a k's segment.  U is accepted and
// ignored: the repetitions run in a counted scalar loop (add_times).
#define AFMM_ACC_CONFIGS(X) \
    X(4, 16, 8, 1, 16)      \
    X(4, 16, 8, 2, 16)      \
    X(4, 16, 8, 4, 16)      \
    X(2, 16, 16, 1, 16)     \
    X(2, 16, 16, 2, 16)     \
    X(2, 16, 16, 4, 16)     \
    X(4, 8, 16, 1, 16)      \
    X(8, 8, 8, 1, 16)       \
    X(4, 4, 8, 1, 16)       \
    X(2, 32, 8, 2, 8)       \
    X(1, 32, 16, 2, 8)      \
    X(1, 64, 8, 2, 8)       \
    X(1, 64, 8, 1, 8)       \
    X(2, 32, 8, 1, 16)      \
    X(1, 16, 16, 1, 16)     \
    X(2, 16, 8, 1, 16)      \
    X(1, 16, 8, 1, 8)       \
    X(1, 16, 16, 1, 8)      \
    X(1, 32, 8, 1, 8)       \
    X(2, 16, 8, 1, 8)       \
    X(1, 16, 8, 1, 16)      \
    X(4, 16, 4, 1, 16)      \
    X(4, 16, 4, 1, 8)       \
    X(4, 32, 4, 1, 8)

bool rep_acc_usable(const StrictArgs& a, int C) {
    // buffer-resource byte offsets of one band's segments and of the count
    // bytes in 31 bits
    const int64_t lim = (int64_t)1 << 31;
    return round_up(a.n_k, kAccKP) * kWave * C * 8 < lim &&
           round_up(a.n_r, kRowPad) * a.ldp < lim;
}

bool rep_acc_supported(int R, int C, int W, int U, int KP) {
#define AFMM_CASE(r, c, w, u, kp) \
    if (R == r && C == c && W == w && U == u && KP == kp) return true;
    AFMM_ACC_CONFIGS(AFMM_CASE)
#undef AFMM_CASE
    return false;
}

hipError_t launch_rep_acc(const StrictArgs& a, const AccLists& L, int R, int C, int W, int U,
                          int KP, hipStream_t s) {
#define AFMM_CASE(r, c, w, u, kp) \
    if (R == r && C == c && W == w && U == u && KP == kp) return launch_acc<r, c, w, kp>(a, L, s);
    AFMM_ACC_CONFIGS(AFMM_CASE)
#undef AFMM_CASE
    return hipErrorInvalidValue;
}

}  // namespace afmm
