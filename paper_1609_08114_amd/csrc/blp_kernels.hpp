// Device-side declarations shared by the solver's HIP kernels and the host
// runtime that launches them.  gfx950 (CDNA4) only: 64-lane wavefronts.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace blp {

constexpr int ST_OPTIMAL = 0, ST_INFEASIBLE = 1, ST_UNBOUNDED = 2, ST_ITER_LIMIT = 3, ST_NUMERICAL = 4;
constexpr int ST_INTERNAL = -1;  // an LP reached a kernel it does not fit (scheduling bug)
constexpr int ID_NONE = 0x7fffffff;
// pivots a recorded trace may hold per LP (the replay keeps them in LDS)
constexpr int kTraceMaxPivots = 256;

// Row flag bits kept in LDS per constraint row.
constexpr unsigned char RF_GE = 1;    // user wrote ">="
constexpr unsigned char RF_ART = 2;   // "<=" form has a negative rhs: surplus + artificial
constexpr unsigned char RF_DEAD = 4;  // redundant row found at the end of phase 1

// Everything a solve kernel needs, passed by value.
struct KParams {
    // batch description (device pointers; per-LP arrays NULL for uniform batches)
    int64_t count;
    int32_t uniform, um, un, ukind;
    const int32_t* m;
    const int32_t* n;
    const int32_t* kind;
    const int64_t* a_off;
    const int64_t* row_off;
    const int64_t* col_off;
    const double* A;
    const double* b;
    const int8_t* sense;
    const double* c;
    const double* l;
    const double* u;
    // outputs
    int32_t* status;
    int32_t* iters;
    double* obj;
    double* x;
    double* y;
    // method options
    int32_t max_iter, bland_after;  // <= 0: per-LP defaults 50 (m + n) and max(m, n)
    double eps_price, eps_piv, eps_feas;
    // work lists: bin `bin` holds bin_len[bin] LP indices at list + bin_off[bin].
    // list == NULL means the identity list 0..count-1.
    const int32_t* list;
    const int32_t* bin_off;
    const int32_t* bin_len;
    int32_t* bin_head;  // persistent mode: next entry to take (atomic), bin b's at bin_head[b * kHeadStride]
    int32_t bin;
    int32_t direct;       // 1: entry = direct_first + blockIdx.x, no queue
    int64_t chunk;        // shared-constraint mode: LPs taken per queue pop
    int32_t shared_in;    // 1: every LP reads A, b and sense at offset 0 (one shared constraint set)
    int32_t box_shared;   // 1: every hyperbox LP reads l and u at offset 0 (one shared box)
    int64_t direct_first;
    int64_t direct_end;   // kernels with several LPs per workgroup: positions >= direct_end are not taken (0: none)
    // streaming kernel workspace: one slot of ws_slot doubles per workgroup
    double* ws;
    int64_t ws_slot;
    int32_t ws_ld;   // leading dimension (rows, multiple of 16)
    int32_t ws_cols; // columns available per slot
    int32_t ws_lds;  // doubles of dynamic LDS for on-chip columns (0: none)
    // pivot trace of the 112 x 112 block tile: LP k's record at
    // trace + k * trace_stride is [count, row 0, slot 0, row 1, slot 1, ...]
    int32_t* trace;
    int32_t trace_stride;
    // phase cycle counters (only with -DBLP_PHASE_TIMERS; NULL otherwise)
    unsigned long long* timers;
    // entering rule: 0 largest coefficient, 1 random positive coefficient
    int32_t pivot_rule;
    // streaming workspace: 0 column-major (element (i, j) at ws[j*ws_ld + i]),
    // 1 row-major (at ws[i*ws_cols + j])
    int32_t layout;
    uint64_t seed;
};

// Workgroup barrier for communication through LDS only: each wave waits for
// its own LDS operations, not for its global loads and stores, so output
// stores drain and prefetches stay in flight across it.  The simplex kernels
// that keep their tableau in registers share data only through LDS.
__device__ __forceinline__ void lds_barrier() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup", "local");
    __builtin_amdgcn_s_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup", "local");
}

// Optional in-kernel phase timers (s_memtime cycles of wave 0, summed over
// workgroups): build with -DBLP_PHASE_TIMERS.  Slots: 0 load, 1 price,
// 2 entering-column publish, 3 ratio test + pivot-row division + barrier,
// 4 pivot update, 5 extraction, 6 pivots, 7 LPs; block-tile kernel only:
// 8 ratio test alone, 9 pivot-row division in the owning wave, 10 pivots
// whose row wave 0 owns; 11 the load up to the rows' preparation, 12 from
// there to the finished tile (block-tile kernel).
enum {
    TM_LOAD = 0, TM_PRICE, TM_PUBCOL, TM_RATIO, TM_PIVOT, TM_EXTRACT, TM_PIVOTS, TM_LPS,
    TM_RTEST, TM_DIV, TM_DIVN, TM_LD_ROWS, TM_LD_TILE, TM_SLOTS
};
#ifdef BLP_PHASE_TIMERS
#define BLP_TDECL unsigned long long tm_acc_[TM_SLOTS] = {}
#define BLP_T(v) const unsigned long long v = __builtin_readcyclecounter()
#define BLP_TACC(slot, a, b) (tm_acc_[slot] += (b) - (a))
#define BLP_TCOUNT(slot, n) (tm_acc_[slot] += (n))
#define BLP_TFLUSH()                                                                  \
    do {                                                                              \
        if (threadIdx.x == 0 && P.timers)                                             \
            for (int s_ = 0; s_ < TM_SLOTS; ++s_) atomicAdd(P.timers + s_, tm_acc_[s_]); \
    } while (0)
#else
#define BLP_TDECL
#define BLP_T(v)
#define BLP_TACC(slot, a, b)
#define BLP_TCOUNT(slot, n)
#define BLP_TFLUSH()
#endif

struct LpRef {
    int32_t m, n;
    int64_t a_off, row_off, col_off;
};

__device__ __forceinline__ LpRef lp_ref(const KParams& P, int64_t k) {
    LpRef r;
    if (P.uniform) {
        r.m = P.um;
        r.n = P.un;
        r.a_off = k * (int64_t)P.um * P.un;
        r.row_off = k * (int64_t)P.um;
        r.col_off = k * (int64_t)P.un;
    } else {
        r.m = P.m[k];
        r.n = P.n[k];
        r.a_off = P.a_off[k];
        r.row_off = P.row_off[k];
        r.col_off = P.col_off[k];
    }
    return r;
}

// Where LP k reads its constraints: its own A, b and sense, or, in a launch
// over one shared constraint set, offset 0 for every LP (the objective and
// the outputs stay per LP).
__device__ __forceinline__ LpRef lp_in(const KParams& P, const LpRef& L) {
    LpRef r = L;
    if (P.shared_in) r.a_off = r.row_off = 0;
    return r;
}

__device__ __forceinline__ int lp_kind(const KParams& P, int64_t k) { return P.uniform ? P.ukind : P.kind[k]; }

// Entry count of this launch's work list.
__device__ __forceinline__ int64_t work_len(const KParams& P) {
    return P.list ? (int64_t)P.bin_len[P.bin] : P.count;
}
__device__ __forceinline__ int64_t work_item(const KParams& P, int64_t q) {
    return P.list ? (int64_t)P.list[P.bin_off[P.bin] + q] : q;
}
// Work-list heads are kHeadStride ints (one 128-byte cache line) apart, so
// that the persistent workgroups' atomics on a head share no line with the
// bins' offsets and lengths, which every pop reads, nor with another bin's
// head.  Sharing a line with the offsets made the 100 x 100 block-tile
// solve ~3% slower.
constexpr int kHeadStride = 32;
__device__ __forceinline__ int* bin_head_of(const KParams& P) { return P.bin_head + P.bin * kHeadStride; }

// Next queue position of this launch's work list (one lane calls it).  On a
// workgroup's first pop the head is read plainly first: when the list is
// empty (or already exhausted) the workgroups of the launch leave without an
// atomic each, which thousands of them would serialise on one address.
// Later pops go straight to the atomic (the extra read would add a memory
// round trip per LP).
__device__ __forceinline__ int pop_position(const KParams& P, int64_t len, bool first) {
    int* head = bin_head_of(P);
    if (first && __hip_atomic_load(head, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) >= len) return (int)len;
    return atomicAdd(head, 1);
}

// ---------------------------------------------------------------------------
// Wave-wide arg-max of (key, id) pairs under the total order
//   a before b  <=>  a.key > b.key, or a.key == b.key and a.id < b.id
// carrying a payload.  Ids are unique within a reduction, so every lane ends
// with the same winner whatever the combination order.  The id (< 2^15) and
// the payload position (< 2^16) travel packed in one dword, id in the high
// half, so comparing packed values orders by id.
// ---------------------------------------------------------------------------
__device__ __forceinline__ bool key_before(double ak, int aid, double bk, int bid) {
    return ak > bk || (ak == bk && aid < bid);
}

constexpr int PACK_NONE = 0x7fffffff;
__device__ __forceinline__ int pack_id(int id, int pos) { return id == ID_NONE ? PACK_NONE : (id << 16) | pos; }
__device__ __forceinline__ int unpack_id(int p) { return p == PACK_NONE ? ID_NONE : (p >> 16); }
__device__ __forceinline__ int unpack_pos(int p) { return p == PACK_NONE ? -1 : (p & 0xffff); }

// Value of the DPP source lane.  With every row enabled (RM = 0xF) the
// controls used here read a valid lane for every lane, so no "old" value is
// needed and the move can fold into its consumer; with a partial row mask the
// disabled rows keep their own value.
template <int CTRL, int RM = 0xF>
__device__ __forceinline__ int dpp_i32(int v) {
    if constexpr (RM == 0xF)
        return __builtin_amdgcn_mov_dpp(v, CTRL, 0xF, 0xF, true);
    else
        return __builtin_amdgcn_update_dpp(v, v, CTRL, RM, 0xF, false);
}
template <int CTRL, int RM = 0xF>
__device__ __forceinline__ double dpp_f64(double v) {
    return __hiloint2double(dpp_i32<CTRL, RM>(__double2hiint(v)), dpp_i32<CTRL, RM>(__double2loint(v)));
}
template <int CTRL, int RM = 0xF>
__device__ __forceinline__ int dpp_min_i32(int v) {
    const int o = dpp_i32<CTRL, RM>(v);
    return o < v ? o : v;
}

// Wave maximum of a signed (hi) or unsigned (lo) dword, valid in lane 63:
// four in-row DPP steps, then row broadcasts 15 and 31 into rows 1 and 3
// (the other rows end with unspecified values; only lane 63 is read).  Each
// step is one max with a DPP operand.
template <int CTRL, int RM>
__device__ __forceinline__ int dpp_src(int v) {
    return __builtin_amdgcn_mov_dpp(v, CTRL, RM, 0xF, RM == 0xF);
}
__device__ __forceinline__ int wave_max_i32(int v) {
    v = max(v, dpp_src<0xB1, 0xF>(v));   // quad_perm [1,0,3,2]
    v = max(v, dpp_src<0x4E, 0xF>(v));   // quad_perm [2,3,0,1]
    v = max(v, dpp_src<0x141, 0xF>(v));  // row_half_mirror
    v = max(v, dpp_src<0x140, 0xF>(v));  // row_mirror
    v = max(v, dpp_src<0x142, 0xA>(v));  // row_bcast:15
    v = max(v, dpp_src<0x143, 0xC>(v));  // row_bcast:31
    return __builtin_amdgcn_readlane(v, 63);
}
__device__ __forceinline__ unsigned wave_max_u32(unsigned v) {
    v = max(v, (unsigned)dpp_src<0xB1, 0xF>((int)v));
    v = max(v, (unsigned)dpp_src<0x4E, 0xF>((int)v));
    v = max(v, (unsigned)dpp_src<0x141, 0xF>((int)v));
    v = max(v, (unsigned)dpp_src<0x140, 0xF>((int)v));
    v = max(v, (unsigned)dpp_src<0x142, 0xA>((int)v));
    v = max(v, (unsigned)dpp_src<0x143, 0xC>((int)v));
    return (unsigned)__builtin_amdgcn_readlane((int)v, 63);
}
__device__ __forceinline__ int wave_min_i32(int v) {
    v = min(v, dpp_src<0xB1, 0xF>(v));
    v = min(v, dpp_src<0x4E, 0xF>(v));
    v = min(v, dpp_src<0x141, 0xF>(v));
    v = min(v, dpp_src<0x140, 0xF>(v));
    v = min(v, dpp_src<0x142, 0xA>(v));
    v = min(v, dpp_src<0x143, 0xC>(v));
    return __builtin_amdgcn_readlane(v, 63);
}

// Wave-wide arg-max of 64-bit integer keys (hi signed, lo unsigned: the
// value hi * 2^32 + lo), ties to the smallest packed (id, pos); the packed
// winner and its key are returned wave-uniform.  For doubles that are all
// >= +0 or -inf, the bit pattern is such a key and orders like the double;
// the bitwise complement of a key reverses the order (a minimum).  Exact
// ties are rare, so the tie passes run only when the ballot of lanes
// holding the maximum has more than one lane.  All 64 lanes must be active.
__device__ __forceinline__ int wave_argmax_i64(int hi, unsigned lo, int pk, int& top_hi, unsigned& top_lo) {
    top_hi = wave_max_i32(hi);
    const bool h_eq = hi == top_hi;
    const uint64_t m1 = __ballot(h_eq);
    if (__popcll(m1) == 1) {
        const int w = __ffsll((long long)m1) - 1;
        top_lo = (unsigned)__builtin_amdgcn_readlane((int)lo, w);
        return __builtin_amdgcn_readlane(pk, w);
    }
    top_lo = wave_max_u32(h_eq ? lo : 0u);
    const bool eq = h_eq & (lo == top_lo);
    const uint64_t m2 = __ballot(eq);
    if (__popcll(m2) == 1) return __builtin_amdgcn_readlane(pk, __ffsll((long long)m2) - 1);
    return wave_min_i32(eq ? pk : PACK_NONE);
}

// All 64 lanes must be active.  On return id/pos are wave-uniform.
// Two passes of six DPP steps each: the maximum key (quad permutes, half-row
// and row mirrors, then row broadcasts 15 and 31 into lane 63), then the
// minimum packed (id, pos) among the lanes holding that key.  Lanes without
// a candidate carry key -inf and id ID_NONE; a NaN key is never chosen.
// Same winner as the pairwise order key_before().
__device__ __forceinline__ void wave_argmax(double& k, int& id, int& pos) {
    double mx = k;
    mx = fmax(mx, dpp_f64<0xB1>(mx));        // quad_perm [1,0,3,2]
    mx = fmax(mx, dpp_f64<0x4E>(mx));        // quad_perm [2,3,0,1]
    mx = fmax(mx, dpp_f64<0x141>(mx));       // row_half_mirror
    mx = fmax(mx, dpp_f64<0x140>(mx));       // row_mirror
    mx = fmax(mx, dpp_f64<0x142, 0xA>(mx));  // row_bcast:15 into rows 1, 3
    mx = fmax(mx, dpp_f64<0x143, 0xC>(mx));  // row_bcast:31 into rows 2, 3
    const double top = __hiloint2double(__builtin_amdgcn_readlane(__double2hiint(mx), 63),
                                        __builtin_amdgcn_readlane(__double2loint(mx), 63));
    int pk = k == top ? pack_id(id, pos) : PACK_NONE;
    pk = dpp_min_i32<0xB1>(pk);
    pk = dpp_min_i32<0x4E>(pk);
    pk = dpp_min_i32<0x141>(pk);
    pk = dpp_min_i32<0x140>(pk);
    pk = dpp_min_i32<0x142, 0xA>(pk);
    pk = dpp_min_i32<0x143, 0xC>(pk);
    pk = __builtin_amdgcn_readlane(pk, 63);
    k = top;
    id = unpack_id(pk);
    pos = unpack_pos(pk);
}

}  // namespace blp
