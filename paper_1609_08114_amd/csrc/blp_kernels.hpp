// Device-side declarations shared by the solver's HIP kernels and the host
// runtime that launches them.  gfx950 (CDNA4) only: 64-lane wavefronts.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace blp {

constexpr int ST_OPTIMAL = 0, ST_INFEASIBLE = 1, ST_UNBOUNDED = 2, ST_ITER_LIMIT = 3, ST_NUMERICAL = 4;
constexpr int ST_INTERNAL = -1;  // an LP reached a kernel it does not fit (scheduling bug)
constexpr int ID_NONE = 0x7fffffff;

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
    int32_t* bin_head;  // persistent mode: next entry to take (atomic)
    int32_t bin;
    int32_t direct;       // 1: entry = direct_first + blockIdx.x, no queue
    int64_t direct_first;
    // streaming kernel workspace: one slot of ws_slot doubles per workgroup
    double* ws;
    int64_t ws_slot;
    int32_t ws_ld;   // leading dimension (rows, multiple of 16)
    int32_t ws_cols; // columns available per slot
    // phase cycle counters (only with -DBLP_PHASE_TIMERS; NULL otherwise)
    unsigned long long* timers;
    // entering rule: 0 largest coefficient, 1 random positive coefficient
    int32_t pivot_rule;
    uint64_t seed;
};

// Optional in-kernel phase timers (s_memtime cycles of wave 0, summed over
// workgroups): build with -DBLP_PHASE_TIMERS.  Slots: 0 load, 1 price,
// 2 entering-column publish, 3 ratio test, 4 pivot update, 5 extraction,
// 6 pivots, 7 LPs.
enum { TM_LOAD = 0, TM_PRICE, TM_PUBCOL, TM_RATIO, TM_PIVOT, TM_EXTRACT, TM_PIVOTS, TM_LPS, TM_SLOTS };
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

__device__ __forceinline__ int lp_kind(const KParams& P, int64_t k) { return P.uniform ? P.ukind : P.kind[k]; }

// Entry count of this launch's work list.
__device__ __forceinline__ int64_t work_len(const KParams& P) {
    return P.list ? (int64_t)P.bin_len[P.bin] : P.count;
}
__device__ __forceinline__ int64_t work_item(const KParams& P, int64_t q) {
    return P.list ? (int64_t)P.list[P.bin_off[P.bin] + q] : q;
}

// ---------------------------------------------------------------------------
// Wave-wide arg-max of (key, id) pairs under the total order
//   a before b  <=>  a.key > b.key, or a.key == b.key and a.id < b.id
// carrying a payload.  Ids are unique within a reduction, so every lane ends
// with the same winner whatever the combination order.  The id (< 2^15) and
// the payload position (< 2^16) travel packed in one dword, id in the high
// half, so comparing packed values orders by id.  Within each 16-lane row
// the exchange uses DPP (quad permutes, then row rotations by 4 and 8);
// across rows, gfx950's permlane16/permlane32 swaps (lane ^ 16, lane ^ 32).
// ---------------------------------------------------------------------------
__device__ __forceinline__ bool key_before(double ak, int aid, double bk, int bid) {
    return ak > bk || (ak == bk && aid < bid);
}

constexpr int PACK_NONE = 0x7fffffff;
__device__ __forceinline__ int pack_id(int id, int pos) { return id == ID_NONE ? PACK_NONE : (id << 16) | pos; }
__device__ __forceinline__ int unpack_id(int p) { return p == PACK_NONE ? ID_NONE : (p >> 16); }
__device__ __forceinline__ int unpack_pos(int p) { return p == PACK_NONE ? -1 : (p & 0xffff); }

template <int CTRL>
__device__ __forceinline__ int dpp_i32(int v) {
    return __builtin_amdgcn_update_dpp(v, v, CTRL, 0xF, 0xF, false);
}

// Value of lane ^ 16 / lane ^ 32 (lane layout of the swaps checked on the
// device: the first result holds the lower source half in the upper lanes).
__device__ __forceinline__ int xor16_i32(int v) {
    const auto r = __builtin_amdgcn_permlane16_swap(v, v, false, false);
    return (threadIdx.x & 16) ? r[0] : r[1];
}
__device__ __forceinline__ int xor32_i32(int v) {
    const auto r = __builtin_amdgcn_permlane32_swap(v, v, false, false);
    return (threadIdx.x & 32) ? r[0] : r[1];
}

template <int CTRL>
__device__ __forceinline__ void argmax_step_dpp(double& k, int& pk) {
    const int lo = dpp_i32<CTRL>(__double2loint(k));
    const int hi = dpp_i32<CTRL>(__double2hiint(k));
    const double ok = __hiloint2double(hi, lo);
    const int opk = dpp_i32<CTRL>(pk);
    if (ok > k || (ok == k && opk < pk)) {
        k = ok;
        pk = opk;
    }
}
template <int X>
__device__ __forceinline__ void argmax_step_swap(double& k, int& pk) {
    const int lo = X == 16 ? xor16_i32(__double2loint(k)) : xor32_i32(__double2loint(k));
    const int hi = X == 16 ? xor16_i32(__double2hiint(k)) : xor32_i32(__double2hiint(k));
    const double ok = __hiloint2double(hi, lo);
    const int opk = X == 16 ? xor16_i32(pk) : xor32_i32(pk);
    if (ok > k || (ok == k && opk < pk)) {
        k = ok;
        pk = opk;
    }
}

// All 64 lanes must be active.  On return id/pos are wave-uniform.
__device__ __forceinline__ void wave_argmax(double& k, int& id, int& pos) {
    int pk = pack_id(id, pos);
    argmax_step_dpp<0xB1>(k, pk);   // quad_perm [1,0,3,2]: lane ^ 1
    argmax_step_dpp<0x4E>(k, pk);   // quad_perm [2,3,0,1]: lane ^ 2
    argmax_step_dpp<0x124>(k, pk);  // row_ror:4
    argmax_step_dpp<0x128>(k, pk);  // row_ror:8
    argmax_step_swap<16>(k, pk);
    argmax_step_swap<32>(k, pk);
    pk = __builtin_amdgcn_readfirstlane(pk);
    id = unpack_id(pk);
    pos = unpack_pos(pk);
}

}  // namespace blp
