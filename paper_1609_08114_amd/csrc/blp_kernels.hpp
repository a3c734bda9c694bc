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
    int32_t ws_ld;   // leading dimension (rows, multiple of 64)
    int32_t ws_cols; // columns available per slot
};

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
// with the same winner whatever the combination order.  Within each 16-lane
// row the exchange uses DPP (quad permutes, then row rotations by 4 and 8);
// across rows, lane shuffles by 16 and 32.
// ---------------------------------------------------------------------------
__device__ __forceinline__ bool key_before(double ak, int aid, double bk, int bid) {
    return ak > bk || (ak == bk && aid < bid);
}

template <int CTRL>
__device__ __forceinline__ int dpp_i32(int v) {
    return __builtin_amdgcn_update_dpp(v, v, CTRL, 0xF, 0xF, false);
}
template <int CTRL>
__device__ __forceinline__ double dpp_f64(double v) {
    int lo = __double2loint(v), hi = __double2hiint(v);
    lo = dpp_i32<CTRL>(lo);
    hi = dpp_i32<CTRL>(hi);
    return __hiloint2double(hi, lo);
}

template <int CTRL>
__device__ __forceinline__ void argmax_dpp_step(double& k, int& id, int& pos) {
    double ok = dpp_f64<CTRL>(k);
    int oid = dpp_i32<CTRL>(id);
    int opos = dpp_i32<CTRL>(pos);
    if (key_before(ok, oid, k, id)) {
        k = ok;
        id = oid;
        pos = opos;
    }
}

__device__ __forceinline__ void argmax_shfl_step(double& k, int& id, int& pos, int mask) {
    double ok = __shfl_xor(k, mask, 64);
    int oid = __shfl_xor(id, mask, 64);
    int opos = __shfl_xor(pos, mask, 64);
    if (key_before(ok, oid, k, id)) {
        k = ok;
        id = oid;
        pos = opos;
    }
}

// All 64 lanes must be active.
__device__ __forceinline__ void wave_argmax(double& k, int& id, int& pos) {
    argmax_dpp_step<0xB1>(k, id, pos);   // quad_perm [1,0,3,2]: lane ^ 1
    argmax_dpp_step<0x4E>(k, id, pos);   // quad_perm [2,3,0,1]: lane ^ 2
    argmax_dpp_step<0x124>(k, id, pos);  // row_ror:4
    argmax_dpp_step<0x128>(k, id, pos);  // row_ror:8
    argmax_shfl_step(k, id, pos, 16);
    argmax_shfl_step(k, id, pos, 32);
    id = __builtin_amdgcn_readfirstlane(id);
    pos = __builtin_amdgcn_readfirstlane(pos);
}

}  // namespace blp
