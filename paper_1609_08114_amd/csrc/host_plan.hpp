// Host-side planning of a solve, from the batch metadata alone: argument
// checks, per-LP offsets, output extents, streaming-workspace sizes, the
// chunk capacity of a memory-limited solve and the copy runs of the
// host-resident pipeline.  Plain C++ (no HIP), so the same code is checked on
// the CPU under AddressSanitizer and UndefinedBehaviorSanitizer.
#pragma once

#include <algorithm>
#include <cstdarg>
#include <cstdint>
#include <cstdio>
#include <string>
#include <vector>

namespace blp {

constexpr int kMaxM = 2046;     // rows of one LP
constexpr int kMaxCols = 4096;  // n + m + 1 (condensed columns, worst case)

// Error codes as in blp.h.
enum { PLAN_OK = 0, PLAN_ERR_ARG = 1, PLAN_ERR_NOMEM = 2, PLAN_ERR_TOO_LARGE = 5 };

struct VariantShape {
    int rows, cols;  // largest tableau (rows incl. objective rows, columns incl. rhs)
    int type1 = 0;   // 1: takes only LPs without artificial rows under the largest-coefficient rule
    int64_t min_count = 0;  // the automatic choice takes it only for batches of at least this many LPs
};

struct PlanIn {
    int64_t count = 0;
    bool uniform = false, shared_box = false;
    const int32_t *m = nullptr, *n = nullptr, *kind = nullptr;
    const int64_t *a_off = nullptr, *row_off = nullptr, *col_off = nullptr;  // NULL: packed
    bool has_A = false, has_b = false, has_sense = false, has_c = false, has_l = false, has_u = false;
    const VariantShape* variants = nullptr;
    int nreg = 0;
    int force = -1;              // -1 automatic, -2 streaming only, >= 0 one variant
    bool remap_streams = false;  // the autotuner sends some register bin to the streaming kernel
    bool stream_all = false;     // size the workspace as if every simplex LP could stream
    bool lpc = true;             // the largest-coefficient rule (type-1-only variants take LPs)
};

struct Plan {
    int code = PLAN_OK;
    std::string msg;
    // metadata: one entry for a uniform batch, else one per LP
    std::vector<int32_t> m, n, kind;
    std::vector<int64_t> a_off, row_off, col_off;  // non-uniform batches: resolved offsets
    bool any_simplex = false, any_box = false;
    int64_t n_box = 0;
    int64_t tot_a = 0, tot_m = 0, tot_n = 0;  // extents of A, rows (b, sense, y), columns (c, l, u, x)
    int max_m = 0, max_n = 0, max_cols = 0;  // over the simplex LPs
    int64_t max_slot = 0;      // largest streaming tableau, doubles (16-row-aligned leading dimension)
    int64_t n_may_stream = 0;  // simplex LPs no register variant is sure to hold
    bool gm_deep = false;      // some LP fits no register tile even without artificial columns
    int box_n = 0;             // shared box: its length
};

inline int plan_fail(Plan& p, int code, const char* fmt, ...) {
    char buf[256];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    p.code = code;
    p.msg = buf;
    return code;
}

// Fills `p` (its vectors keep their capacity across calls).  Returns p.code.
inline int plan_batch(const PlanIn& in, Plan& p) {
    p.code = PLAN_OK;
    p.msg.clear();
    const int64_t K = in.count;
    if (K < 0) return plan_fail(p, PLAN_ERR_ARG, "count out of range");
    if (K > 0 && (!in.m || !in.n || !in.kind)) return plan_fail(p, PLAN_ERR_ARG, "m, n and kind are required");
    const bool uni = in.uniform;
    const int64_t nmeta = uni ? (K > 0 ? 1 : 0) : K;
    p.m.assign(in.m, in.m + nmeta);
    p.n.assign(in.n, in.n + nmeta);
    p.kind.assign(in.kind, in.kind + nmeta);
    p.any_simplex = p.any_box = p.gm_deep = false;
    p.n_box = p.tot_a = p.tot_m = p.tot_n = p.max_slot = p.n_may_stream = 0;
    p.max_m = p.max_n = p.max_cols = p.box_n = 0;
    // no register tile holds the LP even without artificial columns
    auto sure_stream = [&](int m, int n) {
        if (in.force == -2) return true;
        for (int v = 0; v < in.nreg; ++v) {
            if (in.force >= 0 && v != in.force) continue;
            if (in.variants[v].rows >= m + 2 && in.variants[v].cols >= n + 1 && (in.lpc || !in.variants[v].type1))
                return false;
        }
        return true;
    };
    // some register tile holds the LP whatever its artificial columns
    auto sure_register = [&](int m, int n) {
        if (in.stream_all || in.force == -2 || in.remap_streams) return false;
        for (int v = 0; v < in.nreg; ++v) {
            if (in.force >= 0 && v != in.force) continue;
            if (in.variants[v].rows >= m + 2 && in.variants[v].cols >= n + m + 1 && !in.variants[v].type1 &&
                (in.force >= 0 || in.count >= in.variants[v].min_count))
                return true;
        }
        return false;
    };
    for (int64_t k = 0; k < nmeta; ++k) {
        const int m = p.m[k], n = p.n[k], kd = p.kind[k];
        if (kd == 0) {
            if (m < 1 || n < 1) return plan_fail(p, PLAN_ERR_ARG, "LP %lld: simplex LP needs m >= 1 and n >= 1", (long long)k);
            if (m > kMaxM || (int64_t)n + m + 1 > kMaxCols)
                return plan_fail(p, PLAN_ERR_TOO_LARGE, "LP %lld: m=%d n=%d exceeds m <= %d, n + m + 1 <= %d",
                                 (long long)k, m, n, kMaxM, kMaxCols);
            p.any_simplex = true;
            p.max_m = std::max(p.max_m, m);
            p.max_n = std::max(p.max_n, n);
            p.max_cols = std::max(p.max_cols, n + m + 1);
            p.max_slot = std::max<int64_t>(p.max_slot, (int64_t)((m + 2 + 15) / 16) * 16 * (n + m + 1));
            if (!sure_register(m, n)) ++p.n_may_stream;
            if (sure_stream(m, n)) p.gm_deep = true;
        } else if (kd == 1) {
            if (m != 0 || n < 1)
                return plan_fail(p, PLAN_ERR_ARG, "LP %lld: hyperbox LP needs m == 0 and n >= 1", (long long)k);
            p.any_box = true;
            ++p.n_box;
            if (in.shared_box) {
                if (p.box_n == 0) p.box_n = n;
                if (n != p.box_n)
                    return plan_fail(p, PLAN_ERR_ARG, "LP %lld: a shared box needs every hyperbox LP to have n = %d",
                                     (long long)k, p.box_n);
            }
        } else {
            return plan_fail(p, PLAN_ERR_ARG, "LP %lld: kind %d is not 0 or 1", (long long)k, kd);
        }
        p.tot_a += (int64_t)m * n;
        p.tot_m += m;
        p.tot_n += n;
    }
    if (uni) {
        p.n_may_stream *= K;
        p.n_box *= K;
        p.tot_a *= K;
        p.tot_m *= K;
        p.tot_n *= K;
    }
    if (p.any_simplex && (!in.has_A || !in.has_b || !in.has_sense || !in.has_c))
        return plan_fail(p, PLAN_ERR_ARG, "A, b, sense, c required");
    if (p.any_box && (!in.has_c || !in.has_l || !in.has_u))
        return plan_fail(p, PLAN_ERR_ARG, "c, l, u required for hyperbox LPs");
    if (!uni) {
        p.a_off.resize(K);
        p.row_off.resize(K);
        p.col_off.resize(K);
        int64_t ao = 0, ro = 0, co = 0;
        for (int64_t k = 0; k < K; ++k) {
            p.a_off[k] = in.a_off ? in.a_off[k] : ao;
            p.row_off[k] = in.row_off ? in.row_off[k] : ro;
            p.col_off[k] = in.col_off ? in.col_off[k] : co;
            if (p.a_off[k] < 0 || p.row_off[k] < 0 || p.col_off[k] < 0)
                return plan_fail(p, PLAN_ERR_ARG, "LP %lld: negative offset", (long long)k);
            ao += (int64_t)p.m[k] * p.n[k];
            ro += p.m[k];
            co += p.n[k];
        }
        p.tot_a = p.tot_m = p.tot_n = 0;
        for (int64_t k = 0; k < K; ++k) {
            p.tot_a = std::max(p.tot_a, p.a_off[k] + (int64_t)p.m[k] * p.n[k]);
            p.tot_m = std::max(p.tot_m, p.row_off[k] + p.m[k]);
            p.tot_n = std::max(p.tot_n, p.col_off[k] + p.n[k]);
        }
    }
    return PLAN_OK;
}

// Memory-limited solve: with `fixed` bytes held for the whole call and
// `per_lp` bytes per LP of a chunk, the largest chunk that fits `limit`
// (the batch capacity N = S / Y of Sec. 4.5, Eq. (5)); 0 if not even one LP
// fits.  At most `count`.
inline int64_t chunk_capacity(uint64_t limit, uint64_t fixed, uint64_t per_lp, int64_t count) {
    if (per_lp == 0 || fixed >= limit || limit - fixed < per_lp) return 0;
    return (int64_t)std::min<uint64_t>((limit - fixed) / per_lp, (uint64_t)std::max<int64_t>(count, 0));
}

// A contiguous copy of `len` doubles from position `src` of a piece's device
// buffer to position `dst` of the caller's array.
struct CopyRun {
    int64_t dst, src, len;
};

// Runs of the piece [k0, k1) of a host-resident batch: each LP's range
// [off[k], off[k] + len[k]) of the caller's array, which the piece's device
// buffer holds at off[k] - lo; LPs whose ranges follow each other merge into
// one run.  Nothing outside the LPs' own ranges is copied (gaps, or ranges
// of other pieces' LPs between them).  `order` is scratch.
inline void copy_runs(const std::vector<int64_t>& off, const std::vector<int32_t>& len, int64_t k0, int64_t k1,
                      int64_t lo, std::vector<int64_t>& order, std::vector<CopyRun>& runs) {
    runs.clear();
    order.resize((size_t)std::max<int64_t>(0, k1 - k0));
    for (int64_t k = k0; k < k1; ++k) order[(size_t)(k - k0)] = k;
    auto by_off = [&](int64_t a, int64_t b) { return off[a] < off[b]; };
    if (!std::is_sorted(order.begin(), order.end(), by_off)) std::sort(order.begin(), order.end(), by_off);
    int64_t run_lo = -1, run_hi = -1;
    for (size_t q = 0; q <= order.size(); ++q) {
        const bool last = q == order.size();
        const int64_t k = last ? 0 : order[q];
        if (!last && len[k] == 0) continue;
        if (!last && off[k] == run_hi) {
            run_hi += len[k];
            continue;
        }
        if (run_hi > run_lo) runs.push_back({run_lo, run_lo - lo, run_hi - run_lo});
        if (!last) {
            run_lo = off[k];
            run_hi = off[k] + len[k];
        }
    }
}

}  // namespace blp
