// Lane kernel for the smallest size class: one LP per lane, 64 LPs per wave.
//
// A tiny LP (a condensed tableau of a few dozen entries) cannot occupy a
// wave, let alone a workgroup, without leaving most lanes idle: with one LP
// per workgroup (Sec. 4.1's layout) a 5 x 5 LP keeps one lane per tableau
// entry busy for a few instructions between barriers.  Here every lane
// solves its own LP from start to end, with the whole condensed tableau in
// its registers: every loop runs over the compile-time shape R x C (so the
// tableau never needs a dynamic register index) with per-lane masks for the
// LP's own m, n and n_art, and the pivot row / column are picked out with
// selects.  The 64 lanes of a wave take 64 consecutive work-list entries at
// once.  No LDS and no barriers: lanes only share the wave's instruction
// stream, so an LP's cost is the work of the longest-running LP of its wave.
//
// The arithmetic is the same as the other simplex kernels and the CPU
// reference: the condensed tableau of simplex_common.hpp (rows 0..m-1, the
// phase-1 row R-2, the objective row R-1; slot C-1 the rhs), Step 1 over the
// active objective row with the largest-coefficient rule (Sec. 4.2), lowest
// variable id on ties, Bland's lowest index after max(m, n) zero steps;
// Step 2 over rows with a pivot-column entry above eps_piv, ratio rhs /
// entry (0 when the rhs is <= 0), smallest basic id on ties; Step 3 with the
// pivot row divided entry by entry by the pivot element (IEEE division) and
// one fused multiply-add per other entry (Sec. 4.3).  The pivot row is
// stored as the quotients themselves.
#pragma once

#include "blp_kernels.hpp"
#include "simplex_common.hpp"

namespace blp {

// Largest tableau of the lane kernel's variants: R rows (m + 2) by C
// columns (n + n_art + 1).
template <int R, int C, int NWV, int WPE>
__global__ void __launch_bounds__(NWV * 64) __attribute__((amdgpu_waves_per_eu(WPE, WPE)))
simplex_lane_kernel(KParams P) {
    constexpr int MR = R - 2;  // constraint rows
    constexpr int ROW_W = R - 2, ROW_OBJ = R - 1, RHS = C - 1;
    static_assert(R >= 3 && C >= 2 && MR <= 32, "bad lane tile");
    const int lane = threadIdx.x & 63;
    const int wave = threadIdx.x >> 6;
    const int64_t len = work_len(P);
    // direct modes: this wave's 64 positions, bounded by direct_end
    const int64_t dend = P.direct && P.direct_end > 0 && P.direct_end < len ? P.direct_end : len;
    bool first = true;
    for (;;) {
        int64_t q0;
        if (P.direct) {
            if (!first) break;
            q0 = P.direct_first + ((int64_t)blockIdx.x * NWV + wave) * 64;
        } else {
            int v = 0;
            if (lane == 0) {
                int* head = bin_head_of(P);
                // an exhausted (or empty) list: leave without an atomic
                v = first && __hip_atomic_load(head, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) >= len
                        ? (int)len
                        : atomicAdd(head, 64);
            }
            q0 = __shfl(v, 0);
        }
        first = false;
        if (q0 >= dend) break;
        const int64_t q = q0 + lane;
        if (q >= dend) continue;

        // ------------------------------------------------------------ load
        const int k = (int)work_item(P, q);
        const LpRef L = lp_ref(P, k);
        const LpRef Lin = lp_in(P, L);
        const int m = L.m, n = L.n;
        auto write_status_only = [&](int st) __attribute__((always_inline)) {
            for (int j = 0; j < n; ++j) P.x[L.col_off + j] = __builtin_nan("");
            for (int i = 0; i < m; ++i) P.y[L.row_off + i] = __builtin_nan("");
            P.status[k] = st;
            P.iters[k] = 0;
            P.obj[k] = __builtin_nan("");
        };
        if (m > MR || n + 1 > C) {  // never routed here
            write_status_only(ST_INTERNAL);
            continue;
        }
        // rows in "<=" form (Sec. 3): sign, normalised rhs, artificial and
        // ">=" flags (bit i), as prep_row() does
        double sig[MR], bnorm[MR];
        unsigned art = 0, ge = 0;
        int bad = 0, nart = 0;
#pragma unroll
        for (int i = 0; i < MR; ++i) {
            sig[i] = 1.0;
            bnorm[i] = 0.0;
            if (i < m) {
                const double bi = P.b[Lin.row_off + i];
                const int gi = P.sense[Lin.row_off + i] != 0;
                const double ble = gi ? -bi : bi;
                const int ai = ble < 0.0;
                const double sg = ai ? (gi ? 1.0 : -1.0) : (gi ? -1.0 : 1.0);
                sig[i] = sg;
                bnorm[i] = sg * bi;
                bad |= !isfinite(bi);
                art |= (unsigned)ai << i;
                ge |= (unsigned)gi << i;
                nart += ai;
            }
        }
        if (n + nart + 1 > C) {  // never routed here
            write_status_only(ST_INTERNAL);
            continue;
        }
        // constraint rows: structural columns sig_i a_ij, the surplus column
        // of an artificial row (slot n + its rank among those rows) -1, rhs
        double T[R][C];
        int cv[C - 1];  // slot -> variable id
        int bs[MR];     // row -> basic variable id
#pragma unroll
        for (int i = 0; i < MR; ++i) {
            const bool ai = (art >> i) & 1u;
            const int rank = __popc(art & ((1u << i) - 1u));
#pragma unroll
            for (int j = 0; j < RHS; ++j) {
                double v = 0.0;
                if (i < m) {
                    if (j < n) {
                        const double a = P.A[Lin.a_off + (int64_t)i * n + j];
                        bad |= !isfinite(a);
                        v = sig[i] * a;
                    } else if (ai && j == n + rank) {
                        v = -1.0;
                    }
                }
                T[i][j] = v;
            }
            T[i][RHS] = bnorm[i];
            bs[i] = i < m ? (ai ? n + m + i : n + i) : ID_NONE;
        }
        // slot -> variable: structural, then the surplus variables (logical
        // id n + row) of the artificial rows in row order
#pragma unroll
        for (int j = 0; j < RHS; ++j) {
            int v = j < n ? j : ID_NONE;
#pragma unroll
            for (int i = 0; i < MR; ++i)
                if (((art >> i) & 1u) && j == n + __popc(art & ((1u << i) - 1u))) v = n + i;
            cv[j] = v;
        }
        // phase-1 row: the artificial rows summed in increasing row order
        // over the structural columns and the rhs, -1 on the surplus slots;
        // objective row: c_j on the structural slots
#pragma unroll
        for (int j = 0; j < C; ++j) {
            double acc = 0.0;
            if (nart > 0) {
                if (j < n || j == RHS) {
#pragma unroll
                    for (int i = 0; i < MR; ++i)
                        if ((art >> i) & 1u) acc = acc + T[i][j];
                } else if (j < n + nart) {
                    acc = -1.0;
                }
            }
            T[ROW_W][j] = acc;
            double cj = 0.0;
            if (j < n && j < RHS) {
                cj = P.c[L.col_off + j];
                bad |= !isfinite(cj);
            }
            T[ROW_OBJ][j] = cj;
        }
        if (bad) {
            write_status_only(ST_NUMERICAL);
            continue;
        }

        // ------------------------------------------------------ pivot loop
        // mode 1 = phase 1, 2 = phase 2, 3 = driving basic artificials out
        // after a feasible phase 1 (rows in increasing order)
        const double w0 = T[ROW_W][RHS];
        const int max_iter = P.max_iter > 0 ? P.max_iter : 50 * (m + n);
        const int bland_after = P.bland_after > 0 ? P.bland_after : (m > n ? m : n);
        const int id_lim = n + m;
        int mode = nart > 0 ? 1 : 2;
        int iters = 0, degen = 0, st = -1, drive_r = 0;
        unsigned dead = 0;
        for (;;) {
            int l = -1, e = -1, e_id = ID_NONE;
            double rmin = 1.0;
            if (mode == 3) {
                int r0 = -1;
#pragma unroll
                for (int i = 0; i < MR; ++i)
                    if (r0 < 0 && i >= drive_r && i < m && bs[i] >= id_lim && !((dead >> i) & 1u)) r0 = i;
                if (r0 < 0) {
                    mode = 2;
                    degen = 0;
                    continue;
                }
                drive_r = r0 + 1;
                // the lowest-id non-artificial column with a usable entry
#pragma unroll
                for (int j = 0; j < RHS; ++j) {
                    double a = 0.0;
#pragma unroll
                    for (int i = 0; i < MR; ++i) a = i == r0 ? T[i][j] : a;
                    const int v = cv[j];
                    if (v < id_lim && fabs(a) > P.eps_piv && v < e_id) {
                        e_id = v;
                        e = j;
                    }
                }
                if (e < 0) {  // redundant row
                    dead |= 1u << r0;
                    continue;
                }
                l = r0;
            } else {
                // Step 1
                const bool rpc = P.pivot_rule == 1 && degen < bland_after;
                const bool bland = degen >= bland_after;
                int total = 0;
                double bk = -__builtin_inf();
#pragma unroll
                for (int j = 0; j < RHS; ++j) {
                    const double d = mode == 1 ? T[ROW_W][j] : T[ROW_OBJ][j];
                    const int v = cv[j];
                    const bool ok = v < id_lim && d > P.eps_price;
                    total += ok;
                    const double key = bland ? 0.0 : d;
                    if (!rpc && ok && (key > bk || (key == bk && v < e_id))) {
                        bk = key;
                        e_id = v;
                        e = j;
                    }
                }
                if (rpc && total > 0) {
                    // Sec. 4.2's random positive coefficient: the target-th
                    // eligible slot in slot order
                    uint32_t c4[4] = {(uint32_t)iters, (uint32_t)k, 0x52504321u, 0u};
                    philox4x32_10(c4, (uint32_t)P.seed, (uint32_t)(P.seed >> 32));
                    const double u =
                        (double)((uint64_t)(c4[0] >> 5) * 67108864ull + (c4[1] >> 6)) * (1.0 / 9007199254740992.0);
                    int target = (int)(u * total);
                    if (target >= total) target = total - 1;
#pragma unroll
                    for (int j = 0; j < RHS; ++j) {
                        const double d = mode == 1 ? T[ROW_W][j] : T[ROW_OBJ][j];
                        const int v = cv[j];
                        if (v < id_lim && d > P.eps_price) {
                            if (target == 0 && e < 0) {
                                e = j;
                                e_id = v;
                            }
                            --target;
                        }
                    }
                }
                if (e < 0) {
                    if (mode == 2) {
                        st = ST_OPTIMAL;
                        break;
                    }
                    if (T[ROW_W][RHS] > P.eps_feas * (1.0 + w0)) {
                        st = ST_INFEASIBLE;
                        break;
                    }
                    mode = 3;
                    drive_r = 0;
                    continue;
                }
                if (iters >= max_iter) {
                    st = ST_ITER_LIMIT;
                    break;
                }
                // Step 2
                int bid = ID_NONE;
#pragma unroll
                for (int i = 0; i < MR; ++i) {
                    double a = 0.0;
#pragma unroll
                    for (int j = 0; j < RHS; ++j) a = j == e ? T[i][j] : a;
                    if (i < m && !((dead >> i) & 1u) && a > P.eps_piv) {
                        const double bi = T[i][RHS];
                        const double ratio = bi <= 0.0 ? 0.0 : bi / a;
                        if (l < 0 || ratio < rmin || (ratio == rmin && bs[i] < bid)) {
                            l = i;
                            rmin = ratio;
                            bid = bs[i];
                        }
                    }
                }
                if (l < 0) {
                    st = mode == 2 ? ST_UNBOUNDED : ST_NUMERICAL;
                    break;
                }
            }
            // Step 3 on (l, e): the entering slot becomes the leaving
            // variable's column (its old unit column, updated like the rest)
            double f[R];
#pragma unroll
            for (int i = 0; i < R; ++i) {
                double a = 0.0;
#pragma unroll
                for (int j = 0; j < RHS; ++j) a = j == e ? T[i][j] : a;
                f[i] = a;
            }
            double pe = 0.0;
            int lv = ID_NONE;
#pragma unroll
            for (int i = 0; i < MR; ++i) {
                pe = i == l ? f[i] : pe;
                lv = i == l ? bs[i] : lv;
            }
#pragma unroll
            for (int j = 0; j < C; ++j) {
                double tl = 0.0;
#pragma unroll
                for (int i = 0; i < MR; ++i) tl = i == l ? T[i][j] : tl;
                const double pj = (j == e ? 1.0 : tl) / pe;
#pragma unroll
                for (int i = 0; i < R; ++i) {
                    const double base = j == e ? 0.0 : T[i][j];
                    T[i][j] = i == l ? pj : __builtin_fma(-f[i], pj, base);
                }
            }
#pragma unroll
            for (int j = 0; j < RHS; ++j) cv[j] = j == e ? lv : cv[j];
#pragma unroll
            for (int i = 0; i < MR; ++i) bs[i] = i == l ? e_id : bs[i];
            ++iters;
            if (mode != 3) degen = rmin == 0.0 ? degen + 1 : 0;
        }

        // ------------------------------------------------------ extraction
        // every structural and logical variable sits in one slot (nonbasic:
        // x = 0, dual from the objective row) or one row (basic: x = rhs,
        // dual 0); duals d obj / d b_i: -d for "<=" rows, +d for ">=" rows
        const double z = -T[ROW_OBJ][RHS];
        if (st == ST_OPTIMAL && !isfinite(z)) st = ST_NUMERICAL;
        const bool nan_out = st == ST_NUMERICAL;
        const double qnan = __builtin_nan("");
#pragma unroll
        for (int j = 0; j < RHS; ++j) {
            const int v = cv[j];
            if (v < n) {
                P.x[L.col_off + v] = nan_out ? qnan : 0.0;
            } else if (v < n + m) {
                const double d = T[ROW_OBJ][j];
                P.y[L.row_off + (v - n)] = nan_out ? qnan : (((ge >> (v - n)) & 1u) ? d : -d);
            }
        }
#pragma unroll
        for (int i = 0; i < MR; ++i) {
            const int v = bs[i];
            if (i < m) {
                if (v < n) {
                    P.x[L.col_off + v] = nan_out ? qnan : T[i][RHS];
                } else if (v < n + m) {
                    P.y[L.row_off + (v - n)] = nan_out ? qnan : (((ge >> (v - n)) & 1u) ? 0.0 : -0.0);
                }
            }
        }
        P.status[k] = st;
        P.iters[k] = iters;
        P.obj[k] = (st == ST_OPTIMAL || st == ST_ITER_LIMIT) ? z
                   : st == ST_UNBOUNDED                     ? __builtin_inf()
                   : st == ST_INFEASIBLE                    ? -__builtin_inf()
                                                            : qnan;
    }
}

}  // namespace blp
