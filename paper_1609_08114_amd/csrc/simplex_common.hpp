// Per-LP set-up and result extraction shared by the register-tile and the
// streaming simplex kernels.  Both kernels keep the same condensed tableau:
//
//   rows    0..m-1      constraint rows (each user row times its sign s_i)
//           RP-2        phase-1 row (reduced costs of max -sum(artificials))
//           RP-1        objective row d_j = c_j - z_j, -z in the rhs cell
//   columns one per NONBASIC variable plus the right-hand side; a basic
//           variable's column is a unit vector and is not stored.  Column
//           slot j holds variable colvar[j]; row i's basic variable is
//           basis[i].
//
// Variable ids: structural j in [0, n), logical (slack/surplus) of row i is
// n + i, artificial of row i is n + m + i.  Initially the structural
// columns are slots 0..n-1, the surplus columns of the rows that need an
// artificial follow in row order, and the rhs is the last slot.
//
// The values in every stored cell are bit-identical to the same cell of the
// full tableau (x | logicals | artificials | rhs) of the paper's Sec. 3.1
// updated by the Step-3 rule: a pivot on (l, e) turns the entering column's
// slot into the leaving variable's column, whose full-tableau values are
// fma(-f_i, fl(1/PE), 0) off the pivot row and fl(1/PE) on it -- exactly what
// the uniform update below produces after the slot has been zeroed.
#pragma once

#include "blp_kernels.hpp"

namespace blp {

// Rows: sign, rhs (in s_b), flags; returns nonzero if b has a non-finite
// value.  The "<=" form of row i is (a_i, b_i) for "<=" rows and (-a_i, -b_i)
// for ">=" rows (Sec. 3, Eq. (2)); a negative "<=" rhs makes the initial
// basic solution infeasible, so that row is negated back and gets a surplus
// and an artificial variable (the two-phase method of Sec. 3).
__device__ __forceinline__ int prep_row(int i, double bi, int sense, double* s_sig, double* s_b,
                                        unsigned char* s_flag) {
    const int ge = sense != 0;
    const double ble = ge ? -bi : bi;
    const int art = ble < 0.0;
    const double sg = art ? (ge ? 1.0 : -1.0) : (ge ? -1.0 : 1.0);
    s_sig[i] = sg;
    s_b[i] = sg * bi;
    s_flag[i] = (unsigned char)((ge ? RF_GE : 0) | (art ? RF_ART : 0));
    return !isfinite(bi);
}
template <int NT>
__device__ __forceinline__ int prep_rows(const KParams& P, const LpRef& L, int t, double* s_sig, double* s_b,
                                         unsigned char* s_flag) {
    int bad = 0;
    for (int i = t; i < L.m; i += NT) bad |= prep_row(i, P.b[L.row_off + i], P.sense[L.row_off + i], s_sig, s_b, s_flag);
    for (int j = t; j < L.n; j += NT) bad |= !isfinite(P.c[L.col_off + j]);
    return bad;
}

// Wave 0 compacts the rows that need an artificial, in increasing row order
// (the order in which the phase-1 row sums them).
__device__ __forceinline__ void scan_art_rows(int m, int lane, const unsigned char* s_flag, int* s_artrow,
                                              int* s_rank, int* s_nart) {
    int base = 0;
    for (int i0 = 0; i0 < m; i0 += 64) {
        const int i = i0 + lane;
        const bool f = i < m && (s_flag[i] & RF_ART);
        const unsigned long long mask = __ballot(f);
        const int rank = base + __popcll(mask & ((1ull << lane) - 1ull));
        if (f) {
            s_artrow[rank] = i;
            s_rank[i] = rank;
        }
        base += __popcll(mask);
    }
    if (lane == 0) *s_nart = base;
}

// Write one LP's outputs.  s_d must hold the objective row (by slot), s_b the
// rhs column; s_xs (>= n doubles) and s_ys (>= m doubles) are scratch.  The
// barriers order LDS only; the output stores complete asynchronously.
template <int NT>
__device__ __forceinline__ void write_outputs(const KParams& P, const LpRef& L, int k, int t, int st, int iters,
                                              int obj_row, int nslots, const double* s_d, const double* s_b,
                                              const int* s_colvar, const int* s_basis,
                                              const unsigned char* s_flag, double* s_xs, double* s_ys) {
    const int m = L.m, n = L.n;
    for (int j = t; j < n; j += NT) s_xs[j] = 0.0;
    for (int i = t; i < m; i += NT) s_ys[i] = 0.0;
    lds_barrier();
    // x_j = rhs of the row where j is basic; the dual of row i is read from
    // the objective-row entry of its logical variable (zero when basic).
    for (int i = t; i < m; i += NT) {
        const int v = s_basis[i];
        if (v < n) s_xs[v] = s_b[i];
    }
    for (int j = t; j < nslots; j += NT) {
        const int v = s_colvar[j];
        if (v >= n && v < n + m) s_ys[v - n] = s_d[j];
    }
    lds_barrier();
    const double z = -s_b[obj_row];
    if (st == ST_OPTIMAL && !isfinite(z)) st = ST_NUMERICAL;
    const bool nan_out = st == ST_NUMERICAL;
    for (int j = t; j < n; j += NT) P.x[L.col_off + j] = nan_out ? __builtin_nan("") : s_xs[j];
    for (int i = t; i < m; i += NT) {
        const double d = s_ys[i];
        P.y[L.row_off + i] = nan_out ? __builtin_nan("") : ((s_flag[i] & RF_GE) ? d : -d);
    }
    if (t == 0) {
        P.status[k] = st;
        P.iters[k] = iters;
        P.obj[k] = (st == ST_OPTIMAL || st == ST_ITER_LIMIT) ? z
                   : st == ST_UNBOUNDED                     ? __builtin_inf()
                   : st == ST_INFEASIBLE                    ? -__builtin_inf()
                                                            : __builtin_nan("");
    }
}

// Outputs of an LP whose data are not finite (no solve).
template <int NT>
__device__ __forceinline__ void write_numerical(const KParams& P, const LpRef& L, int k, int t, int st) {
    for (int j = t; j < L.n; j += NT) P.x[L.col_off + j] = __builtin_nan("");
    for (int i = t; i < L.m; i += NT) P.y[L.row_off + i] = __builtin_nan("");
    if (t == 0) {
        P.status[k] = st;
        P.iters[k] = 0;
        P.obj[k] = __builtin_nan("");
    }
}

// Step 1 (Sec. 3.1 and the LPC rule of Sec. 4.2): the nonbasic column with
// the largest reduced cost above eps_price, lowest variable id on ties;
// with `bland` set, the lowest variable id above eps_price.  Artificial
// variables (id >= id_lim) never enter.  Every wave computes it.
__device__ __forceinline__ void price(int nslots, int lane, int id_lim, double eps_price, bool bland,
                                      const double* s_d, const int* s_colvar, int& e_id, int& e_pos) {
    double bk = -__builtin_inf();
    int bid = ID_NONE, bpos = -1;
    for (int j = lane; j < nslots; j += 64) {
        const int v = s_colvar[j];
        if (v < id_lim) {
            const double d = s_d[j];
            if (d > eps_price) {
                const double key = bland ? 0.0 : d;
                if (key_before(key, v, bk, bid)) {
                    bk = key;
                    bid = v;
                    bpos = j;
                }
            }
        }
    }
    wave_argmax(bk, bid, bpos);
    e_id = bid;
    e_pos = bpos;
}

// Philox4x32 with 10 rounds (Salmon, Moraes, Dror, Shaw, SC'11): two
// 32x32->64 multiplies per round with the Weyl key schedule.  Used for the
// random entering rule only.
__device__ __forceinline__ void philox4x32_10(uint32_t c[4], uint32_t k0, uint32_t k1) {
    for (int r = 0; r < 10; ++r) {
        if (r > 0) {
            k0 += 0x9E3779B9u;
            k1 += 0xBB67AE85u;
        }
        const uint64_t p0 = (uint64_t)0xD2511F53u * c[0];
        const uint64_t p1 = (uint64_t)0xCD9E8D57u * c[2];
        const uint32_t y0 = (uint32_t)(p1 >> 32) ^ c[1] ^ k0;
        const uint32_t y2 = (uint32_t)(p0 >> 32) ^ c[3] ^ k1;
        c[0] = y0;
        c[1] = (uint32_t)p1;
        c[2] = y2;
        c[3] = (uint32_t)p0;
    }
}

// Sec. 4.2, the "random positive coefficient" rule: a uniformly random
// nonbasic column with reduced cost above eps_price, drawn from Philox keyed
// by the seed and addressed by (LP, pivot count).  Eligible slots are ranked
// in slot order, so the choice is deterministic.  Every wave computes it.
__device__ __forceinline__ void price_rpc(int nslots, int lane, int id_lim, double eps_price, uint64_t seed, int lp,
                                          int iter, const double* s_d, const int* s_colvar, int& e_id, int& e_pos) {
    int total = 0;
    for (int j0 = 0; j0 < nslots; j0 += 64) {
        const int j = j0 + lane;
        const bool ok = j < nslots && s_colvar[j] < id_lim && s_d[j] > eps_price;
        total += __popcll(__ballot(ok));
    }
    e_id = ID_NONE;
    e_pos = -1;
    if (total == 0) return;
    uint32_t c[4] = {(uint32_t)iter, (uint32_t)lp, 0x52504321u, 0u};
    philox4x32_10(c, (uint32_t)seed, (uint32_t)(seed >> 32));
    const double u = (double)((uint64_t)(c[0] >> 5) * 67108864ull + (c[1] >> 6)) * (1.0 / 9007199254740992.0);
    int target = (int)(u * total);
    if (target >= total) target = total - 1;
    for (int j0 = 0; j0 < nslots; j0 += 64) {
        const int j = j0 + lane;
        const bool ok = j < nslots && s_colvar[j] < id_lim && s_d[j] > eps_price;
        unsigned long long mask = __ballot(ok);
        const int cnt = __popcll(mask);
        if (target < cnt) {
            for (int t = 0; t < target; ++t) mask &= mask - 1;  // drop the lowest set bits
            const int pos = j0 + __ffsll((long long)mask) - 1;
            e_pos = __builtin_amdgcn_readfirstlane(pos);
            e_id = s_colvar[e_pos];
            return;
        }
        target -= cnt;
    }
}

// Step 2 (Sec. 3.1): among live rows with a pivot-column entry above
// eps_piv, the minimum ratio rhs / entry (a row whose rhs is <= 0 offers a
// zero step); ties to the smallest basic variable id.  Every wave computes
// it.  Returns the row (or -1) and the minimum ratio.
__device__ __forceinline__ int ratio_test(int m, int lane, double eps_piv, const double* s_f, const double* s_b,
                                          const int* s_basis, const unsigned char* s_flag, double& rmin) {
    double bk = -__builtin_inf();
    int bid = ID_NONE, bpos = -1;
    for (int i = lane; i < m; i += 64) {
        if (s_flag[i] & RF_DEAD) continue;
        const double a = s_f[i];
        if (a > eps_piv) {
            const double bi = s_b[i];
            const double ratio = bi <= 0.0 ? 0.0 : bi / a;
            const int v = s_basis[i];
            if (key_before(-ratio, v, bk, bid)) {
                bk = -ratio;
                bid = v;
                bpos = i;
            }
        }
    }
    wave_argmax(bk, bid, bpos);
    rmin = -bk;
    return bid == ID_NONE ? -1 : bpos;
}

}  // namespace blp
