// Block-tile simplex kernel: one LP per workgroup, the condensed tableau in
// VGPRs as a 2-D block per thread, persistent over a size-binned work list.
//
// Same method, same tableau and the same operation order as the row-tile
// kernel (every stored cell bit-identical to the full tableau of Sec. 3.1
// after the Step-3 update); what changes is where the values live:
//
//  * Thread (trb, tcb) = (t / GC, t % GC) holds rows trb*RB .. trb*RB+RB-1
//    and the strided column slots c*GC + tcb, c = 0..CB-1.  A pivot then
//    needs RB pivot-column values and CB pivot-row values per thread from
//    LDS (RB + CB reads for RB*CB FMAs), and the owners of one row or of one
//    column are GC or GR threads working in parallel, not one thread.
//  * Steps 1 and 2 (Sec. 3.1) read register mirrors of the objective rows,
//    the rhs column, the slot -> variable map and the basis: lane q*64+lane
//    of every wave keeps slot/row q*64+lane and updates it with the same FMA
//    as the tile, so every wave prices and ratio-tests by itself and no
//    barrier is needed to broadcast the result.
//  * The pivot column and the scaled pivot row go through two LDS buffers
//    used alternately, so a pivot has two barriers: after the entering
//    column is published and after the pivot row is published.
//  * The initial tableau is loaded straight from A into the tile (lanes of
//    a row group read consecutive columns).
#pragma once

#include "blp_kernels.hpp"
#include "simplex_common.hpp"

namespace blp {

// Step 1 over register mirrors: slot j = q*64 + lane carries reduced cost
// d[q] and variable cv[q].  Same rule and tie-break as price().
template <int CS>
__device__ __forceinline__ void price_regs(int nslots, int lane, int id_lim, double eps_price, bool bland,
                                           const double (&d)[CS], const int (&cv)[CS], int& e_id, int& e_pos) {
    double bk = -__builtin_inf();
    int bid = ID_NONE, bpos = -1;
#pragma unroll
    for (int q = 0; q < CS; ++q) {
        const int j = q * 64 + lane;
        const int v = cv[q];
        const double key = bland ? 0.0 : d[q];
        const bool take = (j < nslots) & (v < id_lim) & (d[q] > eps_price) &
                          ((key > bk) | ((key == bk) & (v < bid)));
        bk = take ? key : bk;
        bid = take ? v : bid;
        bpos = take ? j : bpos;
    }
    // bk is -inf or >= +0 (eps_price >= 0), so its bit pattern orders like it
    const long long kb = __double_as_longlong(bk);
    int th;
    unsigned tl;
    const int pk = wave_argmax_i64((int)(kb >> 32), (unsigned)kb, pack_id(bid, bpos), th, tl);
    e_id = unpack_id(pk);
    e_pos = unpack_pos(pk);
}

// The random-positive-coefficient rule of Sec. 4.2 over register mirrors;
// the same draw and the same slot-order ranking as price_rpc().
template <int CS>
__device__ __forceinline__ void price_rpc_regs(int nslots, int lane, int id_lim, double eps_price, uint64_t seed,
                                               int lp, int iter, const double (&d)[CS], const int (&cv)[CS],
                                               int& e_id, int& e_pos) {
    bool ok[CS];
    int total = 0;
#pragma unroll
    for (int q = 0; q < CS; ++q) {
        const int j = q * 64 + lane;
        ok[q] = j < nslots && cv[q] < id_lim && d[q] > eps_price;
        total += __popcll(__ballot(ok[q]));
    }
    e_id = ID_NONE;
    e_pos = -1;
    if (total == 0) return;
    uint32_t c[4] = {(uint32_t)iter, (uint32_t)lp, 0x52504321u, 0u};
    philox4x32_10(c, (uint32_t)seed, (uint32_t)(seed >> 32));
    const double u = (double)((uint64_t)(c[0] >> 5) * 67108864ull + (c[1] >> 6)) * (1.0 / 9007199254740992.0);
    int target = (int)(u * total);
    if (target >= total) target = total - 1;
#pragma unroll
    for (int q = 0; q < CS; ++q) {
        unsigned long long mask = __ballot(ok[q]);
        const int cnt = __popcll(mask);
        if (e_pos < 0) {
            if (target < cnt) {
                for (int s = 0; s < target; ++s) mask &= mask - 1;  // drop the lowest set bits
                const int src = __ffsll((long long)mask) - 1;
                e_pos = q * 64 + src;
                e_id = __builtin_amdgcn_readlane(cv[q], src);  // uniform: keeps the pivot loop's branches scalar
            } else {
                target -= cnt;
            }
        }
    }
}

// Step 2 over register mirrors: row i = q*64 + lane has pivot-column entry
// f[q], rhs b[q] and basic variable bs[q]; bit q of `dead` marks a redundant
// row.  Same rule and tie-break as ratio_test().  Returns the row (or -1),
// the minimum ratio and the leaving variable.
template <int RS>
__device__ __forceinline__ int ratio_regs(int m, int lane, double eps_piv, const double (&f)[RS],
                                          const double (&b)[RS], const int (&bs)[RS], unsigned dead, double& rmin,
                                          int& leave_id) {
    double bk = -__builtin_inf();
    int bid = ID_NONE, bpos = -1;
#pragma unroll
    for (int q = 0; q < RS; ++q) {
        const int i = q * 64 + lane;
        const double a = f[q];
        const bool cand = (i < m) & !((dead >> q) & 1u) & (a > eps_piv);
        const double bi = b[q];
        // every lane divides (by 1 where it is no candidate): no branch, so
        // the chains of all RS rows interleave
        double ratio = bi / (cand ? a : 1.0);
        __asm__("" : "+v"(ratio));
        ratio = bi <= 0.0 ? 0.0 : ratio;
        const double key = -ratio;
        const bool take = cand & ((key > bk) | ((key == bk) & (bs[q] < bid)));
        bk = take ? key : bk;
        bid = take ? bs[q] : bid;
        bpos = take ? i : bpos;
    }
    // the lane's smallest ratio (+inf without a candidate) is >= +0: the
    // complement of its bit pattern orders it largest-first
    const long long rb = __double_as_longlong(-bk);
    int th;
    unsigned tl;
    const int pk = wave_argmax_i64(~(int)(rb >> 32), ~(unsigned)rb, pack_id(bid, bpos), th, tl);
    rmin = __longlong_as_double((long long)(((unsigned long long)(unsigned)~th << 32) | (unsigned)~tl));
    leave_id = unpack_id(pk);
    return leave_id == ID_NONE ? -1 : unpack_pos(pk);
}

// x / b rounded to nearest, given y = x / b's reciprocal 1.0 / b (an IEEE
// division) and b_ok = |b| in [2^-500, 2^500]: q = x y is within one ulp of
// x / b, the residual x - b q is exact in one FMA, and q + residual * y
// rounded once is the correctly rounded quotient (Markstein's theorem, IBM J.
// Res. Dev. 34(1), 1990).  x = 0 takes the product (sign of zero).  `ok` is
// false where a step could overflow or underflow (|x| outside [2^-500,
// 2^500] or b outside its range); the caller then divides instead, so the
// result always equals x / b.  No branch here: a row's entries form one
// block of independent chains.
__device__ __forceinline__ double div_rn_fast(double x, double b, double y, bool b_ok, bool& ok) {
    const double q = x * y;
    const double ax = fabs(x);
    const bool zero = x == 0.0;
    ok = zero | (b_ok & (ax >= 0x1p-500) & (ax <= 0x1p500));
    return zero ? q : __builtin_fma(__builtin_fma(-b, q, x), y, q);
}

// Wave-uniform value of a mirror entry (row or slot `idx`).
template <int S>
__device__ __forceinline__ double mirror_at(const double (&v)[S], int idx) {
    double r = 0.0;
#pragma unroll
    for (int q = 0; q < S; ++q)
        if (idx / 64 == q) {
            const int src = idx % 64;
            r = __hiloint2double(__builtin_amdgcn_readlane(__double2hiint(v[q]), src),
                                 __builtin_amdgcn_readlane(__double2loint(v[q]), src));
        }
    return r;
}
template <int S>
__device__ __forceinline__ int mirror_at(const int (&v)[S], int idx) {
    int r = 0;
#pragma unroll
    for (int q = 0; q < S; ++q)
        if (idx / 64 == q) r = __builtin_amdgcn_readlane(v[q], idx % 64);
    return r;
}

// SH: shared-constraint mode.  Every LP k of the launch has the same A, b and
// row senses (read at offset 0) and its own objective c_k (at k*n; x at k*n,
// y at k*m).  A workgroup takes chunks of P.chunk consecutive LPs; after the
// first LP it keeps the tableau and starts the next LP from the current basis,
// which is primal feasible for every objective: only the objective row is
// rebuilt (d_j = c_{var j} - sum_i c_{basis i} T[i][j], -z in the rhs cell)
// and phase 2 resumes, so phase 1 runs once per workgroup.
template <int NW, int GC, int RB, int CB, int WPE, bool SH = false, int TR = 0>
__global__ void __launch_bounds__(NW * 64) __attribute__((amdgpu_waves_per_eu(WPE, WPE)))
simplex_blk_kernel(KParams P) {
    constexpr int NT = NW * 64;
    constexpr int GR = NT / GC;  // row groups
    constexpr int RP = GR * RB;  // tableau rows
    constexpr int CP = GC * CB;  // column slots
    constexpr int ROW_OBJ = RP - 1, ROW_W = RP - 2, COL_RHS = CP - 1;
    constexpr int RS = (RP + 63) / 64, CS = (CP + 63) / 64;
    static_assert(GR * GC == NT && 64 % GC == 0 && RP >= 4 && CP >= 2 && RS <= 32, "bad block tile");

    // pivot column / pivot row, padded to whole waves so that every lane
    // reads its mirror entries without a bounds branch
    __shared__ double s_f[2][RS * 64], s_p[2][CS * 64];
    __shared__ double s_sig[RP], s_b[RP], s_c[CP], s_w[CP];
    __shared__ int s_artrow[RP], s_rank[RP];
    __shared__ unsigned char s_flag[RP];
    __shared__ int s_k, s_nart, s_bad;
    // shared-constraint mode: objective coefficients of the basis, per row
    // group partial sums of the rebuilt objective row, the chunk being served
    __shared__ double s_cb[SH ? RP : 1], s_part[SH ? GR * CP : 1];
    __shared__ int64_t s_cur, s_end;
    __shared__ int s_pending;      // SH: objective handed back to a cold start
    __shared__ double s_sim[3 * NW];  // SH: per-wave sums for the similarity test
    // TR 2: this LP's recorded pivots (count, then row and slot of each)
    __shared__ int s_tr[TR == 2 ? 1 + 2 * kTraceMaxPivots : 1];

    const int t = threadIdx.x;
    const int lane = t & 63;
    const int tcb = t % GC, trb = t / GC;
    const int i0 = trb * RB;  // first row of this thread

    double T[RB][CB];
    double dO[CS], dW[CS], bR[RS];
    int cv[CS], bs[RS];

    BLP_TDECL;
    const int64_t len = work_len(P);
    bool first = true;
    unsigned dead = 0;  // bit q: row q*64 + lane is redundant
    if (SH && t == 0) {
        s_cur = s_end = 0;
        s_pending = -1;
    }
    // Persistent work list: when thread 0 takes an LP it also reserves the
    // next queue position (pf_q); once the LP is loaded it reads that
    // position's list entry (pf_k, -2 = not read yet).  The atomic and the
    // list read then overlap the solve instead of preceding the next load.
    int pf_q = -1, pf_k = -2;
    // next LP index of this workgroup (-1: none); SH takes chunks
    auto pop = [&]() __attribute__((always_inline)) -> int {
        if (t == 0) {
            int kk;
            if (SH && s_pending >= 0) {  // an objective handed back for a cold start
                kk = s_pending;
                s_pending = -1;
            } else if (!SH && !P.direct) {
                if (first) {
                    const int q = pop_position(P, len, true);
                    kk = q < len ? (int)work_item(P, q) : -1;
                } else {
                    kk = pf_k != -2 ? pf_k : (pf_q < len ? (int)work_item(P, pf_q) : -1);
                }
            } else {
                int64_t q;
                if (SH) {
                    if (s_cur >= s_end) {
                        const int64_t c0 = (int64_t)atomicAdd(bin_head_of(P), 1) * P.chunk;
                        s_cur = c0 < len ? c0 : len;
                        s_end = c0 + P.chunk < len ? c0 + P.chunk : len;
                    }
                    q = s_cur < s_end ? s_cur++ : len;
                } else {  // one LP per workgroup (grid and one-LP-per-launch modes)
                    q = first ? P.direct_first + (int64_t)blockIdx.x : len;
                }
                kk = q < len ? (int)work_item(P, q) : -1;
            }
            s_k = kk;
            s_bad = 0;
            if (!SH && !P.direct) {  // reserve the next position (after the LDS write: no wait for it)
                pf_q = kk >= 0 ? atomicAdd(bin_head_of(P), 1) : (int)len;
                pf_k = -2;
            }
        }
        first = false;
        lds_barrier();
        return __builtin_amdgcn_readfirstlane(s_k);
    };
    for (;;) {
        int k = pop();
        if (k < 0) break;
        BLP_T(t_load0);
        if constexpr (TR == 1) {  // no count until the LP is extracted
            if (t == 0) P.trace[(int64_t)k * P.trace_stride] = -1;
        }

        // ------------------------------------------------------------ load
        LpRef L = lp_ref(P, k);
        LpRef Lin = lp_in(P, L);  // where the constraint data are read
        if (SH) Lin.a_off = Lin.row_off = 0;
        const int m = L.m, n = L.n;
        if (m > RP - 2 || n + 1 > CP) {  // never routed here; no LDS write past the arrays
            write_numerical<NT>(P, L, k, t, ST_INTERNAL);
            lds_barrier();
            continue;
        }
        // every load of the LP is issued before any is used, so the rows',
        // costs' and the tile's loads share one memory round trip
        constexpr int RPT = (RP + NT - 1) / NT, CPT = (CP + NT - 1) / NT;
        double lb[RPT], lc[CPT];
        int ls[RPT];
        // (unconditional loads, indices clamped into the LP: m, n >= 1 here;
        // a select on a loaded value would wait for it at once)
#pragma unroll
        for (int u = 0; u < RPT; ++u) {
            const int i = min(t + u * NT, m - 1);
            lb[u] = P.b[Lin.row_off + i];
            ls[u] = P.sense[Lin.row_off + i];
        }
#pragma unroll
        for (int u = 0; u < CPT; ++u) lc[u] = P.c[L.col_off + min(t + u * NT, n - 1)];
        // keep these loads ahead of the tile's: loads complete in issue order,
        // so the rows can be prepared while the tile is still arriving
        __builtin_amdgcn_sched_barrier(0);
        // A straight into the tile (scaled below, once the row signs are known)
        // with range-checked buffer loads: the resource covers this LP's m x n
        // block, so rows >= m read as 0; columns >= n get an offset beyond it.
        // Nothing waits for them before the tile is finished below (the
        // barriers in between order LDS only).
        {
            const __amdgpu_buffer_rsrc_t rs = __builtin_amdgcn_make_buffer_rsrc(
                const_cast<double*>(P.A + Lin.a_off), (short)0, m * n * (int)sizeof(double), 0x00020000);
#pragma unroll
            for (int c = 0; c < CB; ++c) {
                const int j = c * GC + tcb;
                const unsigned cofs = j < n ? (unsigned)(i0 * n + j) * 8u : 0x80000000u;
#pragma unroll
                for (int r = 0; r < RB; ++r)
                    T[r][c] = __builtin_bit_cast(
                        double, __builtin_amdgcn_raw_buffer_load_b64(rs, (int)(cofs + (unsigned)(r * n) * 8u), 0, 0));
            }
        }
        int bad = 0;
#pragma unroll
        for (int u = 0; u < RPT; ++u) {
            const int i = t + u * NT;
            if (i < m) bad |= prep_row(i, lb[u], ls[u], s_sig, s_b, s_flag);
        }
#pragma unroll
        for (int u = 0; u < CPT; ++u) {
            const int j = t + u * NT;
            if (j < n) {
                s_c[j] = lc[u];
                bad |= !isfinite(lc[u]);
            }
        }
        lds_barrier();
        BLP_T(t_ld1);
        BLP_TACC(TM_LD_ROWS, t_load0, t_ld1);
        if (t < 64) scan_art_rows(m, lane, s_flag, s_artrow, s_rank, &s_nart);
        lds_barrier();
        const int nart = __builtin_amdgcn_readfirstlane(s_nart);
        if (n + nart + 1 > CP) {
            write_numerical<NT>(P, L, k, t, ST_INTERNAL);
            lds_barrier();
            continue;
        }
        // Phase-1 row: for each column, the artificial rows summed in row
        // order (one sequential sum per column, columns spread over threads).
        if (nart > 0) {
            for (int j = t; j < CP; j += NT) {
                double acc = 0.0;
                if (j < n) {
                    // 8 loads in flight, then their terms in row order
                    for (int q0 = 0; q0 < nart; q0 += 8) {
                        double v[8];
#pragma unroll
                        for (int u = 0; u < 8; ++u) {
                            const int ii = s_artrow[q0 + u < nart ? q0 + u : q0];
                            v[u] = P.A[Lin.a_off + (int64_t)ii * n + j];
                        }
#pragma unroll
                        for (int u = 0; u < 8; ++u)
                            if (q0 + u < nart) acc = acc + s_sig[s_artrow[q0 + u]] * v[u];
                    }
                } else if (j < n + nart) {
                    acc = -1.0;
                } else if (j == COL_RHS) {
                    for (int q = 0; q < nart; ++q) acc = acc + s_b[s_artrow[q]];
                }
                s_w[j] = acc;
            }
            lds_barrier();
        }
        // finish the tile with selects only (no divergent branch around the
        // tile): row signs on the A block, +0 beyond it, then the rhs column,
        // the surplus columns of the artificial rows and the objective rows
        {
            const bool obj_grp = trb == GR - 1;  // holds rows ROW_W and ROW_OBJ
#pragma unroll
            for (int c = 0; c < CB; ++c) {
                const int j = c * GC + tcb;
                const bool inA = j < n;
                const bool rhs = c == CB - 1 && tcb == GC - 1;
                const bool art = j >= n && j < n + nart;
                const int ar = s_artrow[art ? j - n : 0];
                const double cj = s_c[inA ? j : 0];
                const double wj = nart > 0 ? s_w[j] : 0.0;
#pragma unroll
                for (int r = 0; r < RB; ++r) {
                    const int i = i0 + r;
                    const bool row = i < m;
                    const double sg = s_sig[row ? i : 0];
                    const double bi = s_b[row ? i : 0];
                    bad |= !isfinite(T[r][c]);
                    double v = inA && row ? sg * T[r][c] : 0.0;
                    v = row && rhs ? bi : v;
                    v = row && art ? (ar == i ? -1.0 : 0.0) : v;
                    if (r == RB - 1) v = obj_grp ? (inA ? cj : 0.0) : v;
                    if (r == RB - 2) v = obj_grp ? wj : v;
                    T[r][c] = v;
                }
            }
            // the finished tile and the finiteness flag are computed here:
            // otherwise they sink into the pivot loop, and the raw tile and
            // every input of the selects above stay live across Step 1 (the
            // 160 x 160 tile then spilled)
#pragma unroll
            for (int c = 0; c < CB; ++c)
#pragma unroll
                for (int r = 0; r < RB; ++r) __asm__ volatile("" : "+v"(T[r][c]));
            __asm__ volatile("" : "+v"(bad));
        }
#ifdef BLP_PHASE_TIMERS
        __builtin_amdgcn_s_waitcnt(0);  // the tile's loads have returned
        BLP_T(t_ld2);
        BLP_TACC(TM_LD_TILE, t_ld1, t_ld2);
#endif
        // register mirrors (identical in every wave)
#pragma unroll
        for (int q = 0; q < CS; ++q) {
            const int j = q * 64 + lane;
            dO[q] = j < n ? s_c[j] : 0.0;
            dW[q] = (nart > 0 && j < CP) ? s_w[j] : 0.0;
            cv[q] = j < n ? j : (j < n + nart ? n + s_artrow[j - n] : ID_NONE);
        }
#pragma unroll
        for (int q = 0; q < RS; ++q) {
            const int i = q * 64 + lane;
            bR[q] = i < m ? s_b[i] : (i == ROW_W && nart > 0 ? s_w[COL_RHS] : 0.0);
            bs[q] = i < m ? ((s_flag[i] & RF_ART) ? n + m + i : n + i) : ID_NONE;
        }
        if (bad) atomicOr(&s_bad, 1);
        lds_barrier();
        if (s_bad) {
            write_numerical<NT>(P, L, k, t, ST_NUMERICAL);
            lds_barrier();
            continue;
        }
        if constexpr (TR == 2) {
            // the LP's recorded pivots into LDS; only LPs without artificial
            // rows replay (their pivots are all phase-2 pivots)
            const int32_t* tr = P.trace + (int64_t)k * P.trace_stride;
            const int cnt = tr[0];
            const bool ok = nart == 0 && cnt >= 0 && cnt <= kTraceMaxPivots && 1 + 2 * cnt <= P.trace_stride;
            int badp = 0;
            for (int i = t; ok && i < 1 + 2 * cnt; i += NT) {
                const int v = tr[i];
                s_tr[i] = v;
                // rows in [0, m), slots in [0, n) (no surplus slots here)
                badp |= i > 0 && (v < 0 || v >= ((i & 1) ? m : n));
            }
            if (badp) atomicOr(&s_bad, 1);
            lds_barrier();
            if (!ok || s_bad) {
                write_numerical<NT>(P, L, k, t, ST_INTERNAL);
                lds_barrier();
                continue;
            }
        }
        const double w0 = mirror_at(bR, ROW_W);
        dead = 0;
        int mode = nart > 0 ? 1 : 2;
        const int max_iter = P.max_iter > 0 ? P.max_iter : 50 * (m + n);
        const int bland_after = P.bland_after > 0 ? P.bland_after : (m > n ? m : n);
        const int id_lim = n + m;
        int iters = 0, degen = 0, st = -1;

        // Outputs of LP k straight from the mirrors (wave 0; the mirrors are
        // identical in every wave).  Every structural and logical variable
        // sits in exactly one place, a row (basic: x = rhs, dual 0) or a
        // slot (nonbasic: x = 0, dual from the objective row), so x and y are
        // written by one scatter each, without LDS or barriers; the duals
        // take the same signs as the oracle's (-d for "<=" rows, also on a
        // zero d).  Only s_flag is read, which no other wave writes before
        // the next pop's barrier.
        auto extract = [&]() __attribute__((always_inline)) {
            BLP_T(t_x0);
            if (t < 64) {
                const double z = -mirror_at(bR, ROW_OBJ);
                const int sto = st == ST_OPTIMAL && !isfinite(z) ? ST_NUMERICAL : st;
                const bool nan_out = sto == ST_NUMERICAL;
                const double qnan = __builtin_nan("");
#pragma unroll
                for (int q = 0; q < CS; ++q) {
                    const int j = q * 64 + lane, v = cv[q];
                    if (j < COL_RHS) {
                        if (v < n) {
                            P.x[L.col_off + v] = nan_out ? qnan : 0.0;
                        } else if (v < n + m) {
                            const double d = dO[q];
                            P.y[L.row_off + (v - n)] = nan_out ? qnan : ((s_flag[v - n] & RF_GE) ? d : -d);
                        }
                    }
                }
#pragma unroll
                for (int q = 0; q < RS; ++q) {
                    const int i = q * 64 + lane, v = bs[q];
                    if (i < m) {
                        if (v < n) {
                            P.x[L.col_off + v] = nan_out ? qnan : bR[q];
                        } else if (v < n + m) {
                            P.y[L.row_off + (v - n)] = nan_out ? qnan : ((s_flag[v - n] & RF_GE) ? 0.0 : -0.0);
                        }
                    }
                }
                if (lane == 0) {
                    if constexpr (TR == 1) P.trace[(int64_t)k * P.trace_stride] = 2 + 2 * (iters - 1) < P.trace_stride ? iters : -1;
                    P.status[k] = sto;
                    P.iters[k] = iters;
                    P.obj[k] = (sto == ST_OPTIMAL || sto == ST_ITER_LIMIT) ? z
                               : sto == ST_UNBOUNDED                      ? __builtin_inf()
                               : sto == ST_INFEASIBLE                     ? -__builtin_inf()
                                                                          : qnan;
                }
            }
            BLP_T(t_x1);
            BLP_TACC(TM_EXTRACT, t_x0, t_x1);
            BLP_TCOUNT(TM_PIVOTS, (unsigned long long)iters);
            BLP_TCOUNT(TM_LPS, 1ull);
        };
        // ------------------------------------------------------ pivot loop
        // mode 1 = phase 1, 2 = phase 2, 3 = driving the remaining basic
        // artificials out after a feasible phase 1.  Step 1 for the next
        // pivot runs on the updated mirrors before the tile's rank-1 update,
        // so the two overlap.
        int drive_r = 0, buf = 0;
        int e_id = ID_NONE, e = -1;  // entering variable and slot from Step 1
        auto step1 = [&]() __attribute__((always_inline)) {
            if constexpr (TR == 2) {  // the recorded entering slot
                if (iters < s_tr[0]) {
                    e = s_tr[2 + 2 * iters];
                    e_id = mirror_at(cv, e);
                } else {
                    e_id = ID_NONE;
                }
                return;
            }
            double da[CS];  // the active objective row
#pragma unroll
            for (int q = 0; q < CS; ++q) da[q] = mode == 1 ? dW[q] : dO[q];
            if (P.pivot_rule == 1 && degen < bland_after)
                price_rpc_regs(COL_RHS, lane, id_lim, P.eps_price, P.seed, k, iters, da, cv, e_id, e);
            else
                price_regs(COL_RHS, lane, id_lim, P.eps_price, degen >= bland_after, da, cv, e_id, e);
        };
        step1();
        if (!SH && !P.direct && t == 0 && pf_k == -2) pf_k = pf_q < len ? (int)work_item(P, pf_q) : -1;
        BLP_T(t_load1);
        BLP_TACC(TM_LOAD, t_load0, t_load1);
        for (;;) {
            if (SH && st != -1) {
                // SH: LP k is done (st >= 0) or its objective was not finite
                // (st == -2, outputs written).  Extract it, take the next
                // objective and rebuild the objective row on the current
                // basis; phase 2 resumes from there.  If phase 1 ended the
                // solve (infeasible), every objective gets that outcome.
                if (st >= 0) extract();
                const bool same = st >= 0 && mode != 2;
                k = pop();
                if (k < 0) break;
                L = lp_ref(P, k);
                if (same) continue;
                {
                    // warm start only if the new objective points close to the
                    // previous one (cosine > 0.9); otherwise the previous basis
                    // is usually farther from the new optimum than the slack
                    // basis, and the objective goes back to a cold start
                    double dot = 0.0, nn = 0.0, oo = 0.0;
                    for (int j = t; j < n; j += NT) {
                        const double cn = P.c[L.col_off + j], co = s_c[j];
                        dot += cn * co;
                        nn += cn * cn;
                        oo += co * co;
                    }
                    for (int o = 32; o >= 1; o >>= 1) {
                        dot += __shfl_xor(dot, o);
                        nn += __shfl_xor(nn, o);
                        oo += __shfl_xor(oo, o);
                    }
                    if (lane == 0) {
                        s_sim[3 * (t >> 6)] = dot;
                        s_sim[3 * (t >> 6) + 1] = nn;
                        s_sim[3 * (t >> 6) + 2] = oo;
                    }
                    lds_barrier();
                    dot = nn = oo = 0.0;
                    for (int w = 0; w < NW; ++w) {
                        dot += s_sim[3 * w];
                        nn += s_sim[3 * w + 1];
                        oo += s_sim[3 * w + 2];
                    }
                    if (!(dot > 0.9 * sqrt(nn * oo))) {  // also taken for non-finite c
                        if (t == 0) s_pending = k;
                        lds_barrier();
                        break;
                    }
                }
                int badc = 0;
                for (int j = t; j < n; j += NT) {
                    const double cj = P.c[L.col_off + j];
                    badc |= !isfinite(cj);
                    s_c[j] = cj;
                }
                if (badc) atomicOr(&s_bad, 1);
                lds_barrier();
                if (s_bad) {
                    write_numerical<NT>(P, L, k, t, ST_NUMERICAL);
                    lds_barrier();
                    st = -2;  // written; take the next objective
                    continue;
                }
                if (t < 64) {
#pragma unroll
                    for (int q = 0; q < RS; ++q) {
                        const int i = q * 64 + lane;
                        if (i < RP) s_cb[i] = (i < m && bs[q] < n) ? s_c[bs[q]] : 0.0;
                    }
                }
                lds_barrier();
                // partial sums over this thread's rows, in row order
#pragma unroll
                for (int c = 0; c < CB; ++c) {
                    double acc = 0.0;
#pragma unroll
                    for (int r = 0; r < RB; ++r) acc = __builtin_fma(s_cb[i0 + r], T[r][c], acc);
                    s_part[trb * CP + c * GC + tcb] = acc;
                }
                lds_barrier();
                if (t < 64) {
#pragma unroll
                    for (int q = 0; q < CS; ++q) {
                        const int j = q * 64 + lane;
                        if (j < CP) {
                            double z = 0.0;
                            for (int g = 0; g < GR; ++g) z = z + s_part[g * CP + j];
                            const int v = cv[q];
                            s_p[0][j] = (v < n ? s_c[v] : 0.0) - z;
                        }
                    }
                }
                lds_barrier();
#pragma unroll
                for (int q = 0; q < CS; ++q) {
                    const int j = q * 64 + lane;
                    dO[q] = j < CP ? s_p[0][j] : 0.0;
                }
#pragma unroll
                for (int q = 0; q < RS; ++q)
                    if (q * 64 + lane == ROW_OBJ) bR[q] = s_p[0][COL_RHS];
                if (trb == GR - 1) {
#pragma unroll
                    for (int c = 0; c < CB; ++c) T[RB - 1][c] = s_p[0][c * GC + tcb];
                }
                lds_barrier();
                st = -1;
                iters = 0;
                degen = 0;
                step1();
                continue;
            }
            int l = -1, lv = ID_NONE;
            double rmin = 1.0;
            BLP_T(t_p0);
            if (mode == 3) {
                int r0 = -1;
#pragma unroll
                for (int q = 0; q < RS; ++q) {
                    const int i = q * 64 + lane;
                    const bool cand = i < m && i >= drive_r && bs[q] >= id_lim && !((dead >> q) & 1u);
                    const unsigned long long mk = __ballot(cand);
                    if (r0 < 0 && mk) r0 = q * 64 + __ffsll((long long)mk) - 1;
                }
                if (r0 < 0) {
                    mode = 2;
                    degen = 0;
                    step1();
                    continue;
                }
                drive_r = r0 + 1;
                // row r0 into s_p[buf]; the lowest-id non-artificial column
                // with a usable entry enters
                lds_barrier();
                if (trb == r0 / RB) {
                    const int rr = r0 % RB;
#pragma unroll
                    for (int r = 0; r < RB; ++r)
                        if (r == rr) {
#pragma unroll
                            for (int c = 0; c < CB; ++c) s_p[buf][c * GC + tcb] = T[r][c];
                        }
                }
                lds_barrier();
                double bk = -__builtin_inf();
                int bid = ID_NONE, bpos = -1;
#pragma unroll
                for (int q = 0; q < CS; ++q) {
                    const int j = q * 64 + lane;
                    if (j < COL_RHS) {
                        const int v = cv[q];
                        if (v < id_lim && fabs(s_p[buf][j]) > P.eps_piv && key_before(0.0, v, bk, bid)) {
                            bk = 0.0;
                            bid = v;
                            bpos = j;
                        }
                    }
                }
                wave_argmax(bk, bid, bpos);
                lds_barrier();
                if (bid == ID_NONE) {  // redundant row
                    if (r0 % 64 == lane) dead |= 1u << (r0 / 64);
                    continue;
                }
                l = r0;
                e = bpos;
                e_id = bid;
                lv = mirror_at(bs, r0);
            } else {
                if (e_id == ID_NONE) {
                    if (mode == 2) {
                        st = ST_OPTIMAL;
                        if (SH) continue;
                        break;
                    }
                    if (mirror_at(bR, ROW_W) > P.eps_feas * (1.0 + w0)) {
                        st = ST_INFEASIBLE;
                        if (SH) continue;
                        break;
                    }
                    mode = 3;
                    drive_r = 0;
                    continue;
                }
                if (iters >= max_iter) {
                    st = ST_ITER_LIMIT;
                    if (SH) continue;
                    break;
                }
            }
            BLP_T(t_p1);
            // publish the entering column (f) and clear its slot; the slot
            // becomes the leaving variable's column
            const int e_piv = e;  // Step 1 of the next pivot overwrites e before the update
            {
                const int ce = __builtin_amdgcn_readfirstlane(e / GC), te = e % GC;
                if (tcb == te) {
#pragma unroll
                    for (int c = 0; c < CB; ++c)
                        if (c == ce) {
#pragma unroll
                            for (int r = 0; r < RB; ++r) {
                                s_f[buf][i0 + r] = T[r][c];
                                if (!SH) T[r][c] = 0.0;
                            }
                        }
                }
            }
            lds_barrier();
            BLP_T(t_p2);
            double fr[RS];
#pragma unroll
            for (int q = 0; q < RS; ++q) {
                const int i = q * 64 + lane;
                const double v = s_f[buf][i];
                fr[q] = i < RP ? v : 0.0;
            }
            if (mode != 3) {
                if constexpr (TR == 2) {  // the recorded leaving row
                    l = s_tr[1 + 2 * iters];
                    lv = mirror_at(bs, l);
                } else {
                    l = ratio_regs(m, lane, P.eps_piv, fr, bR, bs, dead, rmin, lv);
                }
                if (l < 0) {
                    st = mode == 2 ? ST_UNBOUNDED : ST_NUMERICAL;
                    if (SH) continue;  // the tile is untouched (SH clears the slot at the update)
                    break;
                }
            }
            const double pe = mirror_at(fr, l);
            if constexpr (TR == 1) {  // record (row, slot) of this pivot
                if (t == 0 && 2 + 2 * iters < P.trace_stride) {
                    int32_t* tr = P.trace + (int64_t)k * P.trace_stride;
                    tr[1 + 2 * iters] = l;
                    tr[2 + 2 * iters] = e_piv;
                }
            }
            BLP_T(t_p2b);
            BLP_TACC(TM_RTEST, t_p2, t_p2b);
            // Step 3's new pivot row.  The owners of row l (GC lanes of one
            // wave) put its entries into s_p[buf] and zero them in the tile;
            // the whole wave holding row l then divides CS entries per lane
            // (LDS operations of one wave complete in order, so no barrier
            // is needed between the two).  After the update the tile's row l
            // is fma(1, p, 0) = p.
            constexpr int ROWS_PER_WAVE = 64 / GC * RB;
            const bool row_wave = t / 64 == l / ROWS_PER_WAVE;
            if (row_wave) {
                if (trb == l / RB) {
                    const int rl = __builtin_amdgcn_readfirstlane(l % RB);
                    const int de = e - tcb;  // slot c*GC + tcb is e iff c*GC == de
#pragma unroll
                    for (int r = 0; r < RB; ++r)
                        if (r == rl) {
#pragma unroll
                            for (int c = 0; c < CB; ++c) {
                                s_p[buf][c * GC + tcb] = c * GC == de ? 1.0 : T[r][c];
                                T[r][c] = 0.0;
                            }
                        }
                }
                __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
                __builtin_amdgcn_wave_barrier();
                __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
                const double y = 1.0 / pe;
                const double ape = fabs(pe);
                const bool pe_ok = ape >= 0x1p-500 && ape <= 0x1p500;
                double xs[CS], ps[CS];
                bool slow = false;
#pragma unroll
                for (int q = 0; q < CS; ++q) {
                    xs[q] = s_p[buf][q * 64 + lane];
                    bool ok;
                    ps[q] = div_rn_fast(xs[q], pe, y, pe_ok, ok);
                    slow |= !ok & (q * 64 + lane < CP);  // padding slots hold no data
                }
                if (slow) {  // extreme magnitudes only: the plain division
#pragma unroll
                    for (int q = 0; q < CS; ++q) ps[q] = xs[q] / pe;
                }
#pragma unroll
                for (int q = 0; q < CS; ++q) s_p[buf][q * 64 + lane] = ps[q];
#ifdef BLP_PHASE_TIMERS
                __builtin_amdgcn_s_waitcnt(0xc07f);  // the row's LDS writes done
                BLP_T(t_p2c);
                BLP_TACC(TM_DIV, t_p2b, t_p2c);
                BLP_TCOUNT(TM_DIVN, 1ull);
#endif
            }
            lds_barrier();
            BLP_T(t_p3);
            double nf[RB], pc[CB];
#pragma unroll
            for (int r = 0; r < RB; ++r) nf[r] = -s_f[buf][i0 + r];
            // only the wave holding row l: the pivot row (zeroed) takes 1 * p
            if (row_wave) {
                const int dl = l - i0;  // row i0 + r is l iff r == dl
#pragma unroll
                for (int r = 0; r < RB; ++r) nf[r] = r == dl ? 1.0 : nf[r];
            }
#pragma unroll
            for (int c = 0; c < CB; ++c) pc[c] = s_p[buf][c * GC + tcb];
            // Step 3 on the mirrors
            {
                const double pr = s_p[buf][COL_RHS];
                const double fO = s_f[buf][ROW_OBJ], fW = s_f[buf][ROW_W];
                const int el = e - lane, ll = l - lane;  // slot / row q*64 + lane is e / l iff q*64 == el / ll
                // slots j >= CP (padding lanes) carry values never read
#pragma unroll
                for (int q = 0; q < CS; ++q) {
                    const double pj = s_p[buf][q * 64 + lane];
                    const bool ent = q * 64 == el;
                    dO[q] = __builtin_fma(-fO, pj, ent ? 0.0 : dO[q]);
                    // the phase-1 row is read only in phase 1 and drive-out
                    if (mode != 2) dW[q] = __builtin_fma(-fW, pj, ent ? 0.0 : dW[q]);
                    cv[q] = ent ? lv : cv[q];
                }
#pragma unroll
                for (int q = 0; q < RS; ++q) {
                    const bool piv = q * 64 == ll;
                    bR[q] = piv ? pr : __builtin_fma(-fr[q], pr, bR[q]);
                    bs[q] = piv ? e_id : bs[q];
                }
            }
            ++iters;
            if (mode != 3) {
                degen = rmin == 0.0 ? degen + 1 : 0;
                step1();  // next pivot's entering column, overlapping the update below
            }
            if (SH) {  // clear the entering slot here, once the pivot is certain
                const int ce = __builtin_amdgcn_readfirstlane(e_piv / GC), te = e_piv % GC;
                if (tcb == te) {
#pragma unroll
                    for (int c = 0; c < CB; ++c)
                        if (c == ce) {
#pragma unroll
                            for (int r = 0; r < RB; ++r)
                                if (i0 + r != l) T[r][c] = 0.0;
                        }
                }
            }
            // Step 3 on the tile; the pivot row becomes p (fma(1, p, +0) = p)
#pragma unroll
            for (int r = 0; r < RB; ++r)
#pragma unroll
                for (int c = 0; c < CB; ++c) T[r][c] = __builtin_fma(nf[r], pc[c], T[r][c]);
            BLP_T(t_p4);
            BLP_TACC(TM_PRICE, t_p0, t_p1);
            BLP_TACC(TM_PUBCOL, t_p1, t_p2);
            BLP_TACC(TM_RATIO, t_p2, t_p3);
            BLP_TACC(TM_PIVOT, t_p3, t_p4);
            buf ^= 1;
        }

        // ------------------------------------------------------ extraction
        if (!SH) extract();
    }
    BLP_TFLUSH();
}

}  // namespace blp
