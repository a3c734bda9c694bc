// Column-split kernel: one LP per workgroup of NW waves, the condensed
// tableau split by columns between the waves, one workgroup barrier per
// pivot.  It takes LPs whose initial basis is feasible (no artificial rows,
// so no phase 1) under the largest-coefficient rule; the scheduler sends
// other LPs to the block-tile or streaming kernels.
//
// Same method, same condensed tableau and the same operation order as the
// other simplex kernels (every stored cell bit-identical to the full tableau
// of Sec. 3.1 after the Step-3 update).  What changes is the distribution:
//
//  * Wave w holds the column slots w*CPW .. w*CPW + CPW - 1 for every
//    constraint row, as a GRW x GCW grid of lanes: lane (ri, ci) = (lane /
//    GCW, lane % GCW) holds rows ri + GRW a (a < RB) of the local slots
//    ci + GCW b (b < CB).  The objective row and the rhs column are not in
//    the tile: they live in register mirrors, the objective row by local
//    slot (lane s holds slot s of its wave) and the rhs column and the basis
//    by row (lane holds rows lane and 64 + lane; the objective row's rhs
//    cell is mirror row 127).  Every wave keeps identical rhs and basis
//    mirrors by applying the same FMAs.
//  * A wave prices its own slots (Step 1 of Sec. 3.1 over its part of the
//    objective row) and at once runs the ratio test (Step 2) on its own best
//    column, which it holds for every row.  Each wave then publishes its
//    candidate -- key, variable, pivot row, minimum ratio and the column
//    itself -- and after ONE barrier every wave picks the same winner by the
//    largest-coefficient rule with the lowest variable id on ties: exactly
//    Step 1 over the whole row followed by Step 2 on the chosen column.
//    (The block-tile kernel needs two barriers per pivot: one to share the
//    entering column, one to share the divided pivot row.)
//  * Step 3 then needs no further exchange between the waves: the owners of
//    row l in each wave put their entries of row l into LDS, every lane of
//    the wave divides the entries it needs itself (LDS is ordered within a
//    wave), and each wave applies the rank-1 update to its own slots with
//    the published pivot column.
#pragma once

#include "blp_kernels.hpp"
#include "simplex_blk.hpp"
#include "simplex_common.hpp"

namespace blp {

// One wave's candidate for the next pivot (written by lane 0 of the wave).
struct ColsRec {
    int khi;      // key bit pattern (a reduced cost above eps_price, or -inf: none)
    unsigned klo;
    int pk;       // pack_id(variable, local slot), PACK_NONE: no candidate
    int l;        // pivot row of the ratio test on that column (-1: none)
    double rmin;  // its minimum ratio
    double pe;    // the pivot element (the column's entry in row l)
};

template <int NW, int GCW, int RB, int CB, int WPE>
__global__ void __launch_bounds__(NW * 64) __attribute__((amdgpu_waves_per_eu(WPE, WPE)))
simplex_cols_kernel(KParams P) {
    constexpr int NT = NW * 64;
    constexpr int GRW = 64 / GCW;    // row groups of a wave
    constexpr int RP = GRW * RB;     // constraint rows held
    constexpr int CPW = GCW * CB;    // column slots per wave
    constexpr int NS = NW * CPW;     // column slots per LP (the rhs is not a slot)
    constexpr int ROW_OBJ = 127;     // mirror row of the objective row's rhs cell
    static_assert(64 % GCW == 0 && RP <= 127 && CPW <= 64 && NT >= RP && NT >= NS, "bad column-split tile");

    // [wave][buffer][row]: the wave's candidate column (rows RP..126 stay
    // zero, row 127 is the objective row's entry); [wave][local slot]: the
    // wave's part of row l; [wave][buffer]: the candidates
    __shared__ double s_col[NW][2][128];
    __shared__ double s_row[NW][64];
    __shared__ ColsRec s_rec[NW][2];
    __shared__ double s_b[RP], s_c[NS];
    __shared__ unsigned char s_flag[RP];
    __shared__ int s_k, s_bad;

    const int t = threadIdx.x;
    const int lane = t & 63;
    const int w = __builtin_amdgcn_readfirstlane(t >> 6);
    const int ri = lane / GCW, ci = lane % GCW;
    const int s0 = w * CPW;  // first global slot of this wave

    double T[RB][CB];
    double bR[2];  // rhs mirror: rows lane, 64 + lane
    int bs[2];     // basis mirror
    double dO;     // objective row at local slot `lane`
    int cv;        // variable of local slot `lane`

    for (int i = t; i < NW * 2 * 128; i += NT) (&s_col[0][0][0])[i] = 0.0;
    // phase cycle counters (-DBLP_PHASE_TIMERS): load, candidate (Steps 1 and
    // 2 of the wave), exchange (record, barrier, winner), pivot row (its
    // publication and division), update (mirrors and tile), extraction
    BLP_TDECL;

    const int64_t len = work_len(P);
    bool first = true;
    int pf_q = -1, pf_k = -2;  // reserved next queue position and its list entry (-2: not read)
    auto pop = [&]() __attribute__((always_inline)) -> int {
        if (t == 0) {
            int kk;
            if (!P.direct) {
                if (first) {
                    const int q = pop_position(P, len, true);
                    kk = q < len ? (int)work_item(P, q) : -1;
                } else {
                    kk = pf_k != -2 ? pf_k : (pf_q < len ? (int)work_item(P, pf_q) : -1);
                }
            } else {
                const int64_t q = first ? P.direct_first + (int64_t)blockIdx.x : len;
                kk = q < len ? (int)work_item(P, q) : -1;
            }
            s_k = kk;
            s_bad = 0;
            if (!P.direct) {
                pf_q = kk >= 0 ? atomicAdd(bin_head_of(P), 1) : (int)len;
                pf_k = -2;
            }
        }
        first = false;
        lds_barrier();
        return __builtin_amdgcn_readfirstlane(s_k);
    };

    for (;;) {
        const int k = pop();
        if (k < 0) break;
        BLP_T(t_load0);

        // ------------------------------------------------------------ load
        const LpRef L = lp_ref(P, k);
        const LpRef Lin = lp_in(P, L);
        const int m = L.m, n = L.n;
        if (m > RP || n > NS || P.pivot_rule != 0) {  // never routed here
            write_numerical<NT>(P, L, k, t, ST_INTERNAL);
            lds_barrier();
            continue;
        }
        // rows, costs and the tile are all in flight before any is used
        const int ir = min(t, m - 1);
        const double lb = P.b[Lin.row_off + ir];
        const int ls = P.sense[Lin.row_off + ir];
        const double lc = P.c[L.col_off + min(t, n - 1)];
        __builtin_amdgcn_sched_barrier(0);
        {
            // range-checked buffer loads over the LP's m x n block: rows >= m
            // read 0, columns >= n get an offset beyond the block
            const __amdgpu_buffer_rsrc_t rs = __builtin_amdgcn_make_buffer_rsrc(
                const_cast<double*>(P.A + Lin.a_off), (short)0, m * n * (int)sizeof(double), 0x00020000);
#pragma unroll
            for (int b = 0; b < CB; ++b) {
                const int j = s0 + ci + GCW * b;
                const unsigned cofs = j < n ? (unsigned)(ri * n + j) * 8u : 0x80000000u;
#pragma unroll
                for (int a = 0; a < RB; ++a)
                    T[a][b] = __builtin_bit_cast(double, __builtin_amdgcn_raw_buffer_load_b64(
                                                             rs, (int)(cofs + (unsigned)(GRW * a * n) * 8u), 0, 0));
            }
        }
        // rows in "<=" form (Sec. 3): a ">=" row is negated; a negative
        // rhs would need an artificial variable, which this kernel does not
        // take (the scheduler never sends such an LP here)
        int bad = 0, art = 0;
        if (t < m) {
            const int ge = ls != 0;
            const double bn = ge ? -lb : lb;
            s_b[t] = bn;
            s_flag[t] = (unsigned char)(ge ? RF_GE : 0);
            bad |= !isfinite(lb);
            art |= bn < 0.0;
        }
        if (t < n) {
            s_c[t] = lc;
            bad |= !isfinite(lc);
        }
        if (art) atomicOr(&s_bad, 2);
        lds_barrier();
        if (s_bad & 2) {
            write_numerical<NT>(P, L, k, t, ST_INTERNAL);
            lds_barrier();
            continue;
        }
        // the tile: the ">=" rows negated (a sign flip), zero beyond the A
        // block (the loads already read 0 there)
        {
            unsigned neg = 0;  // bit a: row ri + GRW a is a ">=" row
#pragma unroll
            for (int a = 0; a < RB; ++a) {
                const int i = ri + GRW * a;
                neg |= (i < m && (s_flag[i] & RF_GE)) ? 1u << a : 0u;
            }
#pragma unroll
            for (int a = 0; a < RB; ++a)
#pragma unroll
                for (int b = 0; b < CB; ++b) {
                    bad |= !isfinite(T[a][b]);
                    T[a][b] = ((neg >> a) & 1u) ? -T[a][b] : T[a][b];
                }
        }
#pragma unroll
        for (int b = 0; b < CB; ++b)
#pragma unroll
            for (int a = 0; a < RB; ++a) __asm__ volatile("" : "+v"(T[a][b]));
        {
            const int j = s0 + lane;
            dO = lane < CPW && j < n ? s_c[j] : 0.0;
            cv = lane < CPW && j < n ? j : ID_NONE;
#pragma unroll
            for (int q = 0; q < 2; ++q) {
                const int i = q * 64 + lane;
                bR[q] = i < m ? s_b[i] : 0.0;
                bs[q] = i < m ? n + i : ID_NONE;
            }
        }
        if (bad) atomicOr(&s_bad, 1);
        lds_barrier();
        if (s_bad) {
            write_numerical<NT>(P, L, k, t, ST_NUMERICAL);
            lds_barrier();
            continue;
        }
        const int max_iter = P.max_iter > 0 ? P.max_iter : 50 * (m + n);
        const int bland_after = P.bland_after > 0 ? P.bland_after : (m > n ? m : n);
        const int id_lim = n + m;
        int iters = 0, degen = 0, st = -1, buf = 0;
        BLP_T(t_load1);
        BLP_TACC(TM_LOAD, t_load0, t_load1);

        // ------------------------------------------------------ pivot loop
        for (;;) {
            BLP_T(t_p0);
            // ---- this wave's candidate (before the barrier)
            int khi;
            unsigned klo;
            int l = -1;
            double rmin = 1.0, pe = 1.0;
            const bool bland = degen >= bland_after;
            const bool ok = lane < CPW && cv < id_lim && dO > P.eps_price;
            const long long kb = __double_as_longlong(ok ? (bland ? 0.0 : dO) : -__builtin_inf());
            const int pk = wave_argmax_i64((int)(kb >> 32), (unsigned)kb, ok ? pack_id(cv, lane) : PACK_NONE, khi, klo);
            if (pk != PACK_NONE) {
                // publish the candidate column, then the ratio test on it
                const int ep = unpack_pos(pk);
                const int be = __builtin_amdgcn_readfirstlane(ep / GCW);
                if (ci == ep % GCW) {
#pragma unroll
                    for (int b = 0; b < CB; ++b)
                        if (b == be) {
#pragma unroll
                            for (int a = 0; a < RB; ++a) s_col[w][buf][ri + GRW * a] = T[a][b];
                            // a distinct end to each case: otherwise the cases
                            // merge into one store of a selected column, which
                            // holds a copy of the column in registers
                            __asm__ volatile("; cols publish %0" ::"i"(b));
                        }
                }
                if (lane == ep) s_col[w][buf][ROW_OBJ] = dO;
                __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
                __builtin_amdgcn_wave_barrier();
                __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
                double fr[2];
#pragma unroll
                for (int q = 0; q < 2; ++q) fr[q] = s_col[w][buf][q * 64 + lane];
                int lvid;
                l = ratio_regs(m, lane, P.eps_piv, fr, bR, bs, 0u, rmin, lvid);
                if (l >= 0) pe = mirror_at(fr, l);
            }
            BLP_T(t_p1);
            if (lane == 0) {
                ColsRec r;
                r.khi = khi;
                r.klo = klo;
                r.pk = pk;
                r.l = l;
                r.rmin = rmin;
                r.pe = pe;
                s_rec[w][buf] = r;
            }
            lds_barrier();
            // ---- the winner (the same in every wave): the larger key, then
            // the smaller packed id; the lowest wave on a full tie (no
            // candidate anywhere).  Lane v reads wave v's record, so that
            // the records arrive in one LDS round trip.
            int rhi = (int)0xfff00000, rpk = PACK_NONE, rl = -1;
            unsigned rlo = 0u;
            double rrm = 1.0, rpe = 1.0;
            if (lane < NW) {
                const ColsRec& r = s_rec[lane][buf];
                rhi = r.khi;
                rlo = r.klo;
                rpk = r.pk;
                rl = r.l;
                rrm = r.rmin;
                rpe = r.pe;
            }
            int W = 0;
            long long kw = 0;
            int pw = PACK_NONE;
#pragma unroll
            for (int v = 0; v < NW; ++v) {
                const int hv = __builtin_amdgcn_readlane(rhi, v);
                const unsigned lv_ = (unsigned)__builtin_amdgcn_readlane((int)rlo, v);
                const int pv = __builtin_amdgcn_readlane(rpk, v);
                const long long kv = (long long)(((unsigned long long)(unsigned)hv << 32) | lv_);
                if (v == 0 || kv > kw || (kv == kw && pv < pw)) {
                    W = v;
                    kw = kv;
                    pw = pv;
                }
            }
            const bool mine = w == W;
            const int cb = buf;
            buf ^= 1;
            if (pw == PACK_NONE) {
                st = ST_OPTIMAL;
                break;
            }
            if (iters >= max_iter) {
                st = ST_ITER_LIMIT;
                break;
            }
            l = __builtin_amdgcn_readlane(rl, W);
            if (l < 0) {
                st = ST_UNBOUNDED;
                break;
            }
            rmin = __hiloint2double(__builtin_amdgcn_readlane(__double2hiint(rrm), W),
                                    __builtin_amdgcn_readlane(__double2loint(rrm), W));
            pe = __hiloint2double(__builtin_amdgcn_readlane(__double2hiint(rpe), W),
                                  __builtin_amdgcn_readlane(__double2loint(rpe), W));
            BLP_T(t_p2);
            const int e_id = unpack_id(pw), ep = unpack_pos(pw);
            const int lv = mirror_at(bs, l);
            // ---- Step 3: the pivot column's entries this lane needs are
            // read first, so that their LDS round trip overlaps the pivot
            // row's publication below
            double nf[RB], f2[2];
#pragma unroll
            for (int a = 0; a < RB; ++a) nf[a] = -s_col[W][cb][ri + GRW * a];
#pragma unroll
            for (int q = 0; q < 2; ++q) f2[q] = s_col[W][cb][q * 64 + lane];
            const double fO = s_col[W][cb][ROW_OBJ];
            const double y = 1.0 / pe;
            const double ape = fabs(pe);
            const bool pe_ok = ape >= 0x1p-500 && ape <= 0x1p500;
            const int al = __builtin_amdgcn_readfirstlane(l / GRW);
            const bool rown = ri == l % GRW;             // this lane holds row l (at a == al)
            const bool ecol = mine && ci == ep % GCW;    // this lane holds the entering slot (at b == be)
            const int be = __builtin_amdgcn_readfirstlane(ep / GCW);
            // this wave's part of row l goes to LDS (the entering slot takes
            // the leaving variable's unit entry); row l and the entering
            // column are zeroed in the tile: the update below rebuilds them
#pragma unroll
            for (int a = 0; a < RB; ++a)
                if (a == al) {
                    if (rown) {
#pragma unroll
                        for (int b = 0; b < CB; ++b) s_row[w][ci + GCW * b] = (ecol && b == be) ? 1.0 : T[a][b];
                    }
#pragma unroll
                    for (int b = 0; b < CB; ++b) T[a][b] = rown ? 0.0 : T[a][b];
                    __asm__ volatile("; cols row %0" ::"i"(a));
                }
            if (mine) {
#pragma unroll
                for (int b = 0; b < CB; ++b)
                    if (b == be) {
#pragma unroll
                        for (int a = 0; a < RB; ++a) T[a][b] = ecol ? 0.0 : T[a][b];
                        __asm__ volatile("; cols zero %0" ::"i"(b));
                    }
            }
            __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
            __builtin_amdgcn_wave_barrier();
            __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
            // p = x / pe for this lane's slots and its mirror slot (one
            // reciprocal and a Markstein correction per entry; the plain
            // division where a magnitude is extreme, so p is always x / pe)
            double pc[CB], pj;
            {
                bool slow = false, okd;
#pragma unroll
                for (int b = 0; b < CB; ++b) {
                    pc[b] = div_rn_fast(s_row[w][ci + GCW * b], pe, y, pe_ok, okd);
                    slow |= !okd;
                }
                pj = div_rn_fast(s_row[w][lane < CPW ? lane : 0], pe, y, pe_ok, okd);
                slow |= !okd;
                if (slow) {
#pragma unroll
                    for (int b = 0; b < CB; ++b) pc[b] = s_row[w][ci + GCW * b] / pe;
                    pj = s_row[w][lane < CPW ? lane : 0] / pe;
                }
            }
            BLP_T(t_p3);
            // mirrors
            {
                const double pr = mirror_at(bR, l) / pe;
                const bool ent = mine && lane == ep;
                dO = __builtin_fma(-fO, pj, ent ? 0.0 : dO);
                cv = ent ? lv : cv;
#pragma unroll
                for (int q = 0; q < 2; ++q) {
                    const bool piv = lane == l - 64 * q;
                    bR[q] = piv ? pr : __builtin_fma(-f2[q], pr, bR[q]);
                    bs[q] = piv ? e_id : bs[q];
                }
            }
            // the rank-1 update of this wave's slots; row l becomes p
#pragma unroll
            for (int a = 0; a < RB; ++a) {
                const double f = (rown && a == al) ? 1.0 : nf[a];
#pragma unroll
                for (int b = 0; b < CB; ++b) T[a][b] = __builtin_fma(f, pc[b], T[a][b]);
            }
            ++iters;
            degen = rmin == 0.0 ? degen + 1 : 0;
            BLP_T(t_p4);
            BLP_TACC(TM_PRICE, t_p0, t_p1);
            BLP_TACC(TM_PUBCOL, t_p1, t_p2);
            BLP_TACC(TM_RATIO, t_p2, t_p3);
            BLP_TACC(TM_PIVOT, t_p3, t_p4);
        }
        BLP_T(t_x0);

        // ------------------------------------------------------ extraction
        // every structural and logical variable sits in one slot (nonbasic:
        // x = 0, dual from the objective row; each wave writes its slots) or
        // one row (basic: x = rhs, dual 0; wave 0 writes the rows)
        {
            const double z = -mirror_at(bR, ROW_OBJ);
            const int sto = st == ST_OPTIMAL && !isfinite(z) ? ST_NUMERICAL : st;
            const bool nan_out = sto == ST_NUMERICAL;
            const double qnan = __builtin_nan("");
            if (lane < CPW) {
                const int v = cv;
                if (v < n) {
                    P.x[L.col_off + v] = nan_out ? qnan : 0.0;
                } else if (v < n + m) {
                    P.y[L.row_off + (v - n)] = nan_out ? qnan : ((s_flag[v - n] & RF_GE) ? dO : -dO);
                }
            }
            if (w == 0) {
#pragma unroll
                for (int q = 0; q < 2; ++q) {
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
                    P.status[k] = sto;
                    P.iters[k] = iters;
                    P.obj[k] = (sto == ST_OPTIMAL || sto == ST_ITER_LIMIT) ? z
                               : sto == ST_UNBOUNDED                      ? __builtin_inf()
                                                                          : qnan;
                }
            }
        }
        BLP_T(t_x1);
        BLP_TACC(TM_EXTRACT, t_x0, t_x1);
        BLP_TCOUNT(TM_PIVOTS, (unsigned long long)iters);
        BLP_TCOUNT(TM_LPS, 1ull);
    }
    BLP_TFLUSH();
}

}  // namespace blp
