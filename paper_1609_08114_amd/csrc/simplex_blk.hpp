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
        if (j < nslots && v < id_lim && d[q] > eps_price) {
            const double key = bland ? 0.0 : d[q];
            if (key_before(key, v, bk, bid)) {
                bk = key;
                bid = v;
                bpos = j;
            }
        }
    }
    wave_argmax(bk, bid, bpos);
    e_id = bid;
    e_pos = bpos;
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
                e_id = __shfl(cv[q], src);
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
        if (i < m && !((dead >> q) & 1u) && a > eps_piv) {
            const double bi = b[q];
            const double ratio = bi <= 0.0 ? 0.0 : bi / a;
            if (key_before(-ratio, bs[q], bk, bid)) {
                bk = -ratio;
                bid = bs[q];
                bpos = i;
            }
        }
    }
    wave_argmax(bk, bid, bpos);
    rmin = -bk;
    leave_id = bid;
    return bid == ID_NONE ? -1 : bpos;
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

template <int NW, int GC, int RB, int CB, int WPE>
__global__ void __launch_bounds__(NW * 64) __attribute__((amdgpu_waves_per_eu(WPE, WPE)))
simplex_blk_kernel(KParams P) {
    constexpr int NT = NW * 64;
    constexpr int GR = NT / GC;  // row groups
    constexpr int RP = GR * RB;  // tableau rows
    constexpr int CP = GC * CB;  // column slots
    constexpr int ROW_OBJ = RP - 1, ROW_W = RP - 2, COL_RHS = CP - 1;
    constexpr int RS = (RP + 63) / 64, CS = (CP + 63) / 64;
    static_assert(GR * GC == NT && 64 % GC == 0 && RP >= 4 && CP >= 2 && RS <= 32, "bad block tile");

    __shared__ double s_f[2][RP], s_p[2][CP];
    __shared__ double s_sig[RP], s_b[RP], s_c[CP], s_w[CP];
    __shared__ int s_colvar[CP], s_basis[RP], s_artrow[RP], s_rank[RP];
    __shared__ unsigned char s_flag[RP];
    __shared__ int s_k, s_nart, s_bad;

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
    for (;;) {
        if (t == 0) {
            int64_t q;
            if (P.direct)
                q = first ? P.direct_first + (int64_t)blockIdx.x : len;
            else
                q = atomicAdd(P.bin_head + P.bin, 1);
            s_k = q < len ? (int)work_item(P, q) : -1;
            s_bad = 0;
        }
        first = false;
        __syncthreads();
        const int k = s_k;
        if (k < 0) break;
        BLP_T(t_load0);

        // ------------------------------------------------------------ load
        const LpRef L = lp_ref(P, k);
        const int m = L.m, n = L.n;
        if (m > RP - 2 || n + 1 > CP) {  // never routed here; no LDS write past the arrays
            write_numerical<NT>(P, L, k, t, ST_INTERNAL);
            __syncthreads();
            continue;
        }
        int bad = prep_rows<NT>(P, L, t, s_sig, s_b, s_flag);
        for (int j = t; j < n; j += NT) s_c[j] = P.c[L.col_off + j];
        // A straight into the tile (scaled below, once the row signs are known)
        {
            const double* A = P.A + L.a_off;
            const bool any = m > 0 && n > 0;
#pragma unroll
            for (int r = 0; r < RB; ++r) {
                const int i = i0 + r;
#pragma unroll
                for (int c = 0; c < CB; ++c) {
                    const int j = c * GC + tcb;
                    const bool in = i < m && j < n;
                    const double a = any ? A[in ? (int64_t)i * n + j : 0] : 0.0;
                    T[r][c] = in ? a : 0.0;
                }
            }
        }
        __syncthreads();
        if (t < 64) scan_art_rows(m, lane, s_flag, s_artrow, s_rank, &s_nart);
        __syncthreads();
        const int nart = s_nart;
        if (n + nart + 1 > CP) {
            write_numerical<NT>(P, L, k, t, ST_INTERNAL);
            __syncthreads();
            continue;
        }
        // Phase-1 row: for each column, the artificial rows summed in row
        // order (one sequential sum per column, columns spread over threads).
        if (nart > 0) {
            for (int j = t; j < CP; j += NT) {
                double acc = 0.0;
                if (j < n) {
                    for (int q = 0; q < nart; ++q) {
                        const int ii = s_artrow[q];
                        acc = acc + s_sig[ii] * P.A[L.a_off + (int64_t)ii * n + j];
                    }
                } else if (j < n + nart) {
                    acc = -1.0;
                } else if (j == COL_RHS) {
                    for (int q = 0; q < nart; ++q) acc = acc + s_b[s_artrow[q]];
                }
                s_w[j] = acc;
            }
            __syncthreads();
        }
        // finish the tile: signs, surplus columns, rhs, objective rows
#pragma unroll
        for (int r = 0; r < RB; ++r) {
            const int i = i0 + r;
            const double sg = s_sig[i < m ? i : 0];
#pragma unroll
            for (int c = 0; c < CB; ++c) {
                const int j = c * GC + tcb;
                double v = 0.0;
                if (i < m) {
                    if (j < n) {
                        bad |= !isfinite(T[r][c]);
                        v = sg * T[r][c];
                    } else if (j < n + nart) {
                        v = s_artrow[j - n] == i ? -1.0 : 0.0;
                    } else if (j == COL_RHS) {
                        v = s_b[i];
                    }
                } else if (i == ROW_OBJ) {
                    v = j < n ? s_c[j] : 0.0;
                } else if (i == ROW_W && nart > 0) {
                    v = s_w[j];
                }
                T[r][c] = v;
            }
        }
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
        __syncthreads();
        if (s_bad) {
            write_numerical<NT>(P, L, k, t, ST_NUMERICAL);
            __syncthreads();
            continue;
        }
        const double w0 = mirror_at(bR, ROW_W);
        const int max_iter = P.max_iter > 0 ? P.max_iter : 50 * (m + n);
        const int bland_after = P.bland_after > 0 ? P.bland_after : (m > n ? m : n);
        const int id_lim = n + m;
        int iters = 0, degen = 0, st = -1;
        unsigned dead = 0;  // bit q: row q*64 + lane is redundant

        // ------------------------------------------------------ pivot loop
        // mode 1 = phase 1, 2 = phase 2, 3 = driving the remaining basic
        // artificials out after a feasible phase 1.
        int mode = nart > 0 ? 1 : 2, drive_r = 0, buf = 0;
        BLP_T(t_load1);
        BLP_TACC(TM_LOAD, t_load0, t_load1);
        for (;;) {
            int e_id, e, l = -1, lv = ID_NONE;
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
                    continue;
                }
                drive_r = r0 + 1;
                // row r0 into s_p[buf]; the lowest-id non-artificial column
                // with a usable entry enters
                __syncthreads();
                if (trb == r0 / RB) {
                    const int rr = r0 % RB;
#pragma unroll
                    for (int r = 0; r < RB; ++r)
                        if (r == rr) {
#pragma unroll
                            for (int c = 0; c < CB; ++c) s_p[buf][c * GC + tcb] = T[r][c];
                        }
                }
                __syncthreads();
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
                __syncthreads();
                if (bid == ID_NONE) {  // redundant row
                    if (r0 % 64 == lane) dead |= 1u << (r0 / 64);
                    continue;
                }
                l = r0;
                e = bpos;
                e_id = bid;
                lv = mirror_at(bs, r0);
            } else {
                double da[CS];  // the active objective row
#pragma unroll
                for (int q = 0; q < CS; ++q) da[q] = mode == 1 ? dW[q] : dO[q];
                if (P.pivot_rule == 1 && degen < bland_after)
                    price_rpc_regs(COL_RHS, lane, id_lim, P.eps_price, P.seed, k, iters, da, cv, e_id, e);
                else
                    price_regs(COL_RHS, lane, id_lim, P.eps_price, degen >= bland_after, da, cv, e_id, e);
                if (e_id == ID_NONE) {
                    if (mode == 2) {
                        st = ST_OPTIMAL;
                        break;
                    }
                    if (mirror_at(bR, ROW_W) > P.eps_feas * (1.0 + w0)) {
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
            }
            BLP_T(t_p1);
            // publish the entering column (f) and clear its slot; the slot
            // becomes the leaving variable's column
            {
                const int ce = __builtin_amdgcn_readfirstlane(e / GC), te = e % GC;
                if (tcb == te) {
#pragma unroll
                    for (int c = 0; c < CB; ++c)
                        if (c == ce) {
#pragma unroll
                            for (int r = 0; r < RB; ++r) {
                                s_f[buf][i0 + r] = T[r][c];
                                T[r][c] = 0.0;
                            }
                        }
                }
            }
            __syncthreads();
            BLP_T(t_p2);
            double fr[RS];
#pragma unroll
            for (int q = 0; q < RS; ++q) {
                const int i = q * 64 + lane;
                fr[q] = i < RP ? s_f[buf][i] : 0.0;
            }
            if (mode != 3) {
                l = ratio_regs(m, lane, P.eps_piv, fr, bR, bs, dead, rmin, lv);
                if (l < 0) {
                    st = mode == 2 ? ST_UNBOUNDED : ST_NUMERICAL;
                    break;
                }
            }
            const double pe = s_f[buf][l];
            // Step 3's new pivot row, divided by the owners of row l
            if (trb == l / RB) {
                const int rl = __builtin_amdgcn_readfirstlane(l % RB);
#pragma unroll
                for (int r = 0; r < RB; ++r)
                    if (r == rl) {
#pragma unroll
                        for (int c = 0; c < CB; ++c) {
                            const int j = c * GC + tcb;
                            const double p = (j == e ? 1.0 : T[r][c]) / pe;
                            s_p[buf][j] = p;
                            T[r][c] = p;
                        }
                    }
            }
            __syncthreads();
            BLP_T(t_p3);
            // rank-1 update; the pivot row keeps p (fma(+0, p, p) = p)
            {
                double nf[RB], pc[CB];
#pragma unroll
                for (int r = 0; r < RB; ++r) nf[r] = i0 + r == l ? 0.0 : -s_f[buf][i0 + r];
#pragma unroll
                for (int c = 0; c < CB; ++c) pc[c] = s_p[buf][c * GC + tcb];
#pragma unroll
                for (int r = 0; r < RB; ++r)
#pragma unroll
                    for (int c = 0; c < CB; ++c) T[r][c] = __builtin_fma(nf[r], pc[c], T[r][c]);
            }
            // the same update on the mirrors
            {
                const double pr = s_p[buf][COL_RHS];
                const double fO = s_f[buf][ROW_OBJ], fW = s_f[buf][ROW_W];
#pragma unroll
                for (int q = 0; q < CS; ++q) {
                    const int j = q * 64 + lane;
                    if (j < CP) {
                        const double pj = s_p[buf][j];
                        if (j == e) {
                            dO[q] = 0.0;
                            dW[q] = 0.0;
                            cv[q] = lv;
                        }
                        dO[q] = __builtin_fma(-fO, pj, dO[q]);
                        dW[q] = __builtin_fma(-fW, pj, dW[q]);
                    }
                }
#pragma unroll
                for (int q = 0; q < RS; ++q) {
                    const int i = q * 64 + lane;
                    if (i == l) {
                        bR[q] = pr;
                        bs[q] = e_id;
                    } else {
                        bR[q] = __builtin_fma(-fr[q], pr, bR[q]);
                    }
                }
            }
            BLP_T(t_p4);
            BLP_TACC(TM_PRICE, t_p0, t_p1);
            BLP_TACC(TM_PUBCOL, t_p1, t_p2);
            BLP_TACC(TM_RATIO, t_p2, t_p3);
            BLP_TACC(TM_PIVOT, t_p3, t_p4);
            ++iters;
            if (mode != 3) degen = rmin == 0.0 ? degen + 1 : 0;
            buf ^= 1;
        }

        // ------------------------------------------------------ extraction
        BLP_T(t_x0);
        __syncthreads();
        if (t < 64) {
#pragma unroll
            for (int q = 0; q < CS; ++q) {
                const int j = q * 64 + lane;
                if (j < CP) {
                    s_p[1][j] = dO[q];
                    s_colvar[j] = cv[q];
                }
            }
#pragma unroll
            for (int q = 0; q < RS; ++q) {
                const int i = q * 64 + lane;
                if (i < RP) s_f[1][i] = bR[q];
                if (i < m) {
                    s_basis[i] = bs[q];
                    if ((dead >> q) & 1u) s_flag[i] |= RF_DEAD;
                }
            }
        }
        __syncthreads();
        write_outputs<NT>(P, L, k, t, st, iters, ROW_OBJ, COL_RHS, s_p[1], s_f[1], s_colvar, s_basis, s_flag, s_p[0],
                          s_f[0]);
        __syncthreads();
        BLP_T(t_x1);
        BLP_TACC(TM_EXTRACT, t_x0, t_x1);
        BLP_TCOUNT(TM_PIVOTS, (unsigned long long)iters);
        BLP_TCOUNT(TM_LPS, 1ull);
    }
    BLP_TFLUSH();
}

}  // namespace blp
