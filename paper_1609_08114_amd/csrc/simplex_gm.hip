// Streaming simplex kernel for tableaux too large for a workgroup's
// registers: one LP per workgroup, the condensed tableau in a per-workgroup
// HBM workspace slot, column-major (element (i, j) at ws[j*ldk + i], ldk =
// m + 2 rounded up to 16 for this LP) so that
// the column operations of Steps 2 and 3 are coalesced (Sec. 4.3).  Each
// pivot streams the whole tableau once (read + write), which is the
// HBM/L2-bound part; Step 1 and Step 2 run on LDS mirrors of the active
// objective row and the rhs column exactly as in the register-tile kernel.
//
// Per pivot: price (LDS) -> load the entering column into LDS -> barrier ->
// ratio test (LDS) -> gather and divide the pivot row into LDS -> barrier ->
// stream the update over all columns (waves take columns, lanes take rows)
// while refreshing the mirrors -> barrier.
//
// On-chip columns: when the launch is given LDS beyond the mirrors
// (P.ws_lds doubles), the first JL column slots of each LP live there instead
// of in the HBM slot (JL = as many columns of this LP's height as fit), so a
// pivot streams only the remaining C - JL columns through HBM; "more data per
// block" in the sense of Sec. 4.5.  The values and the order of every
// operation are the same wherever a column lives.
#include <type_traits>

#include "blp_kernels.hpp"
#include "simplex_common.hpp"
#include "aux_kernels.hpp"

namespace blp {

// Dynamic LDS layout for a launch whose LPs have at most `rows` tableau rows
// (ld, a multiple of 16, at most GM_MAX_LD) and `cols` column slots.
// Largest leading dimension handled (rows incl. objective rows, padded to 16).
constexpr int GM_MAX_LD = 2048;

// a double as the two dwords of a 64-bit buffer access
typedef unsigned int WsPair __attribute__((ext_vector_type(2)));
// byte offset past any slot's end: a buffer load there reads 0, a store is dropped
constexpr unsigned kWsOob = 0x80000000u;

struct GmLds {
    double *d, *p, *b, *f, *sig;
    int *colvar, *basis, *artrow, *rank;
    unsigned char* flag;
    double* T;  // on-chip tableau columns (P.ws_lds doubles)
};
// Bytes of the mirrors; the on-chip columns start at the next 16-byte
// boundary, which lies inside the 64 bytes of slack counted here.
__host__ __device__ inline size_t gm_lds_bytes(int ld, int cols) {
    return (size_t)cols * (8 + 8 + 4) + (size_t)ld * (8 + 8 + 8 + 4 + 4 + 4 + 1) + 64;
}

// QM: 64-row chunks per column held by one lane (ld <= 64 QM).  RM: the
// workspace is row-major instead (element (i, j) at ws[i*ws_cols + j]) with
// the same thread mapping, so the column reads and the update are strided
// across lanes: the non-coalesced variant of Sec. 4.3's comparison, kept for
// the layout measurement; results are identical.
// DEEP (instantiated with QM <= 8): for launches whose bin cannot be empty:
// 32 loads in flight per lane in the update, and on-chip columns in the LDS
// that the host gives beyond the mirrors.
template <int NW, int QM, bool RM, bool DEEP = false>
__global__ void __launch_bounds__(NW * 64) simplex_gm_kernel(KParams P) {
    constexpr int NT = NW * 64;
    extern __shared__ __align__(16) unsigned char smem[];
    const int ld = P.ws_ld, cg_max = P.ws_cols;
    GmLds S;
    S.d = reinterpret_cast<double*>(smem);
    S.p = S.d + cg_max;
    S.b = S.p + cg_max;
    S.f = S.b + ld;
    S.sig = S.f + ld;
    S.colvar = reinterpret_cast<int*>(S.sig + ld);
    S.basis = S.colvar + cg_max;
    S.artrow = S.basis + ld;
    S.rank = S.artrow + ld;
    S.flag = reinterpret_cast<unsigned char*>(S.rank + ld);
    S.T = reinterpret_cast<double*>(((reinterpret_cast<uintptr_t>(S.flag + ld)) + 15) & ~(uintptr_t)15);
    __shared__ int s_k, s_nart, s_bad;

    const int t = threadIdx.x, lane = t & 63, wave = t >> 6;
    BLP_TDECL;
    double* const Tg = P.ws + (int64_t)blockIdx.x * P.ws_slot;

    const int64_t len = work_len(P);
    bool first = true;
    for (;;) {
        if (t == 0) {
            int64_t q;
            if (P.direct)
                q = first ? P.direct_first + (int64_t)blockIdx.x : len;
            else
                q = pop_position(P, len, first);
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
        const LpRef Lin = lp_in(P, L);  // constraint reads
        const int m = L.m, n = L.n;
        if (m > ld - 2 || n + 1 > cg_max) {  // never routed here; no LDS write past the arrays
            write_numerical<NT>(P, L, k, t, ST_INTERNAL);
            __syncthreads();
            continue;
        }
        for (int i = t; i < ld; i += NT) {
            S.flag[i] = 0;
            S.b[i] = 0.0;
        }
        __syncthreads();
        int bad = prep_rows<NT>(P, Lin, t, S.sig, S.b, S.flag);
        __syncthreads();
        if (t < 64) scan_art_rows(m, lane, S.flag, S.artrow, S.rank, &s_nart);
        __syncthreads();
        const int nart = s_nart;
        const int C = n + nart + 1, RHS = C - 1;
        // this LP's tableau: ldk rows (m + 2 rounded up to 16) by C columns
        const int ldk = ((m + 2 + 15) / 16) * 16;
        const int ROW_OBJ = ldk - 1, ROW_W = ldk - 2;
        // workspace index of tableau cell (i, j)
        auto at = [&](int i, int j) -> int64_t { return RM ? (int64_t)i * C + j : (int64_t)j * ldk + i; };
        if (m > ld - 2 || C > cg_max) {
            write_numerical<NT>(P, L, k, t, ST_INTERNAL);
            __syncthreads();
            continue;
        }
        // column slots j < JL are on chip, column-major with an odd stride
        // (the row gathers of Step 3 then spread over the LDS banks)
        const int ldl = ldk + 1;
        const int JL = !DEEP ? 0 : (P.ws_lds / ldl < C ? P.ws_lds / ldl : C);
        auto rd = [&](int i, int j) -> double { return j < JL ? S.T[j * ldl + i] : Tg[at(i, j)]; };
        // this LP's part of the slot as a buffer (ldk x C doubles, either layout)
        const __amdgpu_buffer_rsrc_t wsr =
            __builtin_amdgcn_make_buffer_rsrc(Tg, (short)0, ldk * C * (int)sizeof(double), 0x00020000);
        auto wr = [&](int i, int j, double v) {
            if (j < JL)
                S.T[j * ldl + i] = v;
            else
                Tg[at(i, j)] = v;
        };
        // constraint rows: read A row-major (coalesced), write column-major
        for (int i = wave; i < m; i += NW) {
            const double sg = S.sig[i];
            for (int j = lane; j < n; j += 64) {
                const double a = P.A[Lin.a_off + (int64_t)i * n + j];
                bad |= !isfinite(a);
                wr(i, j, sg * a);
            }
        }
        // the other cells, column by column
        for (int j = wave; j < C; j += NW) {
            const int sur_row = (j >= n && j < RHS) ? S.artrow[j - n] : -1;
            for (int i = lane; i < ldk; i += 64) {
                if (i < m && j < n) continue;  // written above
                double v = 0.0;
                if (i < m) {
                    v = j == RHS ? S.b[i] : (i == sur_row ? -1.0 : 0.0);
                } else if (i == ROW_OBJ) {
                    v = j < n ? P.c[L.col_off + j] : 0.0;
                } else if (i == ROW_W && nart > 0) {
                    double acc = 0.0;
                    if (j < n) {
                        for (int q = 0; q < nart; ++q) {
                            const int ii = S.artrow[q];
                            acc = acc + S.sig[ii] * P.A[Lin.a_off + (int64_t)ii * n + j];
                        }
                    } else if (j < RHS) {
                        acc = -1.0;
                    } else {
                        for (int q = 0; q < nart; ++q) acc = acc + S.b[S.artrow[q]];
                    }
                    v = acc;
                }
                wr(i, j, v);
            }
        }
        if (bad) atomicOr(&s_bad, 1);
        for (int j = t; j < C; j += NT) S.colvar[j] = j < n ? j : (j < RHS ? n + S.artrow[j - n] : ID_NONE);
        for (int i = t; i < m; i += NT) S.basis[i] = (S.flag[i] & RF_ART) ? n + m + i : n + i;
        __syncthreads();
        if (s_bad) {
            write_numerical<NT>(P, L, k, t, ST_NUMERICAL);
            __syncthreads();
            continue;
        }
        int phase = nart > 0 ? 1 : 2;
        auto mirror_row = [&](int row) {
            for (int j = t; j < C; j += NT) S.d[j] = rd(row, j);
        };
        mirror_row(phase == 1 ? ROW_W : ROW_OBJ);
        for (int i = t; i < ldk; i += NT) S.b[i] = rd(i, RHS);
        __syncthreads();
        const double w0 = S.b[ROW_W];
        const int max_iter = P.max_iter > 0 ? P.max_iter : 50 * (m + n);
        const int bland_after = P.bland_after > 0 ? P.bland_after : (m > n ? m : n);
        const int id_lim = n + m;
        int iters = 0, degen = 0, st = -1;

        // ------------------------------------------------------ pivot loop
        BLP_T(t_load1);
        BLP_TACC(TM_LOAD, t_load0, t_load1);
        int mode = phase, drive_r = 0;
        for (;;) {
            BLP_T(t_p0);
            int e_id, e, l = -1;
            double rmin = 1.0;
            if (mode == 3) {
                int r0 = -1;
                for (; drive_r < m; ++drive_r)
                    if (S.basis[drive_r] >= id_lim && !(S.flag[drive_r] & RF_DEAD)) {
                        r0 = drive_r;
                        break;
                    }
                if (r0 < 0) {
                    mode = phase = 2;
                    degen = 0;
                    mirror_row(ROW_OBJ);
                    __syncthreads();
                    continue;
                }
                ++drive_r;
                for (int j = t; j < C; j += NT) S.p[j] = rd(r0, j);
                __syncthreads();
                double bk = -__builtin_inf();
                int bid = ID_NONE, bpos = -1;
                for (int j = lane; j < RHS; j += 64) {
                    const int v = S.colvar[j];
                    if (v < id_lim && fabs(S.p[j]) > P.eps_piv && key_before(0.0, v, bk, bid)) {
                        bk = 0.0;
                        bid = v;
                        bpos = j;
                    }
                }
                wave_argmax(bk, bid, bpos);
                __syncthreads();
                if (bid == ID_NONE) {
                    if (t == 0) S.flag[r0] |= RF_DEAD;
                    __syncthreads();
                    continue;
                }
                l = r0;
                e = bpos;
                e_id = bid;
            } else {
                if (P.pivot_rule == 1 && degen < bland_after)
                    price_rpc(RHS, lane, id_lim, P.eps_price, P.seed, k, iters, S.d, S.colvar, e_id, e);
                else
                    price(RHS, lane, id_lim, P.eps_price, degen >= bland_after, S.d, S.colvar, e_id, e);
                if (e_id == ID_NONE) {
                    if (mode == 2) {
                        st = ST_OPTIMAL;
                        break;
                    }
                    if (S.b[ROW_W] > P.eps_feas * (1.0 + w0)) {
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
            // entering column -> LDS
            BLP_T(t_p1);
            for (int i = t; i < ldk; i += NT) S.f[i] = rd(i, e);
            __syncthreads();
            BLP_T(t_p2);
            if (mode != 3) {
                l = ratio_test(m, lane, P.eps_piv, S.f, S.b, S.basis, S.flag, rmin);
                if (l < 0) {
                    st = mode == 2 ? ST_UNBOUNDED : ST_NUMERICAL;
                    break;
                }
            }
            // Step 3: NewPivotRow = OldPivotRow / PE (the entering slot takes
            // the leaving variable's column, whose pivot-row entry is 1 / PE)
            const double pe = S.f[l];
            for (int j = t; j < C; j += NT) S.p[j] = (j == e ? 1.0 : rd(l, j)) / pe;
            __syncthreads();
            BLP_T(t_p3);
            const int act = phase == 1 ? ROW_W : ROW_OBJ;
            // this lane's rows i = lane + 64 q and their pivot-column entries
            double nf[QM];
#pragma unroll
            for (int q = 0; q < QM; ++q) {
                const int i = lane + 64 * q;
                nf[q] = i < ldk ? -S.f[i] : 0.0;
            }
            // In phase 2 a slot holding an artificial variable never enters
            // again and feeds no output (pricing skips it, duals come from
            // the logical columns), so its column is not updated.  The
            // entering slot's column always is, and its colvar entry is not
            // read here: thread 0 rewrites it below while other waves may
            // still be in these loops.
            const bool skip_art = mode == 2;
            auto updated = [&](int j) { return j == e || j == RHS || !(skip_art && S.colvar[j] >= id_lim); };
            // On-chip columns (a wave takes every NW-th slot).
            // (run while a step's HBM loads are in flight, spread over the
            // wave's HBM steps; the rest after them)
            auto onchip_col = [&](int j) {
                if (!updated(j)) return;
                const bool je = j == e;
                const double pj = S.p[j];
                double* const col = S.T + j * ldl;
#pragma unroll
                for (int q = 0; q < QM; ++q) {
                    const int i = lane + 64 * q;
                    if (i < ldk) {
                        double w = __builtin_fma(nf[q], pj, je ? 0.0 : col[i]);
                        w = i == l ? pj : w;
                        col[i] = w;
                        if (i == act) S.d[j] = w;
                        if (j == RHS) S.b[i] = w;
                    }
                }
            };
            int jl = wave;  // this wave's next on-chip column
            // HBM columns.  A wave streams U columns per step (j0 + u NW),
            // all their loads issued before any is used: with one column per
            // step each wave had QM loads in flight and the update was bound
            // by memory latency, not bandwidth.  Tableaux of 255..510 rows
            // (QM = 8) and the deep instantiation keep 32 loads in flight per
            // lane; otherwise 8 (a launch that finds its bin empty would
            // otherwise hold CUs the register kernels need with its extra
            // VGPRs).  In launches of 8 or more row chunks an LP no taller
            // than half the launch's height runs the loop with half the row
            // chunks and twice the columns per step (the same loads in
            // flight, none of them for rows past ldk).
            // The columns go through a buffer resource over the slot: a dead
            // lane or column gets an offset past its end (the load reads 0,
            // the store is dropped), so loads and stores are issued without
            // branches and the wait before the update counts the loads only.
            constexpr int U = DEEP ? (QM >= 4 ? 32 / QM : 16 / QM) : QM == 8 ? 4 : QM >= 8 ? 1 : 8 / QM;
            auto hbm_update = [&](auto qlc) {
                constexpr int QL = decltype(qlc)::value;
                constexpr int UL = U * QM / QL;
                const int qa = act >> 6;  // the active row's chunk and lane
                const bool lane_act = lane == (act & 63);
                // the wave's on-chip columns spread over its HBM steps
                const int nsteps = C - JL - wave > 0 ? (C - JL - wave + NW * UL - 1) / (NW * UL) : 0;
                const int ncols = JL - wave > 0 ? (JL - wave + NW - 1) / NW : 0;
                const int per = nsteps > 0 ? (ncols + nsteps - 1) / nsteps : 0;
                for (int j0 = JL + wave; j0 < C; j0 += NW * UL) {
                    bool live[UL];
                    double pj[UL], v[UL][QL];
#pragma unroll
                    for (int u = 0; u < UL; ++u) {
                        const int j = j0 + u * NW, jc = j < C ? j : C - 1;
                        const int cv = S.colvar[jc];
                        const double pp = S.p[jc];
                        live[u] = j < C && (j == e || j == RHS || !(skip_art && cv >= id_lim));
                        pj[u] = live[u] ? pp : 0.0;
#pragma unroll
                        for (int q = 0; q < QL; ++q) {
                            const int i = lane + 64 * q;
                            const unsigned o = (live[u] && i < ldk && j != e) ? (unsigned)at(i, j) * 8u : kWsOob;
                            v[u][q] =
                                __builtin_bit_cast(double, __builtin_amdgcn_raw_buffer_load_b64(wsr, (int)o, 0, 0));
                        }
                    }
                    for (int b = 0; b < per && jl < JL; ++b, jl += NW) onchip_col(jl);
                    // straight-line update and stores; the mirrors' entries
                    // are picked out with selects and written afterwards
                    double wa[UL], wr[QL];
#pragma unroll
                    for (int u = 0; u < UL; ++u) {
                        const int j = j0 + u * NW;
                        wa[u] = 0.0;
#pragma unroll
                        for (int q = 0; q < QL; ++q) {
                            const int i = lane + 64 * q;
                            const unsigned o = (live[u] && i < ldk) ? (unsigned)at(i, j) * 8u : kWsOob;
                            double w = __builtin_fma(nf[q], pj[u], v[u][q]);
                            w = i == l ? pj[u] : w;
                            __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(WsPair, w), wsr, (int)o, 0, 0);
                            wa[u] = q == qa ? w : wa[u];
                            if (u == 0) wr[q] = w;
                            else wr[q] = j == RHS ? w : wr[q];
                        }
                    }
                    const int ur = RHS - j0;  // the RHS column's step slot, if it is in this step
                    if (ur >= 0 && ur < NW * UL && ur % NW == 0) {
#pragma unroll
                        for (int q = 0; q < QL; ++q) {
                            const int i = lane + 64 * q;
                            if (i < ldk) S.b[i] = wr[q];
                        }
                    }
                    if (lane_act) {
#pragma unroll
                        for (int u = 0; u < UL; ++u)
                            if (live[u]) S.d[j0 + u * NW] = wa[u];
                    }
                }
            };
            if constexpr (QM >= 8) {
                if (ldk <= 32 * QM)
                    hbm_update(std::integral_constant<int, QM / 2>{});
                else
                    hbm_update(std::integral_constant<int, QM>{});
            } else {
                hbm_update(std::integral_constant<int, QM>{});
            }
            for (; jl < JL; jl += NW) onchip_col(jl);
            if (t == 0) {
                S.colvar[e] = S.basis[l];
                S.basis[l] = e_id;
            }
            __syncthreads();
            BLP_T(t_p4);
            BLP_TACC(TM_PRICE, t_p0, t_p1);
            BLP_TACC(TM_PUBCOL, t_p1, t_p2);
            BLP_TACC(TM_RATIO, t_p2, t_p3);
            BLP_TACC(TM_PIVOT, t_p3, t_p4);
            ++iters;
            if (mode != 3) degen = rmin == 0.0 ? degen + 1 : 0;
        }

        // ------------------------------------------------------ extraction
        BLP_T(t_x0);
        mirror_row(ROW_OBJ);
        __syncthreads();
        write_outputs<NT>(P, L, k, t, st, iters, ROW_OBJ, RHS, S.d, S.b, S.colvar, S.basis, S.flag, S.p, S.f);
        __syncthreads();
        BLP_T(t_x1);
        BLP_TACC(TM_EXTRACT, t_x0, t_x1);
        BLP_TCOUNT(TM_PIVOTS, (unsigned long long)iters);
        BLP_TCOUNT(TM_LPS, 1ull);
    }
    BLP_TFLUSH();
}

template <int QM, bool DEEP = false>
static hipError_t launch_gm_q(const KParams& P, int grid, size_t lds_bytes, hipStream_t s) {
    if (P.layout == 1)
        hipLaunchKernelGGL((simplex_gm_kernel<8, QM, true, DEEP>), dim3(grid), dim3(512), lds_bytes, s, P);
    else
        hipLaunchKernelGGL((simplex_gm_kernel<8, QM, false, DEEP>), dim3(grid), dim3(512), lds_bytes, s, P);
    return hipGetLastError();
}
template <int QM>
static hipError_t launch_gm_d(const KParams& P, int grid, size_t lds_bytes, hipStream_t s, bool deep) {
    return deep ? launch_gm_q<QM, true>(P, grid, lds_bytes, s) : launch_gm_q<QM>(P, grid, lds_bytes, s);
}
static int gm_chunks(int ld) { return ld <= 64 ? 1 : ld <= 128 ? 2 : ld <= 256 ? 4 : ld <= 512 ? 8 : ld <= 1024 ? 16 : 32; }
hipError_t launch_gm(const KParams& P, int grid, size_t lds_bytes, hipStream_t s, bool deep) {
    switch (gm_chunks(P.ws_ld)) {
        case 1: return launch_gm_d<1>(P, grid, lds_bytes, s, deep);
        case 2: return launch_gm_d<2>(P, grid, lds_bytes, s, deep);
        case 4: return launch_gm_d<4>(P, grid, lds_bytes, s, deep);
        case 8: return launch_gm_d<8>(P, grid, lds_bytes, s, deep);
        case 16: return launch_gm_q<16>(P, grid, lds_bytes, s);
        default: return launch_gm_q<32>(P, grid, lds_bytes, s);
    }
}
// the column-major instantiation (occupancy and attributes are the same for
// both layouts)
template <int QM>
static const void* gm_ptr(bool deep) {
    return deep ? reinterpret_cast<const void*>(&simplex_gm_kernel<8, QM, false, true>)
                : reinterpret_cast<const void*>(&simplex_gm_kernel<8, QM, false>);
}
const void* gm_kernel_ptr(int ld, bool deep) {
    switch (gm_chunks(ld)) {
        case 1: return gm_ptr<1>(deep);
        case 2: return gm_ptr<2>(deep);
        case 4: return gm_ptr<4>(deep);
        case 8: return gm_ptr<8>(deep);
        case 16: return reinterpret_cast<const void*>(&simplex_gm_kernel<8, 16, false>);
        default: return reinterpret_cast<const void*>(&simplex_gm_kernel<8, 32, false>);
    }
}
bool gm_has_deep(int ld) { return gm_chunks(ld) <= 8; }
template <int QM, bool DEEP>
static hipError_t gm_allow(int bytes) {
    hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void*>(&simplex_gm_kernel<8, QM, false, DEEP>),
                                       hipFuncAttributeMaxDynamicSharedMemorySize, bytes);
    if (e != hipSuccess) return e;
    return hipFuncSetAttribute(reinterpret_cast<const void*>(&simplex_gm_kernel<8, QM, true, DEEP>),
                               hipFuncAttributeMaxDynamicSharedMemorySize, bytes);
}
hipError_t gm_allow_lds(int ld, bool deep, int bytes) {
    switch (gm_chunks(ld)) {
        case 1: return deep ? gm_allow<1, true>(bytes) : gm_allow<1, false>(bytes);
        case 2: return deep ? gm_allow<2, true>(bytes) : gm_allow<2, false>(bytes);
        case 4: return deep ? gm_allow<4, true>(bytes) : gm_allow<4, false>(bytes);
        case 8: return deep ? gm_allow<8, true>(bytes) : gm_allow<8, false>(bytes);
        case 16: return gm_allow<16, false>(bytes);
        default: return gm_allow<32, false>(bytes);
    }
}
int gm_threads() { return 512; }

}  // namespace blp

namespace blp {
size_t gm_lds_bytes_host(int ld, int cols) { return gm_lds_bytes(ld, cols); }
}  // namespace blp
