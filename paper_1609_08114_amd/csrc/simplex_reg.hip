// Register-tile simplex kernel: one LP per workgroup, the whole condensed
// tableau held in VGPRs, persistent over a size-binned work list.
//
// The paper runs one CUDA block per LP (Sec. 4.1) with the tableau in global
// memory, column-major for coalescing (Sec. 4.3).  On gfx950 a workgroup's
// register file (up to 512 KiB per CU) is the largest and fastest store for
// a tableau of up to a few ten thousand entries, so here it lives in
// registers.  Thread t owns tableau row tr = t / TC and the contiguous
// column block [tc*CT, tc*CT + CT) with tc = t % TC.  The rank-1 update of
// Step 3 (Sec. 4.3) is CT register FMAs per thread per pivot; the pivot
// column f (one value per thread) and the pivot row p (a block per thread,
// read as LDS broadcasts) come through LDS.  Step 1 and Step 2 run on LDS
// mirrors of the active objective row and of the rhs column, reduced with
// wavefront DPP/shuffle arg-max by every wave redundantly (no extra barrier
// to broadcast the result).
//
// A thread's CT columns are kept as vectors of at most 16 doubles, so the
// entering column (a wave-uniform slot) is read and cleared with indexed
// register moves instead of scratch memory; rows never need a dynamic
// register index because each thread holds exactly one row.
//
// Per pivot: price -> owners of the entering column publish f -> barrier ->
// ratio test -> owners of the pivot row publish it -> barrier -> divide by
// the pivot element (Step 3's NewPivotRow) -> barrier -> register update and
// mirrors -> barrier.
#include "aux_kernels.hpp"
#include "blp_kernels.hpp"
#include "simplex_blk.hpp"
#include "simplex_common.hpp"
#include "simplex_cols.hpp"
#include "variants.hpp"

namespace blp {

// Chunk width: a power of two (so indexed register moves apply), at most 16
// doubles (the widest register tuple); CT must be a multiple of it.
template <int CT>
struct TileShape {
    static constexpr int CK = CT % 16 == 0 ? 16 : CT % 8 == 0 ? 8 : CT % 4 == 0 ? 4 : CT % 2 == 0 ? 2 : 1;
    static constexpr int NCH = CT / CK;
    static_assert(CK >= 8 || CT <= 8, "CT must be a multiple of 8 beyond 8 columns per thread");
};

template <int NW, int TC, int CT, int WPE>
__global__ void __launch_bounds__(NW * 64) __attribute__((amdgpu_waves_per_eu(WPE, WPE)))
simplex_reg_kernel(KParams P) {
    constexpr int NT = NW * 64;
    constexpr int RP = NT / TC;  // tableau rows (one per thread row)
    constexpr int CP = TC * CT;  // tableau column slots
    constexpr int ROW_OBJ = RP - 1, ROW_W = RP - 2, COL_RHS = CP - 1;
    constexpr int NCH = TileShape<CT>::NCH, CK = TileShape<CT>::CK;
    static_assert(RP * TC == NT && RP >= 4 && CP >= 2, "bad tile");
    typedef double chunk __attribute__((ext_vector_type(CK)));

    __shared__ double s_d[CP], s_p[CP];
    __shared__ double s_b[RP], s_f[RP], s_sig[RP];
    __shared__ int s_colvar[CP], s_basis[RP], s_artrow[RP], s_rank[RP];
    __shared__ unsigned char s_flag[RP];
    __shared__ int s_k, s_nart, s_bad;
    // Staging area for building the initial tableau, SR rows at a time
    // (row-major, CP columns), filled with coalesced loads.
    constexpr int SR = RP < 32 ? RP : 32;
    __shared__ double s_T[SR * CP];

    const int t = threadIdx.x;
    const int lane = t & 63;
    const int tr = t / TC, tc = t % TC;
    const int j0 = tc * CT;  // first column slot of this thread

    chunk T[NCH];
#define TV(c) T[(c) / CK][(c) % CK]

    BLP_TDECL;
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
        if (m > RP - 2 || n + 1 > CP) {  // never routed here; no LDS write past the arrays
            write_numerical<NT>(P, L, k, t, ST_INTERNAL);
            __syncthreads();
            continue;
        }
        for (int i = t; i < RP; i += NT) {
            s_flag[i] = 0;
            s_b[i] = 0.0;
        }
        __syncthreads();
        int bad = prep_rows<NT>(P, Lin, t, s_sig, s_b, s_flag);
        for (int j = t; j < n; j += NT) s_d[j] = P.c[L.col_off + j];  // objective row source
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
                        acc = acc + s_sig[ii] * P.A[Lin.a_off + (int64_t)ii * n + j];
                    }
                } else if (j < n + nart) {
                    acc = -1.0;
                } else if (j == COL_RHS) {
                    for (int q = 0; q < nart; ++q) acc = acc + s_b[s_artrow[q]];
                }
                s_p[j] = acc;
            }
        }
        // Initial tableau, SR rows at a time: built element-wise in LDS with
        // coalesced loads, then each thread whose row is in the chunk copies
        // its column block (a select keeps the tile out of divergent branches).
        for (int r0 = 0; r0 < RP; r0 += SR) {
            __syncthreads();
            // all of this thread's loads of the chunk are issued before any use
            constexpr int EPT = (SR * CP + NT - 1) / NT;
            double av[EPT];
#pragma unroll
            for (int q = 0; q < EPT; ++q) {
                const int e = t + q * NT;
                const int i = r0 + e / CP, j = e % CP;
                const bool ld = e < SR * CP && i < m && j < n;
                av[q] = ld ? P.A[Lin.a_off + (int64_t)i * n + j] : 0.0;
            }
#pragma unroll
            for (int q = 0; q < EPT; ++q) {
                const int e = t + q * NT;
                if (e >= SR * CP) break;
                const int i = r0 + e / CP, j = e % CP;
                double v = 0.0;
                if (i < m) {
                    if (j < n) {
                        bad |= !isfinite(av[q]);
                        v = s_sig[i] * av[q];
                    } else if (j < n + nart) {
                        v = s_artrow[j - n] == i ? -1.0 : 0.0;
                    } else if (j == COL_RHS) {
                        v = s_b[i];
                    }
                } else if (i == ROW_OBJ) {
                    v = j < n ? s_d[j] : 0.0;
                } else if (i == ROW_W && nart > 0) {
                    v = s_p[j];
                }
                s_T[e] = v;
            }
            __syncthreads();
            const bool mine = tr >= r0 && tr < r0 + SR;
            const double* src = s_T + (mine ? tr - r0 : 0) * CP + j0;
#pragma unroll
            for (int c = 0; c < CT; ++c) {
                const double v = src[c];
                TV(c) = mine ? v : TV(c);
            }
        }
        if (bad) atomicOr(&s_bad, 1);
        for (int j = t; j < CP; j += NT)
            s_colvar[j] = j < n ? j : (j < n + nart && j < COL_RHS ? n + s_artrow[j - n] : ID_NONE);
        for (int i = t; i < m; i += NT) s_basis[i] = (s_flag[i] & RF_ART) ? n + m + i : n + i;
        __syncthreads();
        if (s_bad) {
            write_numerical<NT>(P, L, k, t, ST_NUMERICAL);
            __syncthreads();
            continue;
        }
        int phase = nart > 0 ? 1 : 2;
        // mirrors: active objective row -> s_d, rhs column -> s_b
        if (tr == (phase == 1 ? ROW_W : ROW_OBJ)) {
#pragma unroll
            for (int c = 0; c < CT; ++c) s_d[j0 + c] = TV(c);
        }
        if (tc == TC - 1) s_b[tr] = TV(CT - 1);
        __syncthreads();
        const double w0 = s_b[ROW_W];
        const int max_iter = P.max_iter > 0 ? P.max_iter : 50 * (m + n);
        const int bland_after = P.bland_after > 0 ? P.bland_after : (m > n ? m : n);
        const int id_lim = n + m;
        int iters = 0, degen = 0, st = -1;

        // Publish column slot e into s_f (one value per thread row).
        auto publish_col = [&](int e) __attribute__((always_inline)) {
            const int te = e / CT;
            const int ce = __builtin_amdgcn_readfirstlane(e - te * CT);
            double v = 0.0;
#pragma unroll
            for (int h = 0; h < NCH; ++h) {
                const int idx = ce - h * CK;
                const bool in = (unsigned)idx < (unsigned)CK;
                const double x = T[h][in ? idx : 0];
                v = in ? x : v;
            }
            if (tc == te) s_f[tr] = v;
            __syncthreads();
        };
        // Step 3 on (l, e); s_f holds the pivot column.
        auto pivot = [&](int l, int e, int e_id, double pe) __attribute__((always_inline)) {
            const int te = e / CT;
            const int ce = __builtin_amdgcn_readfirstlane(e - te * CT);
            if (tr == l) {
#pragma unroll
                for (int c = 0; c < CT; ++c) s_p[j0 + c] = TV(c);
            }
            __syncthreads();
            for (int j = t; j < CP; j += NT) s_p[j] = (j == e ? 1.0 : s_p[j]) / pe;
            __syncthreads();
            // the entering slot becomes the leaving variable's column
            {
                // executed by every thread (uniform index), so the tile is
                // never merged across a divergent branch
                const bool own = tc == te;
#pragma unroll
                for (int h = 0; h < NCH; ++h) {
                    const int idx = ce - h * CK;
                    const bool in = (unsigned)idx < (unsigned)CK;
                    const int ix = in ? idx : 0;
                    const double cur = T[h][ix];
                    T[h][ix] = in && own ? 0.0 : cur;
                }
            }
            const double nf = -s_f[tr];
#pragma unroll
            for (int c = 0; c < CT; ++c) {
                TV(c) = __builtin_fma(nf, s_p[j0 + c], TV(c));
                if (c % 16 == 15) __builtin_amdgcn_sched_barrier(0);
            }
            if (tr == l) {
#pragma unroll
                for (int c = 0; c < CT; ++c) TV(c) = s_p[j0 + c];
            }
            if (tr == (phase == 1 ? ROW_W : ROW_OBJ)) {
#pragma unroll
                for (int c = 0; c < CT; ++c) s_d[j0 + c] = TV(c);
            }
            if (tc == TC - 1) s_b[tr] = TV(CT - 1);
            if (t == 0) {
                s_colvar[e] = s_basis[l];
                s_basis[l] = e_id;
            }
            __syncthreads();
        };

        // ------------------------------------------------------ pivot loop
        // One loop, one pivot site: mode 1 = phase 1, 2 = phase 2, 3 = driving
        // the remaining basic artificials out after a feasible phase 1.
        int mode = phase, drive_r = 0;
        BLP_T(t_load1);
        BLP_TACC(TM_LOAD, t_load0, t_load1);
        for (;;) {
            int e_id, e, l = -1;
            double rmin = 1.0;
            BLP_T(t_p0);
            if (mode == 3) {
                int r0 = -1;
                for (; drive_r < m; ++drive_r)
                    if (s_basis[drive_r] >= id_lim && !(s_flag[drive_r] & RF_DEAD)) {
                        r0 = drive_r;
                        break;
                    }
                if (r0 < 0) {
                    mode = phase = 2;
                    degen = 0;
                    if (tr == ROW_OBJ) {
#pragma unroll
                        for (int c = 0; c < CT; ++c) s_d[j0 + c] = TV(c);
                    }
                    __syncthreads();
                    continue;
                }
                ++drive_r;
                // lowest-id non-artificial column with a usable entry in row r0
                if (tr == r0) {
#pragma unroll
                    for (int c = 0; c < CT; ++c) s_p[j0 + c] = TV(c);
                }
                __syncthreads();
                double bk = -__builtin_inf();
                int bid = ID_NONE, bpos = -1;
                for (int j = lane; j < COL_RHS; j += 64) {
                    const int v = s_colvar[j];
                    if (v < id_lim && fabs(s_p[j]) > P.eps_piv && key_before(0.0, v, bk, bid)) {
                        bk = 0.0;
                        bid = v;
                        bpos = j;
                    }
                }
                wave_argmax(bk, bid, bpos);
                __syncthreads();
                if (bid == ID_NONE) {  // redundant row
                    if (t == 0) s_flag[r0] |= RF_DEAD;
                    __syncthreads();
                    continue;
                }
                l = r0;
                e = bpos;
                e_id = bid;
            } else {
                if (P.pivot_rule == 1 && degen < bland_after)
                    price_rpc(COL_RHS, lane, id_lim, P.eps_price, P.seed, k, iters, s_d, s_colvar, e_id, e);
                else
                    price(COL_RHS, lane, id_lim, P.eps_price, degen >= bland_after, s_d, s_colvar, e_id, e);
                if (e_id == ID_NONE) {
                    if (mode == 2) {
                        st = ST_OPTIMAL;
                        break;
                    }
                    if (s_b[ROW_W] > P.eps_feas * (1.0 + w0)) {
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
            publish_col(e);
            BLP_T(t_p2);
            if (mode != 3) {
                l = ratio_test(m, lane, P.eps_piv, s_f, s_b, s_basis, s_flag, rmin);
                if (l < 0) {
                    st = mode == 2 ? ST_UNBOUNDED : ST_NUMERICAL;
                    break;
                }
            }
            BLP_T(t_p3);
            pivot(l, e, e_id, s_f[l]);
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
        if (tr == ROW_OBJ) {
#pragma unroll
            for (int c = 0; c < CT; ++c) s_d[j0 + c] = TV(c);
        }
        __syncthreads();
        write_outputs<NT>(P, L, k, t, st, iters, ROW_OBJ, COL_RHS, s_d, s_b, s_colvar, s_basis, s_flag, s_p, s_f);
        __syncthreads();
        BLP_T(t_x1);
        BLP_TACC(TM_EXTRACT, t_x0, t_x1);
        BLP_TCOUNT(TM_PIVOTS, (unsigned long long)iters);
        BLP_TCOUNT(TM_LPS, 1ull);
    }
    BLP_TFLUSH();
#undef TV
}

// ---------------------------------------------------------------------------
// Instantiations and launchers.
// ---------------------------------------------------------------------------
template <int NW, int TC, int CT, int WPE>
static hipError_t launch_reg(const KParams& P, int grid, hipStream_t s) {
    hipLaunchKernelGGL((simplex_reg_kernel<NW, TC, CT, WPE>), dim3(grid), dim3(NW * 64), 0, s, P);
    return hipGetLastError();
}
template <int NW, int TC, int CT, int WPE>
static const void* kernel_ptr() {
    return reinterpret_cast<const void*>(&simplex_reg_kernel<NW, TC, CT, WPE>);
}

template <int NW, int GC, int RB, int CB, int WPE>
static hipError_t launch_blk(const KParams& P, int grid, hipStream_t s) {
    hipLaunchKernelGGL((simplex_blk_kernel<NW, GC, RB, CB, WPE>), dim3(grid), dim3(NW * 64), 0, s, P);
    return hipGetLastError();
}
template <int NW, int GC, int RB, int CB, int WPE>
static const void* kernel_ptr_blk() {
    return reinterpret_cast<const void*>(&simplex_blk_kernel<NW, GC, RB, CB, WPE>);
}

// ROWS x COLS: the shape the variant claims (ROWS - 2 constraint rows and
// COLS - 1 column slots), which its tile must hold
template <int NW, int GCW, int RB, int CB, int WPE, int ROWS, int COLS>
static hipError_t launch_cols(const KParams& P, int grid, hipStream_t s) {
    static_assert(ROWS - 2 <= 64 / GCW * RB && COLS - 1 <= NW * GCW * CB, "column-split shape");
    hipLaunchKernelGGL((simplex_cols_kernel<NW, GCW, RB, CB, WPE>), dim3(grid), dim3(NW * 64), 0, s, P);
    return hipGetLastError();
}
template <int NW, int GCW, int RB, int CB, int WPE>
static const void* kernel_ptr_cols() {
    return reinterpret_cast<const void*>(&simplex_cols_kernel<NW, GCW, RB, CB, WPE>);
}

// Pivot trace of the 112 x 112 block tile (the kernel of the 100 x 100
// workload): tr 1 records each pivot's (row, slot), tr 2 replays a recorded
// sequence with Steps 1 and 2 replaced by reading it (the rank-1 updates, the
// column and row exchanges and the division stay as they are).
hipError_t launch_blk_trace(const KParams& P, int grid, hipStream_t s, int tr) {
    if (tr == 1)
        hipLaunchKernelGGL((simplex_blk_kernel<4, 16, 7, 7, 2, false, 1>), dim3(grid), dim3(256), 0, s, P);
    else
        hipLaunchKernelGGL((simplex_blk_kernel<4, 16, 7, 7, 2, false, 2>), dim3(grid), dim3(256), 0, s, P);
    return hipGetLastError();
}
const void* blk_trace_kernel_ptr(int tr) {
    return tr == 1 ? reinterpret_cast<const void*>(&simplex_blk_kernel<4, 16, 7, 7, 2, false, 1>)
                   : reinterpret_cast<const void*>(&simplex_blk_kernel<4, 16, 7, 7, 2, false, 2>);
}
void blk_trace_shape(int* rows, int* cols) {
    *rows = 112;
    *cols = 112;
}

// Shared-constraint mode (one A, b; many objectives): the block kernel with a
// 112 x 112 tile.
constexpr int kSharedRows = 112, kSharedCols = 112;
hipError_t launch_shared(const KParams& P, int grid, hipStream_t s) {
    hipLaunchKernelGGL((simplex_blk_kernel<4, 16, 7, 7, 2, true>), dim3(grid), dim3(256), 0, s, P);
    return hipGetLastError();
}
const void* shared_kernel_ptr() { return reinterpret_cast<const void*>(&simplex_blk_kernel<4, 16, 7, 7, 2, true>); }
int shared_threads() { return 256; }
void shared_shape(int* rows, int* cols) {
    *rows = kSharedRows;
    *cols = kSharedCols;
}

#define BLP_BLK_VARIANT(NAME, NW, GC, RB, CB, WPE)                                                    \
    {NAME, (NW) * 64, (NW) * 64 / (GC) * (RB), (GC) * (CB), &launch_blk<NW, GC, RB, CB, WPE>, \
     &kernel_ptr_blk<NW, GC, RB, CB, WPE>, 1, 0},
#define BLP_REG_VARIANT(NAME, NW, TC, CT, WPE)                                                                  \
    {NAME, (NW) * 64, (NW) * 64 / (TC), (TC) * (CT), &launch_reg<NW, TC, CT, WPE>, &kernel_ptr<NW, TC, CT, WPE>, \
     1, 0},
#define BLP_COLS_VARIANT(NAME, NW, GCW, RB, CB, WPE, ROWS, COLS)                                  \
    {NAME, (NW) * 64, ROWS, COLS, &launch_cols<NW, GCW, RB, CB, WPE, ROWS, COLS>,                 \
     &kernel_ptr_cols<NW, GCW, RB, CB, WPE>, 1, 1},
#define BLP_LANE_VARIANT(NAME, R, C, NWV, WPE) \
    {NAME, (NWV) * 64, R, C, &launch_lane<R, C, NWV, WPE>, &kernel_ptr_lane<R, C, NWV, WPE>, (NWV) * 64, 0},

const RegVariant* reg_variants(int* count) {
    static const RegVariant table[] = {BLP_REG_VARIANT_LIST};
    *count = (int)(sizeof(table) / sizeof(table[0]));
    return table;
}

}  // namespace blp
