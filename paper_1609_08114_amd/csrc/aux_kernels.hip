// Scheduling, hyperbox and adjoint kernels.
//
//  - reset_bins / classify / bin_offsets / scatter: build the size-binned
//    work lists on the device.  A simplex LP's condensed tableau has m + 2
//    rows and n + n_art + 1 columns, where n_art (rows whose "<=" form has a
//    negative rhs, Sec. 3) depends on the data, so the bin is chosen here
//    and not on the host.
//  - hyperbox: Eq. (7) of Sec. 6, one LP per thread with the paper's
//    sequential sum (Sec. 6 uses one thread per LP for the same reason).
//  - backward_simplex / backward_hyperbox: the adjoint of the optimum with
//    respect to the data, from the primal and dual solutions.
#include <algorithm>
#include <climits>
#include <cstdint>

#include "aux_kernels.hpp"
#include "blp_kernels.hpp"

namespace blp {

__global__ void reset_bins_kernel(int32_t* counters, int n) {
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) counters[i] = 0;
}

// Waves take LPs round-robin, two LPs per step so that two sets of row loads
// are in flight; each block keeps a bin histogram in LDS and adds it to one
// of kBinStripes copies of the bin counters (stripe = block mod
// kBinStripes), so that thousands of blocks do not serialise on one address.
// bins: 0..nreg-1 register variants, nreg streaming, nreg+1 hyperbox.
// Artificial rows among rows [i0, i0 + 128) of an LP: two wave-widths of
// rows, loads issued unconditionally (indices clamped into the LP) so that
// they are all in flight before the first compare.
struct ArtLoads {
    double ba, bb;
    int sa, sb;
};
__device__ __forceinline__ ArtLoads art_load(const KParams& P, const LpRef& L, int i0, int lane) {
    const int ia = min(i0 + lane, L.m - 1), ib = min(i0 + 64 + lane, L.m - 1);
    return {P.b[L.row_off + ia], P.b[L.row_off + ib], P.sense[L.row_off + ia], P.sense[L.row_off + ib]};
}
__device__ __forceinline__ int art_count(const ArtLoads& a, int m, int i0, int lane) {
    const int ia = i0 + lane, ib = ia + 64;
    return __popcll(__ballot(ia < m && (a.sa != 0 ? -a.ba : a.ba) < 0.0)) +
           __popcll(__ballot(ib < m && (a.sb != 0 ? -a.bb : a.bb) < 0.0));
}
// The variant table spread over the lanes of a wave: lane v < nreg holds
// variant v, loaded once per wave, so that choosing an LP's variant is one
// compare per lane and one wave reduction instead of a loop of table loads.
struct LaneVariant {
    int rows, cols, type1, remap;
    int64_t min_count;
};
__device__ __forceinline__ LaneVariant lane_variant(const VariantTable& vt, int lane) {
    LaneVariant r{0, 0, 1, 0, INT64_MAX};  // lanes past the table never fit
    if (lane < vt.nreg) {
        r.rows = vt.rows[lane];
        r.cols = vt.cols[lane];
        r.type1 = vt.type1[lane];
        r.remap = vt.remap[lane];
        r.min_count = vt.min_count[lane];
    }
    return r;
}
// The LP's bin (all 64 lanes active, result wave-uniform): the forced
// variant if it holds the LP; else the variant of smallest area that holds
// it (the first of equal areas; the area times 32 plus the lane is the key of
// a wave minimum), then the autotuner's remap of that variant.
__device__ __forceinline__ int bin_of(const VariantTable& vt, const LaneVariant& lv, int lane, const LpRef& L,
                                      int nart) {
    const int rows = L.m + 2, cols = L.n + nart + 1;
    // a variant for LPs without artificial rows under the largest-
    // coefficient rule takes only those
    const bool t1 = nart == 0 && vt.lpc;
    if (vt.force >= 0) {
        const int f = vt.force;
        if (f < vt.nreg && __builtin_amdgcn_readlane(lv.rows, f) >= rows &&
            __builtin_amdgcn_readlane(lv.cols, f) >= cols && (t1 || !__builtin_amdgcn_readlane(lv.type1, f)))
            return f;
        return vt.nreg;
    }
    if (vt.force != -1) return vt.nreg;  // streaming only
    const bool fit = lane < vt.nreg && lv.rows >= rows && lv.cols >= cols && (t1 || !lv.type1) &&
                     vt.count >= lv.min_count;
    const int best = wave_min_i32(fit ? ((lv.rows * lv.cols) << 5) | lane : INT_MAX);
    if (best == INT_MAX) return vt.nreg;
    int bin = best & 31;
    const int r = __builtin_amdgcn_readlane(lv.remap, bin);
    if (r >= vt.nreg || t1 || !__builtin_amdgcn_readlane(lv.type1, r)) bin = r;
    return bin;
}

__global__ void __launch_bounds__(256) classify_kernel(KParams P, VariantTable vt, int32_t* binid,
                                                        int32_t* stripes) {
    __shared__ int hist[kMaxVariants + 2];
    const int nbins = vt.nreg + 2;
    for (int b = threadIdx.x; b < nbins; b += blockDim.x) hist[b] = 0;
    __syncthreads();
    const int lane = threadIdx.x & 63;
    const LaneVariant lv = lane_variant(vt, lane);
    const int64_t nwaves = (int64_t)gridDim.x * (blockDim.x >> 6);
    const int wave = __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));  // uniform: scalar branches below
    for (int64_t k = (int64_t)blockIdx.x * (blockDim.x >> 6) + wave; k < P.count; k += 2 * nwaves) {
        // two LPs per step (the second may be absent or a hyperbox): the
        // first 128 rows of both are loaded before either is counted
        const int64_t k2 = k + nwaves < P.count ? k + nwaves : k;
        const bool s1 = lp_kind(P, k) != 1, s2 = lp_kind(P, k2) != 1;
        const LpRef L1 = lp_ref(P, k), L2 = lp_ref(P, k2);
        int n1 = 0, n2 = 0;
        if (s1 || s2) {
            // a hyperbox slot borrows the other LP's rows (loaded, not counted)
            const ArtLoads a1 = art_load(P, s1 ? L1 : L2, 0, lane);
            const ArtLoads a2 = art_load(P, s2 ? L2 : L1, 0, lane);
            n1 = s1 ? art_count(a1, L1.m, 0, lane) : 0;
            n2 = s2 ? art_count(a2, L2.m, 0, lane) : 0;
        }
        for (int i0 = 128; s1 && i0 < L1.m; i0 += 128) n1 += art_count(art_load(P, L1, i0, lane), L1.m, i0, lane);
        for (int i0 = 128; s2 && i0 < L2.m; i0 += 128) n2 += art_count(art_load(P, L2, i0, lane), L2.m, i0, lane);
        const int b1 = s1 ? bin_of(vt, lv, lane, L1, n1) : vt.nreg + 1;
        const int b2 = k2 != k ? (s2 ? bin_of(vt, lv, lane, L2, n2) : vt.nreg + 1) : -1;
        if (lane == 0) {
            binid[k] = b1;
            atomicAdd(&hist[b1], 1);
            if (b2 >= 0) {
                binid[k2] = b2;
                atomicAdd(&hist[b2], 1);
            }
        }
    }
    __syncthreads();
    for (int b = threadIdx.x; b < nbins; b += blockDim.x)
        if (hist[b]) atomicAdd(stripes + (blockIdx.x % kBinStripes) * kStripeStride + b, hist[b]);
}

// Bin sizes (the kBinStripes copies summed) and their exclusive prefix: wave
// w sums bins w, w + 4, ..., one stripe per lane.
__global__ void __launch_bounds__(256) bin_offsets_kernel(const int32_t* stripes, int32_t* bin_count,
                                                          int32_t* bin_off, int nbins) {
    static_assert(kBinStripes == 64, "one stripe per lane");
    __shared__ int total[kMaxVariants + 2];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    int v[(kMaxVariants + 2 + 3) / 4];
#pragma unroll
    for (int u = 0; u < (kMaxVariants + 2 + 3) / 4; ++u) {
        const int b = wave + 4 * u;
        v[u] = b < nbins ? stripes[lane * kStripeStride + b] : 0;
    }
#pragma unroll
    for (int u = 0; u < (kMaxVariants + 2 + 3) / 4; ++u) {
        int acc = v[u];
        for (int o = 32; o >= 1; o >>= 1) acc += __shfl_xor(acc, o);
        const int b = wave + 4 * u;
        if (lane == 0 && b < nbins) total[b] = acc;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        int acc = 0;
        for (int b = 0; b < nbins; ++b) {
            bin_count[b] = total[b];
            bin_off[b] = acc;
            acc += total[b];
        }
    }
}

__global__ void __launch_bounds__(256) scatter_kernel(int64_t count, int nbins, const int32_t* binid,
                                                      const int32_t* bin_off, int32_t* bin_fill, int32_t* list) {
    __shared__ int hist[kMaxVariants + 2], base[kMaxVariants + 2];
    const int64_t chunk = 2048;
    for (int64_t c0 = (int64_t)blockIdx.x * chunk; c0 < count; c0 += (int64_t)gridDim.x * chunk) {
        const int64_t c1 = c0 + chunk < count ? c0 + chunk : count;
        for (int b = threadIdx.x; b < nbins; b += blockDim.x) hist[b] = 0;
        __syncthreads();
        for (int64_t k = c0 + threadIdx.x; k < c1; k += blockDim.x) atomicAdd(&hist[binid[k]], 1);
        __syncthreads();
        for (int b = threadIdx.x; b < nbins; b += blockDim.x) {
            base[b] = hist[b] ? bin_off[b] + atomicAdd(bin_fill + b, hist[b]) : 0;
            hist[b] = 0;
        }
        __syncthreads();
        for (int64_t k = c0 + threadIdx.x; k < c1; k += blockDim.x) {
            const int b = binid[k];
            list[base[b] + atomicAdd(&hist[b], 1)] = (int32_t)k;
        }
        __syncthreads();
    }
}

// Largest-first work lists.  A persistent launch pops its bin in list order,
// and lasts as long as its busiest workgroup: with the long LPs taken first
// and the short ones filling in at the end, the workgroups finish close
// together (list scheduling, longest first).  Work of an LP is estimated as
// pivots x entries per pivot, (m + n)(m + 2)(n + m + 1); LPs are ordered by
// half-octave buckets of it (within a bucket, in scatter order).
constexpr int kWorkBuckets = 64;
__device__ __forceinline__ int work_bucket(const KParams& P, int64_t k) {
    const uint64_t m = (uint32_t)P.m[k], n = (uint32_t)P.n[k];  // m, n >= 0 (checked on the host)
    const uint64_t w = (m + n) * (m + 2) * (n + m + 1) + 1;
    const int e = 63 - __clzll((long long)w);
    const int b = 2 * e + (e > 0 ? (int)((w >> (e - 1)) & 1) : 0);
    return b < kWorkBuckets - 1 ? b : kWorkBuckets - 1;
}
__global__ void __launch_bounds__(1024) order_bins_kernel(KParams P, const int32_t* bin_count,
                                                          const int32_t* bin_off, const int32_t* list,
                                                          int32_t* out) {
    __shared__ int pos[kWorkBuckets];
    const int b = blockIdx.x;  // one workgroup per bin
    const int len = bin_count[b], off = bin_off[b];
    for (int i = threadIdx.x; i < kWorkBuckets; i += blockDim.x) pos[i] = 0;
    __syncthreads();
    for (int q = threadIdx.x; q < len; q += blockDim.x) atomicAdd(&pos[work_bucket(P, list[off + q])], 1);
    __syncthreads();
    if (threadIdx.x == 0) {  // start of each bucket, largest bucket first
        int acc = off;
        for (int i = kWorkBuckets - 1; i >= 0; --i) {
            const int c = pos[i];
            pos[i] = acc;
            acc += c;
        }
    }
    __syncthreads();
    for (int q = threadIdx.x; q < len; q += blockDim.x) {
        const int32_t k = list[off + q];
        out[atomicAdd(&pos[work_bucket(P, k)], 1)] = k;
    }
}

// Eq. (7): maximise c.x over [l, u]: x_i = l_i where c_i < 0, else u_i; the
// value is the sequential fused multiply-add sum in increasing i.
__global__ void hyperbox_kernel(KParams P) {
    const int64_t len = work_len(P);
    for (int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; q < len; q += (int64_t)gridDim.x * blockDim.x) {
        const int64_t k = work_item(P, q);
        const LpRef L = lp_ref(P, k);
        const double* c = P.c + L.col_off;
        const int64_t bo = P.box_shared ? 0 : L.col_off;  // one box for every LP, or its own
        const double* lo = P.l + bo;
        const double* up = P.u + bo;
        double* x = P.x + L.col_off;
        bool bad = false, empty = false;
        double acc = 0.0;
        for (int i = 0; i < L.n; ++i) {
            const double ci = c[i], li = lo[i], ui = up[i];
            bad |= !isfinite(ci) || !isfinite(li) || !isfinite(ui);
            empty |= li > ui;
            const double h = ci < 0.0 ? li : ui;
            acc = __builtin_fma(ci, h, acc);
            x[i] = h;
        }
        if (bad)
            for (int i = 0; i < L.n; ++i) x[i] = __builtin_nan("");
        P.status[k] = bad ? ST_NUMERICAL : (empty ? ST_INFEASIBLE : ST_OPTIMAL);
        P.iters[k] = 0;
        P.obj[k] = bad ? __builtin_nan("") : (empty ? -__builtin_inf() : acc);
    }
}

// Eq. (7) for a uniform batch of n-variable boxes laid out back to back:
// one wave per group of G LPs (64; 32 for n > 16).  c, l, u are read with consecutive lanes on
// consecutive doubles and x is written the same way; c and h go through LDS
// (rows padded to n + 1 doubles against bank conflicts) so that lane i can
// sum LP i's products in increasing order, as the per-LP kernel does.
// Invalid-data flags are OR-ed per LP in LDS.
template <int G>
__global__ void __launch_bounds__(64) hyperbox_tile_kernel(KParams P) {
    extern __shared__ double s_mem[];
    const int N = P.un, NP = N + 1;
    double* s_c = s_mem;
    double* s_h = s_mem + G * NP;
    int* s_fl = reinterpret_cast<int*>(s_h + G * NP);
    const int lane = threadIdx.x;
    const int64_t K = P.count;
    // e / N as a multiply-high: exact for e < 64 * 48 (the fraction of e / N
    // stays below 1 - 1/N, the rounding error below e / 2^32)
    const unsigned magic = (unsigned)((0x100000000ull + N - 1) / N);
    constexpr int UNR = 8;
    for (int64_t g = blockIdx.x; g * G < K; g += gridDim.x) {
        const int64_t k0 = g * G;
        const int nl = (int)(K - k0 < G ? K - k0 : G);
        const int64_t e0 = k0 * N;
        const int ne = nl * N;
        if (lane < G) s_fl[lane] = 0;
        __syncthreads();
        for (int eb = 0; eb < ne; eb += 64 * UNR) {
            double cv[UNR], lv[UNR], uv[UNR];
#pragma unroll
            for (int q = 0; q < UNR; ++q) {
                const int e = eb + q * 64 + lane;
                const int ec = e < ne ? e : 0;
                const int64_t a = e0 + ec;
                // a shared box is read at the variable's index
                const int64_t ab = P.box_shared ? (int64_t)(ec - (int)__umulhi((unsigned)ec, magic) * N) : a;
                cv[q] = P.c[a];
                lv[q] = P.l[ab];
                uv[q] = P.u[ab];
            }
#pragma unroll
            for (int q = 0; q < UNR; ++q) {
                const int e = eb + q * 64 + lane;
                if (e < ne) {
                    const double h = cv[q] < 0.0 ? lv[q] : uv[q];
                    P.x[e0 + e] = h;
                    const int lk = (int)__umulhi((unsigned)e, magic), i = e - lk * N;
                    s_c[lk * NP + i] = cv[q];
                    s_h[lk * NP + i] = h;
                    const int f = ((!isfinite(cv[q]) || !isfinite(lv[q]) || !isfinite(uv[q])) ? 1 : 0) |
                                  (lv[q] > uv[q] ? 2 : 0);
                    if (f) atomicOr(&s_fl[lk], f);
                }
            }
        }
        __syncthreads();
        if (lane < nl) {
            double acc = 0.0;
            for (int i = 0; i < N; ++i) acc = __builtin_fma(s_c[lane * NP + i], s_h[lane * NP + i], acc);
            const int f = s_fl[lane];
            const bool bad = f & 1, empty = f & 2;
            const int64_t k = k0 + lane;
            if (bad) {
                __threadfence();  // after this wave's x = h stores
                for (int i = 0; i < N; ++i) P.x[e0 + (int64_t)lane * N + i] = __builtin_nan("");
            }
            P.status[k] = bad ? ST_NUMERICAL : (empty ? ST_INFEASIBLE : ST_OPTIMAL);
            P.iters[k] = 0;
            P.obj[k] = bad ? __builtin_nan("") : (empty ? -__builtin_inf() : acc);
        }
        __syncthreads();
    }
}

// Adjoint of a uniform hyperbox batch, one thread per variable.
__global__ void __launch_bounds__(256) backward_hyperbox_flat_kernel(KParams P, const double* g, double* dc,
                                                                      double* dl, double* du) {
    const int N = P.un;
    const int64_t E = P.count * (int64_t)N;
    // LP k = e / N advances with e (one division per thread, not per element)
    const int64_t stride = (int64_t)gridDim.x * blockDim.x, e0 = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t dk = stride / N;
    const int dr = (int)(stride - dk * N);
    int64_t k = e0 / N;
    int r = (int)(e0 - k * N);
    for (int64_t e = e0; e < E; e += stride) {
        const bool ok = P.status[k] == ST_OPTIMAL;
        const double gk = ok ? g[k] : 0.0;
        const double ci = P.c[e];
        if (dc) dc[e] = ok ? gk * P.x[e] : 0.0;
        if (dl) dl[e] = ok && ci < 0.0 ? gk * ci : 0.0;
        if (du) du[e] = ok && !(ci < 0.0) ? gk * ci : 0.0;
        k += dk;
        r += dr;
        if (r >= N) {
            r -= N;
            ++k;
        }
    }
}

// Adjoint of a shared box: dl_i = sum over hyperbox LPs k of g_k min(c_ki, 0)
// and du_i of g_k max(c_ki, 0) (zero for LPs that are not OPTIMAL).  A fixed
// summation order, independent of scheduling: block b sums LPs
// [b * 1024, (b + 1) * 1024) -- each thread its four LPs t, t + 256, t + 512,
// t + 768 in that order, then a pairwise tree over the 256 threads -- into
// part[b]; box_shared_final then adds the block sums in block order.
constexpr int kBoxRedLps = 1024;
__global__ void __launch_bounds__(256) box_shared_partial_kernel(KParams P, const double* g, int n, double* part) {
    __shared__ double s_l[256], s_u[256];
    const int t = threadIdx.x;
    const int64_t k0 = (int64_t)blockIdx.x * kBoxRedLps;
    for (int i = 0; i < n; ++i) {
        double al = 0.0, au = 0.0;
        for (int r = 0; r < kBoxRedLps / 256; ++r) {
            const int64_t k = k0 + t + r * 256;
            if (k < P.count && lp_kind(P, k) == 1 && P.status[k] == ST_OPTIMAL) {
                const double ci = P.c[lp_ref(P, k).col_off + i];
                const double gk = g[k];
                al = al + (ci < 0.0 ? gk * ci : 0.0);
                au = au + (ci < 0.0 ? 0.0 : gk * ci);
            }
        }
        s_l[t] = al;
        s_u[t] = au;
        __syncthreads();
        for (int w = 128; w >= 1; w >>= 1) {
            if (t < w) {
                s_l[t] = s_l[t] + s_l[t + w];
                s_u[t] = s_u[t] + s_u[t + w];
            }
            __syncthreads();
        }
        if (t == 0) {
            part[(int64_t)blockIdx.x * 2 * n + i] = s_l[0];
            part[(int64_t)blockIdx.x * 2 * n + n + i] = s_u[0];
        }
        __syncthreads();
    }
}
__global__ void __launch_bounds__(256) box_shared_final_kernel(const double* part, int nblocks, int n, double* dl,
                                                               double* du) {
    for (int i = threadIdx.x; i < 2 * n; i += blockDim.x) {
        double acc = 0.0;
        for (int b = 0; b < nblocks; ++b) acc = acc + part[(int64_t)b * 2 * n + i];
        if (i < n) {
            if (dl) dl[i] = acc;
        } else if (du) {
            du[i - n] = acc;
        }
    }
}

// Adjoint for simplex LPs: dc = g x*, db = g y*, dA = -g y* x*^T.  One
// workgroup per LP; LPs not OPTIMAL get zeros.
__global__ void __launch_bounds__(256) backward_simplex_kernel(KParams P, const double* g, double* dc, double* db,
                                                               double* dA, int stage) {
    // x of the LP, then -(g y) of the LP (when the `stage` doubles of LDS
    // hold them; else read in place): each dA element is one product of two
    // such values, written in element order (coalesced)
    extern __shared__ double s_xy[];
    for (int64_t k = blockIdx.x; k < P.count; k += gridDim.x) {
        if (lp_kind(P, k) != 0) continue;
        const LpRef L = lp_ref(P, k);
        const bool ok = P.status[k] == ST_OPTIMAL;
        const double gk = ok ? g[k] : 0.0;
        const double* x = P.x + L.col_off;
        const double* y = P.y + L.row_off;
        if (dc)
            for (int j = threadIdx.x; j < L.n; j += blockDim.x) dc[L.col_off + j] = ok ? gk * x[j] : 0.0;
        if (db)
            for (int i = threadIdx.x; i < L.m; i += blockDim.x) db[L.row_off + i] = ok ? gk * y[i] : 0.0;
        if (dA && L.n > 0) {
            const bool staged = L.n + L.m <= stage;
            double* sx = s_xy;
            double* sy = s_xy + L.n;
            if (staged) {
                for (int j = threadIdx.x; j < L.n; j += blockDim.x) sx[j] = x[j];
                for (int i = threadIdx.x; i < L.m; i += blockDim.x) sy[i] = -(gk * y[i]);
            }
            __syncthreads();
            // element e = i n + j; (i, j) advance with e instead of a
            // division per element (m n < 2^31 by the size limits).  Not
            // OPTIMAL: zeros (x and y may be NaN; selected away, never
            // multiplied by a zero weight)
            const int n = L.n, mn = L.m * n, step = (int)blockDim.x;
            const int di = step / n, dj = step - di * n;
            int i = (int)threadIdx.x / n, j = (int)threadIdx.x - i * n;
            double* out = dA + L.a_off;
            for (int e = threadIdx.x; e < mn; e += step) {
                out[e] = !ok ? 0.0 : staged ? sy[i] * sx[j] : -(gk * y[i]) * x[j];
                i += di;
                j += dj;
                if (j >= n) {
                    j -= n;
                    ++i;
                }
            }
            __syncthreads();  // the stage is reused by the next LP
        }
    }
}

// Adjoint for hyperbox LPs: dc = g h, dl = g min(c, 0), du = g max(c, 0)
// (with the same c_i < 0 split as the forward pass).  One LP per thread.
__global__ void backward_hyperbox_kernel(KParams P, const double* g, double* dc, double* dl, double* du) {
    const int64_t len = work_len(P);
    for (int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; q < len; q += (int64_t)gridDim.x * blockDim.x) {
        const int64_t k = work_item(P, q);
        const LpRef L = lp_ref(P, k);
        const bool ok = P.status[k] == ST_OPTIMAL;
        const double gk = ok ? g[k] : 0.0;
        for (int i = 0; i < L.n; ++i) {
            const double ci = P.c[L.col_off + i];
            if (dc) dc[L.col_off + i] = ok ? gk * P.x[L.col_off + i] : 0.0;
            if (dl) dl[L.col_off + i] = ok && ci < 0.0 ? gk * ci : 0.0;
            if (du) du[L.col_off + i] = ok && !(ci < 0.0) ? gk * ci : 0.0;
        }
    }
}

// Route of a shared-constraint solve (aux_kernels.hpp: shared_route_of).
__global__ void __launch_bounds__(256) shared_route_kernel(int m, int n, int64_t count, const double* b,
                                                            const int8_t* sense, const double* C, SharedRoute rt,
                                                            int32_t* route_len) {
    __shared__ int s_nart[4], s_close[4];
    const int t = threadIdx.x, lane = t & 63, wave = t >> 6;
    int na = 0;
    for (int i = t; i < m; i += 256) {
        const double bi = b[i];
        na += (sense[i] ? -bi : bi) < 0.0;
    }
    for (int o = 32; o >= 1; o >>= 1) na += __shfl_xor(na, o);
    const int64_t ns = count < 65 ? count : 65;
    int close = 0;
    for (int64_t k = 1 + wave; k < ns; k += 4) {
        const double* u = C + k * n;
        const double* v = C + (k - 1) * n;
        double dot = 0.0, aa = 0.0, bb = 0.0;
        for (int j = lane; j < n; j += 64) {
            dot += u[j] * v[j];
            aa += u[j] * u[j];
            bb += v[j] * v[j];
        }
        for (int o = 32; o >= 1; o >>= 1) {
            dot += __shfl_xor(dot, o);
            aa += __shfl_xor(aa, o);
            bb += __shfl_xor(bb, o);
        }
        close += dot > 0.9 * sqrt(aa * bb);  // false for non-finite objectives
    }
    if (lane == 0) {
        s_nart[wave] = na;
        s_close[wave] = close;
    }
    __syncthreads();
    if (t == 0) {
        const int nart = s_nart[0] + s_nart[1] + s_nart[2] + s_nart[3];
        const int64_t cl = s_close[0] + s_close[1] + s_close[2] + s_close[3];
        const int r = shared_route_of(rt, m, n, nart, ns > 1 && 2 * cl >= ns - 1);
        for (int i = 0; i < rt.nreg + 2; ++i) route_len[i] = i == r ? (int)count : 0;
    }
}

__global__ void iota_kernel(int32_t* list, int64_t count) {
    for (int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; q < count; q += (int64_t)gridDim.x * blockDim.x)
        list[q] = (int32_t)q;
}

// ------------------------------------------------------------------ launchers
hipError_t launch_shared_route(int m, int n, int64_t count, const double* b, const int8_t* sense, const double* C,
                               const SharedRoute& rt, int32_t* route_len, hipStream_t s) {
    hipLaunchKernelGGL(shared_route_kernel, dim3(1), dim3(256), 0, s, m, n, count, b, sense, C, rt, route_len);
    return hipGetLastError();
}

hipError_t launch_iota(int32_t* list, int64_t count, hipStream_t s) {
    int64_t blocks = (count + 255) / 256;
    if (blocks > 4096) blocks = 4096;
    if (blocks < 1) blocks = 1;
    hipLaunchKernelGGL(iota_kernel, dim3((unsigned)blocks), dim3(256), 0, s, list, count);
    return hipGetLastError();
}

hipError_t launch_reset(int32_t* counters, int n, hipStream_t s) {
    hipLaunchKernelGGL(reset_bins_kernel, dim3(1), dim3(256), 0, s, counters, n);
    return hipGetLastError();
}
int classify_blocks(int64_t count) {
    // one LP per wave to start with: the classification is a chain of
    // dependent loads per LP, so more waves in flight finish it sooner
    int64_t blocks = (count + 3) / 4;
    if (blocks > kClassifyMaxBlocks) blocks = kClassifyMaxBlocks;
    if (blocks < 1) blocks = 1;
    return (int)blocks;
}
hipError_t launch_classify(const KParams& P, const VariantTable& vt, int32_t* binid, int32_t* stripes,
                           hipStream_t s) {
    hipLaunchKernelGGL(classify_kernel, dim3((unsigned)classify_blocks(P.count)), dim3(256), 0, s, P, vt, binid,
                       stripes);
    return hipGetLastError();
}
hipError_t launch_bin_offsets(const int32_t* stripes, int32_t* bin_count, int32_t* bin_off, int nbins,
                              hipStream_t s) {
    hipLaunchKernelGGL(bin_offsets_kernel, dim3(1), dim3(256), 0, s, stripes, bin_count, bin_off, nbins);
    return hipGetLastError();
}
hipError_t launch_scatter(int64_t count, int nbins, const int32_t* binid, const int32_t* bin_off, int32_t* bin_fill,
                          int32_t* list, hipStream_t s) {
    int64_t blocks = (count + 2047) / 2048;
    if (blocks > 4096) blocks = 4096;
    if (blocks < 1) blocks = 1;
    hipLaunchKernelGGL(scatter_kernel, dim3((unsigned)blocks), dim3(256), 0, s, count, nbins, binid, bin_off,
                       bin_fill, list);
    return hipGetLastError();
}
hipError_t launch_order_bins(const KParams& P, int nbins, const int32_t* bin_count, const int32_t* bin_off,
                             const int32_t* list, int32_t* out, hipStream_t s) {
    hipLaunchKernelGGL(order_bins_kernel, dim3((unsigned)nbins), dim3(1024), 0, s, P, bin_count, bin_off, list, out);
    return hipGetLastError();
}
static unsigned grid_for(int64_t items, int per_block, int64_t cap) {
    int64_t b = (items + per_block - 1) / per_block;
    if (b > cap) b = cap;
    if (b < 1) b = 1;
    return (unsigned)b;
}
hipError_t launch_hyperbox(const KParams& P, int64_t max_items, hipStream_t s) {
    if (P.uniform && !P.list && P.un >= 1 && P.un <= kBoxTileMaxN) {
        // groups of 64 LPs per wave; 32 for larger n, so that twice as many
        // waves fit the LDS of a CU and keep loads in flight
        if (P.un <= 16) {
            const size_t lds = sizeof(double) * 2 * 64 * (size_t)(P.un + 1) + sizeof(int) * 64;
            hipLaunchKernelGGL(hyperbox_tile_kernel<64>, dim3(grid_for(P.count, 64, 1 << 15)), dim3(64), lds, s, P);
        } else {
            const size_t lds = sizeof(double) * 2 * 32 * (size_t)(P.un + 1) + sizeof(int) * 32;
            hipLaunchKernelGGL(hyperbox_tile_kernel<32>, dim3(grid_for(P.count, 32, 1 << 15)), dim3(64), lds, s, P);
        }
        return hipGetLastError();
    }
    hipLaunchKernelGGL(hyperbox_kernel, dim3(grid_for(max_items, 256, 1 << 16)), dim3(256), 0, s, P);
    return hipGetLastError();
}
hipError_t launch_backward_simplex(const KParams& P, const double* g, double* dc, double* db, double* dA, int max_n,
                                   int max_m, hipStream_t s) {
    const int stage = max_n + max_m > 0 ? max_n + max_m : 1;  // at most 4095 + 2046 doubles
    hipLaunchKernelGGL(backward_simplex_kernel, dim3(grid_for(P.count, 1, 1 << 16)), dim3(256),
                       sizeof(double) * (size_t)stage, s, P, g, dc, db, dA, stage);
    return hipGetLastError();
}
// Adjoint of a shared-constraint solve (one A, b; objectives C, LP k's
// results x_k at X + k n, y_k at Y + k m): w_k = g_k for OPTIMAL LPs, else 0;
// dC[k] = w_k x_k, db = sum_k w_k y_k, dA = -sum_k w_k y_k x_k^T.  The sums
// over k run in increasing k inside chunks of consecutive LPs (one partial
// per chunk), then over the chunks in order: the same bits on every call.
__global__ void __launch_bounds__(256) shared_bwd_dc_kernel(int64_t count, int n, const int32_t* st, const double* g,
                                                            const double* X, double* dC) {
    const int64_t E = count * (int64_t)n;
    const int64_t stride = (int64_t)gridDim.x * blockDim.x, e0 = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t dk = stride / n;
    const int dr = (int)(stride - dk * n);
    int64_t k = e0 / n;
    int r = (int)(e0 - k * n);
    for (int64_t e = e0; e < E; e += stride) {
        dC[e] = st[k] == ST_OPTIMAL ? g[k] * X[e] : 0.0;
        k += dk;
        r += dr;
        if (r >= n) {
            r -= n;
            ++k;
        }
    }
}
// One block per (16 x 16 tile of dA, chunk of LPs): the block stages 64 LPs
// at a time in LDS (w_k y_ki for the tile's 16 rows, x_kj for its 16
// columns; zero for LPs that are not OPTIMAL, whose x and y may be NaN and
// are selected away rather than multiplied by a zero weight), then thread
// (i, j) of the tile sums fma(w_k y_ki, x_kj, .) over them in LP order; the
// tile's first column of threads in the first tile column also sums w_k y_ki
// for db.
__global__ void __launch_bounds__(256) shared_bwd_part_kernel(int64_t count, int m, int n, int64_t chunk,
                                                              const int32_t* st, const double* g, const double* X,
                                                              const double* Y, double* part_a, double* part_b) {
    constexpr int KS = 64;  // LPs per stage
    __shared__ double s_y[KS][16], s_x[KS][16];
    const int tiles_n = (n + 15) / 16;
    const int ti = blockIdx.x / tiles_n, tj = blockIdx.x - ti * tiles_n;
    const int il = (int)threadIdx.x / 16, jl = (int)threadIdx.x % 16;
    const int i = ti * 16 + il, j = tj * 16 + jl;
    const int64_t c = blockIdx.y, k0 = c * chunk, k1 = k0 + chunk < count ? k0 + chunk : count;
    const bool rowsum = tj == 0 && jl == 0 && i < m;
    double acc = 0.0, accb = 0.0;
    for (int64_t kb = k0; kb < k1; kb += KS) {
        for (int e = threadIdx.x; e < KS * 16; e += blockDim.x) {
            const int kk = e / 16, r = e % 16;
            const int64_t k = kb + kk < k1 ? kb + kk : k1 - 1;
            const bool ok = kb + kk < k1 && st[k] == ST_OPTIMAL;
            const int ir = ti * 16 + r < m ? ti * 16 + r : m - 1, jr = tj * 16 + r < n ? tj * 16 + r : n - 1;
            const double yv = Y[k * m + ir], xv = X[k * n + jr], gk = g[k];
            s_y[kk][r] = ok ? gk * yv : 0.0;
            s_x[kk][r] = ok ? xv : 0.0;
        }
        __syncthreads();
        const int kn = k1 - kb < KS ? (int)(k1 - kb) : KS;
        for (int kk = 0; kk < kn; ++kk) {
            const double wy = s_y[kk][il];
            acc = __builtin_fma(wy, s_x[kk][jl], acc);
            accb = accb + wy;
        }
        __syncthreads();
    }
    if (i < m && j < n) part_a[c * (int64_t)m * n + (int64_t)i * n + j] = acc;
    if (rowsum) part_b[c * m + i] = accb;
}
// out[e] = sign * (sum over the chunks, in order, of part[c len + e])
__global__ void __launch_bounds__(256) shared_bwd_final_kernel(int nchunks, int64_t len, const double* part,
                                                               double sign, double* out) {
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < len; e += (int64_t)gridDim.x * blockDim.x) {
        double acc = 0.0;
        for (int c = 0; c < nchunks; ++c) acc = acc + part[(int64_t)c * len + e];
        out[e] = sign * acc;
    }
}

int box_shared_blocks(int64_t count) { return (int)((count + kBoxRedLps - 1) / kBoxRedLps); }
int64_t shared_bwd_chunk(int64_t count, int m, int n) {
    // chunks of at least 1,024 LPs, and partial sums of at most 8M doubles
    const int64_t per = (int64_t)m * n + m;
    const int64_t max_chunks = std::max<int64_t>(1, (int64_t(8) << 20) / per);
    const int64_t chunks =
        std::min<int64_t>(std::min<int64_t>(std::max<int64_t>(1, (count + 1023) / 1024), max_chunks), 65535);
    return (count + chunks - 1) / chunks;
}
hipError_t launch_backward_shared(int64_t count, int m, int n, const int32_t* st, const double* g, const double* X,
                                  const double* Y, double* part, double* dC, double* db, double* dA, hipStream_t s) {
    if (count <= 0) return hipSuccess;
    if (dC) {
        hipLaunchKernelGGL(shared_bwd_dc_kernel, dim3(grid_for(count * (int64_t)n, 256, 1 << 16)), dim3(256), 0, s,
                           count, n, st, g, X, dC);
    }
    if (db || dA) {
        const int64_t chunk = shared_bwd_chunk(count, m, n);
        const int nchunks = (int)((count + chunk - 1) / chunk);
        double* part_a = part;
        double* part_b = part + (int64_t)nchunks * m * n;
        const unsigned tiles = (unsigned)(((m + 15) / 16) * ((n + 15) / 16));
        hipLaunchKernelGGL(shared_bwd_part_kernel, dim3(tiles, (unsigned)nchunks), dim3(256), 0, s, count, m, n, chunk,
                           st, g, X, Y, part_a, part_b);
        if (dA)
            hipLaunchKernelGGL(shared_bwd_final_kernel, dim3(grid_for((int64_t)m * n, 256, 1 << 16)), dim3(256), 0, s,
                               nchunks, (int64_t)m * n, part_a, -1.0, dA);
        if (db)
            hipLaunchKernelGGL(shared_bwd_final_kernel, dim3(grid_for(m, 256, 1 << 16)), dim3(256), 0, s, nchunks,
                               (int64_t)m, part_b, 1.0, db);
    }
    return hipGetLastError();
}
hipError_t launch_backward_box_shared(const KParams& P, int n, const double* g, double* part, double* dl, double* du,
                                      hipStream_t s) {
    const int nb = box_shared_blocks(P.count);
    hipLaunchKernelGGL(box_shared_partial_kernel, dim3((unsigned)nb), dim3(256), 0, s, P, g, n, part);
    hipLaunchKernelGGL(box_shared_final_kernel, dim3(1), dim3(256), 0, s, (const double*)part, nb, n, dl, du);
    return hipGetLastError();
}
hipError_t launch_backward_hyperbox(const KParams& P, int64_t max_items, const double* g, double* dc, double* dl,
                                    double* du, hipStream_t s) {
    if (P.uniform && !P.list && P.un >= 1) {
        hipLaunchKernelGGL(backward_hyperbox_flat_kernel, dim3(grid_for(P.count * (int64_t)P.un, 256, 1 << 16)),
                           dim3(256), 0, s, P, g, dc, dl, du);
        return hipGetLastError();
    }
    hipLaunchKernelGGL(backward_hyperbox_kernel, dim3(grid_for(max_items, 256, 1 << 16)), dim3(256), 0, s, P, g,
                       dc, dl, du);
    return hipGetLastError();
}

}  // namespace blp
