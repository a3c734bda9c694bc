// Host-callable launchers of the solver's kernels.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "blp_kernels.hpp"

namespace blp {

constexpr int kMaxVariants = 24;  // < 32: the classify kernel keys a variant by area * 32 + index
// Widest uniform hyperbox served by the LDS-transposing kernel (LDS per wave:
// 2 * 64 * (n + 1) doubles).
constexpr int kBoxTileMaxN = 48;

// Register-tile variant shapes handed to the classify kernel.
struct VariantTable {
    int nreg;
    int64_t count;  // LPs of the batch
    int force;  // -1 automatic, -2 streaming only, >= 0 one variant
    int rows[kMaxVariants];
    int cols[kMaxVariants];
    int remap[kMaxVariants];  // autotuned replacement of each variant (nreg = streaming)
    int type1[kMaxVariants];  // 1: the variant takes only LPs without artificial rows under LPC
    int64_t min_count[kMaxVariants];  // automatic choice: only for batches of at least this many LPs
    int lpc;                  // 1: the largest-coefficient rule (else the random rule)
};

hipError_t launch_reset(int32_t* counters, int n, hipStream_t s);
// classify adds its blocks' bin histograms into kBinStripes copies of the
// bin counters, one 128-byte line per copy (stripes[stripe * kStripeStride +
// bin], zeroed beforehand), so that the blocks' atomics spread over
// kBinStripes lines; bin_offsets sums the copies into bin_count and writes
// the exclusive prefix to bin_off.
constexpr int kClassifyMaxBlocks = 8192;
constexpr int kBinStripes = 64;
constexpr int kStripeStride = 32;
static_assert(kMaxVariants + 2 <= kStripeStride, "every bin of a stripe on its line");
int classify_blocks(int64_t count);
hipError_t launch_classify(const KParams& P, const VariantTable& vt, int32_t* binid, int32_t* stripes,
                           hipStream_t s);
hipError_t launch_bin_offsets(const int32_t* stripes, int32_t* bin_count, int32_t* bin_off, int nbins,
                              hipStream_t s);
hipError_t launch_scatter(int64_t count, int nbins, const int32_t* binid, const int32_t* bin_off, int32_t* bin_fill,
                          int32_t* list, hipStream_t s);
// Non-uniform batches: copy each bin's segment of `list` into `out` with the
// LPs of most estimated work first (one workgroup per bin).
hipError_t launch_order_bins(const KParams& P, int nbins, const int32_t* bin_count, const int32_t* bin_off,
                             const int32_t* list, int32_t* out, hipStream_t s);
hipError_t launch_hyperbox(const KParams& P, int64_t max_items, hipStream_t s);
// max_n, max_m: the largest n and m of the batch's simplex LPs (the
// workgroup stages x and the scaled y of one LP in LDS)
hipError_t launch_backward_simplex(const KParams& P, const double* g, double* dc, double* db, double* dA, int max_n,
                                   int max_m, hipStream_t s);
hipError_t launch_backward_hyperbox(const KParams& P, int64_t max_items, const double* g, double* dc, double* dl,
                                    double* du, hipStream_t s);
// Shared box: dl, du (length n) summed over the hyperbox LPs in a fixed
// order; `part` holds 2 n doubles per block of box_shared_blocks(count).
int box_shared_blocks(int64_t count);
// Adjoint of a shared-constraint solve: dC (count x n), db (m), dA (m x n);
// `part` holds shared_bwd_chunk's partial sums, (m n + m) doubles per chunk
// of shared_bwd_chunk(count, m, n) LPs.
int64_t shared_bwd_chunk(int64_t count, int m, int n);
hipError_t launch_backward_shared(int64_t count, int m, int n, const int32_t* st, const double* g, const double* X,
                                  const double* Y, double* part, double* dC, double* db, double* dA, hipStream_t s);
hipError_t launch_backward_box_shared(const KParams& P, int n, const double* g, double* part, double* dl, double* du,
                                      hipStream_t s);

// Route of a shared-constraint solve (one A, b, sense; many objectives),
// decided on the device so that the call reads nothing back: bin nreg + 1 is
// the warm-started shared kernel, bins 0..nreg-1 the register variants
// (every objective solved cold), bin nreg the streaming kernel.
struct SharedRoute {
    int nreg;
    int rows[kMaxVariants], cols[kMaxVariants], type1[kMaxVariants];
    int tile_rows, tile_cols;  // tableau of the warm-started kernel
};
// The route for n_art artificial rows; warm_dirs: consecutive objectives
// point in close directions.  Warm starts when the shared tile holds the
// tableau; otherwise the register variant of the shared tile's shape, else
// the one of smallest area (the first of equal areas), that holds it; else
// the streaming kernel.  Variants for LPs without artificial rows only
// (type1) are never taken.
__host__ __device__ inline int shared_route_of(const SharedRoute& rt, int m, int n, int nart, bool warm_dirs) {
    if (warm_dirs && m + 2 <= rt.tile_rows && n + nart + 1 <= rt.tile_cols) return rt.nreg + 1;
    for (int i = 0; i < rt.nreg; ++i)
        if (rt.rows[i] == rt.tile_rows && rt.cols[i] == rt.tile_cols && !rt.type1[i] && m + 2 <= rt.rows[i] &&
            n + nart + 1 <= rt.cols[i])
            return i;
    int v = rt.nreg;
    long best = -1;
    for (int i = 0; i < rt.nreg; ++i)
        if (rt.rows[i] >= m + 2 && rt.cols[i] >= n + nart + 1 && !rt.type1[i]) {
            const long a = (long)rt.rows[i] * rt.cols[i];
            if (best < 0 || a < best) {
                best = a;
                v = i;
            }
        }
    return v;
}
// One workgroup: n_art from b and sense, the close pairs among the first
// 65 objectives (cosine > 0.9, warm when at least half are), then
// route_len[r] = count for the chosen route r and 0 for the others.
hipError_t launch_shared_route(int m, int n, int64_t count, const double* b, const int8_t* sense, const double* C,
                               const SharedRoute& rt, int32_t* route_len, hipStream_t s);
// list[q] = q for q < count
hipError_t launch_iota(int32_t* list, int64_t count, hipStream_t s);

// Shared-constraint kernel (simplex_reg.hip): tableau shape and launcher.
hipError_t launch_shared(const KParams& P, int grid, hipStream_t s);
const void* shared_kernel_ptr();
int shared_threads();
void shared_shape(int* rows, int* cols);

// Pivot trace of the 112 x 112 block tile (simplex_reg.hip): tr 1 records,
// tr 2 replays; 256 threads per workgroup, one LP per workgroup.
hipError_t launch_blk_trace(const KParams& P, int grid, hipStream_t s, int tr);
const void* blk_trace_kernel_ptr(int tr);
void blk_trace_shape(int* rows, int* cols);

// Lane kernel (simplex_lane.hip): launcher and kernel address of the
// variant with an R x C tile, NWV waves per workgroup, WPE waves per SIMD.
template <int R, int C, int NWV, int WPE>
hipError_t launch_lane(const KParams& P, int grid, hipStream_t s);
template <int R, int C, int NWV, int WPE>
const void* kernel_ptr_lane();

// Streaming kernel (simplex_gm.hip).
// deep: the launch's bin is known not to be empty: for tableaux of up to 512
// rows, more loads in flight per lane and on-chip columns in the dynamic LDS
// beyond the mirrors (P.ws_lds doubles; lds_bytes must cover both).
hipError_t launch_gm(const KParams& P, int grid, size_t lds_bytes, hipStream_t s, bool deep = false);
const void* gm_kernel_ptr(int ld, bool deep = false);
// allow `bytes` of dynamic LDS for both layouts' instantiations of a geometry
hipError_t gm_allow_lds(int ld, bool deep, int bytes);
// whether a deep instantiation exists for tableaux of `ld` rows
bool gm_has_deep(int ld);
int gm_threads();
size_t gm_lds_bytes_host(int ld, int cols);

}  // namespace blp
