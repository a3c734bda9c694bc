/*
 * blp -- batched linear programs on one AMD Instinct MI355X (gfx950).
 *
 * C ABI of the solver library (libblp.so).  It solves many independent LPs
 * in one call, each either
 *
 *   simplex kind:  maximise c.x  subject to  a_i.x <= b_i  or  a_i.x >= b_i
 *                  (one sense per row), x >= 0
 *                  -- the standard form of Gurung & Ray, "Solving Batched
 *                  Linear Programs on GPU and Multicore CPU", Sec. 3,
 *                  Eqs. (1)-(3), with ">=" rows (equivalently "<=" rows with
 *                  a negative right-hand side, Sec. 3) handled by the
 *                  two-phase method of Sec. 3;
 *   hyperbox kind: maximise c.x  subject to  l <= x <= u
 *                  -- solved by the closed form of Sec. 6, Eq. (7).
 *
 * Simplex LPs are solved by the dense-tableau simplex iteration of Sec. 3.1
 * (Steps 1-3 with the largest-coefficient entering rule of Sec. 4.2), one LP
 * per GPU workgroup as in Sec. 4.1, in FP64.
 *
 * Conventions shared by every entry point:
 *   - No call throws; each returns a blp_error.  Per-LP outcomes are the
 *     BLP_OPTIMAL.. status codes written to the status array, not errors.
 *   - A handle is not thread-safe: use one handle per host thread.
 *   - Pointers documented as "device" must be HIP device memory of the
 *     handle's device (e.g. torch.Tensor.data_ptr() of a CUDA/HIP tensor);
 *     "host" pointers are ordinary CPU memory.
 *   - Work is ordered on the HIP stream passed in (NULL = default stream);
 *     the caller keeps every input alive until that stream has passed the
 *     call.  A handle's calls reuse its device buffers: a call on another
 *     stream than the handle's previous call first waits (on the device)
 *     for that call's work.
 */
#ifndef BLP_H
#define BLP_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define BLP_ABI_VERSION 5

typedef struct blp_handle_s* blp_handle;

/* Row sense (int8 per row).  Any nonzero value is read as ">=". */
enum { BLP_LE = 0, BLP_GE = 1 };

/* LP kind (int32 per LP). */
enum { BLP_KIND_SIMPLEX = 0, BLP_KIND_HYPERBOX = 1 };

/* Per-LP status (int32 per LP). */
enum {
    BLP_OPTIMAL = 0,    /* optimum found (Sec. 3.1: no positive objective-row coefficient) */
    BLP_INFEASIBLE = 1, /* phase 1 ended above zero (Sec. 3), or a hyperbox with l_i > u_i */
    BLP_UNBOUNDED = 2,  /* no row limits the entering variable (Sec. 3.1) */
    BLP_ITER_LIMIT = 3, /* max_iter pivots done without reaching an optimum */
    BLP_NUMERICAL = 4   /* non-finite input or result */
};

/* Call-level error codes. */
typedef enum {
    BLP_SUCCESS = 0,
    BLP_ERR_ARG = 1,       /* invalid argument; nothing was launched */
    BLP_ERR_NOMEM = 2,     /* device or host allocation failed */
    BLP_ERR_HIP = 3,       /* a HIP runtime call failed (message in blp_last_error) */
    BLP_ERR_STATE = 4,     /* call out of order (e.g. backward before any solve) */
    BLP_ERR_TOO_LARGE = 5  /* an LP exceeds the supported size (see blp_solve_batch) */
} blp_error;

/* Scheduling modes.  They share the kernels and give identical results. */
enum {
    BLP_MODE_PERSISTENT = 0,      /* persistent workgroups pull LPs from size-binned device queues */
    BLP_MODE_GRID = 1,            /* one workgroup per LP, one launch per size bin (Sec. 4.1's layout) */
    BLP_MODE_ONE_PER_LAUNCH = 2   /* one kernel launch per LP (baseline for comparison) */
};

typedef struct {
    int32_t device;        /* HIP device ordinal */
    int32_t mode;          /* BLP_MODE_* */
    int32_t max_iter;      /* pivots per LP; 0 -> 50 (m + n) */
    int32_t bland_after;   /* consecutive zero-step pivots before the lowest-index
                              entering rule takes over; 0 -> max(m, n) */
    double eps_price;      /* entering threshold on reduced costs; 0 -> 1e-9 */
    double eps_piv;        /* minimum pivot-column entry in the ratio test; 0 -> 1e-9 */
    double eps_feas;       /* phase-1 zero test, relative to 1 + initial infeasibility; 0 -> 1e-9 */
    int32_t variant;       /* -1: automatic kernel choice per LP; >= 0 forces one
                              register-tile variant (index into the library's table)
                              and sends LPs that do not fit it to the streaming kernel;
                              -2 forces the streaming kernel for every simplex LP */
    int32_t workers_per_cu;/* persistent mode: workgroups per compute unit; 0 -> from occupancy */
    int32_t profile;       /* nonzero: record HIP events around each kernel class (blp_last_kernel_ms) */
    int32_t graph;         /* nonzero (persistent mode): capture the launch sequence into a hipGraph
                              per batch signature and replay it when the same batch recurs */
    int32_t pivot_rule;    /* BLP_RULE_LPC (default) or BLP_RULE_RPC */
    int32_t layout;        /* streaming kernel's workspace: BLP_LAYOUT_COLUMN (default, the coalesced
                              layout of Sec. 4.3) or BLP_LAYOUT_ROW (same thread mapping on a row-major
                              tableau: the non-coalesced access of Sec. 4.3's comparison).  Results are
                              bit-identical; only speed differs */
    uint64_t seed;         /* RPC only: Philox4x32-10 key; draw = (seed, LP index, pivot count) */
    uint64_t mem_limit;    /* 0: no limit.  Otherwise the bytes of device memory blp_solve_batch may
                              hold for one call: its own result buffers (for outputs passed as NULL),
                              the batch metadata and work lists, and the streaming kernel's
                              workspace.  A batch needing more is solved in consecutive chunks of
                              LPs, each the largest that fits (the batch capacity N = S / Y of
                              Sec. 4.5, Eq. (5), with S the limit and Y the bytes per LP); results
                              are identical.  BLP_ERR_NOMEM if the result buffers or a single LP do
                              not fit. */
    const char* tune_cache;/* NULL, or a file written by blp_autotune: blp_create loads it (same as
                              blp_load_tuning) and fails with its error if it cannot */
} blp_options;

/* Workspace layouts of the streaming kernel (Sec. 4.3). */
enum { BLP_LAYOUT_COLUMN = 0, BLP_LAYOUT_ROW = 1 };

/* Entering rules (Sec. 4.2).  LPC: largest positive reduced cost (Dantzig),
 * lowest variable index on ties.  RPC: a uniformly random column among those
 * with a positive reduced cost, drawn deterministically from Philox4x32-10
 * keyed by the seed and addressed by (LP index, pivot count); the optimum is
 * the same, the pivot path and count differ. */
enum { BLP_RULE_LPC = 0, BLP_RULE_RPC = 1 };

/* A batch.  LP k has m[k] rows and n[k] columns (hyperbox: m[k] = 0).
 * Metadata arrays are HOST memory; data arrays are DEVICE memory.
 *   A      float64, LP k's m x n matrix row-major at A + a_off[k]
 *   b      float64, length m at b + row_off[k]
 *   sense  int8,    length m at sense + row_off[k] (BLP_LE / BLP_GE)
 *   c      float64, length n at c + col_off[k]
 *   l, u   float64, length n at l/u + col_off[k] (hyperbox LPs only; may be
 *          NULL when the batch has none); with shared_box nonzero, one box
 *          of length n at l and u serves every hyperbox LP (all of them must
 *          then have the same n; the many-objectives use of Sec. 6)
 * If `uniform` is nonzero, every LP has m[0], n[0], kind[0] and the offsets
 * are the packed ones (a_off = k m n, row_off = k m, col_off = k n); the
 * offset arrays are then ignored.  Otherwise offsets may be NULL, meaning
 * packed in order (exclusive prefix sums of m n, m and n). */
typedef struct {
    int64_t count;
    int32_t uniform;
    int32_t shared_box;  /* nonzero: the hyperbox LPs share one box (see above) */
    const int32_t* m;
    const int32_t* n;
    const int32_t* kind;
    const int64_t* a_off;
    const int64_t* row_off;
    const int64_t* col_off;
    const double* A;
    const double* b;
    const int8_t* sense;
    const double* c;
    const double* l;
    const double* u;
} blp_batch;

/* Result buffers (DEVICE memory, caller-owned).  Any NULL field makes the
 * handle use its own buffer for that output.
 *   status int32 [count], iters int32 [count] (pivots), obj float64 [count]
 *   x      float64, length n at x + col_off[k]   (primal solution)
 *   y      float64, length m at y + row_off[k]   (y_i = d obj / d b_i)
 * obj is the optimum for BLP_OPTIMAL, the current value for BLP_ITER_LIMIT,
 * +inf for BLP_UNBOUNDED, -inf for BLP_INFEASIBLE and NaN for BLP_NUMERICAL. */
typedef struct {
    int32_t* status;
    int32_t* iters;
    double* obj;
    double* x;
    double* y;
} blp_outputs;

/* Fill *opt with the defaults (device 0, persistent mode, automatic kernels). */
blp_error blp_options_default(blp_options* opt);

/* Create a handle bound to opt->device (opt may be NULL for defaults).
 * The handle owns its device workspace and its own result buffers. */
blp_error blp_create(blp_handle* out, const blp_options* opt);

/* Solve every LP of the batch (stream-ordered; returns before the GPU is
 * done).  Sizes: simplex LPs need 1 <= m <= 2046 and 1 <= n with
 * n + m + 1 <= 4096 (the widest condensed tableau, one column per
 * structural variable and per possible artificial variable, plus the rhs);
 * hyperbox LPs need 1 <= n.  Violations found on the host return
 * BLP_ERR_ARG / BLP_ERR_TOO_LARGE before any launch.  `out` may be NULL.
 * The handle remembers the batch and output pointers for blp_backward and
 * blp_get_solution*, until the next solve. */
blp_error blp_solve_batch(blp_handle h, const blp_batch* batch, const blp_outputs* out, void* hip_stream);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the same
 * solve as blp_solve_batch, with every output buffer required (all five,
 * DEVICE memory) and everything else the solve needs on the device -- batch
 * metadata, work lists, bin counters, the streaming kernel's workspace --
 * taken from a static scratch array of BLP_STATIC_SCRATCH_BYTES per GPU
 * (held by every GPU the library runs on until the process ends).  Calls no
 * hipMalloc, hipFree or other allocating routine; launches eagerly on the
 * stream (the handle's graph and mem_limit options do not apply).  A batch
 * whose metadata and work lists (8 bytes per LP for a uniform batch, 48
 * otherwise) do not fit, or that leaves no room for one streaming workspace
 * slot when it needs one, fails with BLP_ERR_TOO_LARGE before any launch;
 * the streaming kernel runs as many workgroups as the remaining scratch
 * holds slots for (fewer workgroups, the same results).  Every call on a
 * GPU shares that GPU's scratch: calls that overlap on one GPU (on
 * different streams or handles) race and must be ordered by the caller, and
 * blp_backward and blp_get_solution* after this call read the batch
 * metadata from the scratch, so they must come before the next such call
 * on the GPU. */
#define BLP_STATIC_SCRATCH_BYTES (64ull << 20)
blp_error blp_solve_batch_static(blp_handle h, const blp_batch* batch, const blp_outputs* out, void* hip_stream);

/* BLP_STATIC_SCRATCH_BYTES as compiled into the library. */
size_t blp_static_scratch_bytes(void);

/* Host-resident batch with copy/compute overlap (the stream scheme of
 * Sec. 4.4).  Same batch description as blp_solve_batch except that the
 * data arrays (A, b, sense, c, l, u) are HOST memory (page-locked memory
 * gives asynchronous copies) and `out` points to HOST buffers (all five
 * required).  The batch is cut into `chunks` pieces (<= 0: automatic); each
 * piece's upload, solve and download are issued on one of two streams in
 * turn, so transfers of one piece overlap the kernels of the other.
 * Synchronous: returns when every result is in host memory.  Afterwards
 * blp_get_solution* and blp_backward refer to the last piece only. */
blp_error blp_solve_batch_host(blp_handle h, const blp_batch* batch, const blp_outputs* out, int32_t chunks);

/* Shared constraints, many objectives: maximise c_k.x subject to the same rows
 * A x (<= | >=) b and x >= 0, for k = 0..count-1 -- the support-function
 * sampling of Sec. 7, where one polytope is queried in many directions.
 * A (m x n, row-major), b (m), sense (m) and C (count x n, row-major) are
 * device pointers; out->status/iters/obj have count entries, out->x count x n
 * (x of LP k at k*n), out->y count x m (at k*m); all device, caller-owned
 * (C and out may be NULL when count is 0).
 * When consecutive objectives point in close directions (cosine > 0.9 for at
 * least half of the first 64 pairs), each workgroup runs phase 1 once and
 * starts every further objective whose direction is that close to the
 * previous one from the previous optimal basis (only the objective row is
 * rebuilt); other objectives, or every objective when the directions are
 * unrelated, are solved from scratch.  Iteration counts and, at degenerate
 * optima, x and y may therefore differ from independent solves; statuses and
 * optima do not.  Warm starts need m + 2 <= 112 and n + n_art + 1 <= 112
 * (n_art = rows whose "<=" form has a negative rhs); larger constraint sets,
 * up to the limits of blp_solve_batch (m <= 2046, n + m + 1 <= 4096, else
 * BLP_ERR_TOO_LARGE), are solved from scratch for every objective by the
 * smallest register-tile variant that holds them, else the streaming kernel.
 * The route (warm starts, a register variant, or the streaming kernel) is
 * chosen on the device from b, sense and the first 65 objectives, so the
 * call is ordered on the stream and reads nothing back; it allocates its
 * work buffers on first use and when count grows (a call whose count and
 * shape do not exceed an earlier one's allocates nothing, and can be
 * captured in a HIP graph).  A handle whose options force a register-tile
 * variant (variant >= 0) runs the cold solves with that variant, and fails
 * with BLP_ERR_TOO_LARGE if it cannot hold them; to know that, it reads b,
 * sense and the first 65 objectives back to the host once (synchronising
 * the stream).
 * The handle keeps no results of this call (blp_backward and
 * blp_get_solution refer to the last blp_solve_batch). */
blp_error blp_solve_shared(blp_handle h, int32_t m, int32_t n, const double* A, const double* b,
                           const int8_t* sense, int64_t count, const double* C, const blp_outputs* out,
                           void* hip_stream);

/* Adjoint of a blp_solve_shared call for loss = sum_k g[k] obj_k (an
 * extension beyond the paper, valid at non-degenerate optima), from that
 * call's outputs: status (count), x (count x n) and y (count x m).  With
 * w_k = g_k for LPs whose status is BLP_OPTIMAL, else 0:
 * dC = w_k x_k (count x n, row k at k*n), db = sum_k w_k y_k (m),
 * dA = -sum_k w_k y_k x_k^T (m x n, row-major).  All DEVICE memory, caller-
 * owned; any output may be NULL to skip it.  The sums over k run in a fixed
 * order (consecutive LPs in chunks, then the chunks in order), so repeated
 * calls give the same bits.  The handle keeps the partial sums (its
 * workspace grows as needed).  Stream-ordered.  Errors: BLP_ERR_ARG (sizes,
 * a NULL input), BLP_ERR_NOMEM. */
blp_error blp_backward_shared(blp_handle h, int32_t m, int32_t n, int64_t count, const int32_t* status,
                              const double* x, const double* y, const double* g, double* dC, double* db,
                              double* dA, void* hip_stream);

/* Copy LP k's results of the last solve to HOST memory (synchronises the
 * solve's stream).  x (length n) and y (length m) may be NULL. */
blp_error blp_get_solution(blp_handle h, int64_t k, int32_t* status, double* obj, double* x, double* y,
                           int32_t* iters);

/* Copy all results of the last solve, packed like the outputs: with
 * on_device == 0 to HOST memory (synchronises); otherwise to DEVICE memory,
 * ordered on the last solve's stream (returns at once).  Any pointer may be
 * NULL. */
blp_error blp_get_solution_batch(blp_handle h, int32_t* status, int32_t* iters, double* obj, double* x,
                                 double* y, int32_t on_device);

/* Adjoint of the last solve for loss = sum_k g[k] obj_k (an extension beyond
 * the paper; valid at non-degenerate optima where x* and y* are unique).
 * All pointers are DEVICE memory, packed like the batch; any output may be
 * NULL to skip it.  Simplex LP k:  dc = g_k x*,  db = g_k y*,
 * dA = -g_k y* x*^T (row-major at a_off[k]).  Hyperbox LP k:  dc = g_k h,
 * dl_i = g_k min(c_i, 0),  du_i = g_k max(c_i, 0); with a shared box, dl and
 * du have length n and hold the sums of those terms over the hyperbox LPs,
 * added in a fixed order (blocks of 1,024 consecutive LPs, each reduced by a
 * fixed tree, then the block sums in block order), so repeated calls give
 * the same bits.  LPs whose status is not BLP_OPTIMAL get zero gradients.
 * After a solve that mem_limit split into chunks: BLP_ERR_STATE. */
blp_error blp_backward(blp_handle h, const double* g, double* dc, double* db, double* dA, double* dl,
                       double* du, void* hip_stream);

/* Pivot trace of the 100 x 100 class's kernel (the 112 x 112 block tile),
 * to time the rank-1 update of Step 3 (Sec. 4.3) apart from the search of
 * Steps 1 and 2 (Sec. 4.2).  The batch (DEVICE data) must be uniform, simplex
 * LPs only, with m + 2 <= 112 and n + 1 <= 112, and the handle's rule LPC.
 * trace: DEVICE array of count * stride int32, 1 <= stride <= 513; LP k's
 * record at trace + k * stride is [p, l_0, e_0, ..., l_{p-1}, e_{p-1}]: the
 * number of pivots, then each pivot's leaving row and entering slot of the
 * condensed tableau (slot j < n holds structural variable j until a pivot
 * brings another variable there; the slot takes the leaving variable).
 * replay == 0: solve the batch and record every LP's pivots (p = -1 if the
 * LP's data are not finite or its pivots do not fit the stride).
 * replay != 0: solve the batch taking each pivot from the record instead of
 * Steps 1 and 2 (an LP with artificial rows or an invalid record gets status
 * -1 and NaN outputs); for an LP the record run solved to BLP_OPTIMAL the
 * outputs are bit-identical to that run's.  Outputs as in blp_solve_batch;
 * the call is a solve for blp_get_solution and blp_backward.  Stream-ordered;
 * the caller owns `trace`.  Errors: BLP_ERR_ARG (shape, rule, stride, a
 * handle with mem_limit), as blp_solve_batch otherwise. */
blp_error blp_pivot_trace(blp_handle h, const blp_batch* batch, const blp_outputs* out, int32_t* trace,
                          int32_t stride, int32_t replay, void* hip_stream);

/* Number of simplex LPs of the last solve handled by each kernel class:
 * counts[0..n_reg-1] register-tile variants, counts[n_reg] streaming
 * kernel, counts[n_reg+1] hyperbox.  Synchronises.  *n_classes receives
 * n_reg + 2; counts may be NULL to query that number only. */
blp_error blp_last_bins(blp_handle h, int64_t* counts, int32_t* n_classes);

/* Device time of each kernel class in the last solve, from HIP events
 * recorded on the solve's stream around that class's launches (only when
 * the handle was created with opt->profile != 0; otherwise all zero).
 * ms[0..n_reg-1] register-tile variants, ms[n_reg] streaming kernel,
 * ms[n_reg+1] hyperbox kernel, ms[n_reg+2] work-list construction.
 * Synchronises.  *n_entries receives n_reg + 3; ms may be NULL. */
blp_error blp_last_kernel_ms(blp_handle h, double* ms, int32_t* n_entries);

/* Autotuner.  Classifies `batch` (DEVICE data as for blp_solve_batch), then
 * for every size bin that received LPs times each kernel variant able to
 * hold that bin's LPs (register-tile variants of equal or larger shape, and
 * the streaming kernel) on up to `sample` of its LPs, and remaps the bin to
 * the fastest.  The remap applies to later solves on this handle.  Results
 * never depend on it: every variant computes bit-identical outputs.  If
 * cache_path is non-NULL the table is also written there as JSON.
 * Synchronises the stream. */
blp_error blp_autotune(blp_handle h, const blp_batch* batch, int32_t sample, const char* cache_path,
                       void* hip_stream);

/* Load a table written by blp_autotune (same device name and CU count). */
blp_error blp_load_tuning(blp_handle h, const char* cache_path);

/* Current remap: remap[v] is the variant used for LPs whose best-fitting
 * variant is v (v in [0, n_reg)); a value n_reg means the streaming kernel.
 * *n_reg receives the number of register-tile variants. */
blp_error blp_tuning(blp_handle h, int32_t* remap, int32_t* n_reg);

/* Name and maximum tableau shape (rows incl. objective rows, columns incl.
 * rhs) of register-tile variant v; returns BLP_ERR_ARG past the end. */
blp_error blp_variant_info(int32_t v, char* name, int32_t name_len, int32_t* max_rows, int32_t* max_cols);

/* Message of the last failed call on this handle ("" if none). */
const char* blp_last_error(blp_handle h);

/* Release the handle and its device memory (synchronises its device). */
void blp_destroy(blp_handle h);

/* BLP_ABI_VERSION of the library. */
int32_t blp_abi_version(void);

#ifdef __cplusplus
}
#endif

#endif /* BLP_H */
