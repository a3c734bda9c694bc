// Host runtime behind the C ABI of include/blp.h: argument validation, device
// buffers, the size-binned work lists and the kernel launch sequence.
//
// A solve is, on one stream:
//   reset counters -> classify (bin per LP) -> bin offsets -> scatter (work
//   lists) -> one persistent launch per register-tile variant that can
//   receive LPs -> persistent streaming kernel -> hyperbox kernel.
// The persistent kernels pop LP indices from their bin with an atomic head,
// so the host never waits for the device in the default mode.  The grid and
// one-LP-per-launch modes read the bins back to size their launches.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <mutex>
#include <string>
#include <vector>

#include "aux_kernels.hpp"
#include "blp.h"
#include "blp_kernels.hpp"
#include "host_plan.hpp"
#include "variants.hpp"

using namespace blp;

namespace {

struct DevBuf {
    void* p = nullptr;
    size_t bytes = 0;
    // exact: allocate `want` bytes, not the 1.5x growth (memory-limited handles)
    hipError_t reserve(size_t want, bool exact = false) {
        if (want <= bytes) return hipSuccess;
        if (p) {
            hipError_t e = hipFree(p);
            if (e != hipSuccess) return e;
            p = nullptr;
            bytes = 0;
        }
        size_t cap = exact ? want : std::max(want, bytes + bytes / 2);
        hipError_t e = hipMalloc(&p, cap);
        if (e != hipSuccess) {
            p = nullptr;
            return e;
        }
        bytes = cap;
        return hipSuccess;
    }
    void release() {
        if (p) (void)hipFree(p);
        p = nullptr;
        bytes = 0;
    }
    template <class T>
    T* as() const {
        return static_cast<T*>(p);
    }
};

// Bump allocator over one caller-independent device region (the static
// scratch array of the allocation-free entry point): hands out 256-byte
// aligned pieces, never frees.
// Bin counters of a solve, in ints: bin_len, bin_fill and bin_off (nbins
// each), the work-list heads from heads_at(nbins) on (kHeadStride apart,
// each on a cache line of its own), then kBinStripes striped copies of the
// bin counts (kStripeStride apart).  The buffer is 256-byte aligned.
static size_t heads_at(int nbins) { return ((size_t)3 * nbins + kHeadStride - 1) / kHeadStride * kHeadStride; }
static size_t stripes_at(int nbins) { return heads_at(nbins) + (size_t)kHeadStride * nbins; }
static size_t counter_ints(int nbins) { return stripes_at(nbins) + (size_t)kBinStripes * kStripeStride; }

struct Arena {
    char* base = nullptr;
    size_t cap = 0, used = 0;
    void* take(size_t bytes) {
        const size_t at = (used + 255) & ~size_t(255);
        if (at > cap || bytes > cap - at) return nullptr;
        used = at + bytes;
        return base + at;
    }
    size_t left() const {
        const size_t at = (used + 255) & ~size_t(255);
        return at < cap ? cap - at : 0;
    }
};

// The allocation-free entry point's scratch: one copy of this array per
// GPU, kept until the process ends.  Host code never uses the array's name
// as a device address: each device's address is resolved once, with that
// device current, by blp_create (scratch_ptr below).
constexpr size_t kStaticScratchBytes = (size_t)BLP_STATIC_SCRATCH_BYTES;
constexpr int kMaxDevices = 64;
static __device__ __align__(256) char scratch[kStaticScratchBytes];
std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxDevices] = {};

// Device address of `scratch` on `device` (which must be current).
hipError_t scratch_ptr(int device, void** out) {
    *out = nullptr;
    if (device < 0 || device >= kMaxDevices) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_ptr[device]) {
        void* p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return e;
        g_scratch_ptr[device] = p;
    }
    *out = g_scratch_ptr[device];
    return hipSuccess;
}

}  // namespace

struct blp_handle_s {
    blp_options opt;
    std::string err;
    int cu_count = 0;
    size_t lds_per_cu = 0, lds_per_block = 0;  // bytes
    const RegVariant* variants = nullptr;
    int nreg = 0;
    void* scratch = nullptr;  // this device's copy of the static scratch (allocation-free entry point)
    std::vector<int> reg_workers;  // persistent grid per variant
    int gm_occ = 1;
    int direct_v = -1;  // the last solve's one-launch variant (no binning), or -1
    // device buffers
    DevBuf meta;     // m, n, kind (int32) + a_off, row_off, col_off (int64) for non-uniform batches
    DevBuf counters; // bin counters of the last solve (layout: counter_ints)
    DevBuf binid, list;
    DevBuf olist;  // non-uniform batches: the work lists in largest-first order (what the kernels pop)
    DevBuf ws;       // streaming-kernel workspace
    DevBuf own_status, own_iters, own_obj, own_x, own_y;
    // last solve
    bool solved = false;
    KParams last{};
    hipStream_t last_stream = nullptr;
    // Every call's device work reuses the handle's buffers.  order_ev is
    // recorded at the end of each call's work (unless that stream was being
    // captured); a call on another stream first waits for it.
    hipEvent_t order_ev = nullptr;
    bool order_pending = false;
    Plan plan;  // host metadata of the last solve (plan_batch)
    int64_t count = 0;
    bool uniform = false;
    bool any_simplex = false, any_box = false;
    int64_t n_box = 0;
    bool box_shared = false;
    int32_t box_n = 0;      // n of the hyperbox LPs sharing one box
    bool chunked = false;   // the last solve was split by mem_limit
    DevBuf bwd_part;        // shared-box adjoint: per-block partial sums
#ifdef BLP_PHASE_TIMERS
    unsigned long long* timers = nullptr;
#endif
    // kernel-variant remap (autotuner); identity by default
    int remap[kMaxVariants] = {};
    int tuned_deep = -1;  // streaming kernel's loads in flight: -1 automatic, 0 eight, 1 thirty-two
    // captured launch sequence of the last persistent solve
    hipGraphExec_t graph_exec = nullptr;
    std::vector<uint64_t> graph_sig;
    hipStream_t cap_stream = nullptr;
    // persistent kernel classes of a mixed batch run concurrently: forked
    // from the solve stream onto these (default priority) and joined back
    static constexpr int kForks = 3;
    hipStream_t fork[kForks] = {nullptr, nullptr, nullptr};
    hipEvent_t fork_ev = nullptr, join_ev[kForks] = {nullptr, nullptr, nullptr};
    // created once, by blp_create (never inside a capture or a solve)
    hipError_t create_forks() {
        for (int i = 0; i < kForks; ++i) {
            if (!fork[i]) {
                hipError_t e = hipStreamCreateWithFlags(&fork[i], hipStreamNonBlocking);
                if (e != hipSuccess) return e;
            }
            if (!join_ev[i]) {
                hipError_t e = hipEventCreateWithFlags(&join_ev[i], hipEventDisableTiming);
                if (e != hipSuccess) return e;
            }
        }
        if (!fork_ev) return hipEventCreateWithFlags(&fork_ev, hipEventDisableTiming);
        return hipSuccess;
    }
    DevBuf tune;  // autotuner scratch (sample list + counters)
    DevBuf shared_ctr;  // blp_solve_shared: route lengths, zero offsets and queue heads
    DevBuf shared_list; // blp_solve_shared: the identity work list (shared_list_n entries filled)
    int64_t shared_list_n = 0;
    DevBuf shared_ws;   // blp_solve_shared: streaming workspace of the cold route
    // host-resident pipeline: two child handles (own buffers), two streams,
    // two device input/output sets
    blp_handle_s* child[2] = {nullptr, nullptr};
    hipStream_t pipe[2] = {nullptr, nullptr};
    DevBuf pin_in[2], pin_out[2];
    // profiling events: one start/stop pair per kernel class (+1 for binning)
    std::vector<hipEvent_t> ev0, ev1;
    std::vector<char> ev_used;
    // created by blp_create (all classes + binning); later calls only reset
    // the used flags
    hipError_t ensure_events(int n) {
        while ((int)ev0.size() < n) {
            hipEvent_t a, b;
            hipError_t e = hipEventCreate(&a);
            if (e != hipSuccess) return e;
            e = hipEventCreate(&b);
            if (e != hipSuccess) return e;
            ev0.push_back(a);
            ev1.push_back(b);
        }
        ev_used.assign(n, 0);
        return hipSuccess;
    }
    hipError_t mark(int cls, bool start, hipStream_t s) {
        if (!opt.profile) return hipSuccess;
        if (start) ev_used[cls] = 1;
        return hipEventRecord(start ? ev0[cls] : ev1[cls], s);
    }
};

static blp_error fail(blp_handle h, blp_error code, const char* fmt, ...);

// Can variant w (nreg: the streaming kernel) take every LP that the
// scheduler sends to variant v?
static bool can_replace(blp_handle h, int w, int v) {
    if (w >= h->nreg) return true;
    return h->variants[w].max_rows >= h->variants[v].max_rows && h->variants[w].max_cols >= h->variants[v].max_cols &&
           (!h->variants[w].type1_only || h->variants[v].type1_only);
}

// Smallest batch for which the automatic choice may use variant v: a variant
// that packs several LPs into a workgroup (the lane kernel, 64 per wave)
// needs a quarter of its workgroups per CU to beat one LP per wave; smaller
// batches leave most of the GPU idle with it.
static int64_t auto_min_count(blp_handle h, int v) {
    const int64_t per = h->variants[v].lps_per_block;
    return per > 1 ? per * h->cu_count / 4 : 0;
}

// Persistent grid of register variant v for `lps` LPs: its occupancy-sized
// worker count, but no more workgroups than the LPs fill.
static int reg_grid(blp_handle h, int v, int64_t lps) {
    const int64_t per = h->variants[v].lps_per_block;
    const int64_t need = (lps + per - 1) / per;
    return (int)std::max<int64_t>(1, std::min<int64_t>(h->reg_workers[v], need));
}

// Order this call's work after the previous call's (see order_ev).
static hipError_t begin_call(blp_handle h, hipStream_t s) {
    if (h->order_pending && s != h->last_stream) return hipStreamWaitEvent(s, h->order_ev, 0);
    return hipSuccess;
}
static hipError_t end_call(blp_handle h, hipStream_t s) {
    hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
    hipError_t e = hipStreamIsCapturing(s, &cs);
    if (e != hipSuccess) return e;
    h->last_stream = s;
    h->order_pending = false;
    if (cs != hipStreamCaptureStatusNone) return hipSuccess;
    e = hipEventRecord(h->order_ev, s);
    h->order_pending = e == hipSuccess;
    return e;
}
// Host wait for the last call's device work.
static hipError_t wait_last(blp_handle h) {
    return h->order_pending ? hipEventSynchronize(h->order_ev) : hipStreamSynchronize(h->last_stream);
}

static blp_error fail(blp_handle h, blp_error code, const char* fmt, ...) {
    if (h) {
        char buf[512];
        va_list ap;
        va_start(ap, fmt);
        vsnprintf(buf, sizeof buf, fmt, ap);
        va_end(ap);
        h->err = buf;
    }
    return code;
}

#define HIP_TRY(h, expr)                                                                           \
    do {                                                                                           \
        hipError_t e_ = (expr);                                                                    \
        if (e_ != hipSuccess)                                                                      \
            return fail(h, e_ == hipErrorOutOfMemory ? BLP_ERR_NOMEM : BLP_ERR_HIP, "%s: %s (%s)", \
                        #expr, hipGetErrorString(e_), hipGetErrorName(e_));                        \
    } while (0)

extern "C" {

int32_t blp_abi_version(void) { return BLP_ABI_VERSION; }

blp_error blp_options_default(blp_options* opt) {
    if (!opt) return BLP_ERR_ARG;
    std::memset(opt, 0, sizeof *opt);
    opt->device = 0;
    opt->mode = BLP_MODE_PERSISTENT;
    opt->variant = -1;
    return BLP_SUCCESS;
}

blp_error blp_variant_info(int32_t v, char* name, int32_t name_len, int32_t* max_rows, int32_t* max_cols) {
    int nreg = 0;
    const RegVariant* t = reg_variants(&nreg);
    if (v < 0 || v >= nreg) return BLP_ERR_ARG;
    if (name && name_len > 0) {
        std::strncpy(name, t[v].name, (size_t)name_len - 1);
        name[name_len - 1] = 0;
    }
    if (max_rows) *max_rows = t[v].max_rows;
    if (max_cols) *max_cols = t[v].max_cols;
    return BLP_SUCCESS;
}

blp_error blp_create(blp_handle* out, const blp_options* opt) {
    if (!out) return BLP_ERR_ARG;
    *out = nullptr;
    blp_options o;
    blp_options_default(&o);
    if (opt) o = *opt;
    if (o.mode < 0 || o.mode > 2 || o.variant < -2 || o.workers_per_cu < 0) return BLP_ERR_ARG;
    if (o.pivot_rule != BLP_RULE_LPC && o.pivot_rule != BLP_RULE_RPC) return BLP_ERR_ARG;
    if (o.layout != BLP_LAYOUT_COLUMN && o.layout != BLP_LAYOUT_ROW) return BLP_ERR_ARG;
    if (!(o.eps_price >= 0) || !(o.eps_piv >= 0) || !(o.eps_feas >= 0)) return BLP_ERR_ARG;
    int ndev = 0;
    if (hipGetDeviceCount(&ndev) != hipSuccess || ndev <= 0) return BLP_ERR_HIP;
    if (o.device < 0 || o.device >= ndev) return BLP_ERR_ARG;
    if (hipSetDevice(o.device) != hipSuccess) return BLP_ERR_HIP;
    blp_handle h = new (std::nothrow) blp_handle_s();
    if (!h) return BLP_ERR_NOMEM;
    h->opt = o;
    if (h->opt.eps_price == 0) h->opt.eps_price = 1e-9;
    if (h->opt.eps_piv == 0) h->opt.eps_piv = 1e-9;
    if (h->opt.eps_feas == 0) h->opt.eps_feas = 1e-9;
    hipDeviceProp_t prop;
    if (hipGetDeviceProperties(&prop, o.device) != hipSuccess) {
        delete h;
        return BLP_ERR_HIP;
    }
    h->cu_count = prop.multiProcessorCount;
    h->lds_per_cu = prop.maxSharedMemoryPerMultiProcessor;
    h->lds_per_block = std::max(prop.sharedMemPerBlock, prop.sharedMemPerBlockOptin);
    h->variants = reg_variants(&h->nreg);
    for (int v = 0; v < kMaxVariants; ++v) h->remap[v] = v;
    if (o.variant >= h->nreg || h->nreg > kMaxVariants) {
        delete h;
        return BLP_ERR_ARG;
    }
    for (int v = 0; v < h->nreg; ++v) {
        int occ = 0;
        if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&occ, h->variants[v].kernel(), h->variants[v].threads, 0) !=
                hipSuccess ||
            occ < 1)
            occ = 1;
        if (o.workers_per_cu > 0) occ = std::min(occ, (int)o.workers_per_cu);
        h->reg_workers.push_back(occ * h->cu_count);
    }
#ifdef BLP_PHASE_TIMERS
    if (hipMalloc(&h->timers, TM_SLOTS * sizeof(unsigned long long)) == hipSuccess)
        (void)hipMemset(h->timers, 0, TM_SLOTS * sizeof(unsigned long long));
#endif
    // Streams and events the solves use are made here, once: never lazily
    // inside a solve (which may run under a caller's stream capture) and
    // never by the allocation-free entry point.
    hipError_t ce = h->create_forks();
    if (ce == hipSuccess) ce = hipEventCreateWithFlags(&h->order_ev, hipEventDisableTiming);
    if (ce == hipSuccess) ce = scratch_ptr(o.device, &h->scratch);
    if (ce == hipSuccess && h->opt.profile) ce = h->ensure_events(h->nreg + 3);
    if (ce != hipSuccess) {
        blp_destroy(h);
        return ce == hipErrorOutOfMemory ? BLP_ERR_NOMEM : BLP_ERR_HIP;
    }
    if (o.tune_cache) {
        const blp_error te = blp_load_tuning(h, o.tune_cache);
        if (te != BLP_SUCCESS) {
            blp_destroy(h);
            return te;
        }
    }
    h->opt.tune_cache = nullptr;  // the caller's string is not kept
    *out = h;
    return BLP_SUCCESS;
}

void blp_destroy(blp_handle h) {
    if (!h) return;
    (void)hipSetDevice(h->opt.device);
    (void)hipDeviceSynchronize();
#ifdef BLP_PHASE_TIMERS
    if (h->timers) {
        unsigned long long t[TM_SLOTS] = {};
        (void)hipMemcpy(t, h->timers, sizeof t, hipMemcpyDeviceToHost);
        fprintf(stderr,
                "[blp timers] LPs %llu pivots %llu | cycles per LP: load %.0f extract %.0f | per pivot: price %.0f "
                "pubcol %.0f ratio %.0f pivot %.0f | ratio test %.0f, division %.0f over %llu owned pivots | "
                "load: rows %.0f, tile %.0f\n",
                t[TM_LPS], t[TM_PIVOTS], t[TM_LPS] ? (double)t[TM_LOAD] / t[TM_LPS] : 0.0,
                t[TM_LPS] ? (double)t[TM_EXTRACT] / t[TM_LPS] : 0.0,
                t[TM_PIVOTS] ? (double)t[TM_PRICE] / t[TM_PIVOTS] : 0.0,
                t[TM_PIVOTS] ? (double)t[TM_PUBCOL] / t[TM_PIVOTS] : 0.0,
                t[TM_PIVOTS] ? (double)t[TM_RATIO] / t[TM_PIVOTS] : 0.0,
                t[TM_PIVOTS] ? (double)t[TM_PIVOT] / t[TM_PIVOTS] : 0.0,
                t[TM_PIVOTS] ? (double)t[TM_RTEST] / t[TM_PIVOTS] : 0.0,
                t[TM_DIVN] ? (double)t[TM_DIV] / t[TM_DIVN] : 0.0, t[TM_DIVN],
                t[TM_LPS] ? (double)t[TM_LD_ROWS] / t[TM_LPS] : 0.0, t[TM_LPS] ? (double)t[TM_LD_TILE] / t[TM_LPS] : 0.0);
        (void)hipFree(h->timers);
    }
#endif
    // the captured launch sequence and the streams/events go before the
    // buffers its kernels reference
    if (h->graph_exec) (void)hipGraphExecDestroy(h->graph_exec);
    h->graph_exec = nullptr;
    if (h->cap_stream) (void)hipStreamDestroy(h->cap_stream);
    h->cap_stream = nullptr;
    for (int i = 0; i < blp_handle_s::kForks; ++i) {
        if (h->fork[i]) (void)hipStreamDestroy(h->fork[i]);
        if (h->join_ev[i]) (void)hipEventDestroy(h->join_ev[i]);
    }
    if (h->fork_ev) (void)hipEventDestroy(h->fork_ev);
    if (h->order_ev) (void)hipEventDestroy(h->order_ev);
    for (auto e : h->ev0) (void)hipEventDestroy(e);
    for (auto e : h->ev1) (void)hipEventDestroy(e);
    h->meta.release();
    h->counters.release();
    h->binid.release();
    h->list.release();
    h->olist.release();
    h->ws.release();
    h->own_status.release();
    h->own_iters.release();
    h->own_obj.release();
    h->own_x.release();
    h->own_y.release();
    h->tune.release();
    for (int i = 0; i < 2; ++i) {
        if (h->child[i]) blp_destroy(h->child[i]);
        if (h->pipe[i]) (void)hipStreamDestroy(h->pipe[i]);
        h->pin_in[i].release();
        h->pin_out[i].release();
    }
    h->shared_ctr.release();
    h->shared_list.release();
    h->shared_ws.release();
    h->bwd_part.release();
    delete h;
}

const char* blp_last_error(blp_handle h) { return h ? h->err.c_str() : "null handle"; }

// Dynamic LDS of a streaming launch: the mirrors, and for the deep
// instantiation (a bin known to hold LPs) on-chip tableau columns in what the
// CU's LDS has left at the kernel's register-limited occupancy, less 16 KiB
// when workgroups of register kernels may share the CU (`shared`).  Sets
// *bytes, *tab (doubles of on-chip columns) and *occ (workgroups per CU, at
// least 1).
static void gm_lds_plan(blp_handle h, int ld, int cols, bool deep, bool shared, size_t* bytes, int32_t* tab,
                        int* occ) {
    const void* fn = gm_kernel_ptr(ld, deep);
    const size_t mirrors = gm_lds_bytes_host(ld, cols);
    *bytes = mirrors;
    *tab = 0;
    *occ = 1;
    int o = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&o, fn, gm_threads(), mirrors) != hipSuccess || o < 1) return;
    *occ = o;
    hipFuncAttributes fa{};
    if (!deep || !gm_has_deep(ld) || hipFuncGetAttributes(&fa, fn) != hipSuccess) return;
    const size_t kReserve = shared ? (16u << 10) : 0;
    const size_t per = std::min(h->lds_per_cu / (size_t)o, h->lds_per_block);
    if (per <= mirrors + fa.sharedSizeBytes + kReserve + 1024) return;
    const size_t t = (per - mirrors - fa.sharedSizeBytes - kReserve) / sizeof(double);
    const size_t want = mirrors + sizeof(double) * t;
    int o2 = 0;
    if (gm_allow_lds(ld, deep, (int)want) != hipSuccess ||
        hipOccupancyMaxActiveBlocksPerMultiprocessor(&o2, fn, gm_threads(), want) != hipSuccess || o2 < o) {
        (void)hipGetLastError();
        return;
    }
    *bytes = want;
    *tab = (int32_t)t;
}

// Everything one solve needs after validation.
struct SolvePlan {
    KParams P{};
    bool uni = false, any_simplex = false, any_box = false, box_only_uniform = false;
    int64_t n_box = 0;
    int gm_ld = 0, gm_cols = 0, gm_workers = 0;
    bool gm_deep = false;  // the streaming kernel's deep instantiation (deep loads, on-chip columns)
    bool gm_shared = false;  // register kernels may run beside it (keep LDS for them)
    size_t gm_lds = 0;
    std::vector<char> maybe;  // register variants that can receive LPs
    int direct_v = -1;        // >= 0: one launch of this variant, LP k in workgroup k, no binning
    bool may_stream = false;  // some simplex LP may reach the streaming kernel
    // device buffers of this solve (the handle's own, or carved from an arena)
    int32_t* counters = nullptr;
    int32_t* binid = nullptr;
    int32_t* list = nullptr;   // unordered work lists (scatter output)
    int32_t* olist = nullptr;  // largest-first work lists (non-uniform batches)
    int32_t box_n = 0;         // shared box: its length
};

// A device buffer for one solve: the handle's growable buffer `own`, or,
// with an arena (the allocation-free entry point), a piece of the arena.
#define BUF_TRY(h, arena, own, bytes, ptr)                                                              \
    do {                                                                                             \
        const size_t want_ = (bytes);                                                                \
        if (arena) {                                                                                 \
            void* p_ = (arena)->take(want_);                                                         \
            if (!p_)                                                                                 \
                return fail(h, BLP_ERR_TOO_LARGE,                                                    \
                            "static scratch of %zu bytes exhausted (%s needs %zu more bytes)",      \
                            (arena)->cap, #own, want_);                                              \
            (ptr) = static_cast<decltype(ptr)>(p_);                                                  \
        } else {                                                                                     \
            HIP_TRY(h, (own).reserve(want_, (h)->opt.mem_limit > 0));                                \
            (ptr) = static_cast<decltype(ptr)>((own).p);                                             \
        }                                                                                            \
    } while (0)

// Validation, outputs, metadata upload, workspace sizing.  No kernel launch.
// stream_all: size the streaming workspace as if every simplex LP could reach
// the streaming kernel (the autotuner times it on register-variant samples).
// arena: the allocation-free entry point's scratch (every output must then
// be given; nothing is allocated).
// ws_budget (memory-limited handles): bytes the streaming workspace may take.
static blp_error prepare(blp_handle h, const blp_batch* B, const blp_outputs* out, hipStream_t s, SolvePlan& sp,
                         bool stream_all = false, Arena* arena = nullptr, size_t ws_budget = 0) {
    const int64_t K = B->count;
    const bool uni = B->uniform != 0;
    // per-class kernel times report this solve's classes only
    std::fill(h->ev_used.begin(), h->ev_used.end(), (char)0);
    std::vector<VariantShape> shapes((size_t)h->nreg);
    bool remap_streams = false;
    for (int v = 0; v < h->nreg; ++v) {
        shapes[v] = {h->variants[v].max_rows, h->variants[v].max_cols, h->variants[v].type1_only,
                     auto_min_count(h, v)};
        remap_streams |= h->remap[v] >= h->nreg;
    }
    PlanIn in;
    in.count = K;
    in.uniform = uni;
    in.shared_box = B->shared_box != 0;
    in.m = B->m;
    in.n = B->n;
    in.kind = B->kind;
    in.a_off = B->a_off;
    in.row_off = B->row_off;
    in.col_off = B->col_off;
    in.has_A = B->A;
    in.has_b = B->b;
    in.has_sense = B->sense;
    in.has_c = B->c;
    in.has_l = B->l;
    in.has_u = B->u;
    in.variants = shapes.data();
    in.nreg = h->nreg;
    in.force = h->opt.variant;
    in.remap_streams = remap_streams;
    in.lpc = h->opt.pivot_rule == BLP_RULE_LPC;
    in.stream_all = stream_all;
    Plan& pl = h->plan;
    if (plan_batch(in, pl) != PLAN_OK) return fail(h, (blp_error)pl.code, "%s", pl.msg.c_str());
    const bool any_simplex = pl.any_simplex, any_box = pl.any_box;
    const int64_t n_box = pl.n_box, tot_m = pl.tot_m, tot_n = pl.tot_n, max_slot = pl.max_slot;
    const int64_t n_may_stream = pl.n_may_stream;
    sp.may_stream = n_may_stream > 0;
    const int max_m = pl.max_m, max_cols = pl.max_cols;
    // deep when some LP cannot be held by any register tile (the streaming
    // bin is not empty), unless the autotuner chose
    sp.gm_deep = h->tuned_deep >= 0 ? h->tuned_deep != 0 : pl.gm_deep;
    sp.box_n = pl.box_n;

    // ---- outputs
    blp_outputs o{};
    if (out) o = *out;
    if (arena && (!o.status || !o.iters || !o.obj || !o.x || !o.y))
        return fail(h, BLP_ERR_ARG, "all five output buffers are required");
    if (!o.status) {
        HIP_TRY(h, h->own_status.reserve(sizeof(int32_t) * K));
        o.status = h->own_status.as<int32_t>();
    }
    if (!o.iters) {
        HIP_TRY(h, h->own_iters.reserve(sizeof(int32_t) * K));
        o.iters = h->own_iters.as<int32_t>();
    }
    if (!o.obj) {
        HIP_TRY(h, h->own_obj.reserve(sizeof(double) * K));
        o.obj = h->own_obj.as<double>();
    }
    if (!o.x) {
        HIP_TRY(h, h->own_x.reserve(sizeof(double) * std::max<int64_t>(1, tot_n)));
        o.x = h->own_x.as<double>();
    }
    if (!o.y) {
        HIP_TRY(h, h->own_y.reserve(sizeof(double) * std::max<int64_t>(1, tot_m)));
        o.y = h->own_y.as<double>();
    }

    // ---- kernel parameters
    KParams& P = sp.P;
    P = KParams{};
    P.count = K;
    P.uniform = uni ? 1 : 0;
    P.um = h->plan.m[0];
    P.un = h->plan.n[0];
    P.ukind = h->plan.kind[0];
    if (!uni) {
        const size_t bytes = (size_t)K * (3 * sizeof(int32_t) + 3 * sizeof(int64_t));
        char* base = nullptr;
        BUF_TRY(h, arena, h->meta, bytes, base);
        int64_t* offs = reinterpret_cast<int64_t*>(base);
        int32_t* ints = reinterpret_cast<int32_t*>(base + (size_t)K * 3 * sizeof(int64_t));
        HIP_TRY(h, hipMemcpyAsync(offs, pl.a_off.data(), K * sizeof(int64_t), hipMemcpyHostToDevice, s));
        HIP_TRY(h, hipMemcpyAsync(offs + K, pl.row_off.data(), K * sizeof(int64_t), hipMemcpyHostToDevice, s));
        HIP_TRY(h, hipMemcpyAsync(offs + 2 * K, pl.col_off.data(), K * sizeof(int64_t), hipMemcpyHostToDevice, s));
        HIP_TRY(h, hipMemcpyAsync(ints, pl.m.data(), K * sizeof(int32_t), hipMemcpyHostToDevice, s));
        HIP_TRY(h, hipMemcpyAsync(ints + K, pl.n.data(), K * sizeof(int32_t), hipMemcpyHostToDevice, s));
        HIP_TRY(h, hipMemcpyAsync(ints + 2 * K, pl.kind.data(), K * sizeof(int32_t), hipMemcpyHostToDevice, s));
        P.a_off = offs;
        P.row_off = offs + K;
        P.col_off = offs + 2 * K;
        P.m = ints;
        P.n = ints + K;
        P.kind = ints + 2 * K;
    }
    P.A = B->A;
    P.b = B->b;
    P.sense = B->sense;
    P.c = B->c;
    P.l = B->l;
    P.u = B->u;
    P.status = o.status;
    P.iters = o.iters;
    P.obj = o.obj;
    P.x = o.x;
    P.y = o.y;
    P.max_iter = h->opt.max_iter;
    P.bland_after = h->opt.bland_after;
    P.eps_price = h->opt.eps_price;
    P.eps_piv = h->opt.eps_piv;
    P.eps_feas = h->opt.eps_feas;
    P.pivot_rule = h->opt.pivot_rule;
    P.layout = h->opt.layout;
    P.seed = h->opt.seed;
    P.box_shared = (B->shared_box && any_box) ? 1 : 0;
#ifdef BLP_PHASE_TIMERS
    P.timers = h->timers;
#endif
    const int nreg = h->nreg, nbins = nreg + 2;
    BUF_TRY(h, arena, h->counters, sizeof(int32_t) * counter_ints(nbins), sp.counters);
    int32_t* bin_count = sp.counters;
    P.bin_len = bin_count;
    P.bin_off = bin_count + 2 * nbins;
    P.bin_head = bin_count + heads_at(nbins);
    if (h->opt.profile) HIP_TRY(h, h->ensure_events(nbins + 1));

    sp.uni = uni;
    sp.any_simplex = any_simplex;
    sp.any_box = any_box;
    sp.n_box = n_box;
    sp.box_only_uniform = uni && !any_simplex;
    if (!sp.box_only_uniform) {
        BUF_TRY(h, arena, h->binid, sizeof(int32_t) * K, sp.binid);
        BUF_TRY(h, arena, h->list, sizeof(int32_t) * K, sp.list);
        P.list = sp.list;
        if (!uni) {
            BUF_TRY(h, arena, h->olist, sizeof(int32_t) * K, sp.olist);
            P.list = sp.olist;
        }
    }

    // Which register variants can receive an LP?  For a uniform simplex batch
    // only those chosen for some n_art in [0, m]; otherwise all.
    sp.maybe.assign(nreg, 0);
    if (h->opt.variant >= 0) {
        sp.maybe[h->opt.variant] = 1;
    } else if (h->opt.variant == -1 && any_simplex) {
        if (uni) {
            const int m = h->plan.m[0], n = h->plan.n[0];
            for (int nart = 0; nart <= m; ++nart) {
                const bool t1 = nart == 0 && h->opt.pivot_rule == BLP_RULE_LPC;
                int best = -1;
                long barea = -1;
                for (int v = 0; v < nreg; ++v)
                    if (h->variants[v].max_rows >= m + 2 && h->variants[v].max_cols >= n + nart + 1 &&
                        (t1 || !h->variants[v].type1_only) && K >= auto_min_count(h, v)) {
                        long a = (long)h->variants[v].max_rows * h->variants[v].max_cols;
                        if (barea < 0 || a < barea) {
                            barea = a;
                            best = v;
                        }
                    }
                if (best >= 0) {
                    const int r = h->remap[best];
                    const int to = (r >= nreg || t1 || !h->variants[r].type1_only) ? r : best;
                    if (to < nreg) sp.maybe[to] = 1;
                }
            }
        } else {
            std::fill(sp.maybe.begin(), sp.maybe.end(), 1);
        }
    }
    // A uniform batch small enough that every LP gets a place of its own at
    // once (a workgroup, or a lane of the lane kernel once the batch is large
    // enough for it), with a register variant that holds the shape whatever
    // its number of artificial rows: one launch, LP k in workgroup k (lane
    // k mod 64 of wave k / 64).  Binning would only choose among tiles that
    // give the same bits, and it costs four launches, about as long as
    // solving such a batch.
    sp.direct_v = -1;
    if (uni && any_simplex && h->opt.variant == -1 && h->opt.mode == BLP_MODE_PERSISTENT) {
        const int m = h->plan.m[0], n = h->plan.n[0];
        long barea = -1;
        for (int v = 0; v < nreg; ++v) {
            const RegVariant& rv = h->variants[v];
            const int64_t per = rv.lps_per_block;
            if (rv.max_rows >= m + 2 && rv.max_cols >= n + m + 1 && !rv.type1_only && h->remap[v] == v &&
                K <= (int64_t)h->reg_workers[v] * per && (per == 1 || K >= auto_min_count(h, v))) {
                const long a = (long)rv.max_rows * rv.max_cols;
                if (barea < 0 || a < barea) {
                    barea = a;
                    sp.direct_v = v;
                }
            }
        }
    }
    // Streaming-kernel geometry: worst case over the batch's simplex LPs.
    if (any_simplex) {
        sp.gm_ld = ((max_m + 2 + 15) / 16) * 16;  // 128-byte aligned columns
        sp.gm_cols = max_cols;
        int occ = 1;
        sp.gm_shared = std::find(sp.maybe.begin(), sp.maybe.end(), (char)1) != sp.maybe.end();
        gm_lds_plan(h, sp.gm_ld, sp.gm_cols, sp.gm_deep, sp.gm_shared, &sp.gm_lds, &P.ws_lds, &occ);
        if (h->opt.workers_per_cu > 0) occ = std::min(occ, (int)h->opt.workers_per_cu);
        // one workspace slot per streaming workgroup, no more workgroups
        // than LPs that can reach the streaming kernel
        sp.gm_workers = (int)std::max<int64_t>(1, std::min<int64_t>((int64_t)occ * h->cu_count, n_may_stream));
        const size_t slot = (size_t)max_slot;
        if (arena) {
            // as many workspace slots as the scratch still holds (fewer
            // persistent workgroups; the same results)
            const int64_t fit = (int64_t)(arena->left() / (sizeof(double) * slot));
            if (fit < 1)
                return fail(h, BLP_ERR_TOO_LARGE,
                            "static scratch of %zu bytes cannot hold one streaming workspace slot of %zu bytes",
                            arena->cap, sizeof(double) * slot);
            sp.gm_workers = (int)std::min<int64_t>(sp.gm_workers, fit);
        }
        if (ws_budget > 0)
            sp.gm_workers = (int)std::max<int64_t>(
                1, std::min<int64_t>(sp.gm_workers, (int64_t)(ws_budget / (sizeof(double) * slot))));
        BUF_TRY(h, arena, h->ws, sizeof(double) * slot * (size_t)sp.gm_workers, P.ws);
        P.ws_slot = (int64_t)slot;
        P.ws_ld = sp.gm_ld;
        P.ws_cols = sp.gm_cols;
    }
    return BLP_SUCCESS;
}

static VariantTable variant_table(blp_handle h, int64_t count) {
    VariantTable vt{};
    vt.nreg = h->nreg;
    vt.count = count;
    vt.force = h->opt.variant;
    for (int v = 0; v < h->nreg && v < kMaxVariants; ++v) {
        vt.rows[v] = h->variants[v].max_rows;
        vt.cols[v] = h->variants[v].max_cols;
        vt.remap[v] = h->remap[v];
        vt.type1[v] = h->variants[v].type1_only;
        vt.min_count[v] = auto_min_count(h, v);
    }
    vt.lpc = h->opt.pivot_rule == BLP_RULE_LPC;
    return vt;
}

// reset -> classify -> offsets -> scatter
static blp_error enqueue_binning(blp_handle h, SolvePlan& sp, hipStream_t s) {
    if (sp.box_only_uniform) return BLP_SUCCESS;
    const int nbins = h->nreg + 2;
    int32_t* bin_count = sp.counters;
    int32_t* bin_fill = bin_count + nbins;
    HIP_TRY(h, h->mark(nbins, true, s));
    // zero the counters and the striped bin counters (bin_off is rewritten)
    int32_t* stripes = bin_count + stripes_at(nbins);
    HIP_TRY(h, launch_reset(bin_count, (int)counter_ints(nbins), s));
    HIP_TRY(h, launch_classify(sp.P, variant_table(h, sp.P.count), sp.binid, stripes, s));
    HIP_TRY(h, launch_bin_offsets(stripes, bin_count, const_cast<int32_t*>(sp.P.bin_off), nbins, s));
    HIP_TRY(h, launch_scatter(sp.P.count, nbins, sp.binid, sp.P.bin_off, bin_fill, sp.list, s));
    // a uniform batch has one cost per bin; otherwise the kernels pop the
    // bins largest first
    if (!sp.uni)
        HIP_TRY(h, launch_order_bins(sp.P, nbins, bin_count, sp.P.bin_off, sp.list, sp.olist, s));
    HIP_TRY(h, h->mark(nbins, false, s));
    return BLP_SUCCESS;
}

// One persistent launch per kernel class that can receive LPs.  For a mixed
// batch (not uniform, at least kForkMinLps LPs) the launches are forked onto
// internal streams (each waits for the binning on s) and joined back into s:
// the bins of a mixed batch are small, each kernel's duration is set by its
// slowest LP, and run one after another they leave most of the GPU idle.  A
// uniform batch has one dominant class, and there the fork and join would
// only add their own latency.  A captured sequence (graph mode) keeps every
// class on the capturing stream.
static constexpr int64_t kForkMinLps = 2048;
static blp_error enqueue_persistent(blp_handle h, SolvePlan& sp, hipStream_t s, bool capturing = false) {
    const int nreg = h->nreg;
    const int64_t K = sp.P.count;
    KParams P = sp.P;
    P.direct = 0;
    std::vector<int> cls;  // 0..nreg-1 register variants, nreg streaming
    for (int v = 0; v < nreg; ++v)
        if (sp.maybe[v]) cls.push_back(v);
    // the streaming launch is left out when every LP surely fits a register
    // tile (an empty launch still costs a few microseconds on the stream)
    if (sp.any_simplex && sp.may_stream) cls.push_back(nreg);
    const int nc = (int)cls.size();
    const bool forked = !capturing && nc > 1 && !sp.uni && K >= kForkMinLps;
    const int nf = forked ? std::min(nc - 1, (int)blp_handle_s::kForks) : 0;
    if (forked) {
        HIP_TRY(h, hipEventRecord(h->fork_ev, s));
        for (int i = 0; i < nf; ++i) HIP_TRY(h, hipStreamWaitEvent(h->fork[i], h->fork_ev, 0));
    }
    // launches record their first error; the forks are joined back into s
    // in every case, so that work already issued on a fork is ordered before
    // whatever the caller (or the next solve on the handle's buffers) issues
    // on s next
    hipError_t err = hipSuccess;
    const char* what = "";
    for (int i = 0; i < nc && err == hipSuccess; ++i) {
        const int v = cls[i];
        // the last class (the streaming kernel when present) stays on s
        hipStream_t st = (forked && i < nc - 1) ? h->fork[i % nf] : s;
        KParams Q = P;
        Q.bin = v;
        err = h->mark(v, true, st);
        what = "event record";
        if (err == hipSuccess) {
            what = "kernel launch";
            err = v < nreg ? h->variants[v].launch(Q, reg_grid(h, v, K), st)
                           : launch_gm(Q, (int)std::min<int64_t>(sp.gm_workers, K), sp.gm_lds, st, sp.gm_deep);
        }
        if (err == hipSuccess) {
            what = "event record";
            err = h->mark(v, false, st);
        }
    }
    for (int i = 0; i < nf; ++i) {
        hipError_t je = hipEventRecord(h->join_ev[i], h->fork[i]);
        if (je == hipSuccess) je = hipStreamWaitEvent(s, h->join_ev[i], 0);
        if (err == hipSuccess && je != hipSuccess) {
            err = je;
            what = "fork join";
        }
    }
    if (err != hipSuccess)
        return fail(h, err == hipErrorOutOfMemory ? BLP_ERR_NOMEM : BLP_ERR_HIP, "persistent %s: %s (%s)", what,
                    hipGetErrorString(err), hipGetErrorName(err));
    return BLP_SUCCESS;
}

static blp_error enqueue_hyperbox(blp_handle h, SolvePlan& sp, hipStream_t s) {
    if (!sp.any_box) return BLP_SUCCESS;
    KParams Q = sp.P;
    Q.bin = h->nreg + 1;
    Q.direct = 0;
    HIP_TRY(h, h->mark(h->nreg + 1, true, s));
    HIP_TRY(h, launch_hyperbox(Q, sp.box_only_uniform ? sp.P.count : sp.n_box, s));
    HIP_TRY(h, h->mark(h->nreg + 1, false, s));
    return BLP_SUCCESS;
}

// Grid / one-LP-per-launch modes: read the bins back to size the launches.
static blp_error enqueue_baseline(blp_handle h, SolvePlan& sp, hipStream_t s) {
    const int nreg = h->nreg, nbins = nreg + 2, mode = h->opt.mode;
    std::vector<int32_t> cnt(nbins, 0);
    if (!sp.box_only_uniform) {
        HIP_TRY(h, hipMemcpyAsync(cnt.data(), sp.P.bin_len, sizeof(int32_t) * nbins, hipMemcpyDeviceToHost, s));
        HIP_TRY(h, hipStreamSynchronize(s));
    }
    KParams P = sp.P;
    P.direct = 1;
    for (int v = 0; v <= nreg; ++v) {
        const int64_t nv = cnt[v];
        if (nv == 0) continue;
        KParams Q = P;
        Q.bin = v;
        const int64_t chunk = v == nreg ? sp.gm_workers : (mode == BLP_MODE_GRID ? nv : 1);
        const int64_t per = v < nreg ? h->variants[v].lps_per_block : 1;  // LPs per workgroup
        HIP_TRY(h, h->mark(v, true, s));
        for (int64_t first = 0; first < nv; first += chunk) {
            Q.direct_first = first;
            Q.direct_end = std::min<int64_t>(first + chunk, nv);
            const int grid = (int)((std::min<int64_t>(chunk, nv - first) + per - 1) / per);
            if (v == nreg) {
                if (mode == BLP_MODE_GRID) {
                    HIP_TRY(h, launch_gm(Q, grid, sp.gm_lds, s, sp.gm_deep));
                } else {
                    for (int64_t q = first; q < first + grid; ++q) {
                        Q.direct_first = q;
                        HIP_TRY(h, launch_gm(Q, 1, sp.gm_lds, s, sp.gm_deep));
                    }
                }
            } else {
                HIP_TRY(h, h->variants[v].launch(Q, grid, s));
            }
        }
        HIP_TRY(h, h->mark(v, false, s));
    }
    return BLP_SUCCESS;
}

// Signature of everything a captured launch sequence depends on.
static std::vector<uint64_t> graph_signature(blp_handle h, const SolvePlan& sp, hipStream_t s) {
    const KParams& P = sp.P;
    (void)s;
    std::vector<uint64_t> g = {(uint64_t)P.count, (uint64_t)P.uniform, (uint64_t)P.um,
                               (uint64_t)P.un, (uint64_t)P.ukind, (uint64_t)(uintptr_t)P.A, (uint64_t)(uintptr_t)P.b,
                               (uint64_t)(uintptr_t)P.sense, (uint64_t)(uintptr_t)P.c, (uint64_t)(uintptr_t)P.l,
                               (uint64_t)(uintptr_t)P.u, (uint64_t)(uintptr_t)P.status,
                               (uint64_t)(uintptr_t)P.iters, (uint64_t)(uintptr_t)P.obj, (uint64_t)(uintptr_t)P.x,
                               (uint64_t)(uintptr_t)P.y, (uint64_t)(uintptr_t)P.list, (uint64_t)(uintptr_t)P.bin_len,
                               (uint64_t)(uintptr_t)P.ws, (uint64_t)P.ws_slot, (uint64_t)P.ws_ld,
                               (uint64_t)P.ws_cols, (uint64_t)(uintptr_t)P.m, (uint64_t)(uintptr_t)sp.binid,
                               (uint64_t)sp.gm_lds, (uint64_t)sp.gm_workers, (uint64_t)sp.gm_deep};
    for (int v = 0; v < h->nreg; ++v) g.push_back((uint64_t)sp.maybe[v] | ((uint64_t)h->remap[v] << 8));
    g.push_back((uint64_t)(int64_t)sp.direct_v);
    g.push_back((uint64_t)P.pivot_rule);
    g.push_back((uint64_t)P.layout);
    g.push_back(P.seed);
    if (!sp.uni) {
        // metadata content (the device copy is refreshed on every call, but
        // the launch shapes depend only on what is compared here)
        uint64_t f = 1469598103934665603ull;
        auto mix = [&](const void* p, size_t n) {
            const unsigned char* c = static_cast<const unsigned char*>(p);
            for (size_t i = 0; i < n; ++i) f = (f ^ c[i]) * 1099511628211ull;
        };
        mix(h->plan.kind.data(), h->plan.kind.size() * sizeof(int32_t));
        g.push_back(f);
    }
    return g;
}

static void record_solve(blp_handle h, const SolvePlan& sp, int64_t K) {
    h->last = sp.P;
    h->last.direct = 0;
    h->direct_v = sp.direct_v;
    h->count = K;
    h->uniform = sp.uni;
    h->any_simplex = sp.any_simplex;
    h->any_box = sp.any_box;
    h->n_box = sp.n_box;
    h->box_shared = sp.P.box_shared != 0;
    h->box_n = sp.box_n;
    h->chunked = false;
    h->solved = true;
}

static blp_error enqueue_direct(blp_handle h, SolvePlan& sp, hipStream_t s) {
    const int v = sp.direct_v;
    KParams Q = sp.P;
    Q.list = nullptr;  // the identity list
    Q.direct = 1;
    Q.direct_first = 0;
    Q.direct_end = 0;
    Q.bin = v;
    HIP_TRY(h, h->mark(v, true, s));
    const int64_t per = h->variants[v].lps_per_block;
    HIP_TRY(h, h->variants[v].launch(Q, (int)((Q.count + per - 1) / per), s));
    HIP_TRY(h, h->mark(v, false, s));
    return BLP_SUCCESS;
}

static blp_error enqueue_eager(blp_handle h, SolvePlan& sp, hipStream_t s) {
    if (sp.direct_v >= 0 && h->opt.mode == BLP_MODE_PERSISTENT) return enqueue_direct(h, sp, s);
    blp_error e = enqueue_binning(h, sp, s);
    if (e != BLP_SUCCESS) return e;
    e = h->opt.mode == BLP_MODE_PERSISTENT ? enqueue_persistent(h, sp, s) : enqueue_baseline(h, sp, s);
    if (e != BLP_SUCCESS) return e;
    return enqueue_hyperbox(h, sp, s);
}

// A handle with mem_limit S: everything the call allocates fits in S bytes.
// The result buffers the handle provides (outputs passed as NULL), the bin
// counters and one streaming workspace slot of the batch's largest LP are
// fixed; each LP adds Y bytes of metadata and work lists (8 for a uniform
// batch, 48 otherwise).  The batch is solved in consecutive chunks of
// N = (S - fixed) / Y LPs -- the batch capacity of Sec. 4.5, Eq. (5) -- on
// the caller's stream, one after another, into the caller's (or the
// handle's) result buffers; the streaming kernel gets as many workspace slots
// as the rest of the limit holds.  The handle's buffers are released first
// and then sized exactly, so the call never holds more than S.
static blp_error solve_limited(blp_handle h, const blp_batch* B, const blp_outputs* out, hipStream_t s) {
    const int64_t K = B->count;
    const bool uni = B->uniform != 0;
    const uint64_t limit = h->opt.mem_limit;
    // the whole batch's extents and largest streaming slot (arguments are
    // checked again for each chunk by prepare)
    PlanIn in;
    in.count = K;
    in.uniform = uni;
    in.shared_box = B->shared_box != 0;
    in.m = B->m;
    in.n = B->n;
    in.kind = B->kind;
    in.a_off = B->a_off;
    in.row_off = B->row_off;
    in.col_off = B->col_off;
    in.has_A = B->A;
    in.has_b = B->b;
    in.has_sense = B->sense;
    in.has_c = B->c;
    in.has_l = B->l;
    in.has_u = B->u;
    Plan whole;
    if (plan_batch(in, whole) != PLAN_OK) return fail(h, (blp_error)whole.code, "%s", whole.msg.c_str());
    const int64_t tot_m = whole.tot_m, tot_n = whole.tot_n, max_slot = whole.max_slot;
    const bool any_simplex = whole.any_simplex;
    const std::vector<int64_t>& ao = whole.a_off;
    const std::vector<int64_t>& ro = whole.row_off;
    const std::vector<int64_t>& co = whole.col_off;
    const bool own_st = !out || !out->status, own_it = !out || !out->iters, own_ob = !out || !out->obj;
    const bool own_x = !out || !out->x, own_y = !out || !out->y;
    const size_t out_bytes = (own_st ? 4 * (size_t)K : 0) + (own_it ? 4 * (size_t)K : 0) +
                             (own_ob ? 8 * (size_t)K : 0) + (own_x ? 8 * (size_t)std::max<int64_t>(1, tot_n) : 0) +
                             (own_y ? 8 * (size_t)std::max<int64_t>(1, tot_m) : 0);
    const size_t counters = sizeof(int32_t) * counter_ints(h->nreg + 2);
    const size_t slot = any_simplex ? sizeof(double) * (size_t)max_slot : 0;
    const size_t per_lp = uni ? 8 : 48;
    const size_t fixed = out_bytes + counters + slot;
    const int64_t cap = chunk_capacity(limit, fixed, per_lp, K);
    if (cap < 1)
        return fail(h, BLP_ERR_NOMEM,
                    "mem_limit of %llu bytes: %zu bytes of results, %zu of bin counters and a %zu-byte workspace "
                    "slot leave no room for one LP (%zu bytes)",
                    (unsigned long long)limit, out_bytes, counters, slot, per_lp);
    // the buffers are sized for this call alone
    for (DevBuf* b : {&h->meta, &h->counters, &h->binid, &h->list, &h->olist, &h->ws, &h->own_status, &h->own_iters,
                      &h->own_obj, &h->own_x, &h->own_y})
        b->release();
    blp_outputs o = out ? *out : blp_outputs{};
    if (own_st) HIP_TRY(h, h->own_status.reserve(4 * (size_t)K, true));
    if (own_it) HIP_TRY(h, h->own_iters.reserve(4 * (size_t)K, true));
    if (own_ob) HIP_TRY(h, h->own_obj.reserve(8 * (size_t)K, true));
    if (own_x) HIP_TRY(h, h->own_x.reserve(8 * (size_t)std::max<int64_t>(1, tot_n), true));
    if (own_y) HIP_TRY(h, h->own_y.reserve(8 * (size_t)std::max<int64_t>(1, tot_m), true));
    if (own_st) o.status = h->own_status.as<int32_t>();
    if (own_it) o.iters = h->own_iters.as<int32_t>();
    if (own_ob) o.obj = h->own_obj.as<double>();
    if (own_x) o.x = h->own_x.as<double>();
    if (own_y) o.y = h->own_y.as<double>();
    SolvePlan sp;
    int nchunks = 0;
    for (int64_t k0 = 0; k0 < K; k0 += cap, ++nchunks) {
        const int64_t kc = std::min<int64_t>(cap, K - k0);
        blp_batch sub = *B;
        sub.count = kc;
        blp_outputs os = o;
        os.status = o.status + k0;
        os.iters = o.iters + k0;
        os.obj = o.obj + k0;
        if (uni) {
            const int64_t m = B->m[0], n = B->n[0];
            if (B->A) sub.A = B->A + k0 * m * n;
            if (B->b) sub.b = B->b + k0 * m;
            if (B->sense) sub.sense = B->sense + k0 * m;
            if (B->c) sub.c = B->c + k0 * n;
            if (!B->shared_box) {
                if (B->l) sub.l = B->l + k0 * n;
                if (B->u) sub.u = B->u + k0 * n;
            }
            os.x = o.x + k0 * n;
            os.y = o.y + k0 * m;
        } else {  // offsets stay absolute
            sub.m = B->m + k0;
            sub.n = B->n + k0;
            sub.kind = B->kind + k0;
            sub.a_off = ao.data() + k0;
            sub.row_off = ro.data() + k0;
            sub.col_off = co.data() + k0;  // (the whole batch's plan outlives the loop)
        }
        const size_t ws_budget = (size_t)(limit - out_bytes - counters - per_lp * (size_t)kc);
        blp_error e = prepare(h, &sub, &os, s, sp, false, nullptr, std::max<size_t>(ws_budget, 1));
        if (e != BLP_SUCCESS) return e;
        e = enqueue_eager(h, sp, s);
        if (e != BLP_SUCCESS) return e;
    }
    HIP_TRY(h, hipGetLastError());
    // the handle describes the whole batch (results, host metadata); the
    // work lists are those of the last chunk
    record_solve(h, sp, K);
    h->last.status = o.status;
    h->last.iters = o.iters;
    h->last.obj = o.obj;
    h->last.x = o.x;
    h->last.y = o.y;
    h->plan = std::move(whole);
    h->chunked = nchunks > 1;
    return BLP_SUCCESS;
}

blp_error blp_solve_batch(blp_handle h, const blp_batch* B, const blp_outputs* out, void* stream) {
    if (!h) return BLP_ERR_ARG;
    h->err.clear();
    if (!B) return fail(h, BLP_ERR_ARG, "batch is NULL");
    if (B->count < 0 || B->count > 0x7fffffffLL) return fail(h, BLP_ERR_ARG, "count out of range");
    const int64_t K = B->count;
    hipStream_t s = static_cast<hipStream_t>(stream);
    HIP_TRY(h, hipSetDevice(h->opt.device));
    h->solved = false;
    if (K == 0) {
        h->count = 0;
        h->solved = true;
        return BLP_SUCCESS;
    }
    HIP_TRY(h, begin_call(h, s));
    if (h->opt.mem_limit > 0) {
        const blp_error le = solve_limited(h, B, out, s);
        if (le != BLP_SUCCESS) return le;
        HIP_TRY(h, end_call(h, s));
        return BLP_SUCCESS;
    }
    SolvePlan sp;
    blp_error e = prepare(h, B, out, s, sp);
    if (e != BLP_SUCCESS) return e;

    const bool use_graph = h->opt.graph && !h->opt.profile && h->opt.mode == BLP_MODE_PERSISTENT;
    if (use_graph) {
        std::vector<uint64_t> sig = graph_signature(h, sp, s);
        if (!h->graph_exec || sig != h->graph_sig) {
            if (h->graph_exec) {
                (void)hipGraphExecDestroy(h->graph_exec);
                h->graph_exec = nullptr;
            }
            // Capture on an internal stream (the caller's may be the legacy
            // default stream, which cannot capture); the graph is then
            // launched on the caller's stream.
            if (!h->cap_stream) HIP_TRY(h, hipStreamCreateWithFlags(&h->cap_stream, hipStreamNonBlocking));
            hipStream_t cs = h->cap_stream;
            hipGraph_t g = nullptr;
            HIP_TRY(h, hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal));
            blp_error ce = BLP_SUCCESS;
            if (sp.direct_v >= 0) {
                ce = enqueue_direct(h, sp, cs);
            } else {
                ce = enqueue_binning(h, sp, cs);
                if (ce == BLP_SUCCESS) ce = enqueue_persistent(h, sp, cs, true);
                if (ce == BLP_SUCCESS) ce = enqueue_hyperbox(h, sp, cs);
            }
            hipError_t he = hipStreamEndCapture(cs, &g);
            if (ce != BLP_SUCCESS) {
                if (g) (void)hipGraphDestroy(g);
                return ce;
            }
            HIP_TRY(h, he);
            hipError_t ie = hipGraphInstantiate(&h->graph_exec, g, nullptr, nullptr, 0);
            (void)hipGraphDestroy(g);
            HIP_TRY(h, ie);
            h->graph_sig = sig;
        }
        HIP_TRY(h, hipGraphLaunch(h->graph_exec, s));
    } else {
        e = enqueue_eager(h, sp, s);
        if (e != BLP_SUCCESS) return e;
    }
    HIP_TRY(h, hipGetLastError());
    HIP_TRY(h, end_call(h, s));
    record_solve(h, sp, K);
    return BLP_SUCCESS;
}

// Allocation-free variant of blp_solve_batch: the batch metadata, work
// lists, bin counters and streaming workspace come from this device's static
// scratch; the caller passes every output.  Eager launches only (no graph,
// no mem_limit chunking).  The streaming kernel gets as many workspace slots
// as the scratch still holds after the rest.
blp_error blp_solve_batch_static(blp_handle h, const blp_batch* B, const blp_outputs* out, void* stream) {
    if (!h) return BLP_ERR_ARG;
    h->err.clear();
    if (!B) return fail(h, BLP_ERR_ARG, "batch is NULL");
    if (!out || !out->status || !out->iters || !out->obj || !out->x || !out->y)
        return fail(h, BLP_ERR_ARG, "all five output buffers are required");
    if (B->count < 0 || B->count > 0x7fffffffLL) return fail(h, BLP_ERR_ARG, "count out of range");
    if (!h->scratch) return fail(h, BLP_ERR_STATE, "no static scratch on this device");
    const int64_t K = B->count;
    hipStream_t s = static_cast<hipStream_t>(stream);
    HIP_TRY(h, hipSetDevice(h->opt.device));
    h->solved = false;
    if (K == 0) {
        h->count = 0;
        h->solved = true;
        return BLP_SUCCESS;
    }
    HIP_TRY(h, begin_call(h, s));
    Arena arena;
    arena.base = static_cast<char*>(h->scratch);
    arena.cap = kStaticScratchBytes;
    SolvePlan sp;
    blp_error e = prepare(h, B, out, s, sp, false, &arena);
    if (e != BLP_SUCCESS) return e;
    e = enqueue_eager(h, sp, s);
    if (e != BLP_SUCCESS) return e;
    HIP_TRY(h, hipGetLastError());
    HIP_TRY(h, end_call(h, s));
    record_solve(h, sp, K);
    return BLP_SUCCESS;
}

size_t blp_static_scratch_bytes(void) { return kStaticScratchBytes; }

blp_error blp_pivot_trace(blp_handle h, const blp_batch* B, const blp_outputs* out, int32_t* trace, int32_t stride,
                          int32_t replay, void* stream) {
    if (!h) return BLP_ERR_ARG;
    h->err.clear();
    if (!B) return fail(h, BLP_ERR_ARG, "batch is NULL");
    if (B->count < 0 || B->count > 0x7fffffffLL) return fail(h, BLP_ERR_ARG, "count out of range");
    if (stride < 1 || stride > 1 + 2 * kTraceMaxPivots)
        return fail(h, BLP_ERR_ARG, "stride %d outside [1, %d]", stride, 1 + 2 * kTraceMaxPivots);
    if (!B->uniform) return fail(h, BLP_ERR_ARG, "the pivot trace needs a uniform batch");
    if (h->opt.pivot_rule != BLP_RULE_LPC) return fail(h, BLP_ERR_ARG, "the pivot trace needs the rule LPC");
    if (h->opt.mem_limit > 0) return fail(h, BLP_ERR_ARG, "the pivot trace does not split a batch (mem_limit)");
    const int64_t K = B->count;
    hipStream_t s = static_cast<hipStream_t>(stream);
    HIP_TRY(h, hipSetDevice(h->opt.device));
    h->solved = false;
    if (K == 0) {
        h->count = 0;
        h->solved = true;
        return BLP_SUCCESS;
    }
    if (!trace) return fail(h, BLP_ERR_ARG, "trace is NULL");
    if (!B->m || !B->n || !B->kind) return fail(h, BLP_ERR_ARG, "m, n and kind are required");
    int rows = 0, cols = 0;
    blk_trace_shape(&rows, &cols);
    if (B->kind[0] != 0) return fail(h, BLP_ERR_ARG, "the pivot trace needs simplex LPs");
    if (B->m[0] < 1 || B->n[0] < 1 || B->m[0] + 2 > rows || B->n[0] + 1 > cols)
        return fail(h, BLP_ERR_ARG, "the pivot trace needs 1 <= m <= %d and 1 <= n <= %d", rows - 2, cols - 1);
    HIP_TRY(h, begin_call(h, s));
    SolvePlan sp;
    blp_error e = prepare(h, B, out, s, sp);
    if (e != BLP_SUCCESS) return e;
    // one persistent launch over the identity list (no binning), the grid the
    // occupancy allows
    int occ = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&occ, blk_trace_kernel_ptr(replay ? 2 : 1), 256, 0) !=
            hipSuccess ||
        occ < 1)
        occ = 1;
    KParams Q = sp.P;
    Q.list = nullptr;
    Q.direct = 0;
    Q.bin = 0;
    Q.trace = trace;
    Q.trace_stride = stride;
    int v = -1;  // the registered variant of this tile, for the per-class figures
    for (int w = 0; w < h->nreg; ++w)
        if (std::strcmp(h->variants[w].name, "b4_r112_c112") == 0) v = w;
    HIP_TRY(h, launch_reset(Q.bin_head, 1, s));
    if (v >= 0) HIP_TRY(h, h->mark(v, true, s));
    HIP_TRY(h, launch_blk_trace(Q, (int)std::min<int64_t>((int64_t)occ * h->cu_count, K), s, replay ? 2 : 1));
    if (v >= 0) HIP_TRY(h, h->mark(v, false, s));
    HIP_TRY(h, end_call(h, s));
    sp.direct_v = v;
    record_solve(h, sp, K);
    return BLP_SUCCESS;
}

blp_error blp_backward_shared(blp_handle h, int32_t m, int32_t n, int64_t count, const int32_t* status,
                              const double* x, const double* y, const double* g, double* dC, double* db, double* dA,
                              void* stream) {
    if (!h) return BLP_ERR_ARG;
    h->err.clear();
    if (count < 0 || count > 0x7fffffffLL) return fail(h, BLP_ERR_ARG, "count out of range");
    if (m < 1 || n < 1 || m > kMaxM || (int64_t)n + m + 1 > kMaxCols)
        return fail(h, BLP_ERR_ARG, "m and n outside 1 <= m <= %d, n + m + 1 <= %d", kMaxM, kMaxCols);
    if (count == 0 || (!dC && !db && !dA)) return BLP_SUCCESS;
    if (!status || !x || !y || !g) return fail(h, BLP_ERR_ARG, "status, x, y and g are required");
    hipStream_t s = static_cast<hipStream_t>(stream);
    HIP_TRY(h, hipSetDevice(h->opt.device));
    HIP_TRY(h, begin_call(h, s));
    const int64_t chunk = shared_bwd_chunk(count, m, n);
    const int64_t nchunks = (count + chunk - 1) / chunk;
    if (db || dA) HIP_TRY(h, h->bwd_part.reserve(sizeof(double) * (size_t)nchunks * ((size_t)m * n + m)));
    HIP_TRY(h, launch_backward_shared(count, m, n, status, g, x, y, h->bwd_part.as<double>(), dC, db, dA, s));
    HIP_TRY(h, end_call(h, s));
    return BLP_SUCCESS;
}

// ------------------------------------------------ host-resident pipeline
// The warm-started shared kernel: persistent workgroups taking chunks of
// consecutive objectives (the warm starts run along a chunk), at least 8 per
// chunk and about four chunks per workgroup for balance.
static blp_error launch_shared_warm(blp_handle h, KParams& P, hipStream_t s) {
    int occ = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&occ, shared_kernel_ptr(), shared_threads(), 0) != hipSuccess ||
        occ < 1)
        occ = 1;
    const int64_t workers = (int64_t)occ * h->cu_count;
    P.chunk = std::max<int64_t>(8, (P.count + 4 * workers - 1) / (4 * workers));
    const int grid = (int)std::min<int64_t>(workers, (P.count + P.chunk - 1) / P.chunk);
    HIP_TRY(h, launch_shared(P, grid, s));
    return BLP_SUCCESS;
}

// blp_solve_shared on a handle that forces a register variant: the route is
// decided on the host (b, sense and the first 65 objectives read back), so
// that a variant that cannot hold the constraints fails the call.
static blp_error solve_shared_forced(blp_handle h, KParams& P, int rows, int cols, hipStream_t s) {
    const int m = P.um, n = P.un;
    const int64_t count = P.count;
    std::vector<double> hb(m);
    std::vector<int8_t> hs(m);
    const int64_t ns = std::min<int64_t>(count, 65);
    std::vector<double> hc((size_t)std::max<int64_t>(ns, 1) * n);
    HIP_TRY(h, hipMemcpyAsync(hb.data(), P.b, sizeof(double) * m, hipMemcpyDeviceToHost, s));
    HIP_TRY(h, hipMemcpyAsync(hs.data(), P.sense, (size_t)m, hipMemcpyDeviceToHost, s));
    HIP_TRY(h, hipMemcpyAsync(hc.data(), P.c, sizeof(double) * ns * n, hipMemcpyDeviceToHost, s));
    HIP_TRY(h, hipStreamSynchronize(s));
    int close = 0;
    for (int64_t k = 1; k < ns; ++k) {
        double dot = 0.0, aa = 0.0, bb = 0.0;
        for (int j = 0; j < n; ++j) {
            const double u = hc[(size_t)k * n + j], v = hc[(size_t)(k - 1) * n + j];
            dot += u * v;
            aa += u * u;
            bb += v * v;
        }
        close += dot > 0.9 * std::sqrt(aa * bb);
    }
    int nart = 0;
    for (int i = 0; i < m; ++i) nart += (hs[i] ? -hb[i] : hb[i]) < 0.0;
    if (ns > 1 && 2 * close >= ns - 1 && m + 2 <= rows && n + nart + 1 <= cols) return launch_shared_warm(h, P, s);
    const int v = h->opt.variant;
    if (h->variants[v].max_rows < m + 2 || h->variants[v].max_cols < n + nart + 1 ||
        (h->variants[v].type1_only && (nart > 0 || h->opt.pivot_rule != BLP_RULE_LPC)))
        return fail(h, BLP_ERR_TOO_LARGE, "variant %s cannot hold the shared constraints", h->variants[v].name);
    P.shared_in = 1;
    HIP_TRY(h, h->variants[v].launch(P, reg_grid(h, v, count), s));
    return BLP_SUCCESS;
}

blp_error blp_solve_shared(blp_handle h, int32_t m, int32_t n, const double* A, const double* b,
                           const int8_t* sense, int64_t count, const double* C, const blp_outputs* out,
                           void* stream) {
    if (!h) return BLP_ERR_ARG;
    h->err.clear();
    if (count < 0 || count > 0x7fffffffLL) return fail(h, BLP_ERR_ARG, "count out of range");
    if (m < 1 || n < 1) return fail(h, BLP_ERR_ARG, "m and n must be >= 1");
    if (!A || !b || !sense) return fail(h, BLP_ERR_ARG, "A, b and sense are required");
    if (count > 0 && (!C || !out || !out->status || !out->iters || !out->obj || !out->x || !out->y))
        return fail(h, BLP_ERR_ARG, "C and all five output buffers are required");
    if (m > kMaxM || (int64_t)n + m + 1 > kMaxCols)
        return fail(h, BLP_ERR_TOO_LARGE, "shared constraints need m <= %d and n + m + 1 <= %d", kMaxM, kMaxCols);
    int rows = 0, cols = 0;
    shared_shape(&rows, &cols);
    hipStream_t s = static_cast<hipStream_t>(stream);
    HIP_TRY(h, hipSetDevice(h->opt.device));
    if (count == 0) return BLP_SUCCESS;
    HIP_TRY(h, begin_call(h, s));
    KParams P{};
    P.count = count;
    P.uniform = 1;
    P.um = m;
    P.un = n;
    P.ukind = 0;
    P.A = A;
    P.b = b;
    P.sense = sense;
    P.c = C;
    P.status = out->status;
    P.iters = out->iters;
    P.obj = out->obj;
    P.x = out->x;
    P.y = out->y;
    P.max_iter = h->opt.max_iter;
    P.bland_after = h->opt.bland_after;
    P.eps_price = h->opt.eps_price;
    P.eps_piv = h->opt.eps_piv;
    P.eps_feas = h->opt.eps_feas;
    P.pivot_rule = h->opt.pivot_rule;
    P.layout = h->opt.layout;
    P.seed = h->opt.seed;
#ifdef BLP_PHASE_TIMERS
    P.timers = h->timers;
#endif
    const int nreg = h->nreg, nb = nreg + 2;
    // route lengths (nb), zero list offsets (nb), then one queue head per
    // route, each on a cache line of its own
    const size_t heads = ((size_t)2 * nb + kHeadStride - 1) / kHeadStride * kHeadStride;
    const size_t ints = heads + (size_t)kHeadStride * nb;
    HIP_TRY(h, h->shared_ctr.reserve(sizeof(int32_t) * ints));
    int32_t* rb = h->shared_ctr.as<int32_t>();
    HIP_TRY(h, launch_reset(rb, (int)ints, s));
    P.bin_head = rb + heads;
    P.bin = 0;
    if (h->opt.variant >= 0) {
        blp_error e = solve_shared_forced(h, P, rows, cols, s);
        if (e != BLP_SUCCESS) return e;
        HIP_TRY(h, end_call(h, s));
        return BLP_SUCCESS;
    }
    // The route (warm starts, one register variant, or the streaming kernel)
    // depends on b, sense and the first objectives, which are device data:
    // a one-workgroup kernel picks it and writes the work length of every
    // route (count for the chosen one, 0 for the others), and every route
    // that some number of artificial rows could select is launched over the
    // identity list; the others leave at their first look at the list.
    SharedRoute rt{};
    rt.nreg = nreg;
    for (int v = 0; v < nreg && v < kMaxVariants; ++v) {
        rt.rows[v] = h->variants[v].max_rows;
        rt.cols[v] = h->variants[v].max_cols;
        rt.type1[v] = h->variants[v].type1_only;
    }
    rt.tile_rows = rows;
    rt.tile_cols = cols;
    std::vector<char> cand(nb, 0);
    for (int na = 0; na <= m; ++na) {
        cand[shared_route_of(rt, m, n, na, false)] = 1;
        if (count > 1) cand[shared_route_of(rt, m, n, na, true)] = 1;
    }
    if (count > h->shared_list_n) {
        h->shared_list_n = 0;
        HIP_TRY(h, h->shared_list.reserve(sizeof(int32_t) * (size_t)count));
        HIP_TRY(h, launch_iota(h->shared_list.as<int32_t>(), count, s));
        h->shared_list_n = count;
    }
    HIP_TRY(h, launch_shared_route(m, n, count, b, sense, C, rt, rb, s));
    P.list = h->shared_list.as<int32_t>();
    P.bin_len = rb;
    P.bin_off = rb + nb;
    if (cand[nreg + 1]) {
        KParams Q = P;
        Q.bin = nreg + 1;
        blp_error e = launch_shared_warm(h, Q, s);
        if (e != BLP_SUCCESS) return e;
    }
    for (int v = 0; v < nreg; ++v) {
        if (!cand[v]) continue;
        KParams Q = P;
        Q.bin = v;
        Q.shared_in = 1;
        HIP_TRY(h, h->variants[v].launch(Q, reg_grid(h, v, count), s));
    }
    if (cand[nreg]) {
        // the streaming kernel with on-chip columns (nothing else runs beside
        // it), one workspace slot per workgroup for the widest tableau the
        // constraints can give (every row artificial)
        KParams Q = P;
        Q.bin = nreg;
        Q.shared_in = 1;
        const int ld = ((m + 2 + 15) / 16) * 16, gcols = n + m + 1;
        const bool deep = true;
        int occ = 1;
        size_t lds = 0;
        gm_lds_plan(h, ld, gcols, deep, false, &lds, &Q.ws_lds, &occ);
        if (h->opt.workers_per_cu > 0) occ = std::min(occ, (int)h->opt.workers_per_cu);
        const int64_t workers = std::max<int64_t>(1, std::min<int64_t>((int64_t)occ * h->cu_count, count));
        const size_t slot = (size_t)ld * gcols;
        HIP_TRY(h, h->shared_ws.reserve(sizeof(double) * slot * (size_t)workers));
        Q.ws = h->shared_ws.as<double>();
        Q.ws_slot = (int64_t)slot;
        Q.ws_ld = ld;
        Q.ws_cols = gcols;
        HIP_TRY(h, launch_gm(Q, (int)workers, lds, s, deep));
    }
    HIP_TRY(h, end_call(h, s));
    return BLP_SUCCESS;
}

blp_error blp_solve_batch_host(blp_handle h, const blp_batch* B, const blp_outputs* out, int32_t chunks) {
    if (!h) return BLP_ERR_ARG;
    h->err.clear();
    if (!B || !out) return fail(h, BLP_ERR_ARG, "batch and out are required");
    if (!out->status || !out->iters || !out->obj || !out->x || !out->y)
        return fail(h, BLP_ERR_ARG, "all five host output buffers are required");
    if (B->count < 0 || B->count > 0x7fffffffLL) return fail(h, BLP_ERR_ARG, "count out of range");
    const int64_t K = B->count;
    if (K == 0) return BLP_SUCCESS;
    if (!B->m || !B->n || !B->kind) return fail(h, BLP_ERR_ARG, "m, n and kind are required");
    HIP_TRY(h, hipSetDevice(h->opt.device));
    const bool uni = B->uniform != 0;
    // per-LP host offsets
    std::vector<int32_t> m(K), n(K), kind(K);
    std::vector<int64_t> ao(K), ro(K), co(K);
    int64_t a = 0, r = 0, c = 0;
    for (int64_t k = 0; k < K; ++k) {
        m[k] = B->m[uni ? 0 : k];
        n[k] = B->n[uni ? 0 : k];
        kind[k] = B->kind[uni ? 0 : k];
        if (m[k] < 0 || n[k] < 0) return fail(h, BLP_ERR_ARG, "LP %lld: negative size", (long long)k);
        ao[k] = (!uni && B->a_off) ? B->a_off[k] : a;
        ro[k] = (!uni && B->row_off) ? B->row_off[k] : r;
        co[k] = (!uni && B->col_off) ? B->col_off[k] : c;
        a += (int64_t)m[k] * n[k];
        r += m[k];
        c += n[k];
    }
    int64_t box_n = 0;  // shared box: its length (that of any hyperbox LP)
    for (int64_t k = 0; k < K && B->shared_box && !box_n; ++k)
        if (kind[k] == BLP_KIND_HYPERBOX) box_n = n[k];
    if (chunks <= 0) chunks = (int32_t)std::min<int64_t>(8, std::max<int64_t>(1, K / 1024));
    chunks = (int32_t)std::min<int64_t>(chunks, K);
    for (int i = 0; i < 2; ++i) {
        if (!h->child[i]) {
            blp_options o = h->opt;
            o.graph = 0;
            blp_error e = blp_create(&h->child[i], &o);
            if (e != BLP_SUCCESS) return fail(h, e, "child handle: %s", blp_last_error(h->child[i]));
            for (int v = 0; v < kMaxVariants; ++v) h->child[i]->remap[v] = h->remap[v];
        }
        if (!h->pipe[i]) HIP_TRY(h, hipStreamCreateWithFlags(&h->pipe[i], hipStreamNonBlocking));
    }
    struct Range { int64_t lo = INT64_MAX, hi = 0; };
    std::vector<int64_t> order;
    std::vector<CopyRun> runs;
    for (int32_t ch = 0; ch < chunks; ++ch) {
        const int64_t k0 = K * ch / chunks, k1 = K * (ch + 1) / chunks, Kc = k1 - k0;
        const int slot = ch & 1;
        blp_handle ch_h = h->child[slot];
        hipStream_t s = h->pipe[slot];
        // data ranges of this piece (offsets may be arbitrary, not packed)
        Range ra, rr, rc;
        for (int64_t k = k0; k < k1; ++k) {
            ra.lo = std::min(ra.lo, ao[k]);
            ra.hi = std::max(ra.hi, ao[k] + (int64_t)m[k] * n[k]);
            rr.lo = std::min(rr.lo, ro[k]);
            rr.hi = std::max(rr.hi, ro[k] + m[k]);
            rc.lo = std::min(rc.lo, co[k]);
            rc.hi = std::max(rc.hi, co[k] + n[k]);
        }
        const int64_t na = std::max<int64_t>(0, ra.hi - ra.lo), nr = std::max<int64_t>(0, rr.hi - rr.lo),
                      nc = std::max<int64_t>(0, rc.hi - rc.lo);
        // device layout of one piece: A | b | c | l | u (doubles) | sense (bytes)
        const size_t in_bytes = sizeof(double) * (size_t)(na + nr + 3 * nc) + (size_t)nr + 64;
        const size_t out_bytes = sizeof(double) * (size_t)(Kc + nc + nr) + 2 * sizeof(int32_t) * (size_t)Kc + 64;
        // the previous piece on this stream must be done with the buffers
        HIP_TRY(h, hipStreamSynchronize(s));
        HIP_TRY(h, h->pin_in[slot].reserve(in_bytes));
        HIP_TRY(h, h->pin_out[slot].reserve(out_bytes));
        double* dA = h->pin_in[slot].as<double>();
        double* db = dA + na;
        double* dc = db + nr;
        double* dl = dc + nc;
        double* du = dl + nc;
        int8_t* dsense = reinterpret_cast<int8_t*>(du + nc);
        double* oobj = h->pin_out[slot].as<double>();
        double* ox = oobj + Kc;
        double* oy = ox + nc;
        int32_t* ost = reinterpret_cast<int32_t*>(oy + nr);
        int32_t* oit = ost + Kc;
        auto up = [&](void* dst, const void* src, size_t bytes) -> hipError_t {
            return (src && bytes) ? hipMemcpyAsync(dst, src, bytes, hipMemcpyHostToDevice, s) : hipSuccess;
        };
        HIP_TRY(h, up(dA, B->A ? B->A + ra.lo : nullptr, sizeof(double) * na));
        HIP_TRY(h, up(db, B->b ? B->b + rr.lo : nullptr, sizeof(double) * nr));
        HIP_TRY(h, up(dsense, B->sense ? B->sense + rr.lo : nullptr, (size_t)nr));
        HIP_TRY(h, up(dc, B->c ? B->c + rc.lo : nullptr, sizeof(double) * nc));
        if (B->shared_box) {  // the one box (at most nc long: some LP of the piece has its length)
            HIP_TRY(h, up(dl, B->l ? B->l : nullptr, sizeof(double) * std::min<int64_t>(box_n, nc)));
            HIP_TRY(h, up(du, B->u ? B->u : nullptr, sizeof(double) * std::min<int64_t>(box_n, nc)));
        } else {
            HIP_TRY(h, up(dl, B->l ? B->l + rc.lo : nullptr, sizeof(double) * nc));
            HIP_TRY(h, up(du, B->u ? B->u + rc.lo : nullptr, sizeof(double) * nc));
        }
        std::vector<int64_t> cao(Kc), cro(Kc), cco(Kc);
        for (int64_t k = k0; k < k1; ++k) {
            cao[k - k0] = ao[k] - ra.lo;
            cro[k - k0] = ro[k] - rr.lo;
            cco[k - k0] = co[k] - rc.lo;
        }
        blp_batch cb{};
        cb.count = Kc;
        cb.uniform = uni ? 1 : 0;
        cb.shared_box = B->shared_box;
        cb.m = uni ? m.data() : m.data() + k0;
        cb.n = uni ? n.data() : n.data() + k0;
        cb.kind = uni ? kind.data() : kind.data() + k0;
        cb.a_off = cao.data();
        cb.row_off = cro.data();
        cb.col_off = cco.data();
        cb.A = B->A ? dA : nullptr;
        cb.b = B->b ? db : nullptr;
        cb.sense = B->sense ? dsense : nullptr;
        cb.c = B->c ? dc : nullptr;
        cb.l = B->l ? dl : nullptr;
        cb.u = B->u ? du : nullptr;
        blp_outputs co_{ost, oit, oobj, ox, oy};
        blp_error e = blp_solve_batch(ch_h, &cb, &co_, s);
        if (e != BLP_SUCCESS) return fail(h, e, "piece %d: %s", ch, blp_last_error(ch_h));
        // results back; x/y of each LP land at the caller's offsets.  Only
        // the piece's own LPs' ranges are copied (one copy per run of LPs
        // whose ranges follow each other): with gapped or interleaved
        // offsets the piece's device buffer holds nothing meaningful
        // between them, and another piece may own those positions.
        HIP_TRY(h, hipMemcpyAsync(out->status + k0, ost, sizeof(int32_t) * Kc, hipMemcpyDeviceToHost, s));
        HIP_TRY(h, hipMemcpyAsync(out->iters + k0, oit, sizeof(int32_t) * Kc, hipMemcpyDeviceToHost, s));
        HIP_TRY(h, hipMemcpyAsync(out->obj + k0, oobj, sizeof(double) * Kc, hipMemcpyDeviceToHost, s));
        for (int pass = 0; pass < 2; ++pass) {
            copy_runs(pass == 0 ? co : ro, pass == 0 ? n : m, k0, k1, pass == 0 ? rc.lo : rr.lo, order, runs);
            double* dst = pass == 0 ? out->x : out->y;
            const double* src = pass == 0 ? ox : oy;
            for (const CopyRun& r : runs)
                HIP_TRY(h, hipMemcpyAsync(dst + r.dst, src + r.src, sizeof(double) * r.len, hipMemcpyDeviceToHost, s));
        }
    }
    for (int i = 0; i < 2; ++i) HIP_TRY(h, hipStreamSynchronize(h->pipe[i]));
    return BLP_SUCCESS;
}

static void lp_offsets(blp_handle h, int64_t k, int* m, int* n, int64_t* ro, int64_t* co) {
    if (h->uniform) {
        *m = h->plan.m[0];
        *n = h->plan.n[0];
        *ro = k * (int64_t)*m;
        *co = k * (int64_t)*n;
    } else {
        *m = h->plan.m[k];
        *n = h->plan.n[k];
        *ro = h->plan.row_off[k];
        *co = h->plan.col_off[k];
    }
}

blp_error blp_get_solution(blp_handle h, int64_t k, int32_t* status, double* obj, double* x, double* y,
                           int32_t* iters) {
    if (!h) return BLP_ERR_ARG;
    if (!h->solved) return fail(h, BLP_ERR_STATE, "no solve yet");
    if (k < 0 || k >= h->count) return fail(h, BLP_ERR_ARG, "k out of range");
    HIP_TRY(h, hipSetDevice(h->opt.device));
    HIP_TRY(h, wait_last(h));
    int m, n;
    int64_t ro, co;
    lp_offsets(h, k, &m, &n, &ro, &co);
    const KParams& P = h->last;
    if (status) HIP_TRY(h, hipMemcpy(status, P.status + k, sizeof(int32_t), hipMemcpyDeviceToHost));
    if (iters) HIP_TRY(h, hipMemcpy(iters, P.iters + k, sizeof(int32_t), hipMemcpyDeviceToHost));
    if (obj) HIP_TRY(h, hipMemcpy(obj, P.obj + k, sizeof(double), hipMemcpyDeviceToHost));
    if (x && n > 0) HIP_TRY(h, hipMemcpy(x, P.x + co, sizeof(double) * n, hipMemcpyDeviceToHost));
    if (y && m > 0) HIP_TRY(h, hipMemcpy(y, P.y + ro, sizeof(double) * m, hipMemcpyDeviceToHost));
    return BLP_SUCCESS;
}

blp_error blp_get_solution_batch(blp_handle h, int32_t* status, int32_t* iters, double* obj, double* x,
                                 double* y, int32_t on_device) {
    if (!h) return BLP_ERR_ARG;
    if (!h->solved) return fail(h, BLP_ERR_STATE, "no solve yet");
    HIP_TRY(h, hipSetDevice(h->opt.device));
    if (!on_device) HIP_TRY(h, wait_last(h));
    const int64_t K = h->count;
    if (K == 0) return BLP_SUCCESS;
    int64_t tot_m = 0, tot_n = 0;
    for (int64_t k = 0; k < (h->uniform ? 1 : K); ++k) {
        int m, n;
        int64_t ro, co;
        lp_offsets(h, k, &m, &n, &ro, &co);
        tot_m = std::max(tot_m, ro + m);
        tot_n = std::max(tot_n, co + n);
    }
    if (h->uniform) {
        tot_m = K * (int64_t)h->plan.m[0];
        tot_n = K * (int64_t)h->plan.n[0];
    }
    const KParams& P = h->last;
    if (on_device) {
        // device to device on the last solve's stream (ordered after it)
        const hipStream_t s = h->last_stream;
        if (status)
            HIP_TRY(h, hipMemcpyAsync(status, P.status, sizeof(int32_t) * K, hipMemcpyDeviceToDevice, s));
        if (iters) HIP_TRY(h, hipMemcpyAsync(iters, P.iters, sizeof(int32_t) * K, hipMemcpyDeviceToDevice, s));
        if (obj) HIP_TRY(h, hipMemcpyAsync(obj, P.obj, sizeof(double) * K, hipMemcpyDeviceToDevice, s));
        if (x && tot_n > 0) HIP_TRY(h, hipMemcpyAsync(x, P.x, sizeof(double) * tot_n, hipMemcpyDeviceToDevice, s));
        if (y && tot_m > 0) HIP_TRY(h, hipMemcpyAsync(y, P.y, sizeof(double) * tot_m, hipMemcpyDeviceToDevice, s));
        return BLP_SUCCESS;
    }
    if (status) HIP_TRY(h, hipMemcpy(status, P.status, sizeof(int32_t) * K, hipMemcpyDeviceToHost));
    if (iters) HIP_TRY(h, hipMemcpy(iters, P.iters, sizeof(int32_t) * K, hipMemcpyDeviceToHost));
    if (obj) HIP_TRY(h, hipMemcpy(obj, P.obj, sizeof(double) * K, hipMemcpyDeviceToHost));
    if (x && tot_n > 0) HIP_TRY(h, hipMemcpy(x, P.x, sizeof(double) * tot_n, hipMemcpyDeviceToHost));
    if (y && tot_m > 0) HIP_TRY(h, hipMemcpy(y, P.y, sizeof(double) * tot_m, hipMemcpyDeviceToHost));
    return BLP_SUCCESS;
}

blp_error blp_backward(blp_handle h, const double* g, double* dc, double* db, double* dA, double* dl, double* du,
                       void* stream) {
    if (!h) return BLP_ERR_ARG;
    h->err.clear();
    if (!h->solved) return fail(h, BLP_ERR_STATE, "backward before any solve");
    if (h->chunked) return fail(h, BLP_ERR_STATE, "backward after a solve that mem_limit split into chunks");
    if (h->count == 0) return BLP_SUCCESS;
    if (!g) return fail(h, BLP_ERR_ARG, "g is NULL");
    hipStream_t s = static_cast<hipStream_t>(stream);
    HIP_TRY(h, hipSetDevice(h->opt.device));
    HIP_TRY(h, begin_call(h, s));
    KParams P = h->last;
    if (h->any_simplex && (dc || db || dA))
        HIP_TRY(h, launch_backward_simplex(P, g, dc, db, dA, h->plan.max_n, h->plan.max_m, s));
    if (h->any_box && (dc || dl || du)) {
        KParams Q = P;
        Q.bin = h->nreg + 1;
        if (h->box_shared) {
            // per-LP dc; dl, du summed over the LPs into the one box
            if (dc) HIP_TRY(h, launch_backward_hyperbox(Q, P.list ? h->n_box : h->count, g, dc, nullptr, nullptr, s));
            if (dl || du) {
                const size_t nb = (size_t)box_shared_blocks(P.count);
                HIP_TRY(h, h->bwd_part.reserve(sizeof(double) * 2 * (size_t)h->box_n * nb));
                HIP_TRY(h, launch_backward_box_shared(Q, h->box_n, g, h->bwd_part.as<double>(), dl, du, s));
            }
        } else {
            HIP_TRY(h, launch_backward_hyperbox(Q, P.list ? h->n_box : h->count, g, dc, dl, du, s));
        }
    }
    HIP_TRY(h, end_call(h, s));
    return BLP_SUCCESS;
}

// ---------------------------------------------------------------- autotuner
static blp_error write_tuning(blp_handle h, const char* path) {
    hipDeviceProp_t prop;
    HIP_TRY(h, hipGetDeviceProperties(&prop, h->opt.device));
    FILE* f = std::fopen(path, "w");
    if (!f) return fail(h, BLP_ERR_ARG, "cannot write %s", path);
    std::fprintf(f, "{\n  \"arch\": \"%s\",\n  \"cus\": %d,\n  \"remap\": {", prop.gcnArchName, h->cu_count);
    for (int v = 0; v < h->nreg; ++v)
        std::fprintf(f, "%s\n    \"%s\": \"%s\"", v ? "," : "", h->variants[v].name,
                     h->remap[v] < h->nreg ? h->variants[h->remap[v]].name : "streaming");
    std::fprintf(f, "\n  },\n  \"streaming_deep\": %d\n}\n", h->tuned_deep);
    std::fclose(f);
    return BLP_SUCCESS;
}

blp_error blp_load_tuning(blp_handle h, const char* path) {
    if (!h || !path) return BLP_ERR_ARG;
    FILE* f = std::fopen(path, "r");
    if (!f) return fail(h, BLP_ERR_ARG, "cannot read %s", path);
    std::string txt;
    char buf[4096];
    size_t nr;
    while ((nr = std::fread(buf, 1, sizeof buf, f)) > 0) txt.append(buf, nr);
    std::fclose(f);
    hipDeviceProp_t prop;
    HIP_TRY(h, hipGetDeviceProperties(&prop, h->opt.device));
    char want[256];
    std::snprintf(want, sizeof want, "\"arch\": \"%s\"", prop.gcnArchName);
    char cus[64];
    std::snprintf(cus, sizeof cus, "\"cus\": %d", h->cu_count);
    if (txt.find(want) == std::string::npos || txt.find(cus) == std::string::npos)
        return fail(h, BLP_ERR_ARG, "%s was tuned for another device", path);
    auto index_of = [&](const std::string& name) {
        if (name == "streaming") return h->nreg;
        for (int v = 0; v < h->nreg; ++v)
            if (name == h->variants[v].name) return v;
        return -1;
    };
    int remap[kMaxVariants];
    for (int v = 0; v < kMaxVariants; ++v) remap[v] = v;
    for (int v = 0; v < h->nreg; ++v) {
        const std::string key = std::string("\"") + h->variants[v].name + "\": \"";
        const size_t p = txt.find(key);
        if (p == std::string::npos) continue;
        const size_t q = txt.find('"', p + key.size());
        if (q == std::string::npos) return fail(h, BLP_ERR_ARG, "malformed %s", path);
        const int w = index_of(txt.substr(p + key.size(), q - p - key.size()));
        if (w < 0) return fail(h, BLP_ERR_ARG, "unknown variant in %s", path);
        // a replacement must hold every LP of the original bin
        if (!can_replace(h, w, v))
            return fail(h, BLP_ERR_ARG, "%s maps %s to a variant that cannot hold its LPs", path,
                        h->variants[v].name);
        remap[v] = w;
    }
    for (int v = 0; v < kMaxVariants; ++v) h->remap[v] = remap[v];
    // the streaming kernel's depth (absent in older tables: automatic)
    h->tuned_deep = -1;
    const size_t dp = txt.find("\"streaming_deep\": ");
    if (dp != std::string::npos) {
        const int d = std::atoi(txt.c_str() + dp + std::strlen("\"streaming_deep\": "));
        if (d < -1 || d > 1) return fail(h, BLP_ERR_ARG, "malformed streaming_deep in %s", path);
        h->tuned_deep = d;
    }
    if (h->graph_exec) {
        (void)hipGraphExecDestroy(h->graph_exec);
        h->graph_exec = nullptr;
    }
    return BLP_SUCCESS;
}

blp_error blp_tuning(blp_handle h, int32_t* remap, int32_t* n_reg) {
    if (!h) return BLP_ERR_ARG;
    if (n_reg) *n_reg = h->nreg;
    if (remap)
        for (int v = 0; v < h->nreg; ++v) remap[v] = h->remap[v];
    return BLP_SUCCESS;
}

blp_error blp_autotune(blp_handle h, const blp_batch* B, int32_t sample, const char* cache_path, void* stream) {
    if (!h) return BLP_ERR_ARG;
    h->err.clear();
    if (!B || B->count <= 0 || sample <= 0) return fail(h, BLP_ERR_ARG, "autotune needs a non-empty batch and sample > 0");
    hipStream_t s = static_cast<hipStream_t>(stream);
    HIP_TRY(h, hipSetDevice(h->opt.device));
    HIP_TRY(h, begin_call(h, s));
    const int nreg = h->nreg, nbins = nreg + 2;
    // classify with the untuned table
    int saved[kMaxVariants];
    for (int v = 0; v < kMaxVariants; ++v) {
        saved[v] = h->remap[v];
        h->remap[v] = v;
    }
    const int saved_force = h->opt.variant, saved_deep = h->tuned_deep;
    h->opt.variant = -1;
    h->tuned_deep = -1;
    SolvePlan sp;
    blp_error e = prepare(h, B, nullptr, s, sp, /*stream_all=*/true);
    if (e == BLP_SUCCESS) e = enqueue_binning(h, sp, s);
    h->opt.variant = saved_force;
    h->tuned_deep = saved_deep;
    if (e != BLP_SUCCESS || sp.box_only_uniform) {
        for (int v = 0; v < kMaxVariants; ++v) h->remap[v] = saved[v];
        return e;
    }
    std::vector<int32_t> cnt(nbins), off(nbins);
    HIP_TRY(h, hipMemcpyAsync(cnt.data(), sp.P.bin_len, sizeof(int32_t) * nbins, hipMemcpyDeviceToHost, s));
    HIP_TRY(h, hipMemcpyAsync(off.data(), sp.P.bin_off, sizeof(int32_t) * nbins, hipMemcpyDeviceToHost, s));
    HIP_TRY(h, hipStreamSynchronize(s));
    hipEvent_t e0, e1;
    HIP_TRY(h, hipEventCreate(&e0));
    HIP_TRY(h, hipEventCreate(&e1));
    for (int v = 0; v < nreg; ++v) {
        if (cnt[v] == 0) continue;
        const int S = std::min<int>(sample, cnt[v]);
        // scratch: [bin_off = 0, bin_len = S, bin_head] + S list entries
        HIP_TRY(h, h->tune.reserve(sizeof(int32_t) * (4 + (size_t)S)));
        int32_t* tb = h->tune.as<int32_t>();
        int32_t hdr[3] = {0, S, 0};
        HIP_TRY(h, hipMemcpyAsync(tb, hdr, sizeof hdr, hipMemcpyHostToDevice, s));
        HIP_TRY(h, hipMemcpyAsync(tb + 4, sp.list + off[v], sizeof(int32_t) * S,
                                  hipMemcpyDeviceToDevice, s));
        KParams Q = sp.P;
        Q.list = tb + 4;
        Q.bin_off = tb;
        Q.bin_len = tb + 1;
        Q.bin_head = tb + 2;
        Q.bin = 0;
        Q.direct = 0;
        float best_ms = -1.f;
        int best = v;
        for (int w = 0; w <= nreg; ++w) {
            if (!can_replace(h, w, v)) continue;
            float ms = 0.f;
            for (int rep = 0; rep < 2; ++rep) {  // the second run is timed
                HIP_TRY(h, launch_reset(tb + 2, 1, s));
                HIP_TRY(h, hipEventRecord(e0, s));
                if (w < nreg) {
                    HIP_TRY(h, h->variants[w].launch(Q, reg_grid(h, w, S), s));
                } else {
                    HIP_TRY(h, launch_gm(Q, (int)std::min<int64_t>(sp.gm_workers, S), sp.gm_lds, s, sp.gm_deep));
                }
                HIP_TRY(h, hipEventRecord(e1, s));
                HIP_TRY(h, hipEventSynchronize(e1));
                HIP_TRY(h, hipEventElapsedTime(&ms, e0, e1));
            }
            if (best_ms < 0 || ms < best_ms) {
                best_ms = ms;
                best = w;
            }
        }
        saved[v] = best;
    }
    // the streaming kernel's loads in flight per lane (8 or 32), timed on a
    // sample of the streaming bin, each depth with its own occupancy-sized
    // grid (never more workgroups than the workspace has slots)
    int deep = saved_deep;
    if (cnt[nreg] > 0) {
        const int S = std::min<int>(sample, cnt[nreg]);
        HIP_TRY(h, h->tune.reserve(sizeof(int32_t) * (4 + (size_t)S)));
        int32_t* tb = h->tune.as<int32_t>();
        int32_t hdr[3] = {0, S, 0};
        HIP_TRY(h, hipMemcpyAsync(tb, hdr, sizeof hdr, hipMemcpyHostToDevice, s));
        HIP_TRY(h, hipMemcpyAsync(tb + 4, sp.list + off[nreg], sizeof(int32_t) * S, hipMemcpyDeviceToDevice, s));
        KParams Q = sp.P;
        Q.list = tb + 4;
        Q.bin_off = tb;
        Q.bin_len = tb + 1;
        Q.bin_head = tb + 2;
        Q.bin = 0;
        Q.direct = 0;
        float best_ms = -1.f;
        for (int d = 0; d < 2; ++d) {
            int occ = 1;
            size_t lds = 0;
            gm_lds_plan(h, sp.gm_ld, sp.gm_cols, d != 0, sp.gm_shared, &lds, &Q.ws_lds, &occ);
            const int grid = (int)std::min<int64_t>(std::min<int64_t>((int64_t)occ * h->cu_count, sp.gm_workers), S);
            float ms = 0.f;
            for (int rep = 0; rep < 2; ++rep) {  // the second run is timed
                HIP_TRY(h, launch_reset(tb + 2, 1, s));
                HIP_TRY(h, hipEventRecord(e0, s));
                HIP_TRY(h, launch_gm(Q, grid, lds, s, d != 0));
                HIP_TRY(h, hipEventRecord(e1, s));
                HIP_TRY(h, hipEventSynchronize(e1));
                HIP_TRY(h, hipEventElapsedTime(&ms, e0, e1));
            }
            if (best_ms < 0 || ms < best_ms) {
                best_ms = ms;
                deep = d;
            }
        }
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    for (int v = 0; v < kMaxVariants; ++v) h->remap[v] = saved[v];
    h->tuned_deep = deep;
    if (h->graph_exec) {
        (void)hipGraphExecDestroy(h->graph_exec);
        h->graph_exec = nullptr;
    }
    HIP_TRY(h, end_call(h, s));
    h->solved = false;  // the handle's outputs hold tuning runs, not a solve
    if (cache_path) return write_tuning(h, cache_path);
    return BLP_SUCCESS;
}

blp_error blp_last_kernel_ms(blp_handle h, double* ms, int32_t* n_entries) {
    if (!h) return BLP_ERR_ARG;
    const int n = h->nreg + 3;
    if (n_entries) *n_entries = n;
    if (!ms) return BLP_SUCCESS;
    for (int i = 0; i < n; ++i) ms[i] = 0.0;
    if (!h->solved) return fail(h, BLP_ERR_STATE, "no solve yet");
    if (!h->opt.profile || h->count == 0) return BLP_SUCCESS;
    HIP_TRY(h, hipSetDevice(h->opt.device));
    HIP_TRY(h, wait_last(h));
    for (int i = 0; i < n && i < (int)h->ev_used.size(); ++i) {
        if (!h->ev_used[i]) continue;
        float t = 0.f;
        HIP_TRY(h, hipEventElapsedTime(&t, h->ev0[i], h->ev1[i]));
        ms[i] = t;
    }
    return BLP_SUCCESS;
}

blp_error blp_last_bins(blp_handle h, int64_t* counts, int32_t* n_classes) {
    if (!h) return BLP_ERR_ARG;
    const int nbins = h->nreg + 2;
    if (n_classes) *n_classes = nbins;
    if (!counts) return BLP_SUCCESS;
    if (!h->solved) return fail(h, BLP_ERR_STATE, "no solve yet");
    HIP_TRY(h, hipSetDevice(h->opt.device));
    HIP_TRY(h, wait_last(h));
    std::vector<int32_t> c(nbins, 0);
    if (h->direct_v >= 0) {
        c[h->direct_v] = (int32_t)h->count;
    } else if (h->last.list) {
        HIP_TRY(h, hipMemcpy(c.data(), h->last.bin_len, sizeof(int32_t) * nbins, hipMemcpyDeviceToHost));
    } else {
        c[h->nreg + 1] = (int32_t)h->count;
    }
    for (int b = 0; b < nbins; ++b) counts[b] = c[b];
    return BLP_SUCCESS;
}

}  // extern "C"
