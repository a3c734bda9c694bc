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
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <string>
#include <vector>

#include "aux_kernels.hpp"
#include "blp.h"
#include "blp_kernels.hpp"
#include "variants.hpp"

using namespace blp;

namespace {

constexpr int kMaxM = 2046;     // rows of one LP
constexpr int kMaxCols = 4096;  // n + m + 1 (condensed columns, worst case)

struct DevBuf {
    void* p = nullptr;
    size_t bytes = 0;
    hipError_t reserve(size_t want) {
        if (want <= bytes) return hipSuccess;
        if (p) {
            hipError_t e = hipFree(p);
            if (e != hipSuccess) return e;
            p = nullptr;
            bytes = 0;
        }
        size_t cap = std::max(want, bytes + bytes / 2);
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

}  // namespace

struct blp_handle_s {
    blp_options opt;
    std::string err;
    int cu_count = 0;
    const RegVariant* variants = nullptr;
    int nreg = 0;
    std::vector<int> reg_workers;  // persistent grid per variant
    int gm_occ = 1;
    // device buffers
    DevBuf meta;     // m, n, kind (int32) + a_off, row_off, col_off (int64) for non-uniform batches
    DevBuf counters; // bin_count, bin_fill, bin_head, bin_off (4 x nbins int32)
    DevBuf binid, list;
    DevBuf ws;       // streaming-kernel workspace
    DevBuf own_status, own_iters, own_obj, own_x, own_y;
    // last solve
    bool solved = false;
    KParams last{};
    hipStream_t last_stream = nullptr;
    std::vector<int32_t> h_m, h_n, h_kind;
    std::vector<int64_t> h_row_off, h_col_off, h_a_off;
    int64_t count = 0;
    bool uniform = false;
    bool any_simplex = false, any_box = false;
    int64_t n_box = 0;
};

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
    h->variants = reg_variants(&h->nreg);
    if (o.variant >= h->nreg) {
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
    *out = h;
    return BLP_SUCCESS;
}

void blp_destroy(blp_handle h) {
    if (!h) return;
    (void)hipSetDevice(h->opt.device);
    (void)hipDeviceSynchronize();
    h->meta.release();
    h->counters.release();
    h->binid.release();
    h->list.release();
    h->ws.release();
    h->own_status.release();
    h->own_iters.release();
    h->own_obj.release();
    h->own_x.release();
    h->own_y.release();
    delete h;
}

const char* blp_last_error(blp_handle h) { return h ? h->err.c_str() : "null handle"; }

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
    if (!B->m || !B->n || !B->kind) return fail(h, BLP_ERR_ARG, "m, n and kind are required");
    // ---- host-side validation and packed offsets
    const bool uni = B->uniform != 0;
    const int64_t nmeta = uni ? 1 : K;
    h->h_m.assign(B->m, B->m + nmeta);
    h->h_n.assign(B->n, B->n + nmeta);
    h->h_kind.assign(B->kind, B->kind + nmeta);
    bool any_simplex = false, any_box = false;
    int64_t n_box = 0, tot_a = 0, tot_m = 0, tot_n = 0;
    int max_m = 0, max_cols = 0;
    for (int64_t k = 0; k < nmeta; ++k) {
        const int m = h->h_m[k], n = h->h_n[k], kd = h->h_kind[k];
        if (kd == BLP_KIND_SIMPLEX) {
            if (m < 1 || n < 1) return fail(h, BLP_ERR_ARG, "LP %lld: simplex LP needs m >= 1 and n >= 1", (long long)k);
            if (m > kMaxM || (int64_t)n + m + 1 > kMaxCols)
                return fail(h, BLP_ERR_TOO_LARGE, "LP %lld: m=%d n=%d exceeds m <= %d, n + m + 1 <= %d",
                            (long long)k, m, n, kMaxM, kMaxCols);
            any_simplex = true;
            max_m = std::max(max_m, m);
            max_cols = std::max(max_cols, n + m + 1);
        } else if (kd == BLP_KIND_HYPERBOX) {
            if (m != 0 || n < 1) return fail(h, BLP_ERR_ARG, "LP %lld: hyperbox LP needs m == 0 and n >= 1", (long long)k);
            any_box = true;
            ++n_box;
        } else {
            return fail(h, BLP_ERR_ARG, "LP %lld: kind %d is not 0 or 1", (long long)k, kd);
        }
        tot_a += (int64_t)m * n;
        tot_m += m;
        tot_n += n;
    }
    if (uni) {
        n_box *= K;
        tot_a *= K;
        tot_m *= K;
        tot_n *= K;
    }
    if (any_simplex && (!B->A || !B->b || !B->sense || !B->c)) return fail(h, BLP_ERR_ARG, "A, b, sense, c required");
    if (any_box && (!B->c || !B->l || !B->u)) return fail(h, BLP_ERR_ARG, "c, l, u required for hyperbox LPs");
    if (!uni) {
        h->h_a_off.resize(K);
        h->h_row_off.resize(K);
        h->h_col_off.resize(K);
        int64_t ao = 0, ro = 0, co = 0;
        for (int64_t k = 0; k < K; ++k) {
            h->h_a_off[k] = B->a_off ? B->a_off[k] : ao;
            h->h_row_off[k] = B->row_off ? B->row_off[k] : ro;
            h->h_col_off[k] = B->col_off ? B->col_off[k] : co;
            if (h->h_a_off[k] < 0 || h->h_row_off[k] < 0 || h->h_col_off[k] < 0)
                return fail(h, BLP_ERR_ARG, "LP %lld: negative offset", (long long)k);
            ao += (int64_t)h->h_m[k] * h->h_n[k];
            ro += h->h_m[k];
            co += h->h_n[k];
        }
        if (!B->a_off || !B->row_off || !B->col_off) {
            tot_a = std::max(tot_a, ao);
            tot_m = std::max(tot_m, ro);
            tot_n = std::max(tot_n, co);
        }
        for (int64_t k = 0; k < K; ++k) {
            tot_a = std::max(tot_a, h->h_a_off[k] + (int64_t)h->h_m[k] * h->h_n[k]);
            tot_m = std::max(tot_m, h->h_row_off[k] + h->h_m[k]);
            tot_n = std::max(tot_n, h->h_col_off[k] + h->h_n[k]);
        }
    }

    // ---- outputs
    blp_outputs o{};
    if (out) o = *out;
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
    KParams P{};
    P.count = K;
    P.uniform = uni ? 1 : 0;
    P.um = h->h_m[0];
    P.un = h->h_n[0];
    P.ukind = h->h_kind[0];
    if (!uni) {
        const size_t bytes = (size_t)K * (3 * sizeof(int32_t) + 3 * sizeof(int64_t));
        HIP_TRY(h, h->meta.reserve(bytes));
        char* base = h->meta.as<char>();
        int64_t* offs = reinterpret_cast<int64_t*>(base);
        int32_t* ints = reinterpret_cast<int32_t*>(base + (size_t)K * 3 * sizeof(int64_t));
        HIP_TRY(h, hipMemcpyAsync(offs, h->h_a_off.data(), K * sizeof(int64_t), hipMemcpyHostToDevice, s));
        HIP_TRY(h, hipMemcpyAsync(offs + K, h->h_row_off.data(), K * sizeof(int64_t), hipMemcpyHostToDevice, s));
        HIP_TRY(h, hipMemcpyAsync(offs + 2 * K, h->h_col_off.data(), K * sizeof(int64_t), hipMemcpyHostToDevice, s));
        HIP_TRY(h, hipMemcpyAsync(ints, h->h_m.data(), K * sizeof(int32_t), hipMemcpyHostToDevice, s));
        HIP_TRY(h, hipMemcpyAsync(ints + K, h->h_n.data(), K * sizeof(int32_t), hipMemcpyHostToDevice, s));
        HIP_TRY(h, hipMemcpyAsync(ints + 2 * K, h->h_kind.data(), K * sizeof(int32_t), hipMemcpyHostToDevice, s));
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

    const int nreg = h->nreg, nbins = nreg + 2;
    const int BIN_GM = nreg, BIN_BOX = nreg + 1;
    HIP_TRY(h, h->counters.reserve(sizeof(int32_t) * 4 * nbins));
    int32_t* bin_count = h->counters.as<int32_t>();
    int32_t* bin_fill = bin_count + nbins;
    int32_t* bin_head = bin_fill + nbins;
    int32_t* bin_off = bin_head + nbins;
    P.bin_off = bin_off;
    P.bin_len = bin_count;
    P.bin_head = bin_head;

    // ---- binning (not needed for an all-hyperbox uniform batch)
    const bool box_only_uniform = uni && !any_simplex;
    if (!box_only_uniform) {
        HIP_TRY(h, h->binid.reserve(sizeof(int32_t) * K));
        HIP_TRY(h, h->list.reserve(sizeof(int32_t) * K));
        VariantTable vt{};
        vt.nreg = nreg;
        vt.force = h->opt.variant;
        for (int v = 0; v < nreg && v < kMaxVariants; ++v) {
            vt.rows[v] = h->variants[v].max_rows;
            vt.cols[v] = h->variants[v].max_cols;
        }
        HIP_TRY(h, launch_reset(bin_count, 3 * nbins, s));
        HIP_TRY(h, launch_classify(P, vt, h->binid.as<int32_t>(), bin_count, s));
        HIP_TRY(h, launch_bin_offsets(bin_count, bin_off, nbins, s));
        HIP_TRY(h, launch_scatter(K, h->binid.as<int32_t>(), bin_off, bin_fill, h->list.as<int32_t>(), s));
        P.list = h->list.as<int32_t>();
    } else {
        P.list = nullptr;
    }

    // Which register variants can receive an LP?  For a uniform simplex batch
    // only those chosen for some n_art in [0, m]; otherwise all.
    std::vector<char> maybe(nreg, 0);
    if (h->opt.variant >= 0) {
        maybe[h->opt.variant] = 1;
    } else if (h->opt.variant == -1) {
        if (uni && any_simplex) {
            const int m = h->h_m[0], n = h->h_n[0];
            for (int nart = 0; nart <= m; ++nart) {
                int best = -1;
                long barea = -1;
                for (int v = 0; v < nreg; ++v)
                    if (h->variants[v].max_rows >= m + 2 && h->variants[v].max_cols >= n + nart + 1) {
                        long a = (long)h->variants[v].max_rows * h->variants[v].max_cols;
                        if (barea < 0 || a < barea) {
                            barea = a;
                            best = v;
                        }
                    }
                if (best >= 0) maybe[best] = 1;
            }
        } else if (any_simplex) {
            std::fill(maybe.begin(), maybe.end(), 1);
        }
    }
    // Streaming-kernel geometry: worst case over the batch's simplex LPs.
    const int gm_ld = ((max_m + 2 + 63) / 64) * 64;
    const int gm_cols = max_cols;
    const size_t gm_lds = any_simplex ? gm_lds_bytes_host(gm_ld, gm_cols) : 0;
    int gm_workers = 0;
    if (any_simplex) {
        int occ = 0;
        if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&occ, gm_kernel_ptr(), gm_threads(), gm_lds) != hipSuccess ||
            occ < 1)
            occ = 1;
        if (h->opt.workers_per_cu > 0) occ = std::min(occ, (int)h->opt.workers_per_cu);
        gm_workers = occ * h->cu_count;
        const size_t slot = (size_t)gm_ld * gm_cols;
        HIP_TRY(h, h->ws.reserve(sizeof(double) * slot * (size_t)gm_workers));
        P.ws = h->ws.as<double>();
        P.ws_slot = (int64_t)slot;
        P.ws_ld = gm_ld;
        P.ws_cols = gm_cols;
    }

    const int mode = h->opt.mode;
    if (mode == BLP_MODE_PERSISTENT) {
        P.direct = 0;
        for (int v = 0; v < nreg; ++v) {
            if (!maybe[v]) continue;
            KParams Q = P;
            Q.bin = v;
            const int grid = (int)std::min<int64_t>(h->reg_workers[v], K);
            HIP_TRY(h, h->variants[v].launch(Q, grid, s));
        }
        if (any_simplex) {
            KParams Q = P;
            Q.bin = BIN_GM;
            const int grid = (int)std::min<int64_t>(gm_workers, K);
            HIP_TRY(h, launch_gm(Q, grid, gm_lds, s));
        }
    } else {
        // grid / one-per-launch: read the bins back to size the launches
        std::vector<int32_t> cnt(nbins, 0);
        if (!box_only_uniform) {
            HIP_TRY(h, hipMemcpyAsync(cnt.data(), bin_count, sizeof(int32_t) * nbins, hipMemcpyDeviceToHost, s));
            HIP_TRY(h, hipStreamSynchronize(s));
        }
        P.direct = 1;
        for (int v = 0; v <= nreg; ++v) {
            const int64_t nv = cnt[v];
            if (nv == 0) continue;
            KParams Q = P;
            Q.bin = v;
            const int64_t chunk = v == BIN_GM ? gm_workers : (mode == BLP_MODE_GRID ? nv : 1);
            for (int64_t first = 0; first < nv; first += chunk) {
                Q.direct_first = first;
                const int grid = (int)std::min<int64_t>(chunk, nv - first);
                if (v == BIN_GM) {
                    if (mode == BLP_MODE_GRID) {
                        HIP_TRY(h, launch_gm(Q, grid, gm_lds, s));
                    } else {
                        for (int64_t q = first; q < first + grid; ++q) {
                            Q.direct_first = q;
                            HIP_TRY(h, launch_gm(Q, 1, gm_lds, s));
                        }
                    }
                } else {
                    HIP_TRY(h, h->variants[v].launch(Q, grid, s));
                }
            }
        }
        P.direct = 0;
    }
    if (any_box) {
        KParams Q = P;
        Q.bin = BIN_BOX;
        Q.direct = 0;
        HIP_TRY(h, launch_hyperbox(Q, box_only_uniform ? K : n_box, s));
    }
    HIP_TRY(h, hipGetLastError());

    h->last = P;
    h->last_stream = s;
    h->count = K;
    h->uniform = uni;
    h->any_simplex = any_simplex;
    h->any_box = any_box;
    h->n_box = n_box;
    h->solved = true;
    return BLP_SUCCESS;
}

static void lp_offsets(blp_handle h, int64_t k, int* m, int* n, int64_t* ro, int64_t* co) {
    if (h->uniform) {
        *m = h->h_m[0];
        *n = h->h_n[0];
        *ro = k * (int64_t)*m;
        *co = k * (int64_t)*n;
    } else {
        *m = h->h_m[k];
        *n = h->h_n[k];
        *ro = h->h_row_off[k];
        *co = h->h_col_off[k];
    }
}

blp_error blp_get_solution(blp_handle h, int64_t k, int32_t* status, double* obj, double* x, double* y,
                           int32_t* iters) {
    if (!h) return BLP_ERR_ARG;
    if (!h->solved) return fail(h, BLP_ERR_STATE, "no solve yet");
    if (k < 0 || k >= h->count) return fail(h, BLP_ERR_ARG, "k out of range");
    HIP_TRY(h, hipSetDevice(h->opt.device));
    HIP_TRY(h, hipStreamSynchronize(h->last_stream));
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
                                 double* y) {
    if (!h) return BLP_ERR_ARG;
    if (!h->solved) return fail(h, BLP_ERR_STATE, "no solve yet");
    HIP_TRY(h, hipSetDevice(h->opt.device));
    HIP_TRY(h, hipStreamSynchronize(h->last_stream));
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
        tot_m = K * (int64_t)h->h_m[0];
        tot_n = K * (int64_t)h->h_n[0];
    }
    const KParams& P = h->last;
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
    if (h->count == 0) return BLP_SUCCESS;
    if (!g) return fail(h, BLP_ERR_ARG, "g is NULL");
    hipStream_t s = static_cast<hipStream_t>(stream);
    HIP_TRY(h, hipSetDevice(h->opt.device));
    KParams P = h->last;
    if (h->any_simplex && (dc || db || dA)) HIP_TRY(h, launch_backward_simplex(P, g, dc, db, dA, s));
    if (h->any_box && (dc || dl || du)) {
        KParams Q = P;
        Q.bin = h->nreg + 1;
        HIP_TRY(h, launch_backward_hyperbox(Q, P.list ? h->n_box : h->count, g, dc, dl, du, s));
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
    HIP_TRY(h, hipStreamSynchronize(h->last_stream));
    std::vector<int32_t> c(nbins, 0);
    if (h->last.list) {
        HIP_TRY(h, hipMemcpy(c.data(), h->last.bin_len, sizeof(int32_t) * nbins, hipMemcpyDeviceToHost));
    } else {
        c[h->nreg + 1] = (int32_t)h->count;
    }
    for (int b = 0; b < nbins; ++b) counts[b] = c[b];
    return BLP_SUCCESS;
}

}  // extern "C"
