/*
 * Seeded synthetic LP inputs for the batched simplex solver and its oracle.
 *
 * This module only draws random numbers and lays them out; it contains none
 * of the simplex arithmetic.  Both the GPU path's tests/benchmarks and the CPU
 * oracle's tests take their inputs from here, so the two always see the same
 * bytes.
 *
 * Random source: Philox4x32-10, the counter-based generator of Salmon, Moraes,
 * Dror and Shaw ("Parallel Random Numbers: As Easy as 1, 2, 3", SC'11).  One
 * generator call per drawn value, keyed by the config seed and addressed by
 * (LP id, field, element index), so any subset of a batch can be regenerated
 * independently and in any order.
 *
 * Workload shapes follow the paper's three LP families (abstract; Sec. 4.6 and
 * Sec. 6): type 1 = all rows "<=" with b > 0 (origin feasible), type 2 = half
 * "<=" rows and half ">=" rows built around an interior point x0 (origin
 * infeasible, needs phase 1), type 3 = hyperbox l <= x <= u (Eq. 7).
 */
#include <math.h>
#include <stdint.h>
#include <string.h>

#define PHILOX_M0 0xD2511F53u
#define PHILOX_M1 0xCD9E8D57u
#define PHILOX_W0 0x9E3779B9u
#define PHILOX_W1 0xBB67AE85u

/* One Philox4x32 round: two 32x32->64 multiplies, xor with the other words
 * and the round key, then a word permutation. */
static inline void philox_round(uint32_t x[4], const uint32_t k[2]) {
    uint64_t p0 = (uint64_t)PHILOX_M0 * (uint64_t)x[0];
    uint64_t p1 = (uint64_t)PHILOX_M1 * (uint64_t)x[2];
    uint32_t hi0 = (uint32_t)(p0 >> 32), lo0 = (uint32_t)p0;
    uint32_t hi1 = (uint32_t)(p1 >> 32), lo1 = (uint32_t)p1;
    uint32_t y0 = hi1 ^ x[1] ^ k[0];
    uint32_t y2 = hi0 ^ x[3] ^ k[1];
    x[0] = y0;
    x[1] = lo1;
    x[2] = y2;
    x[3] = lo0;
}

/* Philox4x32 with 10 rounds; the key is bumped by the Weyl constants between
 * rounds. */
void lpgen_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4]) {
    uint32_t x[4] = {ctr[0], ctr[1], ctr[2], ctr[3]};
    uint32_t k[2] = {key[0], key[1]};
    for (int r = 0; r < 10; ++r) {
        if (r > 0) {
            k[0] += PHILOX_W0;
            k[1] += PHILOX_W1;
        }
        philox_round(x, k);
    }
    memcpy(out, x, sizeof x);
}

/* Field identifiers: which input array a drawn value belongs to. */
enum {
    F_A = 1, F_B = 2, F_C = 3, F_X0 = 4, F_DELTA = 5, F_M = 6, F_N = 7,
    F_CLASS = 8, F_L = 9, F_U = 10, F_G = 11, F_W = 12
};

static inline void draw(uint64_t seed, uint64_t lp, uint32_t field, uint32_t idx, uint32_t out[4]) {
    uint32_t ctr[4] = {idx, (uint32_t)lp, field, (uint32_t)(lp >> 32)};
    uint32_t key[2] = {(uint32_t)seed, (uint32_t)(seed >> 32)};
    lpgen_philox4x32_10(ctr, key, out);
}

/* 53-bit uniform in [0, 1) from the first two output words. */
static inline double u53(const uint32_t w[4]) {
    uint64_t a = w[0] >> 5, b = w[1] >> 6; /* 27 + 26 bits */
    return (double)(a * 67108864ull + b) * (1.0 / 9007199254740992.0);
}

double lpgen_uniform(uint64_t seed, uint64_t lp, uint32_t field, uint32_t idx) {
    uint32_t w[4];
    draw(seed, lp, field, idx, w);
    return u53(w);
}

static inline double unif(uint64_t seed, uint64_t lp, uint32_t field, uint32_t idx, double lo, double hi) {
    return lo + (hi - lo) * lpgen_uniform(seed, lp, field, idx);
}

/* Integer uniform on {lo..hi}. */
int32_t lpgen_uniform_int(uint64_t seed, uint64_t lp, uint32_t field, uint32_t idx, int32_t lo, int32_t hi) {
    double u = lpgen_uniform(seed, lp, field, idx);
    int32_t v = lo + (int32_t)floor(u * (double)(hi - lo + 1));
    return v > hi ? hi : v;
}

/* Standard normal by Box-Muller from the four output words of one call. */
double lpgen_normal(uint64_t seed, uint64_t lp, uint32_t field, uint32_t idx) {
    uint32_t w[4];
    draw(seed, lp, field, idx, w);
    double u1 = 1.0 - u53(w); /* (0, 1] */
    uint32_t w2[4] = {w[2], w[3], 0, 0};
    double u2 = u53(w2);
    return sqrt(-2.0 * log(u1)) * cos(6.283185307179586 * u2);
}

/* Distribution parameters for one workload. */
typedef struct {
    double a_lo, a_hi;      /* A_ij ~ U(a_lo, a_hi)                     */
    double b_lo, b_hi;      /* type 1: b_i ~ U(b_lo, b_hi)              */
    double c_lo, c_hi;      /* simplex: c_j ~ U(c_lo, c_hi)             */
    double x0_lo, x0_hi;    /* type 2: interior point x0 ~ U(..)^n      */
    double d_lo, d_hi;      /* type 2: row offset delta_i ~ U(..)       */
    double l_lo, l_hi;      /* hyperbox: l_i ~ U(..)                    */
    double u_lo, u_hi;      /* hyperbox: u_i ~ U(..)                    */
    int32_t box_c_unit;     /* hyperbox: 1 -> c = g/|g|, g ~ N(0, I)    */
    int32_t pad_;
} lpgen_params;

/* Fill one LP.  type: 1, 2 (simplex) or 3 (hyperbox).  A is row-major m x n.
 * For hyperbox LPs m is ignored and c, l, u (length n) are written. */
static void gen_one(uint64_t seed, uint64_t lp, int32_t type, int32_t m, int32_t n,
                    const lpgen_params* p, double* A, double* b, int8_t* sense,
                    double* c, double* l, double* u) {
    if (type == 3) {
        for (int32_t j = 0; j < n; ++j) {
            l[j] = unif(seed, lp, F_L, (uint32_t)j, p->l_lo, p->l_hi);
            u[j] = unif(seed, lp, F_U, (uint32_t)j, p->u_lo, p->u_hi);
            c[j] = lpgen_normal(seed, lp, F_G, (uint32_t)j);
        }
        if (p->box_c_unit) {
            double s = 0.0;
            for (int32_t j = 0; j < n; ++j) s += c[j] * c[j];
            s = sqrt(s);
            if (s > 0.0)
                for (int32_t j = 0; j < n; ++j) c[j] = c[j] / s;
        }
        return;
    }
    for (int32_t i = 0; i < m; ++i)
        for (int32_t j = 0; j < n; ++j)
            A[(int64_t)i * n + j] = unif(seed, lp, F_A, (uint32_t)((int64_t)i * n + j), p->a_lo, p->a_hi);
    for (int32_t j = 0; j < n; ++j) c[j] = unif(seed, lp, F_C, (uint32_t)j, p->c_lo, p->c_hi);
    if (type == 1) {
        for (int32_t i = 0; i < m; ++i) {
            b[i] = unif(seed, lp, F_B, (uint32_t)i, p->b_lo, p->b_hi);
            sense[i] = 0;
        }
        return;
    }
    /* type 2: the first floor(m/2) rows are "<=", the rest ">="; both pass
     * through x0 with a random margin so x0 is strictly feasible. */
    double x0[4096];
    for (int32_t j = 0; j < n; ++j) x0[j] = unif(seed, lp, F_X0, (uint32_t)j, p->x0_lo, p->x0_hi);
    int32_t n_le = m / 2;
    for (int32_t i = 0; i < m; ++i) {
        double ax = 0.0;
        for (int32_t j = 0; j < n; ++j) ax += A[(int64_t)i * n + j] * x0[j];
        double d = unif(seed, lp, F_DELTA, (uint32_t)i, p->d_lo, p->d_hi);
        if (i < n_le) {
            b[i] = ax + d;
            sense[i] = 0;
        } else {
            b[i] = ax - d;
            sense[i] = 1;
        }
    }
}

/* Fill a batch.  lp_ids[k] is the generator address of batch entry k; the
 * offsets locate each LP's slices in the packed output arrays (A by a_off,
 * b/sense by row_off, c/l/u by col_off).  Entries are independent, so the
 * loop is split across OpenMP threads. */
void lpgen_batch(uint64_t seed, int64_t count, const int64_t* lp_ids, const int32_t* type,
                 const int32_t* m, const int32_t* n, const int64_t* a_off, const int64_t* row_off,
                 const int64_t* col_off, const lpgen_params* p, double* A, double* b, int8_t* sense,
                 double* c, double* l, double* u) {
#pragma omp parallel for schedule(dynamic, 16)
    for (int64_t k = 0; k < count; ++k) {
        int32_t t = type[k];
        gen_one(seed, (uint64_t)lp_ids[k], t, m[k], n[k], p,
                t == 3 ? 0 : A + a_off[k], t == 3 ? 0 : b + row_off[k], t == 3 ? 0 : sense + row_off[k],
                c + col_off[k], t == 3 ? l + col_off[k] : 0, t == 3 ? u + col_off[k] : 0);
    }
}

/* Per-LP shape/class draws for mixed workloads: m, n ~ U{lo..hi}; the class
 * comes from one uniform compared against cumulative fractions. */
void lpgen_shapes(uint64_t seed, int64_t count, const int64_t* lp_ids, int32_t mn_lo, int32_t mn_hi,
                  int32_t square, double frac_t1, double frac_t2, int32_t* type, int32_t* m, int32_t* n) {
#pragma omp parallel for schedule(static)
    for (int64_t k = 0; k < count; ++k) {
        uint64_t lp = (uint64_t)lp_ids[k];
        int32_t mm = lpgen_uniform_int(seed, lp, F_M, 0, mn_lo, mn_hi);
        int32_t nn = square ? mm : lpgen_uniform_int(seed, lp, F_N, 0, mn_lo, mn_hi);
        double u = lpgen_uniform(seed, lp, F_CLASS, 0);
        int32_t t = u < frac_t1 ? 1 : (u < frac_t1 + frac_t2 ? 2 : 3);
        type[k] = t;
        m[k] = t == 3 ? 0 : mm;
        n[k] = nn;
    }
}

/* Loss weights w_k ~ U(lo, hi). */
void lpgen_weights(uint64_t seed, int64_t count, const int64_t* lp_ids, double lo, double hi, double* w) {
#pragma omp parallel for schedule(static)
    for (int64_t k = 0; k < count; ++k) w[k] = unif(seed, (uint64_t)lp_ids[k], F_W, 0, lo, hi);
}
