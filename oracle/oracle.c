/*
 * ORACLE -- test infrastructure only.
 *
 * A plain, slow, deliberately unoptimised CPU implementation of what the
 * batched LP solver computes, used to check the GPU path.  Only the test
 * suite, the smoke check and the benchmark's CPU-baseline leg may load it; the
 * solver itself never calls it, and the two share no code.
 *
 * What it computes (Gurung & Ray, "Solving Batched Linear Programs on GPU and
 * Multicore CPU"):
 *   - Sec. 3, Eqs. (1)-(3): maximise sum_j c_j x_j subject to
 *     sum_j a_ij x_j <= b_i (or >= b_i), x >= 0.
 *   - Sec. 3, Eq. (4): one logical (slack) variable per row; the initial basis
 *     is the logical variables, which is infeasible when a row's right-hand
 *     side is negative in "<=" form.  Such LPs go through the two-phase method
 *     of Sec. 3: artificial variables whose sum is the auxiliary objective,
 *     phase II only if that optimum is zero.
 *   - Sec. 3.1, Steps 1-3 on a dense simplex tableau: entering column = index
 *     of the largest objective-row coefficient (the LPC rule of Sec. 4.2),
 *     leaving row = minimum ratio over rows, pivot = divide the pivot row by
 *     the pivot element, subtract PivotCol_i * NewPivotRow_j from every other
 *     row (Sec. 4.3, the step-3 update).
 *   - Sec. 3.1 halt conditions: unbounded when no row limits the entering
 *     variable, optimal when no objective-row coefficient is positive.
 *   - Sec. 6, Eq. (7): hyperbox LPs in closed form.
 *
 * Readings where the paper is silent or loose (each one is listed with its
 * reason in the design notes of the repository):
 *   R1  the ratio test uses the standard tableau sign convention: candidate
 *       rows have T[i][e] > eps_piv, ratio T[i][rhs] / T[i][e];
 *   R2  "minimum positive ratio" admits zero: a candidate row whose rhs is
 *       <= 0 offers a step of exactly 0 (degenerate pivot);
 *   R3  no INT_MAX sentinel is needed here (plain loop); "no candidate" means
 *       unbounded;
 *   R4  optimality: every eligible objective coefficient <= eps_price;
 *   R5  entering ties go to the lowest column (= variable) index;
 *   R6  leaving ties (equal computed ratios) go to the smallest basic
 *       variable index;
 *   R7  after max(m, n) consecutive degenerate pivots the entering rule
 *       switches to "lowest index with a positive coefficient" (Bland) until
 *       a pivot with a nonzero step;
 *   R8  eps_price = eps_piv = eps_feas = 1e-9 by default;
 *   R9  one artificial variable per row whose "<=" form has a negative rhs;
 *   R10 phase 1 ends feasible when the auxiliary value is within
 *       eps_feas * (1 + w0) of zero; artificials still basic are pivoted out
 *       on the lowest-index non-artificial column with |entry| > eps_piv,
 *       otherwise their row is redundant ("dead") and ignored afterwards;
 *       artificial columns never enter the basis;
 *   R11 the update covers every row except the pivot row, objective rows
 *       included;
 *   R12 pricing scans every non-artificial column, logical ones included;
 *   R13 at most max_iter pivots (default 50 (m + n)), then ITER_LIMIT;
 *   R14 hyperbox: h_i = l_i if c_i < 0 else u_i (Eq. 7's "otherwise" case
 *       takes the upper bound when c_i = 0); the sum runs in increasing i;
 *   R15 hyperbox with some l_i > u_i is infeasible;
 *   R18 everything in IEEE binary64; the update is one fused multiply-add per
 *       element, the pivot row one IEEE division per element.
 *
 * Tableau used here (the paper's Fig. "Formation of the Simplex Tableau"
 * with the basis kept in its own array): R = m + 1 (+1 for the phase-1 row)
 * rows, C = n + m + n_art + 1 columns ordered x_1..x_n, logical variables in
 * row order, artificial variables in row order, right-hand side.  Row m is
 * the objective row holding d_j = c_j - z_j and -z in its rhs cell; row m+1
 * is the phase-1 row.  Stored row-major, the plainest layout.
 *
 * Compile with -ffp-contract=off so that only the explicit fma() calls fuse.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

enum { ST_OPTIMAL = 0, ST_INFEASIBLE = 1, ST_UNBOUNDED = 2, ST_ITER_LIMIT = 3, ST_NUMERICAL = 4 };

typedef struct {
    int32_t max_iter;     /* <= 0: 50 * (m + n)                   */
    int32_t bland_after;  /* <= 0: max(m, n) degenerate pivots     */
    double eps_price;     /* <= 0: 1e-9                            */
    double eps_piv;       /* <= 0: 1e-9                            */
    double eps_feas;      /* <= 0: 1e-9                            */
} oracle_opts;

typedef struct {
    int32_t m, n, R, C, n_art;
    double* T;          /* R x C, row-major */
    int32_t* basis;     /* m: column index of the basic variable of each row */
    uint8_t* dead;      /* m: redundant row found at the end of phase 1 */
    int32_t* trace;     /* optional (row, col) per pivot */
    int32_t trace_cap;
} tab_t;

#define T_(tb, i, j) ((tb)->T[(int64_t)(i) * (tb)->C + (j)])

/* Step 3 (Sec. 4.3): NewPivotRow = OldPivotRow / PE; every other row i gets
 * NewRow_ij = OldRow_ij - PivotCol_i * NewPivotRow_j.  The pivot column then
 * becomes the unit vector of the entering variable. */
static void pivot(tab_t* tb, int32_t l, int32_t e, int32_t iter) {
    const int32_t R = tb->R, C = tb->C;
    double* f = (double*)malloc(sizeof(double) * (size_t)R);
    double* p = (double*)malloc(sizeof(double) * (size_t)C);
    double pe = T_(tb, l, e);
    for (int32_t i = 0; i < R; ++i) f[i] = T_(tb, i, e);
    for (int32_t j = 0; j < C; ++j) p[j] = T_(tb, l, j) / pe;
    for (int32_t i = 0; i < R; ++i) {
        if (i == l) continue;
        for (int32_t j = 0; j < C; ++j) T_(tb, i, j) = fma(-f[i], p[j], T_(tb, i, j));
    }
    for (int32_t j = 0; j < C; ++j) T_(tb, l, j) = p[j];
    for (int32_t i = 0; i < R; ++i) T_(tb, i, e) = (i == l) ? 1.0 : 0.0;
    tb->basis[l] = e;
    if (tb->trace && iter < tb->trace_cap) {
        tb->trace[2 * iter] = l;
        tb->trace[2 * iter + 1] = e;
    }
    free(f);
    free(p);
}

/* Solve one LP.  A is m x n row-major; sense[i] == 0 means "<=", anything
 * else ">=".  Outputs: status, iteration (pivot) count, objective, x[n],
 * y[m] = d(objective)/d(b_i), and optionally the final basis (column indices
 * of the full tableau) and the pivot trace.  Returns 0, or -1 on bad sizes. */
int oracle_simplex(int32_t m, int32_t n, const double* A, const double* b, const int8_t* sense,
                   const double* c, const oracle_opts* o, int32_t* status, int32_t* iters, double* obj,
                   double* x, double* y, int32_t* basis_out, int32_t* trace, int32_t trace_cap) {
    if (m <= 0 || n <= 0) return -1;
    const double eps_price = (o && o->eps_price > 0) ? o->eps_price : 1e-9;
    const double eps_piv = (o && o->eps_piv > 0) ? o->eps_piv : 1e-9;
    const double eps_feas = (o && o->eps_feas > 0) ? o->eps_feas : 1e-9;
    const int32_t max_iter = (o && o->max_iter > 0) ? o->max_iter : 50 * (m + n);
    const int32_t bland_after = (o && o->bland_after > 0) ? o->bland_after : (m > n ? m : n);

    /* Non-finite data: no solve. */
    int bad = 0;
    for (int64_t k = 0; k < (int64_t)m * n; ++k) bad |= !isfinite(A[k]);
    for (int32_t i = 0; i < m; ++i) bad |= !isfinite(b[i]);
    for (int32_t j = 0; j < n; ++j) bad |= !isfinite(c[j]);
    if (bad) {
        *status = ST_NUMERICAL;
        *iters = 0;
        *obj = NAN;
        for (int32_t j = 0; j < n; ++j) x[j] = NAN;
        for (int32_t i = 0; i < m; ++i) y[i] = NAN;
        if (basis_out)
            for (int32_t i = 0; i < m; ++i) basis_out[i] = -1;
        return 0;
    }

    /* Sec. 3: bring each row to "<=" form (a ">=" row is negated).  A row
     * whose "<=" right-hand side is negative makes the origin infeasible; it
     * is negated back (so its rhs is positive) and gets a surplus (-1) plus an
     * artificial (+1) variable.  Every other row gets a slack (+1).
     * s[i] is the overall sign applied to the user's row. */
    double* s = (double*)malloc(sizeof(double) * (size_t)m);
    uint8_t* art = (uint8_t*)malloc((size_t)m);
    int32_t n_art = 0;
    for (int32_t i = 0; i < m; ++i) {
        int ge = sense[i] != 0;
        double b_le = ge ? -b[i] : b[i];
        art[i] = b_le < 0.0;
        s[i] = art[i] ? (ge ? 1.0 : -1.0) : (ge ? -1.0 : 1.0);
        n_art += art[i];
    }

    tab_t tb;
    tb.m = m;
    tb.n = n;
    tb.n_art = n_art;
    tb.R = m + 1 + (n_art > 0);
    tb.C = n + m + n_art + 1;
    tb.T = (double*)calloc((size_t)tb.R * (size_t)tb.C, sizeof(double));
    tb.basis = (int32_t*)malloc(sizeof(int32_t) * (size_t)m);
    tb.dead = (uint8_t*)calloc((size_t)m, 1);
    tb.trace = trace;
    tb.trace_cap = trace ? trace_cap : 0;
    const int32_t rhs = tb.C - 1, jart = n + m; /* first artificial column */
    const int32_t row_obj = m, row_w = m + 1;

    /* Tableau: constraint rows, Eq. (4) in tableau form. */
    int32_t r = 0;
    for (int32_t i = 0; i < m; ++i) {
        for (int32_t j = 0; j < n; ++j) T_(&tb, i, j) = s[i] * A[(int64_t)i * n + j];
        T_(&tb, i, n + i) = art[i] ? -1.0 : 1.0;
        if (art[i]) {
            T_(&tb, i, jart + r) = 1.0;
            tb.basis[i] = jart + r;
            ++r;
        } else {
            tb.basis[i] = n + i;
        }
        T_(&tb, i, rhs) = s[i] * b[i];
    }
    /* Objective row: d_j = c_j for the structural variables, -z = 0. */
    for (int32_t j = 0; j < n; ++j) T_(&tb, row_obj, j) = c[j];
    /* Phase-1 row: reduced costs of maximising -(sum of artificials), i.e.
     * the sum of the artificial rows over every non-artificial column and the
     * rhs, added in increasing row order; zero on the artificial columns. */
    double w0 = 0.0;
    if (n_art > 0) {
        for (int32_t j = 0; j < tb.C; ++j) {
            if (j >= jart && j < rhs) continue;
            double acc = 0.0;
            for (int32_t i = 0; i < m; ++i)
                if (art[i]) acc = acc + T_(&tb, i, j);
            T_(&tb, row_w, j) = acc;
        }
        w0 = T_(&tb, row_w, rhs);
    }

    int32_t phase = n_art > 0 ? 1 : 2;
    int32_t it = 0, degen_run = 0, st = -1;
    for (;;) {
        const int32_t ro = phase == 1 ? row_w : row_obj;
        /* Step 1 (LPC): largest positive coefficient, lowest index on ties;
         * Bland's lowest positive index while anti-cycling is active. */
        int32_t e = -1;
        double best = 0.0;
        for (int32_t j = 0; j < jart; ++j) {
            double v = T_(&tb, ro, j);
            if (!(v > eps_price)) continue;
            if (degen_run >= bland_after) {
                e = j;
                break;
            }
            if (e < 0 || v > best) {
                e = j;
                best = v;
            }
        }
        if (e < 0) {
            if (phase == 2) {
                st = ST_OPTIMAL;
                break;
            }
            /* End of phase 1. */
            if (T_(&tb, row_w, rhs) > eps_feas * (1.0 + w0)) {
                st = ST_INFEASIBLE;
                break;
            }
            for (int32_t i = 0; i < m; ++i) {
                if (tb.basis[i] < jart || tb.dead[i]) continue;
                int32_t jj = -1;
                for (int32_t j = 0; j < jart; ++j)
                    if (fabs(T_(&tb, i, j)) > eps_piv) {
                        jj = j;
                        break;
                    }
                if (jj < 0) {
                    tb.dead[i] = 1;
                } else {
                    pivot(&tb, i, jj, it);
                    ++it;
                }
            }
            phase = 2;
            degen_run = 0;
            continue;
        }
        if (it >= max_iter) {
            st = ST_ITER_LIMIT;
            break;
        }
        /* Step 2: minimum ratio over rows with a positive pivot-column
         * entry; ties to the smallest basic variable index. */
        int32_t l = -1;
        double rmin = 0.0;
        for (int32_t i = 0; i < m; ++i) {
            if (tb.dead[i]) continue;
            double a = T_(&tb, i, e);
            if (!(a > eps_piv)) continue;
            double bi = T_(&tb, i, rhs);
            double ratio = bi <= 0.0 ? 0.0 : bi / a;
            if (l < 0 || ratio < rmin || (ratio == rmin && tb.basis[i] < tb.basis[l])) {
                l = i;
                rmin = ratio;
            }
        }
        if (l < 0) {
            /* Phase 1 is bounded below by zero; no limiting row there can
             * only come from corrupted numbers. */
            st = phase == 2 ? ST_UNBOUNDED : ST_NUMERICAL;
            break;
        }
        /* Step 3. */
        pivot(&tb, l, e, it);
        ++it;
        degen_run = rmin == 0.0 ? degen_run + 1 : 0;
    }

    /* Extraction.  -z sits in the objective row's rhs cell; a structural
     * variable's value is the rhs of the row where it is basic; the dual of
     * row i is read from the objective-row entry of its logical column (the
     * sign makes it d(objective)/d(b_i) in the caller's orientation). */
    double z = -T_(&tb, row_obj, rhs);
    if (st == ST_OPTIMAL && !isfinite(z)) st = ST_NUMERICAL;
    *status = st;
    *iters = it;
    *obj = st == ST_OPTIMAL || st == ST_ITER_LIMIT ? z
         : st == ST_UNBOUNDED ? INFINITY
         : st == ST_INFEASIBLE ? -INFINITY : NAN;
    for (int32_t j = 0; j < n; ++j) x[j] = 0.0;
    for (int32_t i = 0; i < m; ++i)
        if (tb.basis[i] < n) x[tb.basis[i]] = T_(&tb, i, rhs);
    for (int32_t i = 0; i < m; ++i) {
        double d = T_(&tb, row_obj, n + i);
        y[i] = sense[i] == 0 ? -d : d;
    }
    if (st == ST_NUMERICAL) {
        for (int32_t j = 0; j < n; ++j) x[j] = NAN;
        for (int32_t i = 0; i < m; ++i) y[i] = NAN;
    }
    if (basis_out)
        for (int32_t i = 0; i < m; ++i) basis_out[i] = tb.dead[i] ? -1 - tb.basis[i] : tb.basis[i];
    free(tb.T);
    free(tb.basis);
    free(tb.dead);
    free(s);
    free(art);
    return 0;
}

/* Sec. 6, Eq. (7): the maximum of c.x over the box [l, u] takes x_i = l_i
 * where c_i < 0 and u_i otherwise; the value is summed sequentially. */
void oracle_hyperbox(int32_t n, const double* c, const double* l, const double* u, int32_t* status,
                     double* obj, double* x) {
    int bad = 0, empty = 0;
    for (int32_t i = 0; i < n; ++i) {
        bad |= !isfinite(c[i]) || !isfinite(l[i]) || !isfinite(u[i]);
        empty |= l[i] > u[i];
    }
    if (bad) {
        *status = ST_NUMERICAL;
        *obj = NAN;
        for (int32_t i = 0; i < n; ++i) x[i] = NAN;
        return;
    }
    double acc = 0.0;
    for (int32_t i = 0; i < n; ++i) {
        x[i] = c[i] < 0.0 ? l[i] : u[i];
        acc = fma(c[i], x[i], acc);
    }
    *status = empty ? ST_INFEASIBLE : ST_OPTIMAL;
    *obj = empty ? -INFINITY : acc;
}

/* A batch in the packed layout of the solver's C ABI: LP k has m[k] rows and
 * n[k] columns, kind[k] 0 (simplex) or 1 (hyperbox), its A at a_off[k], its
 * b/sense/y at row_off[k], its c/l/u/x at col_off[k].  One LP per OpenMP
 * thread, the multicore scheme of the paper's Sec. 5. */
void oracle_batch(int64_t count, const int32_t* m, const int32_t* n, const int32_t* kind,
                  const int64_t* a_off, const int64_t* row_off, const int64_t* col_off, const double* A,
                  const double* b, const int8_t* sense, const double* c, const double* l, const double* u,
                  const oracle_opts* o, int32_t* status, int32_t* iters, double* obj, double* x, double* y) {
#pragma omp parallel for schedule(dynamic, 1)
    for (int64_t k = 0; k < count; ++k) {
        if (kind[k] == 1) {
            oracle_hyperbox(n[k], c + col_off[k], l + col_off[k], u + col_off[k], status + k, obj + k,
                            x + col_off[k]);
            iters[k] = 0;
        } else {
            oracle_simplex(m[k], n[k], A + a_off[k], b + row_off[k], sense + row_off[k], c + col_off[k], o,
                           status + k, iters + k, obj + k, x + col_off[k], y + row_off[k], NULL, NULL, 0);
        }
    }
}
