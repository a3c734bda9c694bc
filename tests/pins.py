"""Independent checks that pin the CPU oracle to the paper and to mathematics.

Each ``pin_*`` function takes a loaded oracle library (the real one, or a
deliberately broken copy built by the mutation test) and raises
AssertionError when the oracle disagrees with something fixed outside it:
brute-force vertex enumeration, closed forms, LP duality recomputed by an
independent LU solve, the Klee-Minty pivot count of Dantzig's rule, crafted
statuses, the hyperbox closed form of Eq. (7) against vertex enumeration, and
an external solver (scipy HiGHS).  None of them retypes the oracle's tableau
arithmetic.
"""
from __future__ import annotations

import itertools

import numpy as np

import lpgen
import oracle

REL = 1e-9


def rel_err(a, b):
    return abs(a - b) / max(1.0, abs(b))


# --------------------------------------------------------------------------
# Brute force: enumerate every vertex of {G x <= h}
# --------------------------------------------------------------------------
def _le_form(A, b, sense):
    sg = np.where(np.asarray(sense) == 0, 1.0, -1.0)
    return sg[:, None] * A, sg * b


def _best_vertex(G, h, c):
    n = G.shape[1]
    best, arg = -np.inf, None
    for S in itertools.combinations(range(G.shape[0]), n):
        GS = G[list(S)]
        if abs(np.linalg.det(GS)) < 1e-10:
            continue
        x = np.linalg.solve(GS, h[list(S)])
        if np.all(G @ x <= h + 1e-9 * (1 + np.abs(h))):
            v = float(c @ x)
            if v > best:
                best, arg = v, x
    return best, arg


def brute_force(A, b, sense, c, box=1e6):
    """Return (status, obj) by vertex enumeration.

    Feasibility and the optimum come from the vertices of
    {A x (<=,>=) b, 0 <= x <= box}; unboundedness from the recession cone:
    the LP is unbounded iff it is feasible and some d >= 0 with A_le d <= 0,
    d <= 1 has c.d > 0 (again found by vertex enumeration).
    Status: 0 optimal, 1 infeasible, 2 unbounded.
    """
    A = np.asarray(A, float)
    m, n = A.shape
    c = np.asarray(c, float)
    Al, bl = _le_form(A, np.asarray(b, float), sense)
    I = np.eye(n)
    G = np.vstack([Al, -I, I])
    b1, x1 = _best_vertex(G, np.concatenate([bl, np.zeros(n), np.full(n, box)]), c)
    if x1 is None:
        return 1, -np.inf
    r, _ = _best_vertex(G, np.concatenate([np.zeros(m), np.zeros(n), np.ones(n)]), c)
    if r > 1e-9:
        return 2, np.inf
    return 0, b1


def pin_bruteforce(L, cases=300, seed=7):
    rng = np.random.default_rng(seed)
    seen = {0: 0, 1: 0, 2: 0}
    for t in range(cases):
        m = int(rng.integers(1, 6))
        n = int(rng.integers(1, 4))
        A = rng.integers(-3, 7, size=(m, n)).astype(float)
        b = rng.integers(-4, 11, size=m).astype(float)
        c = rng.integers(-2, 6, size=n).astype(float)
        sense = rng.integers(0, 2, size=m).astype(np.int8)
        st, ob = brute_force(A, b, sense, c)
        r = oracle.solve(A, b, c, sense, library=L)
        assert r["status"] == st, (t, A, b, c, sense, r, st, ob)
        seen[st] += 1
        if st == 0:
            assert rel_err(r["obj"], ob) <= 1e-8, (t, r["obj"], ob)
    # the family must exercise every outcome
    assert min(seen.values()) > 5, seen


def pin_bruteforce_float(L, cases=150, seed=11):
    """Continuous data, feasible origin and mixed rows: opt to 1e-9."""
    rng = np.random.default_rng(seed)
    for t in range(cases):
        m = int(rng.integers(1, 7))
        n = int(rng.integers(1, 5))
        A = rng.uniform(-2, 10, size=(m, n))
        x0 = rng.uniform(0.5, 2.0, size=n)
        sense = rng.integers(0, 2, size=m).astype(np.int8)
        ax = A @ x0
        b = np.where(sense == 0, ax + rng.uniform(0.5, 3, m), ax - rng.uniform(0.5, 3, m))
        c = rng.uniform(-1, 5, size=n)
        st, ob = brute_force(A, b, sense, c)
        r = oracle.solve(A, b, c, sense, library=L)
        assert r["status"] == st, (t, r, st)
        if st == 0:
            assert rel_err(r["obj"], ob) <= REL, (t, r["obj"], ob)


# --------------------------------------------------------------------------
# Closed forms
# --------------------------------------------------------------------------
def pin_closed_forms(L, seed=3):
    rng = np.random.default_rng(seed)
    for _ in range(40):
        n = int(rng.integers(1, 30))
        a = rng.uniform(1, 10, n)
        bb = float(rng.uniform(10, 100))
        c = rng.uniform(1, 10, n)
        r = oracle.solve(a[None, :], [bb], c, library=L)
        assert r["status"] == 0 and rel_err(r["obj"], bb * float(np.max(c / a))) <= REL
        # single constraint: its dual is the best value-per-unit ratio
        assert rel_err(r["y"][0], float(np.max(c / a))) <= REL
    for _ in range(40):
        m = int(rng.integers(1, 30))
        a = rng.uniform(1, 10, m)
        b = rng.uniform(10, 100, m)
        cc = float(rng.uniform(1, 10))
        r = oracle.solve(a[:, None], b, [cc], library=L)
        assert r["status"] == 0 and rel_err(r["obj"], cc * float(np.min(b / a))) <= REL
        assert rel_err(r["x"][0], float(np.min(b / a))) <= REL
    for _ in range(20):
        n = int(rng.integers(1, 40))
        a = rng.uniform(1, 10, n)
        b = rng.uniform(10, 100, n)
        c = rng.uniform(1, 10, n)
        r = oracle.solve(np.diag(a), b, c, library=L)
        assert r["status"] == 0 and rel_err(r["obj"], float(np.sum(c * b / a))) <= REL
        assert np.allclose(r["x"], b / a, rtol=1e-12) and np.allclose(r["y"], c / a, rtol=1e-12)
        # ">=" form of the same box: -a_j x_j >= -b_j
        r2 = oracle.solve(-np.diag(a), -b, c, np.ones(n, np.int8), library=L)
        assert r2["status"] == 0 and rel_err(r2["obj"], float(np.sum(c * b / a))) <= REL
        assert np.allclose(r2["y"], -c / a, rtol=1e-12)


# --------------------------------------------------------------------------
# Duality certificates with an independent LU recomputation
# --------------------------------------------------------------------------
def _check_certificate(A, b, sense, c, r, tag):
    m, n = A.shape
    x, y = r["x"], r["y"]
    scale = max(1.0, float(np.abs(b).max()), float(np.abs(A).max()))
    tol = 1e-9 * scale
    ax = A @ x
    le = np.asarray(sense) == 0
    assert (x >= -tol).all(), tag
    assert (ax[le] <= b[le] + tol * (1 + np.abs(b[le]))).all(), tag
    assert (ax[~le] >= b[~le] - tol * (1 + np.abs(b[~le]))).all(), tag
    assert (y[le] >= -tol).all() and (y[~le] <= tol).all(), tag
    ytA = A.T @ y
    assert (ytA >= c - 1e-8 * (1 + np.abs(c))).all(), tag
    assert rel_err(float(c @ x), float(b @ y)) <= 1e-9 * scale, (tag, c @ x, b @ y)
    assert rel_err(r["obj"], float(c @ x)) <= 1e-9 * scale, tag
    slack = np.where(le, b - ax, ax - b)
    assert (np.abs(y * slack) <= 1e-7 * (1 + np.abs(y) * (1 + np.abs(b)))).all(), tag
    assert (np.abs(x * (ytA - c)) <= 1e-7 * (1 + np.abs(x) * (1 + np.abs(c)))).all(), tag
    # LU: the oracle's final basis, refactored from the original data.
    g = np.where(le, 1.0, -1.0)
    M = np.hstack([A, np.diag(g)])
    cost = np.concatenate([c, np.zeros(m)])
    basis = r["basis"]
    if (basis < 0).any() or (basis >= n + m).any():
        return  # a redundant row or an artificial left basic: no square basis
    B = M[:, basis]
    xB = np.linalg.solve(B, b)
    yl = np.linalg.solve(B.T, cost[basis])
    xf = np.zeros(n + m)
    xf[basis] = xB
    assert np.allclose(xf[:n], x, rtol=1e-9, atol=1e-9 * scale), tag
    assert np.allclose(yl, y, rtol=1e-9, atol=1e-9 * scale), tag


def pin_duality(L, seed=5):
    rng = np.random.default_rng(seed)
    # type-1 workloads from the generator
    bt = lpgen.config(1, range(60))
    for k in range(bt.count):
        lp = bt.lp(k)
        r = oracle.solve(lp["A"], lp["b"], lp["c"], lp["sense"], library=L)
        assert r["status"] == 0
        _check_certificate(lp["A"], lp["b"], lp["sense"], lp["c"], r, ("cfg1", k))
    bt = lpgen.config(2, range(4))
    for k in range(bt.count):
        lp = bt.lp(k)
        r = oracle.solve(lp["A"], lp["b"], lp["c"], lp["sense"], library=L)
        assert r["status"] == 0
        _check_certificate(lp["A"], lp["b"], lp["sense"], lp["c"], r, ("cfg2", k))
    # mixed "<=" / ">=" rows through an interior point, negative rhs included
    for t in range(60):
        m = int(rng.integers(2, 25))
        n = int(rng.integers(2, 25))
        A = rng.uniform(-3, 10, size=(m, n))
        x0 = rng.uniform(1, 5, n)
        sense = rng.integers(0, 2, m).astype(np.int8)
        ax = A @ x0
        b = np.where(sense == 0, ax + rng.uniform(1, 10, m), ax - rng.uniform(1, 10, m))
        # keep it bounded: one all-positive "<=" row
        A[0] = rng.uniform(1, 10, n)
        sense[0] = 0
        b[0] = A[0] @ x0 + 5.0
        c = rng.uniform(-5, 10, n)
        r = oracle.solve(A, b, c, sense, library=L)
        assert r["status"] == 0, (t, r["status"])
        _check_certificate(A, b, sense, c, r, ("mixed", t))


# --------------------------------------------------------------------------
# Klee-Minty: Dantzig's largest-coefficient rule visits every vertex
# --------------------------------------------------------------------------
def klee_minty(n):
    A = np.zeros((n, n))
    for i in range(n):
        for j in range(i):
            A[i, j] = 2.0 * 10.0 ** (i - j)
        A[i, i] = 1.0
    b = np.array([100.0 ** i for i in range(n)])
    c = np.array([10.0 ** (n - 1 - j) for j in range(n)])
    return A, b, c


def pin_klee_minty(L):
    for n in range(2, 9):
        A, b, c = klee_minty(n)
        r = oracle.solve(A, b, c, library=L)
        assert r["status"] == 0
        assert r["obj"] == 100.0 ** (n - 1), (n, r["obj"])
        assert r["iters"] == 2 ** n - 1, (n, r["iters"])
        x = np.zeros(n)
        x[-1] = 100.0 ** (n - 1)
        assert np.array_equal(r["x"], x)


# --------------------------------------------------------------------------
# Crafted outcomes
# --------------------------------------------------------------------------
def pin_statuses(L):
    # infeasible: x1 + x2 <= 1 and x1 + x2 >= 2
    r = oracle.solve([[1, 1], [1, 1]], [1, 2], [1, 1], [0, 1], library=L)
    assert r["status"] == oracle.INFEASIBLE and r["obj"] == -np.inf
    # infeasible through a negative "<=" rhs with nonnegative row: x1 + x2 <= -1
    r = oracle.solve([[1, 1]], [-1], [1, 1], library=L)
    assert r["status"] == oracle.INFEASIBLE
    # unbounded: max x1 s.t. x1 - x2 <= 1
    r = oracle.solve([[1, -1]], [1], [1, 0], library=L)
    assert r["status"] == oracle.UNBOUNDED and r["obj"] == np.inf
    # unbounded after phase 1: x1 + x2 >= 2, max x1
    r = oracle.solve([[1, 1]], [2], [1, 0], [1], library=L)
    assert r["status"] == oracle.UNBOUNDED
    # optimum at the origin (c <= 0): zero pivots
    r = oracle.solve([[1, 2], [3, 1]], [4, 5], [-1, -2], library=L)
    assert r["status"] == 0 and r["iters"] == 0 and r["obj"] == 0.0
    # non-finite input
    r = oracle.solve([[1, np.nan]], [1], [1, 1], library=L)
    assert r["status"] == oracle.NUMERICAL and np.isnan(r["obj"]) and r["iters"] == 0
    r = oracle.solve([[1, 1]], [np.inf], [1, 1], library=L)
    assert r["status"] == oracle.NUMERICAL
    # iteration limit
    A, b, c = klee_minty(5)
    r = oracle.solve(A, b, c, max_iter=3, library=L)
    assert r["status"] == oracle.ITER_LIMIT and r["iters"] == 3
    # duplicated rows: x1 + x2 >= 2 twice and x1 + x2 <= 2 -> x1 + x2 = 2; both
    # artificials must leave the basis (degenerate phase-1 end)
    r = oracle.solve([[1, 1], [1, 1], [1, 1]], [2, 2, 2], [1, 2], [1, 1, 0], library=L)
    assert r["status"] == 0 and rel_err(r["obj"], 4.0) <= REL
    assert rel_err(float(r["x"].sum()), 2.0) <= REL
    # degenerate: zero right-hand sides
    A = np.array([[1.0, -1.0], [-1.0, 1.0], [1.0, 1.0]])
    r = oracle.solve(A, [0, 0, 4], [1, 1], library=L)
    assert r["status"] == 0 and rel_err(r["obj"], 4.0) <= REL
    assert abs(r["x"][0] - r["x"][1]) <= 1e-12


def pin_degenerate_cycling(L):
    """A degenerate instance (Beale's structure: two rows with zero rhs) on
    which the largest-coefficient rule with the smallest-basic-index leaving
    tie-break cycles forever; with the anti-cycling switch the optimum, 1.25
    at x = (1, 0, 1, 0), is reached.  The optimum is confirmed by vertex
    enumeration here and by HiGHS."""
    A = np.array([[0.25, -8.0, -1.0, 9.0], [0.5, -12.0, -0.5, 3.0], [0.0, 0.0, 1.0, 0.0]])
    b = np.array([0.0, 0.0, 1.0])
    c = np.array([0.75, -20.0, 0.5, -6.0])
    st, ob = brute_force(A, b, np.zeros(3, np.int8), c)
    assert st == 0 and rel_err(ob, 1.25) <= 1e-12
    r = oracle.solve(A, b, c, library=L)
    assert r["status"] == 0, r
    assert rel_err(r["obj"], 1.25) <= REL, r["obj"]
    assert np.allclose(r["x"], [1.0, 0.0, 1.0, 0.0], atol=1e-12)
    # without the anti-cycling switch the same rules cycle at objective 0
    r = oracle.solve(A, b, c, bland_after=10 ** 6, max_iter=200, library=L)
    assert r["status"] == oracle.ITER_LIMIT and r["obj"] == 0.0


# --------------------------------------------------------------------------
# Hyperbox, Eq. (7)
# --------------------------------------------------------------------------
def pin_hyperbox(L, seed=9):
    rng = np.random.default_rng(seed)
    for t in range(200):
        n = int(rng.integers(1, 11))
        c = rng.normal(size=n)
        lo = rng.uniform(-10, -1, n)
        hi = rng.uniform(1, 10, n)
        r = oracle.hyperbox(c, lo, hi, library=L)
        verts = np.array(list(itertools.product(*zip(lo, hi))))
        vals = verts @ c
        assert r["status"] == 0
        assert rel_err(r["obj"], float(vals.max())) <= 1e-12, (t, r["obj"], vals.max())
        assert rel_err(float(c @ r["x"]), float(vals.max())) <= 1e-12
        assert ((r["x"] == lo) | (r["x"] == hi)).all()
    # zero objective coefficient takes the upper bound (Eq. 7, "otherwise")
    r = oracle.hyperbox([0.0, -1.0, 2.0], [-1.0, -2.0, -3.0], [4.0, 5.0, 6.0], library=L)
    assert list(r["x"]) == [4.0, -2.0, 6.0] and r["obj"] == 14.0
    # empty box
    r = oracle.hyperbox([1.0, 1.0], [0.0, 2.0], [1.0, 1.0], library=L)
    assert r["status"] == oracle.INFEASIBLE and r["obj"] == -np.inf
    r = oracle.hyperbox([1.0, np.nan], [0.0, 0.0], [1.0, 1.0], library=L)
    assert r["status"] == oracle.NUMERICAL


# --------------------------------------------------------------------------
# External solver on the workload recipes
# --------------------------------------------------------------------------
def pin_external(L, per_cfg=(40, 6, 2)):
    from scipy.optimize import linprog
    for cfg, cnt in zip((1, 2, 3), per_cfg):
        bt = lpgen.config(cfg, range(cnt))
        for k in range(cnt):
            lp = bt.lp(k)
            A, b, c, s = lp["A"], lp["b"], lp["c"], lp["sense"]
            r = oracle.solve(A, b, c, s, library=L)
            Al, bl = _le_form(A, b, s)
            h = linprog(-c, A_ub=Al, b_ub=bl, bounds=(0, None), method="highs",
                        options={"primal_feasibility_tolerance": 1e-10, "dual_feasibility_tolerance": 1e-10})
            assert h.status == 0 and r["status"] == 0
            assert rel_err(r["obj"], -h.fun) <= 1e-9, (cfg, k, r["obj"], -h.fun)


# --------------------------------------------------------------------------
# Monotone progress along the pivot path (phase 2 of type-1 LPs)
# --------------------------------------------------------------------------
def pin_monotone(L, seed=13):
    bt = lpgen.config(2, range(2))
    for k in range(bt.count):
        lp = bt.lp(k)
        A, b, c = lp["A"], lp["b"], lp["c"]
        full = oracle.solve(A, b, c, library=L)
        prev = 0.0
        for it in range(1, full["iters"] + 1):
            r = oracle.solve(A, b, c, max_iter=it, library=L)
            assert r["obj"] >= prev - 1e-9 * max(1.0, abs(prev)), (k, it)
            assert (A @ r["x"] <= b + 1e-9 * b).all() and (r["x"] >= -1e-12).all(), (k, it)
            assert rel_err(float(c @ r["x"]), r["obj"]) <= 1e-9
            prev = r["obj"]
        assert rel_err(prev, full["obj"]) <= 1e-12


# --------------------------------------------------------------------------
# The batch driver: packed layout with arbitrary offsets, mixed kinds
# --------------------------------------------------------------------------
def _scattered_batch(seed=17):
    """Mixed simplex / hyperbox LPs (tiny brute-force cases with every
    outcome, diagonal closed forms, generator LPs of both types, non-finite
    members) stored in a permuted order at gapped, non-monotone offsets; the
    gaps hold NaN so that a read at a wrong offset changes the outcome.
    Returns (lps, batch arrays, expected (status, obj) per LP or None)."""
    rng = np.random.default_rng(seed)
    lps, expect = [], []
    while len(lps) < 24:  # tiny LPs, brute force, every outcome
        m, n = int(rng.integers(1, 5)), int(rng.integers(1, 4))
        A = rng.integers(-3, 7, size=(m, n)).astype(float)
        b = rng.integers(-4, 11, size=m).astype(float)
        c = rng.integers(-2, 6, size=n).astype(float)
        sense = rng.integers(0, 2, size=m).astype(np.int8)
        lps.append({"A": A, "b": b, "c": c, "sense": sense})
        expect.append(brute_force(A, b, sense, c))
    for _ in range(6):  # diagonal: opt = sum c_j b_j / a_jj
        n = int(rng.integers(1, 12))
        a, b, c = rng.uniform(1, 10, n), rng.uniform(10, 100, n), rng.uniform(1, 10, n)
        lps.append({"A": np.diag(a), "b": b, "c": c, "sense": np.zeros(n, np.int8)})
        expect.append((0, float(np.sum(c * b / a))))
    g1 = lpgen.config(1, range(4))
    g4 = lpgen.config(4, [i for i in range(400) if lpgen.config(4, [i]).m[0] <= 24][:6])
    for bt in (g1, g4):
        for k in range(bt.count):
            d = bt.lp(k)
            lps.append({kk: np.array(v) for kk, v in d.items() if kk in ("A", "b", "c", "sense", "l", "u")})
            expect.append(None)
    for t in range(8):  # hyperbox: Eq. (7) against box-vertex enumeration
        n = int(rng.integers(1, 7))
        c, lo, hi = rng.normal(size=n), rng.uniform(-10, -1, n), rng.uniform(1, 10, n)
        if t == 6:
            lo[0], hi[0] = 2.0, 1.0  # empty box
        lps.append({"c": c, "l": lo, "u": hi})
        if t == 6:
            expect.append((1, -np.inf))
        else:
            verts = np.array(list(itertools.product(*zip(lo, hi))))
            expect.append((0, float((verts @ c).max())))
    lps.append({"A": np.array([[1.0, np.nan]]), "b": np.array([1.0]), "c": np.array([1.0, 1.0]),
                "sense": np.zeros(1, np.int8)})
    expect.append((4, np.nan))
    lps.append({"c": np.array([np.nan, 1.0]), "l": np.array([-1.0, -1.0]), "u": np.array([1.0, 1.0])})
    expect.append((4, np.nan))
    K = len(lps)
    order = rng.permutation(K)  # storage order differs from LP order
    m = np.array([0 if "l" in d else d["A"].shape[0] for d in lps], np.int32)
    n = np.array([len(d["c"]) for d in lps], np.int32)
    kind = np.array([1 if "l" in d else 0 for d in lps], np.int32)
    a_off, row_off, col_off = (np.zeros(K, np.int64) for _ in range(3))
    pa = pr = pc = 0
    for k in order:
        pa += int(rng.integers(0, 5))
        pr += int(rng.integers(0, 4))
        pc += int(rng.integers(0, 4))
        a_off[k], row_off[k], col_off[k] = pa, pr, pc
        pa += int(m[k]) * int(n[k])
        pr += int(m[k])
        pc += int(n[k])
    A = np.full(pa + 3, np.nan)
    b = np.full(pr + 3, np.nan)
    sense = np.full(pr + 3, 1, np.int8)
    c = np.full(pc + 3, np.nan)
    l = np.full(pc + 3, np.nan)
    u = np.full(pc + 3, np.nan)
    for k, d in enumerate(lps):
        co, nn = int(col_off[k]), int(n[k])
        c[co:co + nn] = d["c"]
        if kind[k]:
            l[co:co + nn], u[co:co + nn] = d["l"], d["u"]
        else:
            ao, ro, mm = int(a_off[k]), int(row_off[k]), int(m[k])
            A[ao:ao + mm * nn] = d["A"].ravel()
            b[ro:ro + mm] = d["b"]
            sense[ro:ro + mm] = d["sense"]
    return lps, (K, m, n, kind, a_off, row_off, col_off, A, b, sense, c, l, u), expect


def pin_batch_driver(L):
    """oracle_batch on a scattered batch: every LP's status, iterations,
    objective, x and y equal (bit for bit) the single-LP routines' results at
    that LP's own offsets, outcomes match brute force / closed forms, and no
    output position outside the LPs' ranges is written."""
    import ctypes
    lps, arrs, expect = _scattered_batch()
    K, m, n, kind, a_off, row_off, col_off, A, b, sense, c, l, u = arrs
    SENT = 1234.5
    st = np.full(K, -7, np.int32)
    it = np.full(K, -7, np.int32)
    ob = np.full(K, SENT)
    # outputs padded past both packed ranges, so that a driver writing at the
    # wrong offsets stays inside the arrays (and is caught by the sentinel)
    pad = max(c.shape[0], b.shape[0]) + 64
    x = np.full(pad, SENT)
    y = np.full(pad, SENT)
    P = lambda a: a.ctypes.data_as(ctypes.c_void_p)
    L.oracle_batch(K, P(m), P(n), P(kind), P(a_off), P(row_off), P(col_off), P(A), P(b), P(sense), P(c),
                   P(l), P(u), ctypes.byref(oracle.Opts(0, 0, 0.0, 0.0, 0.0)), P(st), P(it), P(ob), P(x), P(y))
    xw = np.zeros(x.shape[0], bool)
    yw = np.zeros(y.shape[0], bool)
    for k, d in enumerate(lps):
        co, nn = int(col_off[k]), int(n[k])
        if kind[k]:
            r = oracle.hyperbox(d["c"], d["l"], d["u"], library=L)
            r["iters"], r["y"] = 0, np.zeros(0)
        else:
            r = oracle.solve(d["A"], d["b"], d["c"], d["sense"], library=L)
        ro, mm = int(row_off[k]), int(m[k])
        assert st[k] == r["status"] and it[k] == r["iters"], (k, st[k], r["status"], it[k], r["iters"])
        assert np.array_equal(np.array([ob[k]]).view(np.int64), np.array([r["obj"]]).view(np.int64)), k
        assert np.array_equal(x[co:co + nn].view(np.int64), r["x"].view(np.int64)), k
        if not kind[k]:
            assert np.array_equal(y[ro:ro + mm].view(np.int64), r["y"].view(np.int64)), k
            yw[ro:ro + mm] = True
        xw[co:co + nn] = True
        if expect[k] is not None:
            est, eob = expect[k]
            assert st[k] == est, (k, st[k], est)
            if est == 0:
                assert rel_err(ob[k], eob) <= 1e-8, (k, ob[k], eob)
    assert (x[~xw] == SENT).all() and (y[~yw] == SENT).all(), "output written outside the LPs' ranges"
    assert set(np.unique(st)) >= {0, 1, 2, 4}


ALL_PINS = [pin_bruteforce, pin_bruteforce_float, pin_closed_forms, pin_duality, pin_klee_minty,
            pin_statuses, pin_degenerate_cycling, pin_hyperbox, pin_external, pin_monotone,
            pin_batch_driver]
