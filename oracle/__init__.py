"""ORACLE -- test infrastructure only.

ctypes wrapper around ``liboracle.so`` (built from ``oracle.c``): a plain FP64
CPU dense-tableau two-phase simplex and the hyperbox closed form, written from
the paper (Secs. 3, 3.1, 4.2-4.3 and 6, Eqs. (1)-(4) and (7)).  Only the test
suite, ``__graft_entry__.smoke()`` and ``bench.py``'s CPU-baseline leg may
import this package; the solver never does.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "liboracle.so")
SOURCES = [os.path.join(_HERE, "oracle.c")]

OPTIMAL, INFEASIBLE, UNBOUNDED, ITER_LIMIT, NUMERICAL = range(5)
STATUS_NAMES = {0: "OPTIMAL", 1: "INFEASIBLE", 2: "UNBOUNDED", 3: "ITER_LIMIT", 4: "NUMERICAL"}


class Opts(ctypes.Structure):
    _fields_ = [("max_iter", ctypes.c_int32), ("bland_after", ctypes.c_int32),
                ("eps_price", ctypes.c_double), ("eps_piv", ctypes.c_double), ("eps_feas", ctypes.c_double)]


def build(cc: str = "gcc", src: str | None = None, out: str | None = None, extra=()) -> str:
    """Compile the oracle with plain gcc.  ``-ffp-contract=off`` keeps every
    multiply-add unfused except the explicit fma() of the pivot update."""
    import subprocess
    out = out or LIB_PATH
    cmd = [cc, "-O2", "-ffp-contract=off", "-fno-fast-math", "-fPIC", "-shared", "-fopenmp", *extra,
           "-o", out + ".tmp", *(src and [src] or SOURCES), "-lm"]
    subprocess.check_call(cmd)
    os.replace(out + ".tmp", out)
    return out


def _bind(path: str) -> ctypes.CDLL:
    L = ctypes.CDLL(path)
    vp = ctypes.c_void_p
    L.oracle_simplex.argtypes = [ctypes.c_int32, ctypes.c_int32, vp, vp, vp, vp, ctypes.POINTER(Opts),
                                 vp, vp, vp, vp, vp, vp, vp, ctypes.c_int32]
    L.oracle_simplex.restype = ctypes.c_int
    L.oracle_hyperbox.argtypes = [ctypes.c_int32, vp, vp, vp, vp, vp, vp]
    L.oracle_hyperbox.restype = None
    L.oracle_batch.argtypes = [ctypes.c_int64] + [vp] * 12 + [ctypes.POINTER(Opts)] + [vp] * 5
    L.oracle_batch.restype = None
    return L


_lib = None


def lib(path: str | None = None) -> ctypes.CDLL:
    global _lib
    if path is not None:
        return _bind(path)
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is not built; run __graft_entry__.build()")
        _lib = _bind(LIB_PATH)
    return _lib


def _p(a):
    return None if a is None else a.ctypes.data_as(ctypes.c_void_p)


def _opts(max_iter=0, bland_after=0, eps_price=0.0, eps_piv=0.0, eps_feas=0.0):
    return Opts(max_iter, bland_after, eps_price, eps_piv, eps_feas)


def solve(A, b, c, sense=None, *, max_iter=0, bland_after=0, eps_price=0.0, eps_piv=0.0, eps_feas=0.0,
          trace=False, library: ctypes.CDLL | None = None) -> dict:
    """Solve one LP: max c.x s.t. A x (<= or >=) b, x >= 0.

    Returns status, iters, obj, x, y (= d obj / d b), basis (full-tableau
    column index per row, -1-col for a redundant row) and, with
    ``trace=True``, the (row, column) of every pivot.
    """
    A = np.ascontiguousarray(A, dtype=np.float64)
    m, n = A.shape
    b = np.ascontiguousarray(b, dtype=np.float64)
    c = np.ascontiguousarray(c, dtype=np.float64)
    sense = np.zeros(m, np.int8) if sense is None else np.ascontiguousarray(sense, dtype=np.int8)
    st = np.zeros(1, np.int32)
    it = np.zeros(1, np.int32)
    ob = np.zeros(1, np.float64)
    x = np.zeros(n, np.float64)
    y = np.zeros(m, np.float64)
    basis = np.zeros(m, np.int32)
    cap = (max_iter if max_iter > 0 else 50 * (m + n)) + m + 1
    tr = np.full(2 * cap, -1, np.int32) if trace else None
    L = library or lib()
    rc = L.oracle_simplex(m, n, _p(A), _p(b), _p(sense), _p(c),
                          ctypes.byref(_opts(max_iter, bland_after, eps_price, eps_piv, eps_feas)),
                          _p(st), _p(it), _p(ob), _p(x), _p(y), _p(basis), _p(tr), cap if trace else 0)
    if rc != 0:
        raise ValueError("oracle_simplex: bad sizes")
    out = {"status": int(st[0]), "iters": int(it[0]), "obj": float(ob[0]), "x": x, "y": y, "basis": basis}
    if trace:
        k = min(int(it[0]), cap)
        out["trace"] = tr[: 2 * k].reshape(k, 2)
    return out


def hyperbox(c, l, u, library: ctypes.CDLL | None = None) -> dict:
    c = np.ascontiguousarray(c, dtype=np.float64)
    l = np.ascontiguousarray(l, dtype=np.float64)
    u = np.ascontiguousarray(u, dtype=np.float64)
    n = c.shape[0]
    st = np.zeros(1, np.int32)
    ob = np.zeros(1, np.float64)
    x = np.zeros(n, np.float64)
    (library or lib()).oracle_hyperbox(n, _p(c), _p(l), _p(u), _p(st), _p(ob), _p(x))
    return {"status": int(st[0]), "obj": float(ob[0]), "x": x}


def solve_batch(batch, *, max_iter=0, eps_price=0.0, eps_piv=0.0, eps_feas=0.0) -> dict:
    """Solve a packed batch (``lpgen.Batch`` layout) with one LP per thread."""
    K = batch.count
    st = np.zeros(K, np.int32)
    it = np.zeros(K, np.int32)
    ob = np.zeros(K, np.float64)
    x = np.zeros(max(1, batch.c.shape[0]), np.float64)
    y = np.zeros(max(1, batch.b.shape[0]), np.float64)
    lib().oracle_batch(K, _p(batch.m), _p(batch.n), _p(batch.kind), _p(batch.a_off), _p(batch.row_off),
                       _p(batch.col_off), _p(batch.A), _p(batch.b), _p(batch.sense), _p(batch.c), _p(batch.l),
                       _p(batch.u), ctypes.byref(_opts(max_iter, 0, eps_price, eps_piv, eps_feas)),
                       _p(st), _p(it), _p(ob), _p(x), _p(y))
    return {"status": st, "iters": it, "obj": ob, "x": x, "y": y}
