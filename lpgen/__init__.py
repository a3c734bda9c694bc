"""Seeded synthetic LP batches (inputs only; no simplex arithmetic here).

The C library ``liblpgen.so`` (built from ``lpgen.c``) draws every value from
Philox4x32-10 keyed by (config seed, LP id, field, element index).  This
wrapper knows the five workload recipes and returns packed numpy arrays in the
layout the solver's C ABI takes:

* ``A``: each LP's m x n matrix, row-major, packed at ``a_off[k]``;
* ``b``, ``sense``: length m at ``row_off[k]`` (sense 0 = "<=", 1 = ">=");
* ``c`` (and ``l``, ``u`` for hyperbox LPs): length n at ``col_off[k]``;
* ``kind``: 0 = simplex LP, 1 = hyperbox LP.

Workload recipes (the paper's LP families, abstract and Secs. 4.6, 6):

1. type 1, K=1,000, m=n=5; A~U(1,10), b~U(10,100), c~U(1,10)
2. type 1, K=50,000, m=n=100, same distributions
3. type 2, K=10,000, m=n=200; rows 0..99 "<=", 100..199 ">=" through an
   interior point x0~U(1,5)^n with margin U(1,10); A~U(1,10), c~U(1,10)
4. mixed, K=200,000; m, n ~ U{5..300}; 40% type 1, 40% type 2, 20% hyperbox
   (l~U(-10,-1), u~U(1,10), c~N(0,1))
5. 20,000 type-1 LPs with m=n~U{20..150}; 4,000,000 hyperbox LPs with n=5 and
   6,000,000 with n=28 (c = g/|g|, g~N(0,I)); loss weights w~U(0,1)
"""
from __future__ import annotations

import ctypes
import os
from dataclasses import dataclass, field

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "liblpgen.so")
SOURCES = [os.path.join(_HERE, "lpgen.c")]

SEEDS = {1: 1001, 2: 1002, 3: 1003, 4: 1004, 5: 1005}
BATCH_SIZES = {1: 1_000, 2: 50_000, 3: 10_000, 4: 200_000}
CFG5_SIMPLEX = 20_000
CFG5_BOX5 = 4_000_000
CFG5_BOX28 = 6_000_000


class Params(ctypes.Structure):
    _fields_ = [
        ("a_lo", ctypes.c_double), ("a_hi", ctypes.c_double),
        ("b_lo", ctypes.c_double), ("b_hi", ctypes.c_double),
        ("c_lo", ctypes.c_double), ("c_hi", ctypes.c_double),
        ("x0_lo", ctypes.c_double), ("x0_hi", ctypes.c_double),
        ("d_lo", ctypes.c_double), ("d_hi", ctypes.c_double),
        ("l_lo", ctypes.c_double), ("l_hi", ctypes.c_double),
        ("u_lo", ctypes.c_double), ("u_hi", ctypes.c_double),
        ("box_c_unit", ctypes.c_int32), ("pad_", ctypes.c_int32),
    ]


def default_params(box_c_unit: bool = False) -> Params:
    return Params(1.0, 10.0, 10.0, 100.0, 1.0, 10.0, 1.0, 5.0, 1.0, 10.0,
                  -10.0, -1.0, 1.0, 10.0, 1 if box_c_unit else 0, 0)


def build(cc: str = "gcc") -> str:
    """Compile liblpgen.so next to its source (plain gcc, OpenMP)."""
    import subprocess
    cmd = [cc, "-O2", "-ffp-contract=off", "-fPIC", "-shared", "-fopenmp",
           "-o", LIB_PATH + ".tmp", *SOURCES, "-lm"]
    subprocess.check_call(cmd)
    os.replace(LIB_PATH + ".tmp", LIB_PATH)
    return LIB_PATH


_lib = None


def lib() -> ctypes.CDLL:
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is not built; run __graft_entry__.build()")
        L = ctypes.CDLL(LIB_PATH)
        P = ctypes.POINTER
        L.lpgen_philox4x32_10.argtypes = [P(ctypes.c_uint32), P(ctypes.c_uint32), P(ctypes.c_uint32)]
        L.lpgen_philox4x32_10.restype = None
        L.lpgen_uniform.argtypes = [ctypes.c_uint64, ctypes.c_uint64, ctypes.c_uint32, ctypes.c_uint32]
        L.lpgen_uniform.restype = ctypes.c_double
        L.lpgen_uniform_int.argtypes = [ctypes.c_uint64, ctypes.c_uint64, ctypes.c_uint32, ctypes.c_uint32,
                                        ctypes.c_int32, ctypes.c_int32]
        L.lpgen_uniform_int.restype = ctypes.c_int32
        L.lpgen_normal.argtypes = [ctypes.c_uint64, ctypes.c_uint64, ctypes.c_uint32, ctypes.c_uint32]
        L.lpgen_normal.restype = ctypes.c_double
        vp = ctypes.c_void_p
        L.lpgen_batch.argtypes = [ctypes.c_uint64, ctypes.c_int64] + [vp] * 7 + [P(Params)] + [vp] * 6
        L.lpgen_batch.restype = None
        L.lpgen_shapes.argtypes = [ctypes.c_uint64, ctypes.c_int64, vp, ctypes.c_int32, ctypes.c_int32,
                                   ctypes.c_int32, ctypes.c_double, ctypes.c_double, vp, vp, vp]
        L.lpgen_shapes.restype = None
        L.lpgen_weights.argtypes = [ctypes.c_uint64, ctypes.c_int64, vp, ctypes.c_double, ctypes.c_double, vp]
        L.lpgen_weights.restype = None
        _lib = L
    return _lib


def philox4x32_10(ctr, key):
    c = (ctypes.c_uint32 * 4)(*ctr)
    k = (ctypes.c_uint32 * 2)(*key)
    o = (ctypes.c_uint32 * 4)()
    lib().lpgen_philox4x32_10(c, k, o)
    return list(o)


def _ptr(a: np.ndarray | None):
    return None if a is None else a.ctypes.data_as(ctypes.c_void_p)


@dataclass
class Batch:
    """A packed batch of LPs (host numpy arrays)."""
    m: np.ndarray            # int32 [K] (0 for hyperbox LPs)
    n: np.ndarray            # int32 [K]
    kind: np.ndarray         # int32 [K]: 0 simplex, 1 hyperbox
    a_off: np.ndarray        # int64 [K]
    row_off: np.ndarray      # int64 [K]
    col_off: np.ndarray      # int64 [K]
    A: np.ndarray            # float64 [sum m*n]
    b: np.ndarray            # float64 [sum m]
    sense: np.ndarray        # int8 [sum m]
    c: np.ndarray            # float64 [sum n]
    l: np.ndarray            # float64 [sum n] (hyperbox entries only meaningful)
    u: np.ndarray            # float64 [sum n]
    lp_ids: np.ndarray       # int64 [K] generator addresses
    gen_type: np.ndarray     # int32 [K]: 1, 2 or 3
    meta: dict = field(default_factory=dict)

    @property
    def count(self) -> int:
        return int(self.m.shape[0])

    @property
    def uniform(self) -> bool:
        return bool(self.count > 0 and (self.m == self.m[0]).all() and (self.n == self.n[0]).all()
                    and (self.kind == self.kind[0]).all())

    def lp(self, k: int) -> dict:
        """Views of LP k's arrays."""
        m, n = int(self.m[k]), int(self.n[k])
        ao, ro, co = int(self.a_off[k]), int(self.row_off[k]), int(self.col_off[k])
        d = {"m": m, "n": n, "kind": int(self.kind[k]), "c": self.c[co:co + n]}
        if self.kind[k] == 0:
            d.update(A=self.A[ao:ao + m * n].reshape(m, n), b=self.b[ro:ro + m], sense=self.sense[ro:ro + m])
        else:
            d.update(l=self.l[co:co + n], u=self.u[co:co + n])
        return d


def offsets(m: np.ndarray, n: np.ndarray):
    """Packed offsets for per-LP slices (exclusive prefix sums)."""
    m64, n64 = m.astype(np.int64), n.astype(np.int64)
    a_off = np.zeros_like(m64)
    row_off = np.zeros_like(m64)
    col_off = np.zeros_like(m64)
    if len(m64):
        a_off[1:] = np.cumsum(m64 * n64)[:-1]
        row_off[1:] = np.cumsum(m64)[:-1]
        col_off[1:] = np.cumsum(n64)[:-1]
    return a_off, row_off, col_off


def make_batch(seed: int, lp_ids, gen_type, m, n, params: Params | None = None) -> Batch:
    """Generate LPs with explicit ids, generator types (1, 2, 3) and shapes."""
    lp_ids = np.ascontiguousarray(lp_ids, dtype=np.int64)
    gen_type = np.ascontiguousarray(gen_type, dtype=np.int32)
    m = np.ascontiguousarray(m, dtype=np.int32).copy()
    n = np.ascontiguousarray(n, dtype=np.int32)
    m[gen_type == 3] = 0
    if (n > 4096).any() or (m > 4096).any():
        raise ValueError("generator supports m, n <= 4096")
    kind = (gen_type == 3).astype(np.int32)
    a_off, row_off, col_off = offsets(m, n)
    K = len(m)
    tot_a = int((m.astype(np.int64) * n).sum())
    tot_m = int(m.astype(np.int64).sum())
    tot_n = int(n.astype(np.int64).sum())
    A = np.zeros(tot_a, np.float64)
    b = np.zeros(tot_m, np.float64)
    sense = np.zeros(tot_m, np.int8)
    c = np.zeros(tot_n, np.float64)
    l = np.zeros(tot_n, np.float64)
    u = np.zeros(tot_n, np.float64)
    p = params or default_params()
    if K:
        lib().lpgen_batch(seed, K, _ptr(lp_ids), _ptr(gen_type), _ptr(m), _ptr(n), _ptr(a_off), _ptr(row_off),
                          _ptr(col_off), ctypes.byref(p), _ptr(A), _ptr(b), _ptr(sense), _ptr(c), _ptr(l), _ptr(u))
    return Batch(m, n, kind, a_off, row_off, col_off, A, b, sense, c, l, u, lp_ids, gen_type)


def shapes(seed: int, lp_ids, mn_lo: int, mn_hi: int, square: bool, frac_t1: float, frac_t2: float):
    lp_ids = np.ascontiguousarray(lp_ids, dtype=np.int64)
    K = len(lp_ids)
    t = np.zeros(K, np.int32)
    m = np.zeros(K, np.int32)
    n = np.zeros(K, np.int32)
    if K:
        lib().lpgen_shapes(seed, K, _ptr(lp_ids), mn_lo, mn_hi, 1 if square else 0, frac_t1, frac_t2,
                           _ptr(t), _ptr(m), _ptr(n))
    return t, m, n


def weights(seed: int, lp_ids, lo: float = 0.0, hi: float = 1.0) -> np.ndarray:
    lp_ids = np.ascontiguousarray(lp_ids, dtype=np.int64)
    w = np.zeros(len(lp_ids), np.float64)
    if len(lp_ids):
        lib().lpgen_weights(seed, len(lp_ids), _ptr(lp_ids), lo, hi, _ptr(w))
    return w


def config(cfg: int, lp_ids=None, part: str | None = None) -> Batch:
    """Batch for workload ``cfg`` (1..5), restricted to ``lp_ids`` if given.

    Config 5 has three parts addressed by ``part``: "simplex" (20,000 type-1
    LPs, m=n~U{20..150}), "box5" (n=5) and "box28" (n=28); LP ids restart at 0
    in each part and the parts use distinct seeds (1005, 1015, 1025).
    """
    seed = SEEDS[cfg]
    if cfg in (1, 2, 3):
        K = BATCH_SIZES[cfg]
        ids = np.arange(K, dtype=np.int64) if lp_ids is None else np.asarray(lp_ids, np.int64)
        dim = {1: 5, 2: 100, 3: 200}[cfg]
        t = np.full(len(ids), 1 if cfg < 3 else 2, np.int32)
        dims = np.full(len(ids), dim, np.int32)
        bt = make_batch(seed, ids, t, dims, dims)
    elif cfg == 4:
        K = BATCH_SIZES[4]
        ids = np.arange(K, dtype=np.int64) if lp_ids is None else np.asarray(lp_ids, np.int64)
        t, m, n = shapes(seed, ids, 5, 300, False, 0.4, 0.4)
        bt = make_batch(seed, ids, t, m, n)
    elif cfg == 5:
        part = part or "simplex"
        if part == "simplex":
            K = CFG5_SIMPLEX
            ids = np.arange(K, dtype=np.int64) if lp_ids is None else np.asarray(lp_ids, np.int64)
            t, m, n = shapes(seed, ids, 20, 150, True, 1.0, 0.0)
            bt = make_batch(seed, ids, t, m, n)
        elif part in ("box5", "box28"):
            K = CFG5_BOX5 if part == "box5" else CFG5_BOX28
            s = seed + (10 if part == "box5" else 20)
            ids = np.arange(K, dtype=np.int64) if lp_ids is None else np.asarray(lp_ids, np.int64)
            dim = 5 if part == "box5" else 28
            t = np.full(len(ids), 3, np.int32)
            dims = np.full(len(ids), dim, np.int32)
            bt = make_batch(s, ids, t, dims, dims, default_params(box_c_unit=True))
            seed = s
        else:
            raise ValueError(part)
    else:
        raise ValueError(cfg)
    bt.meta = {"config": cfg, "seed": seed, "part": part}
    return bt
