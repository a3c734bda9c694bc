"""Batched LP solving on one AMD MI355X: Python binding of libblp.so.

The functions named ``blp_*`` are thin ctypes wrappers of the C ABI in
``include/blp.h`` (argument marshalling only; every step of the solve runs in
the library's HIP kernels).  PyTorch is used for device memory and streams.
If the library has not been built, importing the binding works but any call
raises: there is no CPU fallback.
"""
from __future__ import annotations

import ctypes
import os
from dataclasses import dataclass

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
# BLP_LIBRARY may name another build of the same library (the phase-timer
# build); there is no fallback when it is missing
LIB_PATH = os.environ.get("BLP_LIBRARY") or os.path.join(HERE, "libblp.so")

BLP_LE, BLP_GE = 0, 1
BLP_KIND_SIMPLEX, BLP_KIND_HYPERBOX = 0, 1
BLP_OPTIMAL, BLP_INFEASIBLE, BLP_UNBOUNDED, BLP_ITER_LIMIT, BLP_NUMERICAL = range(5)
BLP_SUCCESS, BLP_ERR_ARG, BLP_ERR_NOMEM, BLP_ERR_HIP, BLP_ERR_STATE, BLP_ERR_TOO_LARGE = range(6)
BLP_MODE_PERSISTENT, BLP_MODE_GRID, BLP_MODE_ONE_PER_LAUNCH = range(3)
BLP_RULE_LPC, BLP_RULE_RPC = range(2)
BLP_LAYOUT_COLUMN, BLP_LAYOUT_ROW = range(2)
ERROR_NAMES = {0: "SUCCESS", 1: "ERR_ARG", 2: "ERR_NOMEM", 3: "ERR_HIP", 4: "ERR_STATE", 5: "ERR_TOO_LARGE"}

# Every entry point that include/blp.h declares.
EXPORTS = ["blp_abi_version", "blp_options_default", "blp_create", "blp_destroy", "blp_last_error",
           "blp_solve_batch", "blp_get_solution", "blp_get_solution_batch", "blp_backward", "blp_last_bins",
           "blp_variant_info", "blp_last_kernel_ms", "blp_autotune", "blp_load_tuning", "blp_tuning",
           "blp_solve_batch_host", "blp_solve_shared", "blp_solve_batch_static", "blp_static_scratch_bytes",
           "blp_pivot_trace", "blp_backward_shared"]


class blp_options(ctypes.Structure):
    _fields_ = [("device", ctypes.c_int32), ("mode", ctypes.c_int32), ("max_iter", ctypes.c_int32),
                ("bland_after", ctypes.c_int32), ("eps_price", ctypes.c_double), ("eps_piv", ctypes.c_double),
                ("eps_feas", ctypes.c_double), ("variant", ctypes.c_int32), ("workers_per_cu", ctypes.c_int32),
                ("profile", ctypes.c_int32), ("graph", ctypes.c_int32), ("pivot_rule", ctypes.c_int32),
                ("layout", ctypes.c_int32), ("seed", ctypes.c_uint64), ("mem_limit", ctypes.c_uint64),
                ("tune_cache", ctypes.c_char_p)]


class blp_batch(ctypes.Structure):
    _fields_ = [("count", ctypes.c_int64), ("uniform", ctypes.c_int32), ("shared_box", ctypes.c_int32),
                ("m", ctypes.c_void_p), ("n", ctypes.c_void_p), ("kind", ctypes.c_void_p),
                ("a_off", ctypes.c_void_p), ("row_off", ctypes.c_void_p), ("col_off", ctypes.c_void_p),
                ("A", ctypes.c_void_p), ("b", ctypes.c_void_p), ("sense", ctypes.c_void_p),
                ("c", ctypes.c_void_p), ("l", ctypes.c_void_p), ("u", ctypes.c_void_p)]


class blp_outputs(ctypes.Structure):
    _fields_ = [("status", ctypes.c_void_p), ("iters", ctypes.c_void_p), ("obj", ctypes.c_void_p),
                ("x", ctypes.c_void_p), ("y", ctypes.c_void_p)]


class BlpError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"{ERROR_NAMES.get(code, code)}: {msg}")
        self.code = code


_lib = None


def lib() -> ctypes.CDLL:
    """The loaded library; raises if it has not been built (no fallback)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is not built; run __graft_entry__.build() (no CPU fallback exists)")
        L = ctypes.CDLL(LIB_PATH)
        vp, i32, i64 = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64
        P = ctypes.POINTER
        L.blp_abi_version.restype = i32
        L.blp_abi_version.argtypes = []
        L.blp_options_default.argtypes = [P(blp_options)]
        L.blp_create.argtypes = [P(vp), P(blp_options)]
        L.blp_destroy.argtypes = [vp]
        L.blp_destroy.restype = None
        L.blp_last_error.argtypes = [vp]
        L.blp_last_error.restype = ctypes.c_char_p
        L.blp_solve_batch.argtypes = [vp, P(blp_batch), P(blp_outputs), vp]
        L.blp_get_solution.argtypes = [vp, i64, vp, vp, vp, vp, vp]
        L.blp_get_solution_batch.argtypes = [vp, vp, vp, vp, vp, vp, i32]
        L.blp_backward.argtypes = [vp, vp, vp, vp, vp, vp, vp, vp]
        L.blp_last_bins.argtypes = [vp, vp, P(i32)]
        L.blp_variant_info.argtypes = [i32, ctypes.c_char_p, i32, P(i32), P(i32)]
        L.blp_last_kernel_ms.argtypes = [vp, vp, P(i32)]
        L.blp_autotune.argtypes = [vp, P(blp_batch), i32, ctypes.c_char_p, vp]
        L.blp_load_tuning.argtypes = [vp, ctypes.c_char_p]
        L.blp_tuning.argtypes = [vp, vp, P(i32)]
        L.blp_solve_batch_host.argtypes = [vp, P(blp_batch), P(blp_outputs), i32]
        L.blp_solve_shared.argtypes = [vp, i32, i32, vp, vp, vp, i64, vp, P(blp_outputs), vp]
        L.blp_solve_batch_static.argtypes = [vp, P(blp_batch), P(blp_outputs), vp]
        L.blp_pivot_trace.argtypes = [vp, P(blp_batch), P(blp_outputs), vp, i32, i32, vp]
        L.blp_backward_shared.argtypes = [vp, i32, i32, i64, vp, vp, vp, vp, vp, vp, vp, vp]
        L.blp_static_scratch_bytes.argtypes = []
        L.blp_static_scratch_bytes.restype = ctypes.c_size_t
        for f in EXPORTS:
            if f not in ("blp_abi_version", "blp_destroy", "blp_last_error", "blp_static_scratch_bytes"):
                getattr(L, f).restype = ctypes.c_int
        _lib = L
    return _lib


# ---------------------------------------------------------------------------
# Same-name wrappers of the C ABI
# ---------------------------------------------------------------------------
def blp_abi_version() -> int:
    return lib().blp_abi_version()


def blp_options_default() -> blp_options:
    o = blp_options()
    _check(None, lib().blp_options_default(ctypes.byref(o)))
    return o


def blp_create(opt: blp_options | None = None) -> ctypes.c_void_p:
    h = ctypes.c_void_p()
    _check(None, lib().blp_create(ctypes.byref(h), ctypes.byref(opt) if opt is not None else None))
    return h


def blp_destroy(h) -> None:
    lib().blp_destroy(h)


def blp_last_error(h) -> str:
    return (lib().blp_last_error(h) or b"").decode()


def blp_solve_batch(h, batch: blp_batch, out: blp_outputs | None = None, stream: int | None = None) -> None:
    _check(h, lib().blp_solve_batch(h, ctypes.byref(batch), ctypes.byref(out) if out is not None else None,
                                    stream))


def blp_solve_batch_static(h, batch: blp_batch, out: blp_outputs, stream: int | None = None) -> None:
    _check(h, lib().blp_solve_batch_static(h, ctypes.byref(batch), ctypes.byref(out), stream))


def blp_static_scratch_bytes() -> int:
    return lib().blp_static_scratch_bytes()


def blp_pivot_trace(h, batch: blp_batch, out: blp_outputs | None, trace: int, stride: int, replay: bool,
                    stream: int | None = None) -> None:
    _check(h, lib().blp_pivot_trace(h, ctypes.byref(batch), ctypes.byref(out) if out is not None else None, trace,
                                    stride, 1 if replay else 0, stream))


def blp_backward_shared(h, m: int, n: int, count: int, status, x, y, g, dC, db, dA,
                        stream: int | None = None) -> None:
    _check(h, lib().blp_backward_shared(h, m, n, count, status, x, y, g, dC, db, dA, stream))


def blp_solve_batch_host(h, batch: blp_batch, out: blp_outputs, chunks: int = 0) -> None:
    _check(h, lib().blp_solve_batch_host(h, ctypes.byref(batch), ctypes.byref(out), chunks))


def blp_solve_shared(h, m: int, n: int, A, b, sense, count: int, C, out: blp_outputs,
                     stream: int | None = None) -> None:
    _check(h, lib().blp_solve_shared(h, m, n, A, b, sense, count, C, ctypes.byref(out), stream))


def blp_get_solution(h, k: int, status=None, obj=None, x=None, y=None, iters=None) -> None:
    _check(h, lib().blp_get_solution(h, k, status, obj, x, y, iters))


def blp_get_solution_batch(h, status=None, iters=None, obj=None, x=None, y=None, on_device: int = 0) -> None:
    _check(h, lib().blp_get_solution_batch(h, status, iters, obj, x, y, on_device))


def blp_backward(h, g, dc=None, db=None, dA=None, dl=None, du=None, stream: int | None = None) -> None:
    _check(h, lib().blp_backward(h, g, dc, db, dA, dl, du, stream))


def blp_last_bins(h) -> np.ndarray:
    n = ctypes.c_int32()
    _check(h, lib().blp_last_bins(h, None, ctypes.byref(n)))
    out = np.zeros(n.value, np.int64)
    _check(h, lib().blp_last_bins(h, out.ctypes.data_as(ctypes.c_void_p), ctypes.byref(n)))
    return out


def blp_last_kernel_ms(h) -> np.ndarray:
    n = ctypes.c_int32()
    _check(h, lib().blp_last_kernel_ms(h, None, ctypes.byref(n)))
    out = np.zeros(n.value, np.float64)
    _check(h, lib().blp_last_kernel_ms(h, out.ctypes.data_as(ctypes.c_void_p), ctypes.byref(n)))
    return out


def blp_autotune(h, batch: blp_batch, sample: int = 512, cache_path: str | None = None,
                 stream: int | None = None) -> None:
    _check(h, lib().blp_autotune(h, ctypes.byref(batch), sample,
                                 cache_path.encode() if cache_path else None, stream))


def blp_load_tuning(h, cache_path: str) -> None:
    _check(h, lib().blp_load_tuning(h, cache_path.encode()))


def blp_tuning(h) -> np.ndarray:
    n = ctypes.c_int32()
    _check(h, lib().blp_tuning(h, None, ctypes.byref(n)))
    out = np.zeros(n.value, np.int32)
    _check(h, lib().blp_tuning(h, out.ctypes.data_as(ctypes.c_void_p), ctypes.byref(n)))
    return out


def blp_variant_info(v: int):
    name = ctypes.create_string_buffer(64)
    r, c = ctypes.c_int32(), ctypes.c_int32()
    rc = lib().blp_variant_info(v, name, 64, ctypes.byref(r), ctypes.byref(c))
    if rc != 0:
        return None
    return name.value.decode(), r.value, c.value


def variants() -> list:
    out, v = [], 0
    while True:
        info = blp_variant_info(v)
        if info is None:
            return out
        out.append(info)
        v += 1


def _check(h, rc: int) -> None:
    if rc != 0:
        raise BlpError(rc, blp_last_error(h) if h is not None else "")


# ---------------------------------------------------------------------------
# Torch-facing helpers (device memory and streams only)
# ---------------------------------------------------------------------------
def _ptr(t):
    return None if t is None else ctypes.c_void_p(t.data_ptr())


@dataclass
class DeviceBatch:
    """A packed batch whose data arrays live in device memory (torch tensors)
    and whose metadata stays on the host (numpy), as the C ABI takes them."""
    m: np.ndarray
    n: np.ndarray
    kind: np.ndarray
    a_off: np.ndarray
    row_off: np.ndarray
    col_off: np.ndarray
    A: object
    b: object
    sense: object
    c: object
    l: object
    u: object
    uniform: bool
    shared_box: bool = False  # l and u: one box of length n for every hyperbox LP

    @property
    def count(self) -> int:
        return int(self.m.shape[0]) if not self.uniform else self._count

    @classmethod
    def from_host(cls, hb, device="cuda", uniform: bool | None = None, shared_box: bool = False) -> "DeviceBatch":
        """Copy a packed host batch to the device.  With `shared_box`, hb.l
        and hb.u hold the one box (length n) of every hyperbox LP."""
        import torch
        uni = hb.uniform if uniform is None else uniform

        def dev(a, dt):
            return torch.from_numpy(np.ascontiguousarray(a)).to(device=device, dtype=dt)

        has_box = bool((hb.kind == 1).any())
        db = cls(m=hb.m, n=hb.n, kind=hb.kind, a_off=hb.a_off, row_off=hb.row_off, col_off=hb.col_off,
                 A=dev(hb.A if hb.A.size else np.zeros(1), torch.float64),
                 b=dev(hb.b if hb.b.size else np.zeros(1), torch.float64),
                 sense=dev(hb.sense if hb.sense.size else np.zeros(1, np.int8), torch.int8),
                 c=dev(hb.c, torch.float64),
                 l=dev(hb.l, torch.float64) if has_box else None,
                 u=dev(hb.u, torch.float64) if has_box else None, uniform=uni, shared_box=shared_box)
        db._count = hb.count
        return db

    def c_struct(self) -> blp_batch:
        K = self.count
        self._keep = [np.ascontiguousarray(a) for a in (self.m, self.n, self.kind, self.a_off, self.row_off,
                                                       self.col_off)]
        m, n, kind, ao, ro, co = [a.ctypes.data_as(ctypes.c_void_p) for a in self._keep]
        return blp_batch(K, 1 if self.uniform else 0, 1 if self.shared_box else 0, m, n, kind,
                         None if self.uniform else ao, None if self.uniform else ro, None if self.uniform else co,
                         _ptr(self.A), _ptr(self.b), _ptr(self.sense), _ptr(self.c), _ptr(self.l), _ptr(self.u))


class Solver:
    """A handle plus device result tensors.  One per host thread."""

    def __init__(self, device: int = 0, mode: int = BLP_MODE_PERSISTENT, variant: int = -1, max_iter: int = 0,
                 workers_per_cu: int = 0, bland_after: int = 0, profile: bool = False, graph: bool = False,
                 pivot_rule: int = BLP_RULE_LPC, seed: int = 0, layout: int = BLP_LAYOUT_COLUMN,
                 mem_limit: int = 0, tune_cache: str | None = None):
        o = blp_options_default()
        o.device, o.mode, o.variant, o.max_iter = device, mode, variant, max_iter
        o.workers_per_cu, o.bland_after, o.profile = workers_per_cu, bland_after, 1 if profile else 0
        o.graph = 1 if graph else 0
        o.pivot_rule, o.seed, o.layout = pivot_rule, seed, layout
        o.mem_limit = mem_limit
        o.tune_cache = tune_cache.encode() if tune_cache else None
        self.device = device
        self.h = blp_create(o)

    def close(self):
        if self.h:
            blp_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def solve(self, db: DeviceBatch, stream=None, outputs: dict | None = None) -> dict:
        """Solve on `stream` (torch stream or None for the current one).
        Returns device tensors status, iters, obj, x, y."""
        import torch
        dev = torch.device("cuda", self.device)
        K = db.count
        tot_m = int(db.m[0]) * K if db.uniform else int((db.row_off + db.m).max(initial=0))
        tot_n = int(db.n[0]) * K if db.uniform else int((db.col_off + db.n).max(initial=0))
        if outputs is None:
            outputs = {"status": torch.empty(max(K, 1), dtype=torch.int32, device=dev),
                       "iters": torch.empty(max(K, 1), dtype=torch.int32, device=dev),
                       "obj": torch.empty(max(K, 1), dtype=torch.float64, device=dev),
                       "x": torch.empty(max(tot_n, 1), dtype=torch.float64, device=dev),
                       "y": torch.empty(max(tot_m, 1), dtype=torch.float64, device=dev)}
        o = blp_outputs(*[_ptr(outputs[k]) for k in ("status", "iters", "obj", "x", "y")])
        st = stream if stream is not None else torch.cuda.current_stream(dev)
        self._batch = db.c_struct()
        blp_solve_batch(self.h, self._batch, o, st.cuda_stream)
        self._last = (db, outputs)
        return outputs

    def pivot_trace(self, db: DeviceBatch, trace, stride: int, replay: bool, stream=None,
                    outputs: dict | None = None) -> dict:
        """blp_pivot_trace on a uniform batch: record each LP's pivots into
        `trace` (int32 device tensor of count * stride) or replay them.
        Returns device tensors status, iters, obj, x, y."""
        import torch
        dev = torch.device("cuda", self.device)
        K = db.count
        if outputs is None:
            outputs = {"status": torch.empty(max(K, 1), dtype=torch.int32, device=dev),
                       "iters": torch.empty(max(K, 1), dtype=torch.int32, device=dev),
                       "obj": torch.empty(max(K, 1), dtype=torch.float64, device=dev),
                       "x": torch.empty(max(int(db.n[0]) * K, 1), dtype=torch.float64, device=dev),
                       "y": torch.empty(max(int(db.m[0]) * K, 1), dtype=torch.float64, device=dev)}
        o = blp_outputs(*[_ptr(outputs[k]) for k in ("status", "iters", "obj", "x", "y")])
        st = stream if stream is not None else torch.cuda.current_stream(dev)
        self._batch = db.c_struct()
        blp_pivot_trace(self.h, self._batch, o, _ptr(trace), stride, replay, st.cuda_stream)
        self._last = (db, outputs)
        return outputs

    def solve_shared(self, A, b, sense, C, stream=None) -> dict:
        """One constraint set (A: m x n, b, sense: m; device tensors) with the
        objectives in the rows of C (count x n).  Returns device tensors
        status, iters, obj (count), x (count x n), y (count x m)."""
        import torch
        dev = torch.device("cuda", self.device)
        m, n = int(b.numel()), int(C.shape[1])
        K = int(C.shape[0])
        out = {"status": torch.empty(max(K, 1), dtype=torch.int32, device=dev),
               "iters": torch.empty(max(K, 1), dtype=torch.int32, device=dev),
               "obj": torch.empty(max(K, 1), dtype=torch.float64, device=dev),
               "x": torch.empty(max(K * n, 1), dtype=torch.float64, device=dev),
               "y": torch.empty(max(K * m, 1), dtype=torch.float64, device=dev)}
        o = blp_outputs(*[_ptr(out[k]) for k in ("status", "iters", "obj", "x", "y")])
        st = stream if stream is not None else torch.cuda.current_stream(dev)
        blp_solve_shared(self.h, m, n, _ptr(A), _ptr(b), _ptr(sense), K, _ptr(C), o, st.cuda_stream)
        return out

    def backward_shared(self, out: dict, m: int, n: int, g, stream=None, want=("dC", "db", "dA")) -> dict:
        """Gradients of sum_k g[k] obj_k after solve_shared (its output dict
        `out`): dC (count x n), db (m), dA (m x n), new device tensors."""
        import torch
        K = int(g.numel())
        dev = g.device
        res = {"dC": torch.empty(max(K * n, 1), dtype=torch.float64, device=dev) if "dC" in want else None,
               "db": torch.empty(m, dtype=torch.float64, device=dev) if "db" in want else None,
               "dA": torch.empty(m * n, dtype=torch.float64, device=dev) if "dA" in want else None}
        st = stream if stream is not None else torch.cuda.current_stream(dev)
        blp_backward_shared(self.h, m, n, K, _ptr(out["status"]), _ptr(out["x"]), _ptr(out["y"]), _ptr(g),
                            _ptr(res["dC"]), _ptr(res["db"]), _ptr(res["dA"]), st.cuda_stream)
        return res

    def autotune(self, db: DeviceBatch, sample: int = 512, cache_path: str | None = None, stream=None) -> None:
        import torch
        st = stream if stream is not None else torch.cuda.current_stream(torch.device("cuda", self.device))
        self._tune_batch = db.c_struct()
        blp_autotune(self.h, self._tune_batch, sample, cache_path, st.cuda_stream)

    def backward(self, g, stream=None, want=("dc", "db", "dA", "dl", "du"), out: dict | None = None) -> dict:
        """Gradients of sum_k g[k] obj_k into new tensors (or into `out`,
        the dict a previous call returned: nothing is allocated then)."""
        import torch
        db, _ = self._last
        dev = g.device
        if out is not None:
            res = out
        else:
            res = {}
            for k in want:
                src = {"dc": db.c, "db": db.b, "dA": db.A, "dl": db.l, "du": db.u}[k]
                if k in ("dl", "du") and src is not None and getattr(db, "shared_box", False):
                    src = src[:int(db.n[db.kind == 1][0])]
                res[k] = None if src is None else torch.zeros_like(src)
        st = stream if stream is not None else torch.cuda.current_stream(dev)
        blp_backward(self.h, _ptr(g), _ptr(res.get("dc")), _ptr(res.get("db")), _ptr(res.get("dA")),
                     _ptr(res.get("dl")), _ptr(res.get("du")), st.cuda_stream)
        return res
