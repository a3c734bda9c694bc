"""Boundary options on the GPU: memory-limited (chunked) solves, the tuning
cache option, one box shared by many hyperbox LPs (Sec. 6's many-objectives
use) with its adjoint, and on-device result copies."""
import ctypes

import numpy as np
import pytest

import lpgen
import oracle
from solve_util import compare, gpu_solve

pytestmark = pytest.mark.gpu


def _bits(a):
    return np.asarray(a).view(np.int64)


def _same(a, b, K, tag, nx=None, ny=None):
    """Bitwise equal results; x and y over their first nx / ny entries (the
    batch's packed extents)."""
    for k in ("status", "iters"):
        assert np.array_equal(np.asarray(a[k])[:K], np.asarray(b[k])[:K]), (tag, k)
    for k in ("obj",):
        assert np.array_equal(_bits(np.asarray(a[k])[:K]), _bits(np.asarray(b[k])[:K])), (tag, k)
    for k, lim in (("x", nx), ("y", ny)):
        n = min(len(a[k]), len(b[k])) if lim is None else lim
        assert np.array_equal(_bits(a[k][:n]), _bits(b[k][:n])), (tag, k)


def test_mem_limit_chunks_identical():
    """A limit that holds the results plus only a few dozen LPs' lists: the
    batch is solved in chunks (Eq. (5)'s capacity) with the same bits as one
    unlimited solve, and as the oracle."""
    import torch

    import paper_1609_08114_amd as blp
    for hb, per_lp, tag in ((lpgen.config(4, range(0, 200)), 48, "mixed"), (lpgen.config(2, range(400)), 8, "uniform")):
        print(f"[boundary] mem_limit {tag}", flush=True)
        ref = gpu_solve(hb)
        K = hb.count
        # (the results go to the caller's tensors) bin counters, one
        # streaming slot of the largest LP, then room for 37 LPs
        m, n = hb.m.astype(np.int64), hb.n.astype(np.int64)
        slot = int((((m + 2 + 15) // 16) * 16 * (n + m + 1) * 8)[hb.kind == 0].max())
        # bin counters: lengths, fill counts and offsets, the work-list heads
        # one 128-byte line apart, then 64 striped copies of the counts, one
        # 128-byte line each
        nbins = len(blp.variants()) + 2
        counters = 4 * (-(-3 * nbins // 32) * 32 + 32 * nbins + 64 * 32)
        limit = counters + slot + 37 * per_lp
        s = blp.Solver(mem_limit=limit)
        try:
            db = blp.DeviceBatch.from_host(hb)
            out = s.solve(db)
            torch.cuda.synchronize()
            g = {k: v.cpu().numpy() for k, v in out.items()}
            # the handle reports every LP of the chunked solve
            st = np.zeros(1, np.int32)
            ob = np.zeros(1)
            blp.blp_get_solution(s.h, K - 3, st.ctypes.data_as(ctypes.c_void_p), ob.ctypes.data_as(ctypes.c_void_p),
                                 None, None, None)
            assert st[0] == ref["status"][K - 3] and ob[0] == ref["obj"][K - 3]
            with pytest.raises(blp.BlpError) as ei:
                s.backward(torch.ones(K, dtype=torch.float64, device="cuda"), want=("dc",))
            assert ei.value.code == blp.BLP_ERR_STATE
        finally:
            s.close()
        _same(g, ref, K, tag, hb.c.size, hb.b.size)
        gg = {k: (v[:K] if k in ("status", "iters", "obj") else v) for k, v in g.items()}
        compare(hb, gg, oracle.solve_batch(hb), strict=True, tag="mem-limit-" + tag)
    # a limit below one LP's needs
    s = blp.Solver(mem_limit=4096)
    try:
        with pytest.raises(blp.BlpError) as ei:
            s.solve(blp.DeviceBatch.from_host(lpgen.config(3, range(2))))
        assert ei.value.code == blp.BLP_ERR_NOMEM
    finally:
        s.close()


def test_tune_cache_option(tmp_path):
    import torch

    import paper_1609_08114_amd as blp
    hb = lpgen.config(5, range(400), part="simplex")
    db = blp.DeviceBatch.from_host(hb)
    path = str(tmp_path / "tune.json")
    s = blp.Solver()
    s.autotune(db, sample=16, cache_path=path)
    remap = blp.blp_tuning(s.h)
    s.close()
    s2 = blp.Solver(tune_cache=path)
    try:
        assert np.array_equal(blp.blp_tuning(s2.h), remap)
        out = s2.solve(db)
        torch.cuda.synchronize()
        g = {k: v.cpu().numpy() for k, v in out.items()}
    finally:
        s2.close()
    K = hb.count
    compare(hb, {k: (v[:K] if k in ("status", "iters", "obj") else v) for k, v in g.items()},
            oracle.solve_batch(hb), strict=True, tag="tune-cache")
    with pytest.raises(blp.BlpError):
        blp.Solver(tune_cache=str(tmp_path / "missing.json"))


def _box_batch(K, n, seed, with_simplex=False):
    """K hyperbox LPs with their own unit objectives, one box [l, u] for all
    (and optionally interleaved simplex LPs)."""
    rng = np.random.default_rng(seed)
    lo = rng.uniform(-10, -1, n)
    hi = rng.uniform(1, 10, n)
    lo[0] = 0.0  # a zero lower bound and a zero objective coefficient below
    C = rng.normal(size=(K, n))
    C /= np.linalg.norm(C, axis=1, keepdims=True)
    C[3, 1] = 0.0
    per = lpgen.make_batch(1, np.arange(K), np.full(K, 3, np.int32), np.zeros(K, np.int32), np.full(K, n, np.int32))
    per.c[:] = C.ravel()
    per.l[:] = np.tile(lo, K)
    per.u[:] = np.tile(hi, K)
    if not with_simplex:
        shared = lpgen.make_batch(1, np.arange(K), np.full(K, 3, np.int32), np.zeros(K, np.int32),
                                  np.full(K, n, np.int32))
        shared.c[:] = C.ravel()
        shared.l = lo.copy()
        shared.u = hi.copy()
        return per, shared, lo, hi
    # interleave simplex LPs of workload 1
    cfg = lpgen.config(1, range(K // 4))
    kinds = []
    parts = []
    for k in range(K):
        parts.append(("box", k))
        if k % 4 == 0 and k // 4 < cfg.count:
            parts.append(("lp", k // 4))
    lps = []
    for kind, i in parts:
        if kind == "box":
            lps.append(dict(c=C[i], l=lo, u=hi))
        else:
            d = cfg.lp(i)
            lps.append(dict(A=d["A"], b=d["b"], c=d["c"], sense=d["sense"]))
    from solve_util import crafted_batch
    per = crafted_batch(lps)
    shared = crafted_batch(lps)
    shared.l = lo.copy()
    shared.u = hi.copy()
    return per, shared, lo, hi


@pytest.mark.parametrize("mixed", [False, True])
def test_shared_box_matches_oracle_and_its_adjoint(mixed):
    import torch

    import paper_1609_08114_amd as blp
    K, n = 5000, 7
    per, shared, lo, hi = _box_batch(K, n, seed=31, with_simplex=mixed)
    KK = per.count
    o = oracle.solve_batch(per)
    s = blp.Solver()
    try:
        dbs = blp.DeviceBatch.from_host(shared, shared_box=True)
        out = s.solve(dbs)
        torch.cuda.synchronize()
        g = {k: v.cpu().numpy() for k, v in out.items()}
        w = torch.from_numpy(lpgen.weights(77, np.arange(KK))).to("cuda")
        gr1 = s.backward(w)
        gr2 = s.backward(w)
        torch.cuda.synchronize()
        dc = gr1["dc"].cpu().numpy()
        dl, du = gr1["dl"].cpu().numpy(), gr1["du"].cpu().numpy()
        assert np.array_equal(_bits(dl), _bits(gr2["dl"].cpu().numpy()))  # fixed summation order
        assert np.array_equal(_bits(du), _bits(gr2["du"].cpu().numpy()))
    finally:
        s.close()
    gg = {k: (v[:KK] if k in ("status", "iters", "obj") else v) for k, v in g.items()}
    compare(per, gg, o, strict=True, tag="shared-box")
    # the per-LP-box solve gives the same bits
    _same(gpu_solve(per), g, KK, "per-lp-box", per.c.size, per.b.size)
    # adjoint: dc = w x per LP; dl, du = sums of w min(c, 0), w max(c, 0)
    wn = w.cpu().numpy()
    box = per.kind == 1
    ok = box & (o["status"] == 0)
    Cb = np.stack([per.c[per.col_off[k]:per.col_off[k] + n] for k in np.nonzero(box)[0]])
    wb = np.where(ok[box], wn[box], 0.0)
    want_l = (wb[:, None] * np.minimum(Cb, 0.0)).sum(axis=0)
    want_u = (wb[:, None] * np.where(Cb < 0.0, 0.0, Cb)).sum(axis=0)
    assert np.allclose(dl, want_l, rtol=1e-12, atol=1e-12) and np.allclose(du, want_u, rtol=1e-12, atol=1e-12)
    for k in np.nonzero(box)[0][:200]:
        co = per.col_off[k]
        assert np.array_equal(_bits(dc[co:co + n]), _bits(wn[k] * o["x"][co:co + n]))


def test_shared_box_host_pipeline():
    per, shared, lo, hi = _box_batch(3000, 5, seed=5, with_simplex=True)
    g = _host_solve_shared(shared, 3)
    compare(per, g, oracle.solve_batch(per), strict=True, tag="host-shared-box")


def _host_solve_shared(hb, chunks):
    import paper_1609_08114_amd as blp
    s = blp.Solver()
    K = hb.count
    st = np.zeros(K, np.int32)
    it = np.zeros(K, np.int32)
    ob = np.zeros(K)
    x = np.zeros(hb.c.size)
    y = np.zeros(max(1, hb.b.size))
    keep = [np.ascontiguousarray(a) for a in (hb.m, hb.n, hb.kind, hb.a_off, hb.row_off, hb.col_off)]
    P = lambda a: a.ctypes.data_as(ctypes.c_void_p)
    b = blp.blp_batch(K, 0, 1, *[P(a) for a in keep], P(hb.A), P(hb.b), P(hb.sense), P(hb.c), P(hb.l), P(hb.u))
    o = blp.blp_outputs(P(st), P(it), P(ob), P(x), P(y))
    try:
        blp.blp_solve_batch_host(s.h, b, o, chunks)
    finally:
        s.close()
    return {"status": st, "iters": it, "obj": ob, "x": x, "y": y}


def test_solution_batch_on_device():
    import torch

    import paper_1609_08114_amd as blp
    hb = lpgen.config(4, range(300, 380))
    s = blp.Solver()
    try:
        db = blp.DeviceBatch.from_host(hb)
        s.solve(db)
        K = hb.count
        nx, ny = hb.c.size, hb.b.size
        dev = {"status": torch.full((K,), -1, dtype=torch.int32, device="cuda"),
               "iters": torch.full((K,), -1, dtype=torch.int32, device="cuda"),
               "obj": torch.zeros(K, dtype=torch.float64, device="cuda"),
               "x": torch.zeros(nx, dtype=torch.float64, device="cuda"),
               "y": torch.zeros(ny, dtype=torch.float64, device="cuda")}
        P = lambda t: ctypes.c_void_p(t.data_ptr())
        blp.blp_get_solution_batch(s.h, P(dev["status"]), P(dev["iters"]), P(dev["obj"]), P(dev["x"]), P(dev["y"]),
                                   on_device=1)
        host = {"status": np.zeros(K, np.int32), "iters": np.zeros(K, np.int32), "obj": np.zeros(K),
                "x": np.zeros(nx), "y": np.zeros(ny)}
        Q = lambda a: a.ctypes.data_as(ctypes.c_void_p)
        blp.blp_get_solution_batch(s.h, Q(host["status"]), Q(host["iters"]), Q(host["obj"]), Q(host["x"]),
                                   Q(host["y"]))
        torch.cuda.synchronize()
    finally:
        s.close()
    _same({k: v.cpu().numpy() for k, v in dev.items()}, host, K, "on-device", nx, ny)
    compare(hb, host, oracle.solve_batch(hb), strict=True, tag="solution-batch")
