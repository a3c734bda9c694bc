"""Shared constraints, many objectives (blp_solve_shared, the support-function
sampling of Sec. 7): every objective's status and optimum against the
oracle solving that LP on its own.  The warm-started pivot path differs from
a cold solve, so objectives are compared to 1e-9 relative (not bit for bit)
and x, y only where the optimum is non-degenerate."""
import numpy as np
import pytest

import lpgen
import oracle
from solve_util import REL, crafted_batch

pytestmark = pytest.mark.gpu


def _shared_gpu(A, b, sense, C, variant=-1):
    import torch

    import paper_1609_08114_amd as blp
    dev = torch.device("cuda")
    s = blp.Solver(variant=variant)
    try:
        out = s.solve_shared(torch.from_numpy(np.ascontiguousarray(A, np.float64).ravel()).to(dev),
                             torch.from_numpy(np.ascontiguousarray(b, np.float64)).to(dev),
                             torch.from_numpy(np.ascontiguousarray(sense, np.int8)).to(dev),
                             torch.from_numpy(np.ascontiguousarray(C, np.float64)).to(dev))
        torch.cuda.synchronize()
        K, n, m = C.shape[0], C.shape[1], len(b)
        return {"status": out["status"][:K].cpu().numpy(), "iters": out["iters"][:K].cpu().numpy(),
                "obj": out["obj"][:K].cpu().numpy(), "x": out["x"][:K * n].cpu().numpy().reshape(K, n),
                "y": out["y"][:K * m].cpu().numpy().reshape(K, m)}
    finally:
        s.close()


def _oracle(A, b, sense, C):
    lps = [dict(A=A, b=b, c=c, sense=sense) for c in C]
    return oracle.solve_batch(crafted_batch(lps))


def _check(A, b, sense, C, tag, variant=-1):
    g = _shared_gpu(A, b, sense, C, variant)
    o = _oracle(A, b, sense, C)
    K, n = C.shape
    m = len(b)
    bad = np.nonzero(g["status"] != o["status"])[0]
    assert bad.size == 0, f"{tag}: status differs at {bad[:10]}: {g['status'][bad[:10]]} vs {o['status'][bad[:10]]}"
    ok = o["status"] == oracle.OPTIMAL
    rel = np.abs(g["obj"][ok] - o["obj"][ok]) / np.maximum(1.0, np.abs(o["obj"][ok]))
    assert (rel <= REL).all(), f"{tag}: obj relerr {rel.max():.3e}"
    inf = np.isin(o["status"], (oracle.INFEASIBLE, oracle.UNBOUNDED))
    assert np.array_equal(g["obj"][inf], o["obj"][inf]), tag
    # x and y where the optimum is unique (basic values and reduced costs away from 0)
    ox = o["x"].reshape(K, n)
    oy = o["y"].reshape(K, m)
    checked = 0
    for k in np.nonzero(ok)[0]:
        x, y = ox[k], oy[k]
        slack = np.where(np.asarray(sense) == 0, b - A @ x, A @ x - b)
        scale = max(1.0, float(np.abs(b).max()))
        nbasic = (x > 1e-7 * scale).sum() + (slack > 1e-7 * scale).sum()
        d = C[k] - A.T @ y
        if nbasic != m or (np.abs(d[x <= 1e-7 * scale]) <= 1e-7).any() or (np.abs(y[slack <= 1e-7 * scale]) <= 1e-7).any():
            continue
        assert np.allclose(g["x"][k], x, rtol=1e-9, atol=1e-9 * scale), (tag, k)
        assert np.allclose(g["y"][k], y, rtol=1e-9, atol=1e-9 * max(1.0, np.abs(y).max())), (tag, k)
        checked += 1
    return g, o, checked


def test_type1_polytope_many_directions():
    # one workload-2 polytope (m = n = 100), 600 objectives: 300 from the
    # workload's own distribution, 300 unit directions (support function)
    hb = lpgen.config(2, [7])
    lp = hb.lp(0)
    A, b, sense = lp["A"], lp["b"], lp["sense"]
    rng = np.random.default_rng(21)
    C1 = rng.uniform(1, 10, size=(300, 100))
    G = rng.normal(size=(300, 100))
    C2 = G / np.linalg.norm(G, axis=1, keepdims=True)
    g, o, checked = _check(A, b, sense, np.vstack([C1, C2]), "type1")
    assert (o["status"] == oracle.OPTIMAL).all() and checked > 100


def test_directions_swept_along_a_circle():
    # support-function sampling: directions cos(t) u + sin(t) v, t stepping
    # around a circle; neighbouring optima share most of their basis, so the
    # warm starts need far fewer pivots than cold solves
    hb = lpgen.config(2, [11])
    lp = hb.lp(0)
    A, b, sense = lp["A"], lp["b"], lp["sense"]
    rng = np.random.default_rng(4)
    u, v = rng.normal(size=(2, 100))
    t = np.linspace(0.0, 2.0 * np.pi, 2048, endpoint=False)
    C = np.cos(t)[:, None] * u + np.sin(t)[:, None] * v
    g, o, _ = _check(A, b, sense, C, "sweep")
    assert g["iters"].mean() < 0.5 * o["iters"].mean(), (g["iters"].mean(), o["iters"].mean())


def test_type2_polytope_phase1_once():
    # ">=" rows: the origin is infeasible, phase 1 runs once per workgroup
    hb = lpgen.config(4, range(0, 400))
    k = next(i for i in range(hb.count) if hb.kind[i] == 0 and 20 <= hb.m[i] <= 60 and 20 <= hb.n[i] <= 60
             and (hb.sense[hb.row_off[i]:hb.row_off[i] + hb.m[i]] != 0).any())
    lp = hb.lp(k)
    A, b, sense = lp["A"], lp["b"], lp["sense"]
    n = A.shape[1]
    rng = np.random.default_rng(5)
    G = rng.normal(size=(400, n))
    C = G / np.linalg.norm(G, axis=1, keepdims=True)
    g, o, _ = _check(A, b, sense, C, "type2")
    assert (o["status"] == oracle.OPTIMAL).all()
    # the same polytope swept around a circle: warm starts after one phase 1
    u, v = rng.normal(size=(2, n))
    t = np.linspace(0.0, 2.0 * np.pi, 600, endpoint=False)
    Cs = np.cos(t)[:, None] * u + np.sin(t)[:, None] * v
    g, o, _ = _check(A, b, sense, Cs, "type2-sweep")
    assert g["iters"].mean() < 0.5 * o["iters"].mean()


def test_mixed_outcomes_and_bad_objectives():
    # an unbounded recession direction for some objectives, NaN in one
    A = np.array([[1.0, -1.0, 0.0], [-1.0, 1.0, 0.0], [0.0, 0.0, 1.0], [1.0, 1.0, 1.0]])
    b = np.array([2.0, 3.0, 5.0, 1.0])
    sense = np.array([0, 0, 0, 1], np.int8)  # a strip in (x1, x2), unbounded along (1, 1)
    rng = np.random.default_rng(9)
    C = rng.integers(-3, 4, size=(500, 3)).astype(float)
    C[17, 1] = np.nan
    g = _shared_gpu(A, b, sense, C)
    assert g["status"][17] == oracle.NUMERICAL
    keep = np.ones(len(C), bool)
    keep[17] = False
    _check(A, b, sense, C[keep], "mixed")
    st = _oracle(A, b, sense, C[keep])["status"]
    assert set(np.unique(st)) >= {oracle.OPTIMAL, oracle.UNBOUNDED}


def test_mixed_outcomes_along_a_sweep():
    # warm starts through optimal and unbounded objectives, one of them NaN
    A = np.array([[1.0, -1.0, 0.0], [-1.0, 1.0, 0.0], [0.0, 0.0, 1.0], [1.0, 1.0, 1.0]])
    b = np.array([2.0, 3.0, 5.0, 1.0])
    sense = np.array([0, 0, 0, 1], np.int8)
    t = np.linspace(0.0, 4.0 * np.pi, 800, endpoint=False)
    C = np.stack([np.cos(t), np.sin(t), 0.3 + 0.2 * np.cos(3 * t)], axis=1)
    C[401, 0] = np.nan
    g = _shared_gpu(A, b, sense, C)
    assert g["status"][401] == oracle.NUMERICAL
    keep = np.ones(len(C), bool)
    keep[401] = False
    g2, o, _ = _check(A, b, sense, C[keep], "mixed-sweep")
    assert set(np.unique(o["status"])) >= {oracle.OPTIMAL, oracle.UNBOUNDED}
    # the statuses of the full run agree with the run without the NaN objective
    assert np.array_equal(g["status"][keep], g2["status"])


def test_infeasible_constraints():
    A = np.array([[1.0, 1.0], [1.0, 1.0]])
    b = np.array([1.0, 3.0])
    sense = np.array([0, 1], np.int8)
    C = np.random.default_rng(2).normal(size=(50, 2))
    g, o, _ = _check(A, b, sense, C, "infeasible")
    assert (g["status"] == oracle.INFEASIBLE).all()
    t = np.linspace(0.0, 1.0, 200)
    Cs = np.stack([1.0 + 0.1 * t, 1.0 - 0.1 * t], axis=1)  # close directions: the warm-start kernel
    g, o, _ = _check(A, b, sense, Cs, "infeasible-sweep")
    assert (g["status"] == oracle.INFEASIBLE).all()


def test_cold_route_on_every_register_variant():
    # unrelated directions take the cold route; forcing each register-tile
    # variant in turn checks that every kernel reads the one shared
    # constraint set (A, b, sense at offset 0) and not per-LP offsets
    import paper_1609_08114_amd as blp
    rng = np.random.default_rng(13)
    m, n = 5, 5
    A = rng.uniform(0.5, 2.0, size=(m, n))
    b = rng.uniform(5.0, 10.0, size=m)
    sense = np.zeros(m, np.int8)
    sense[2] = 1  # one ">=" row: phase 1 with one artificial
    b[2] = 1.0
    C = rng.normal(size=(300, n))
    le = np.zeros(m, np.int8)  # the same rows as "<=": no artificial variable
    for v, (name, _, _) in enumerate(blp.variants()):
        print(f"[shared-cold] variant {name}", flush=True)
        g, o, _ = _check(A, b, le, C, f"cold-{name}-type1", variant=v)
        assert (o["status"] == oracle.OPTIMAL).any()
        try:
            g, o, _ = _check(A, b, sense, C, f"cold-{name}", variant=v)
        except blp.BlpError as e:
            # a variant for LPs without artificial rows (it held the 5 x 5
            # set above) refuses this one, which needs phase 1
            assert e.code == blp.BLP_ERR_TOO_LARGE and name in str(e), e
            continue
        assert (o["status"] == oracle.OPTIMAL).any()


def test_beyond_the_shared_tile():
    """Constraint sets larger than the 112 x 112 tile of the warm-start
    kernel take the cold route: a 130 x 130 type-1 set in the register tile
    that holds it, and workload 3's first 200 x 200 set (rows of both senses,
    phase 1) in the streaming kernel; every objective against the oracle."""
    rng = np.random.default_rng(31)
    m = n = 130
    A = rng.uniform(1.0, 10.0, size=(m, n))
    b = rng.uniform(10.0, 100.0, size=m)
    C = rng.normal(size=(120, n))
    C[:60] = np.abs(C[:60])  # half of them in the positive orthant
    _check(A, b, np.zeros(m, np.int8), C, "shared-130")
    h3 = lpgen.config(3, range(0, 1))
    m3, n3 = int(h3.m[0]), int(h3.n[0])
    A3 = h3.A[:m3 * n3].reshape(m3, n3)
    C3 = np.vstack([h3.c[:n3], rng.uniform(1.0, 10.0, size=(15, n3))])
    _check(A3, h3.b[:m3], h3.sense[:m3], C3, "shared-200-streaming")


def test_shared_errors():
    import torch

    import paper_1609_08114_amd as blp
    s = blp.Solver()
    dev = torch.device("cuda")
    A = torch.ones(2100 * 5, dtype=torch.float64, device=dev)
    b = torch.ones(2100, dtype=torch.float64, device=dev)
    sense = torch.zeros(2100, dtype=torch.int8, device=dev)
    C = torch.ones(3, 5, dtype=torch.float64, device=dev)
    with pytest.raises(blp.BlpError) as ei:
        s.solve_shared(A, b, sense, C)  # more rows than any LP may have
    assert ei.value.code == blp.BLP_ERR_TOO_LARGE
    out = s.solve_shared(A[:10], b[:2], sense[:2], C[:0])
    torch.cuda.synchronize()
    assert out["status"].numel() == 1  # nothing solved, nothing written
    s.close()


def test_shared_adjoint():
    """blp_backward_shared after solve_shared: dC, db and dA against the
    formulas on the same x, y, status (w_k = g_k at OPTIMAL LPs, else 0), and
    against the per-LP adjoint of blp_backward summed over the objectives;
    repeated calls give the same bits."""
    import torch

    import paper_1609_08114_amd as blp
    rng = np.random.default_rng(41)
    m, n, K = 24, 20, 3000
    A = rng.uniform(1.0, 10.0, size=(m, n))
    b = rng.uniform(10.0, 100.0, size=m)
    sense = np.zeros(m, np.int8)
    C = rng.normal(size=(K, n))
    C[5] = np.nan  # a NUMERICAL objective: no gradient
    dev = torch.device("cuda")
    s = blp.Solver()
    try:
        tA = torch.from_numpy(A.ravel()).to(dev)
        tb = torch.from_numpy(b).to(dev)
        ts = torch.from_numpy(sense).to(dev)
        out = s.solve_shared(tA, tb, ts, torch.from_numpy(C).to(dev))
        g = torch.from_numpy(rng.uniform(0.0, 1.0, size=K)).to(dev)
        r1 = s.backward_shared(out, m, n, g)
        r2 = s.backward_shared(out, m, n, g)
        torch.cuda.synchronize()
        st = out["status"][:K].cpu().numpy()
        X = out["x"][:K * n].cpu().numpy().reshape(K, n)
        Y = out["y"][:K * m].cpu().numpy().reshape(K, m)
        w = np.where(st == 0, g.cpu().numpy(), 0.0)
        assert st[5] == blp.BLP_NUMERICAL and (st == 0).sum() > K // 2
        got = {k: v.cpu().numpy() for k, v in r1.items()}
        for k in got:
            assert np.array_equal(got[k].view(np.int64), r2[k].cpu().numpy().view(np.int64)), k
        dC = np.where(st[:, None] == 0, w[:, None] * np.nan_to_num(X), 0.0)
        assert np.array_equal(got["dC"].reshape(K, n), dC)
        wy = np.where(st[:, None] == 0, w[:, None] * np.nan_to_num(Y), 0.0)
        db = wy.sum(axis=0)
        dA = -(wy.T @ np.where(st[:, None] == 0, np.nan_to_num(X), 0.0))
        scale_b = (np.abs(wy).sum(axis=0) + 1.0)
        assert (np.abs(got["db"] - db) <= 1e-12 * scale_b).all()
        scale_a = np.abs(wy).T @ np.abs(np.where(st[:, None] == 0, np.nan_to_num(X), 0.0)) + 1.0
        assert (np.abs(got["dA"].reshape(m, n) - dA) <= 1e-12 * scale_a).all()
    finally:
        s.close()
    # the per-LP adjoint of the same LPs solved as an ordinary batch, summed
    ok = st == 0
    lps = [dict(A=A, b=b, c=C[k], sense=sense) for k in np.nonzero(ok)[0][:400]]
    hb = crafted_batch(lps)
    s2 = blp.Solver()
    try:
        db_ = blp.DeviceBatch.from_host(hb)
        o2 = s2.solve(db_)
        gk = torch.from_numpy(w[ok][:400].copy()).to(dev)
        grads = s2.backward(gk)
        torch.cuda.synchronize()
        per_dA = grads["dA"].cpu().numpy().reshape(len(lps), m, n).sum(axis=0)
        sel = np.zeros(K)
        sel[np.nonzero(ok)[0][:400]] = 1.0
        s3 = blp.Solver()
        out3 = s3.solve_shared(tA, tb, ts, torch.from_numpy(C).to(dev))
        r3 = s3.backward_shared(out3, m, n, torch.from_numpy(sel * g.cpu().numpy()).to(dev))
        torch.cuda.synchronize()
        s3.close()
        tot = np.abs(per_dA).max() + 1.0
        assert np.abs(r3["dA"].cpu().numpy().reshape(m, n) - per_dA).max() <= 1e-9 * tot
        assert o2["status"][:len(lps)].cpu().numpy().max() == 0
    finally:
        s2.close()


def test_shared_solve_is_stream_ordered():
    """The route of a shared-constraint solve is chosen on the device and
    nothing is read back, so the call can be captured in a graph once an
    eager call has sized its buffers: every replay (with other work on the
    GPU between them) gives the eager call's bits, for a swept circle (warm
    starts), random directions (cold, register tile) and a two-phase 200 x
    200 set (cold, streaming kernel)."""
    import torch

    import paper_1609_08114_amd as blp
    dev = torch.device("cuda")
    rng = np.random.default_rng(8)
    lp = lpgen.config(2, [11]).lp(0)
    u, v = rng.normal(size=(2, 100))
    t = np.linspace(0.0, 2.0 * np.pi, 600, endpoint=False)
    sweep = np.cos(t)[:, None] * u + np.sin(t)[:, None] * v
    h3 = lpgen.config(3, range(0, 1))
    m3, n3 = int(h3.m[0]), int(h3.n[0])
    cases = [("sweep", lp["A"], lp["b"], lp["sense"], sweep),
             ("random", lp["A"], lp["b"], lp["sense"], rng.normal(size=(300, 100))),
             ("streaming", h3.A[:m3 * n3].reshape(m3, n3), h3.b[:m3], h3.sense[:m3],
              rng.uniform(1.0, 10.0, size=(24, n3)))]
    for tag, A, b, sense, C in cases:
        print(f"[shared] graph capture {tag}", flush=True)
        Ad = torch.from_numpy(np.ascontiguousarray(A, np.float64).ravel()).to(dev)
        bd = torch.from_numpy(np.ascontiguousarray(b, np.float64)).to(dev)
        sd = torch.from_numpy(np.ascontiguousarray(sense, np.int8)).to(dev)
        Cd = torch.from_numpy(np.ascontiguousarray(C, np.float64)).to(dev)
        s = blp.Solver()
        st = torch.cuda.Stream()
        try:
            with torch.cuda.stream(st):
                ref = {k: v.clone() for k, v in s.solve_shared(Ad, bd, sd, Cd).items()}
            torch.cuda.synchronize()
            g = torch.cuda.CUDAGraph()
            with torch.cuda.graph(g, stream=st):
                out = s.solve_shared(Ad, bd, sd, Cd)
            torch.cuda.synchronize()
            for rep in range(3):
                for k in out:
                    out[k].fill_(-7)
                noise = torch.randn(1 << 16, device=dev).sum()
                g.replay()
                torch.cuda.synchronize()
                for k in ("status", "iters", "obj", "x", "y"):
                    assert torch.equal(out[k].view(torch.int32) if out[k].dtype == torch.float64 else out[k],
                                       ref[k].view(torch.int32) if ref[k].dtype == torch.float64 else ref[k]), \
                        (tag, rep, k)
                del noise
            del g
        finally:
            s.close()
        o = _oracle(A, b, sense, C)
        K = C.shape[0]
        st_ = ref["status"][:K].cpu().numpy()
        assert np.array_equal(st_, o["status"]), tag
        ok = o["status"] == oracle.OPTIMAL
        obj = ref["obj"][:K].cpu().numpy()
        assert (np.abs(obj[ok] - o["obj"][ok]) <= REL * np.maximum(1.0, np.abs(o["obj"][ok]))).all(), tag
