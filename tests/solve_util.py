"""Helpers shared by the GPU tests: run the HIP solver and the oracle on the
same generated batch and compare."""
from __future__ import annotations

import numpy as np

import lpgen
import oracle

REL = 1e-9  # objective relative-error bar


def gpu_solve(hb: lpgen.Batch, uniform: bool | None = None, **solver_kw) -> dict:
    import torch

    import paper_1609_08114_amd as blp
    s = blp.Solver(**solver_kw)
    try:
        db = blp.DeviceBatch.from_host(hb, uniform=uniform)
        out = s.solve(db)
        torch.cuda.synchronize()
        res = {k: v.cpu().numpy() for k, v in out.items()}
        res["bins"] = blp.blp_last_bins(s.h)
    finally:
        s.close()
    K = hb.count
    res["status"] = res["status"][:K]
    res["iters"] = res["iters"][:K]
    res["obj"] = res["obj"][:K]
    return res


def oracle_solve(hb: lpgen.Batch, **kw) -> dict:
    return oracle.solve_batch(hb, **kw)


def compare(hb: lpgen.Batch, g: dict, o: dict, strict: bool = True, tag: str = "") -> None:
    """Status exact; objective within 1e-9 relative.  With `strict`, also the
    iteration counts, and objective / x / y bit-for-bit (the GPU takes the
    oracle's pivot path)."""
    st_g, st_o = g["status"], o["status"]
    bad = np.nonzero(st_g != st_o)[0]
    assert bad.size == 0, f"{tag}: status differs at LPs {bad[:10]}: gpu {st_g[bad[:10]]} oracle {st_o[bad[:10]]}"
    ok = st_o == oracle.OPTIMAL
    og, oo = g["obj"][ok], o["obj"][ok]
    rel = np.abs(og - oo) / np.maximum(1.0, np.abs(oo))
    assert (rel <= REL).all(), f"{tag}: obj relerr {rel.max():.3e} at LP {np.nonzero(ok)[0][rel.argmax()]}"
    inf = np.isin(st_o, (oracle.INFEASIBLE, oracle.UNBOUNDED))
    assert np.array_equal(g["obj"][inf], o["obj"][inf]), tag
    if strict:
        it = np.nonzero(g["iters"] != o["iters"])[0]
        assert it.size == 0, f"{tag}: iteration counts differ at {it[:10]}: {g['iters'][it[:10]]} vs {o['iters'][it[:10]]}"
        fin = np.isfinite(o["obj"])
        assert np.array_equal(g["obj"][fin].view(np.int64), o["obj"][fin].view(np.int64)), f"{tag}: obj bits"
        nx = hb.c.shape[0]
        ny = hb.b.shape[0]
        xg, xo = g["x"][:nx], o["x"][:nx]
        yg, yo = g["y"][:ny], o["y"][:ny]
        assert np.array_equal(np.nan_to_num(xg, nan=7.0), np.nan_to_num(xo, nan=7.0)), f"{tag}: x bits"
        assert np.array_equal(np.nan_to_num(yg, nan=7.0), np.nan_to_num(yo, nan=7.0)), f"{tag}: y bits"


def crafted_batch(lps: list) -> lpgen.Batch:
    """Pack a list of dicts {A, b, c, sense} / {c, l, u} into a Batch."""
    K = len(lps)
    m = np.array([0 if "l" in d else np.asarray(d["A"]).shape[0] for d in lps], np.int32)
    n = np.array([len(d["c"]) for d in lps], np.int32)
    kind = np.array([1 if "l" in d else 0 for d in lps], np.int32)
    a_off, row_off, col_off = lpgen.offsets(m, n)
    A = np.zeros(int((m.astype(np.int64) * n).sum()))
    b = np.zeros(int(m.sum()))
    sense = np.zeros(int(m.sum()), np.int8)
    c = np.zeros(int(n.sum()))
    l = np.zeros(int(n.sum()))
    u = np.zeros(int(n.sum()))
    for k, d in enumerate(lps):
        co, nn = int(col_off[k]), int(n[k])
        c[co:co + nn] = d["c"]
        if kind[k] == 1:
            l[co:co + nn] = d["l"]
            u[co:co + nn] = d["u"]
        else:
            mm, ao, ro = int(m[k]), int(a_off[k]), int(row_off[k])
            A[ao:ao + mm * nn] = np.asarray(d["A"], float).ravel()
            b[ro:ro + mm] = d["b"]
            sense[ro:ro + mm] = d.get("sense", np.zeros(mm, np.int8))
    return lpgen.Batch(m, n, kind, a_off, row_off, col_off, A, b, sense, c, l, u,
                       np.arange(K, dtype=np.int64), np.where(kind == 1, 3, 1).astype(np.int32))


def scattered_batch(seed: int = 17) -> lpgen.Batch:
    """The mixed batch of the oracle's batch-driver pin: simplex and hyperbox
    LPs with every outcome, stored in a permuted order at gapped offsets
    (NaN in the gaps)."""
    import pins
    _, arrs, _ = pins._scattered_batch(seed)
    K, m, n, kind, a_off, row_off, col_off, A, b, sense, c, l, u = arrs
    return lpgen.Batch(m, n, kind, a_off, row_off, col_off, A, b, sense, c, l, u,
                       np.arange(K, dtype=np.int64), np.where(kind == 1, 3, 1).astype(np.int32))


def compare_scattered(hb: lpgen.Batch, g: dict, o: dict, tag: str = "") -> None:
    """compare() for batches with gapped offsets: x and y only at the LPs'
    own ranges (the gaps of the output buffers belong to nobody)."""
    K = hb.count
    xw = np.zeros(hb.c.shape[0], bool)
    yw = np.zeros(max(1, hb.b.shape[0]), bool)
    for k in range(K):
        xw[hb.col_off[k]:hb.col_off[k] + hb.n[k]] = True
        yw[hb.row_off[k]:hb.row_off[k] + hb.m[k]] = True
    gg = dict(g)
    oo = dict(o)
    def fit(a, size):  # outputs may end at the last LP's range, before the inputs' padding
        a = np.asarray(a)[:size]
        return np.concatenate([a, np.zeros(size - a.size, a.dtype)]) if a.size < size else a
    for d in (gg, oo):
        d["x"] = np.where(xw, fit(d["x"], xw.size), 0.0)
        d["y"] = np.where(yw, fit(d["y"], yw.size), 0.0)
    compare(hb, gg, oo, strict=True, tag=tag)
