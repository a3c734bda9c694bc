"""Parity at the workloads' full sizes, in the persistent launch that bench.py
times, on outputs the oracle recomputes one LP at a time (a seeded random
sample), and at the largest LP shapes the library accepts (closed forms)."""
import numpy as np
import pytest

import lpgen
import oracle
from solve_util import compare, crafted_batch, gpu_solve

pytestmark = pytest.mark.gpu


def _check_sample(cfg, K, part=None, S=400, seed=0):
    print(f"[fullsize] cfg {cfg} {part or ''} K={K}: generating", flush=True)
    hb = lpgen.config(cfg, range(K), part=part) if part else lpgen.config(cfg, range(K))
    print(f"[fullsize] cfg {cfg} {part or ''} K={K}: solving", flush=True)
    g = gpu_solve(hb)
    print(f"[fullsize] cfg {cfg} {part or ''}: oracle on {min(S, K)} sampled LPs", flush=True)
    rng = np.random.default_rng(seed)
    idx = np.sort(rng.choice(K, size=min(S, K), replace=False))
    sub = lpgen.config(cfg, idx, part=part) if part else lpgen.config(cfg, idx)
    o = oracle.solve_batch(sub)
    # the sampled LPs' rows of the full solve, repacked like the sample
    gs = {"status": g["status"][idx], "iters": g["iters"][idx], "obj": g["obj"][idx]}
    xs, ys = [], []
    for k in idx:
        co, n = int(hb.col_off[k]), int(hb.n[k])
        ro, m = int(hb.row_off[k]), int(hb.m[k])
        xs.append(g["x"][co:co + n])
        ys.append(g["y"][ro:ro + m])
    gs["x"] = np.concatenate(xs)
    gs["y"] = np.concatenate(ys) if ys else np.zeros(0)
    compare(sub, gs, o, strict=True, tag=f"cfg{cfg}{part or ''}-full")
    del hb
    return g


def test_workload2_full_batch():
    # the bench workload: 50,000 LPs, m = n = 100, one persistent launch
    g = _check_sample(2, 50_000, S=2000, seed=2)
    assert (g["status"] == 0).all()


def test_workload3_full_batch():
    # 10,000 type-2 LPs, m = n = 200 (streaming kernel), ~2,000 pivots each
    _check_sample(3, 10_000, S=24, seed=3)


def test_workload4_full_batch():
    # the uneven batch at its stated size: 200,000 LPs with m, n ~ U{5..300}
    # (40% type 1, 40% type 2, 20% hyperbox) in one persistent solve (every
    # size class: register tiles, streaming kernel, hyperbox); 2,000 seeded
    # random LPs recomputed by the oracle, strict
    g = _check_sample(4, 200_000, S=2000, seed=4)
    assert (g["status"] == 0).all()
    bins = g["bins"]
    assert bins.sum() == 200_000 and bins[-1] > 30_000 and bins[-2] > 0


def test_workload5_simplex_full():
    # 20,000 type-1 LPs with m = n ~ U{20..150} (several register variants)
    g = _check_sample(5, 20_000, part="simplex", S=2000, seed=5)
    assert (g["status"] == 0).all()


def test_workload5_hyperbox_full():
    for part in ("box5", "box28"):
        hb = lpgen.config(5, None, part=part)
        print(f"[fullsize] cfg 5 {part} K={hb.count}", flush=True)
        g = gpu_solve(hb)
        o = oracle.solve_batch(hb)
        assert np.array_equal(g["status"], o["status"])
        assert np.array_equal(g["obj"].view(np.int64), o["obj"].view(np.int64))
        assert np.array_equal(g["x"][:hb.c.size].view(np.int64), o["x"].view(np.int64))


def test_largest_shapes_closed_forms():
    # m = 2046 rows, one column: opt = c * min_i b_i / a_i; one row,
    # n = 4094 columns: opt = b * max_j c_j / a_j (both exact in FP64 here:
    # the divisions are the only roundings on either side)
    rng = np.random.default_rng(1)
    m = 2046
    a = rng.integers(1, 50, size=(m, 1)).astype(float)
    b = rng.integers(1, 1000, size=m).astype(float)
    n = 4094
    a2 = rng.integers(1, 50, size=(1, n)).astype(float)
    c2 = rng.integers(1, 1000, size=n).astype(float)
    hb = crafted_batch([dict(A=a, b=b, c=[3.0]), dict(A=a2, b=[7.0], c=c2)])
    g = gpu_solve(hb)
    o = oracle.solve_batch(hb)
    compare(hb, g, o, strict=True, tag="largest")
    assert g["status"][0] == 0 and g["status"][1] == 0
    assert g["obj"][0] == pytest.approx(3.0 * (b / a[:, 0]).min(), rel=1e-15)
    assert g["obj"][1] == pytest.approx(7.0 * (c2 / a2[0]).max(), rel=1e-15)
    # one row too many is refused before any launch
    import paper_1609_08114_amd as blp
    big = crafted_batch([dict(A=np.ones((2047, 1)), b=np.ones(2047), c=[1.0])])
    with pytest.raises(blp.BlpError) as ei:
        gpu_solve(big)
    assert ei.value.code == blp.BLP_ERR_TOO_LARGE
