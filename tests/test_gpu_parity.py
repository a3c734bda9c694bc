"""GPU parity: the HIP solver (through the C ABI) against the CPU oracle."""
import numpy as np
import pytest

import lpgen
import oracle
import pins
from solve_util import compare, crafted_batch, gpu_solve, oracle_solve

pytestmark = pytest.mark.gpu


def _both(hb, strict=True, tag="", okw=None, **kw):
    print(f"[parity] {tag}: K={hb.count}", flush=True)
    g = gpu_solve(hb, **kw)
    o = oracle_solve(hb, **(okw or {}))
    compare(hb, g, o, strict=strict, tag=tag)
    return g, o


def test_config1_all():
    # 1,000 type-1 LPs, m = n = 5 (the one-LP-per-launch workload)
    g, o = _both(lpgen.config(1), tag="cfg1")
    assert (o["status"] == 0).all()


def test_config2_sample():
    g, o = _both(lpgen.config(2, range(0, 300)), tag="cfg2")
    assert (o["status"] == 0).all()


def test_config3_sample():
    _both(lpgen.config(3, range(0, 12)), tag="cfg3")


def test_config4_sample():
    g, o = _both(lpgen.config(4, range(0, 160)), tag="cfg4")
    bins = g["bins"]
    assert bins.sum() == 160 and bins[-1] > 0 and bins[-2] > 0  # hyperbox and streaming both used


def test_config5_parts():
    _both(lpgen.config(5, range(0, 60), part="simplex"), tag="cfg5-simplex")
    _both(lpgen.config(5, range(0, 20000), part="box5"), tag="cfg5-box5")
    _both(lpgen.config(5, range(0, 5000), part="box28"), tag="cfg5-box28")


def test_small_random_families():
    """Integer and continuous tiny LPs with every outcome (optimal,
    infeasible, unbounded), mixed row senses and negative right-hand sides."""
    rng = np.random.default_rng(7)
    lps = []
    for _ in range(400):
        m = int(rng.integers(1, 6))
        n = int(rng.integers(1, 4))
        lps.append(dict(A=rng.integers(-3, 7, size=(m, n)).astype(float), b=rng.integers(-4, 11, size=m).astype(float),
                        c=rng.integers(-2, 6, size=n).astype(float), sense=rng.integers(0, 2, size=m).astype(np.int8)))
    for _ in range(200):
        m = int(rng.integers(1, 30))
        n = int(rng.integers(1, 30))
        A = rng.uniform(-2, 10, size=(m, n))
        x0 = rng.uniform(0.5, 2.0, size=n)
        sense = rng.integers(0, 2, size=m).astype(np.int8)
        ax = A @ x0
        b = np.where(sense == 0, ax + rng.uniform(0.5, 3, m), ax - rng.uniform(0.5, 3, m))
        lps.append(dict(A=A, b=b, c=rng.uniform(-1, 5, size=n), sense=sense))
    hb = crafted_batch(lps)
    g, o = _both(hb, tag="small-families")
    assert set(np.unique(o["status"])) >= {0, 1, 2}


def test_crafted_statuses():
    A, b, c = pins.klee_minty(7)
    beale = dict(A=[[0.25, -8.0, -1.0, 9.0], [0.5, -12.0, -0.5, 3.0], [0.0, 0.0, 1.0, 0.0]], b=[0, 0, 1],
                 c=[0.75, -20.0, 0.5, -6.0])
    lps = [
        dict(A=[[1, 1], [1, 1]], b=[1, 2], c=[1, 1], sense=[0, 1]),          # infeasible
        dict(A=[[1, 1]], b=[-1], c=[1, 1]),                                  # infeasible, negative rhs
        dict(A=[[1, -1]], b=[1], c=[1, 0]),                                  # unbounded
        dict(A=[[1, 1]], b=[2], c=[1, 0], sense=[1]),                        # unbounded after phase 1
        dict(A=[[1, 2], [3, 1]], b=[4, 5], c=[-1, -2]),                      # optimal at the origin
        dict(A=[[1, np.nan]], b=[1], c=[1, 1]),                              # non-finite data
        dict(A=[[1, 1]], b=[np.inf], c=[1, 1]),
        dict(A=[[1, 1], [1, 1], [1, 1]], b=[2, 2, 2], c=[1, 2], sense=[1, 1, 0]),  # duplicated rows
        dict(A=[[1.0, -1.0], [-1.0, 1.0], [1.0, 1.0]], b=[0, 0, 4], c=[1, 1]),    # degenerate
        beale,                                                               # cycles without anti-cycling
        dict(A=A, b=b, c=c),                                                 # Klee-Minty, 2^7 - 1 pivots
        dict(c=[0.0, -1.0, 2.0], l=[-1.0, -2.0, -3.0], u=[4.0, 5.0, 6.0]),   # hyperbox, tie at c = 0
        dict(c=[1.0, 1.0], l=[0.0, 2.0], u=[1.0, 1.0]),                      # empty box
        dict(c=[1.0, np.nan], l=[0.0, 0.0], u=[1.0, 1.0]),
    ]
    hb = crafted_batch(lps)
    g, o = _both(hb, tag="crafted")
    want = [1, 1, 2, 2, 0, 4, 4, 0, 0, 0, 0, 0, 1, 4]
    assert list(g["status"]) == want
    assert g["iters"][10] == 2 ** 7 - 1 and g["obj"][10] == 100.0 ** 6
    assert g["obj"][9] == o["obj"][9] and abs(g["obj"][9] - 1.25) < 1e-12


def test_iteration_limit():
    A, b, c = pins.klee_minty(6)
    hb = crafted_batch([dict(A=A, b=b, c=c)] * 3)
    g = gpu_solve(hb, max_iter=5)
    o = oracle_solve(hb, max_iter=5)
    compare(hb, g, o, tag="iter-limit")
    assert (g["status"] == oracle.ITER_LIMIT).all() and (g["iters"] == 5).all()


@pytest.mark.parametrize("mode", [1, 2])
def test_modes_identical(mode):
    hb = lpgen.config(4, range(1000, 1060))
    a = gpu_solve(hb)
    b = gpu_solve(hb, mode=mode)
    for k in ("status", "iters"):
        assert np.array_equal(a[k], b[k])
    for k in ("obj", "x", "y"):
        assert np.array_equal(a[k].view(np.int64), b[k].view(np.int64)), k


def test_every_kernel_variant_identical():
    """Forcing each register-tile variant (LPs that do not fit go to the
    streaming kernel) and forcing the streaming kernel gives the same bits."""
    import paper_1609_08114_amd as blp
    hb = lpgen.config(4, range(2000, 2080))
    ref = gpu_solve(hb, variant=-2)
    o = oracle_solve(hb)
    compare(hb, ref, o, tag="streaming-only")
    for v in range(len(blp.variants())):
        g = gpu_solve(hb, variant=v)
        for k in ("status", "iters"):
            assert np.array_equal(ref[k], g[k]), (v, k)
        for k in ("obj", "x", "y"):
            assert np.array_equal(ref[k].view(np.int64), g[k].view(np.int64)), (v, k)


def _crafted_lps():
    A, b, c = pins.klee_minty(7)
    beale = dict(A=[[0.25, -8.0, -1.0, 9.0], [0.5, -12.0, -0.5, 3.0], [0.0, 0.0, 1.0, 0.0]], b=[0, 0, 1],
                 c=[0.75, -20.0, 0.5, -6.0])
    lps = [
        dict(A=[[1, 1], [1, 1]], b=[1, 2], c=[1, 1], sense=[0, 1]),
        dict(A=[[1, 1]], b=[-1], c=[1, 1]),
        dict(A=[[1, -1]], b=[1], c=[1, 0]),
        dict(A=[[1, 1]], b=[2], c=[1, 0], sense=[1]),
        dict(A=[[1, 2], [3, 1]], b=[4, 5], c=[-1, -2]),
        dict(A=[[1, 1], [1, 1], [1, 1]], b=[2, 2, 2], c=[1, 2], sense=[1, 1, 0]),
        dict(A=[[1, 1, 0], [1, 1, 0], [0, 1, 1], [0, 1, 1]], b=[3, 3, 2, 2], c=[1, 2, 1], sense=[1, 1, 1, 0]),
        dict(A=[[1.0, -1.0], [-1.0, 1.0], [1.0, 1.0]], b=[0, 0, 4], c=[1, 1]),
        beale,
        dict(A=A, b=b, c=c),
    ]
    rng = np.random.default_rng(11)
    for _ in range(300):
        m = int(rng.integers(1, 7))
        n = int(rng.integers(1, 5))
        lps.append(dict(A=rng.integers(-3, 7, size=(m, n)).astype(float), b=rng.integers(-4, 11, size=m).astype(float),
                        c=rng.integers(-2, 6, size=n).astype(float), sense=rng.integers(0, 2, size=m).astype(np.int8)))
    # redundant equality-like pairs: a >= row and a <= row with the same data
    for _ in range(60):
        m = int(rng.integers(2, 6))
        n = int(rng.integers(2, 5))
        A = rng.integers(1, 5, size=(m, n)).astype(float)
        b = rng.integers(2, 9, size=m).astype(float)
        A = np.vstack([A, A[:1]])
        b = np.concatenate([b, b[:1]])
        sense = np.zeros(m + 1, np.int8)
        sense[0] = 1
        lps.append(dict(A=A, b=b, c=rng.integers(-1, 5, size=n).astype(float), sense=sense))
    return lps


def test_every_variant_on_crafted_and_degenerate():
    """Each register-tile variant, forced, on the crafted statuses, repeated
    rows with mixed senses (phase-1 drive-out), degenerate and cycling LPs:
    identical bits to the oracle's strict comparison."""
    import paper_1609_08114_amd as blp
    hb = crafted_batch(_crafted_lps())
    o = oracle_solve(hb)
    assert set(np.unique(o["status"])) >= {0, 1, 2}
    for v in range(len(blp.variants())):
        print(f"[parity] crafted variant {v}", flush=True)
        g = gpu_solve(hb, variant=v)
        compare(hb, g, o, strict=True, tag=f"crafted-v{v}")


def test_ragged_and_empty():
    # LPs of every size class in one batch, not in order, plus zero-size batch
    rng = np.random.default_rng(3)
    ids = rng.permutation(np.arange(3000, 3400))[:90]
    hb = lpgen.config(4, ids)
    _both(hb, tag="ragged")
    empty = crafted_batch([])
    g = gpu_solve(empty)
    assert g["status"].size == 0


def test_determinism():
    hb = lpgen.config(2, range(300, 400))
    a = gpu_solve(hb)
    b = gpu_solve(hb)
    for k in ("obj", "x", "y"):
        assert np.array_equal(a[k].view(np.int64), b[k].view(np.int64))


def test_lane_kernel_tiny_lps():
    """The smallest size class runs one LP per lane (64 per wave): a few
    thousand tiny LPs of every outcome, strict against the oracle, spread
    over both lane variants and several waves with a partial last wave; the
    grid and one-LP-per-launch modes and the random entering rule give the
    same bits as the other register kernels."""
    import paper_1609_08114_amd as blp
    rng = np.random.default_rng(23)
    lps = []
    for t in range(3001):
        m = int(rng.integers(1, 6))
        n = int(rng.integers(1, 6))
        if t % 3 == 0:  # continuous, through an interior point, mixed senses
            A = rng.uniform(-2, 10, size=(m, n))
            x0 = rng.uniform(0.5, 2.0, size=n)
            sense = rng.integers(0, 2, size=m).astype(np.int8)
            ax = A @ x0
            b = np.where(sense == 0, ax + rng.uniform(0.5, 3, m), ax - rng.uniform(0.5, 3, m))
            c = rng.uniform(-1, 5, size=n)
        else:
            A = rng.integers(-3, 7, size=(m, n)).astype(float)
            b = rng.integers(-4, 11, size=m).astype(float)
            c = rng.integers(-2, 6, size=n).astype(float)
            sense = rng.integers(0, 2, size=m).astype(np.int8)
        lps.append(dict(A=A, b=b, c=c, sense=sense))
    # six copies: the automatic choice takes the lane kernel only for
    # batches that give it a quarter of a workgroup per CU (16,384 LPs)
    hb = crafted_batch(lps * 6)
    g, o = _both(hb, tag="lane-tiny")
    names = [v[0] for v in blp.variants()]
    lane = [i for i, nm in enumerate(names) if nm.startswith("l64_")]
    assert len(lane) == 2 and all(g["bins"][i] > 64 for i in lane), g["bins"]
    assert set(np.unique(o["status"])) >= {0, 1, 2}
    # a small batch leaves it to one LP per wave, with the same bits
    small = crafted_batch(lps)
    gs = gpu_solve(small)
    assert all(gs["bins"][i] == 0 for i in lane), gs["bins"]
    K = len(lps)
    for k in ("status", "iters"):
        assert np.array_equal(gs[k], g[k][:K]), k
    assert np.array_equal(gs["obj"].view(np.int64), g["obj"][:K].view(np.int64))
    sub = crafted_batch(lps[:700])
    a = gpu_solve(sub, variant=lane[0])
    for mode in (1, 2):
        b = gpu_solve(sub, mode=mode, variant=lane[0])
        for k in ("status", "iters"):
            assert np.array_equal(a[k], b[k]), (mode, k)
        for k in ("obj", "x", "y"):
            assert np.array_equal(a[k].view(np.int64), b[k].view(np.int64)), (mode, k)
    # random entering rule: the lane kernel and the row-tile kernel draw the
    # same pivots
    w1 = names.index("w1_r8_c8")
    cfg1 = lpgen.config(1, range(1000))
    r_lane = gpu_solve(cfg1, variant=lane[0], pivot_rule=blp.BLP_RULE_RPC, seed=3)
    r_row = gpu_solve(cfg1, variant=w1, pivot_rule=blp.BLP_RULE_RPC, seed=3)
    assert r_lane["bins"][lane[0]] == 1000
    for k in ("status", "iters"):
        assert np.array_equal(r_lane[k], r_row[k]), k
    for k in ("obj", "x", "y"):
        assert np.array_equal(r_lane[k].view(np.int64), r_row[k].view(np.int64)), k
