"""Runtime features on the GPU: hipGraph replay, autotuner, profiling hooks,
error paths that reach the device."""
import json

import numpy as np
import pytest

import lpgen
import oracle
from solve_util import compare, compare_scattered, crafted_batch, gpu_solve, scattered_batch

pytestmark = pytest.mark.gpu


def _bits(a):
    return np.asarray(a).view(np.int64)


def test_graph_replay_matches_eager():
    import torch

    import paper_1609_08114_amd as blp
    hb = lpgen.config(4, range(500, 620))
    ref = gpu_solve(hb)
    compare(hb, ref, oracle.solve_batch(hb), strict=True, tag="eager")
    db = blp.DeviceBatch.from_host(hb)
    s = blp.Solver(graph=True)
    outs = []
    for rep in range(4):
        out = s.solve(db)
        torch.cuda.synchronize()
        # eager work between replays
        junk = torch.randn(1000, device="cuda").sum().item()
        outs.append({k: v.cpu().numpy().copy() for k, v in out.items()})
    # a different batch forces a new capture, then the first one again
    hb2 = lpgen.config(1, range(100))
    out2 = s.solve(blp.DeviceBatch.from_host(hb2))
    torch.cuda.synchronize()
    ref2 = gpu_solve(hb2)
    assert np.array_equal(_bits(out2["obj"][:100].cpu().numpy()), _bits(ref2["obj"]))
    compare(hb2, ref2, oracle.solve_batch(hb2), strict=True, tag="cfg1")
    out3 = s.solve(db)
    torch.cuda.synchronize()
    outs.append({k: v.cpu().numpy().copy() for k, v in out3.items()})
    s.close()
    K = hb.count
    ora = oracle.solve_batch(hb)
    for rep, o in enumerate(outs):
        compare(hb, {k: (v[:K] if k in ("status", "iters", "obj") else v) for k, v in o.items()}, ora, strict=True,
                tag=f"replay {rep}")
        assert np.array_equal(o["status"][:K], ref["status"])
        assert np.array_equal(_bits(o["obj"][:K]), _bits(ref["obj"]))
        assert np.array_equal(_bits(o["x"][:hb.c.size]), _bits(ref["x"][:hb.c.size]))


def test_autotune_remap_and_cache(tmp_path):
    import torch

    import paper_1609_08114_amd as blp
    hb = lpgen.config(4, range(700, 900))
    db = blp.DeviceBatch.from_host(hb)
    ref = gpu_solve(hb)
    s = blp.Solver()
    path = str(tmp_path / "tune.json")
    s.autotune(db, sample=32, cache_path=path)
    remap = blp.blp_tuning(s.h)
    vs = blp.variants()
    for v, w in enumerate(remap):
        if w < len(vs):
            assert vs[w][1] >= vs[v][1] and vs[w][2] >= vs[v][2]
    tab = json.load(open(path))
    assert tab["cus"] > 0 and set(tab["remap"]) == {v[0] for v in vs}
    # this batch has LPs that only the streaming kernel holds: its depth is tuned
    assert tab["streaming_deep"] in (0, 1), tab
    out = s.solve(db)
    torch.cuda.synchronize()
    K = hb.count
    assert np.array_equal(out["status"][:K].cpu().numpy(), ref["status"])
    assert np.array_equal(_bits(out["obj"][:K].cpu().numpy()), _bits(ref["obj"]))
    tuned = {k: v.cpu().numpy() for k, v in out.items()}
    for k in ("status", "iters", "obj"):
        tuned[k] = tuned[k][:K]
    compare(hb, tuned, oracle.solve_batch(hb), strict=True, tag="autotuned")
    s.close()
    s2 = blp.Solver()
    blp.blp_load_tuning(s2.h, path)
    assert np.array_equal(blp.blp_tuning(s2.h), remap)
    s2.close()


@pytest.mark.parametrize("deep", [0, 1])
def test_streaming_kernel_every_size(tmp_path, deep):
    """Every LP through the streaming kernel (a tuning file that remaps each
    register variant to it), with shallow loads and HBM columns only (deep 0)
    or deep loads and on-chip columns (deep 1): LPs of 5..300 rows and
    columns, so that tableaux of every height class run, some wholly on chip
    and some split between LDS and HBM, plus the crafted statuses; strict
    against the oracle."""
    import torch

    import paper_1609_08114_amd as blp
    from test_gpu_parity import _crafted_lps
    w4 = lpgen.config(4, range(1200, 1280))
    lps = []
    for k in range(w4.count):
        m, n, co = int(w4.m[k]), int(w4.n[k]), int(w4.col_off[k])
        if w4.kind[k] == 1:
            lps.append(dict(c=w4.c[co:co + n], l=w4.l[co:co + n], u=w4.u[co:co + n]))
        else:
            ao, ro = int(w4.a_off[k]), int(w4.row_off[k])
            lps.append(dict(A=w4.A[ao:ao + m * n].reshape(m, n), b=w4.b[ro:ro + m], c=w4.c[co:co + n],
                            sense=w4.sense[ro:ro + m]))
    hb = crafted_batch(lps + _crafted_lps())
    props = torch.cuda.get_device_properties(0)
    names = [v[0] for v in blp.variants()]
    path = str(tmp_path / "all_streaming.json")
    with open(path, "w") as f:
        json.dump({"arch": props.gcnArchName, "cus": props.multi_processor_count,
                   "remap": {v: "streaming" for v in names}, "streaming_deep": deep}, f, indent=2)
    g = gpu_solve(hb, tune_cache=path)
    bins = g["bins"]
    assert bins[len(names)] == int((hb.kind == 0).sum()), bins
    compare(hb, g, oracle.solve_batch(hb), strict=True, tag=f"streaming-deep{deep}")


def test_small_uniform_batch_runs_as_one_launch():
    """A uniform batch whose LPs all get a workgroup at once runs as one
    launch (LP k in workgroup k) of a variant that holds its shape for any
    number of artificial rows, with no binning launches: strict against the
    oracle, and the same bits in graph mode; a uniform batch too large for
    that is still binned."""
    import torch

    import paper_1609_08114_amd as blp
    hb = lpgen.config(1, range(1000))
    db = blp.DeviceBatch.from_host(hb)
    s = blp.Solver(profile=True)
    out = s.solve(db)
    torch.cuda.synchronize()
    bins = blp.blp_last_bins(s.h)
    ms = blp.blp_last_kernel_ms(s.h)
    s.close()
    nz = np.nonzero(bins)[0]
    assert len(nz) == 1 and bins[nz[0]] == 1000, bins
    _, rows, cols = blp.variants()[nz[0]]
    assert rows >= 5 + 2 and cols >= 5 + 5 + 1
    assert ms[nz[0]] > 0 and ms[-1] == 0, ms  # no binning
    g = {k: v.cpu().numpy() for k, v in out.items()}
    for k in ("status", "iters", "obj"):
        g[k] = g[k][:1000]
    compare(hb, g, oracle.solve_batch(hb), strict=True, tag="one-launch")
    gg = gpu_solve(hb, graph=True)
    for k in ("obj", "x", "y"):
        assert np.array_equal(_bits(gg[k]), _bits(g[k])), k
    big = lpgen.config(1, range(200_000))
    gb = gpu_solve(big)
    assert gb["bins"].sum() == 200_000 and gb["bins"][nz[0]] < 200_000, gb["bins"]
    assert np.array_equal(_bits(gb["obj"][:1000]), _bits(g["obj"]))


def test_uniform_lane_batch_runs_as_one_launch():
    """A uniform batch of tiny LPs large enough for the lane kernel (one LP
    per lane) and small enough for all of them to be resident at once runs
    as one launch of the lane tile that holds the shape for any number of
    artificial rows (7 x 11 for 5 x 5 LPs), with no binning: strict against
    the oracle, and the same bits as the binned solve of a larger batch
    with the same leading LPs."""
    import torch

    import paper_1609_08114_amd as blp
    K = 20_000
    hb = lpgen.config(1, range(K))
    db = blp.DeviceBatch.from_host(hb)
    s = blp.Solver(profile=True)
    out = s.solve(db)
    torch.cuda.synchronize()
    bins = blp.blp_last_bins(s.h)
    ms = blp.blp_last_kernel_ms(s.h)
    s.close()
    nz = np.nonzero(bins)[0]
    assert len(nz) == 1 and bins[nz[0]] == K, bins
    name, rows, cols = blp.variants()[nz[0]]
    assert name.startswith("l64_") and rows >= 5 + 2 and cols >= 5 + 5 + 1, name
    assert ms[nz[0]] > 0 and ms[-1] == 0, ms  # no binning
    g = {k: v.cpu().numpy() for k, v in out.items()}
    for k in ("status", "iters", "obj"):
        g[k] = g[k][:K]
    compare(hb, g, oracle.solve_batch(hb), strict=True, tag="one-launch lane")
    gg = gpu_solve(hb, graph=True)
    for k in ("obj", "x", "y"):
        assert np.array_equal(_bits(gg[k]), _bits(g[k])), k
    big = lpgen.config(1, range(300_000))
    gb = gpu_solve(big)
    assert gb["bins"].sum() == 300_000 and gb["bins"][nz[0]] < 300_000, gb["bins"]
    assert np.array_equal(_bits(gb["obj"][:K]), _bits(g["obj"]))


def test_profile_and_bins():
    import torch

    import paper_1609_08114_amd as blp
    hb = lpgen.config(4, range(0, 300))
    db = blp.DeviceBatch.from_host(hb)
    s = blp.Solver(profile=True)
    s.solve(db)
    ms = blp.blp_last_kernel_ms(s.h)
    bins = blp.blp_last_bins(s.h)
    s.close()
    assert bins.sum() == 300
    assert (ms >= 0).all() and ms.sum() > 0
    assert len(ms) == len(bins) + 1


def test_errors_from_the_device_side():
    import torch

    import paper_1609_08114_amd as blp
    s = blp.Solver()
    hb = lpgen.config(1, range(4))
    db = blp.DeviceBatch.from_host(hb)
    bad = db.c_struct()
    bad.A = None
    with pytest.raises(blp.BlpError) as ei:
        blp.blp_solve_batch(s.h, bad)
    assert ei.value.code == blp.BLP_ERR_ARG
    # backward before any solve
    s2 = blp.Solver()
    g = torch.ones(4, dtype=torch.float64, device="cuda")
    with pytest.raises(blp.BlpError) as ei:
        blp.blp_backward(s2.h, blp._ptr(g))
    assert ei.value.code == blp.BLP_ERR_STATE
    # too large
    hb_big = lpgen.make_batch(1, [0], [1], [2047], [3])
    dbb = blp.DeviceBatch.from_host(hb_big)
    with pytest.raises(blp.BlpError) as ei:
        s.solve(dbb)
    assert ei.value.code == blp.BLP_ERR_TOO_LARGE
    # get_solution copies one LP to the host
    s.solve(db)
    st = np.zeros(1, np.int32)
    ob = np.zeros(1)
    x = np.zeros(5)
    blp.blp_get_solution(s.h, 2, st.ctypes.data_as(blp.ctypes.c_void_p), ob.ctypes.data_as(blp.ctypes.c_void_p),
                         x.ctypes.data_as(blp.ctypes.c_void_p), None, None)
    ref = gpu_solve(hb)
    assert st[0] == 0 and ob[0] == ref["obj"][2]
    s.close()
    s2.close()


def test_rpc_rule_reaches_the_same_optimum():
    """Sec. 4.2's random-positive-coefficient rule: same status and optimum as
    the oracle (which uses the largest-coefficient rule), more pivots on
    average, deterministic for a given seed.  The pivot path is not compared
    (parity unpinned for the path; only the optimum is unique)."""
    import paper_1609_08114_amd as blp
    from solve_util import compare, crafted_batch, oracle_solve
    for hb, tag in ((lpgen.config(1, range(1000)), "cfg1"), (lpgen.config(2, range(200)), "cfg2"),
                    (lpgen.config(4, range(60)), "cfg4")):
        o = oracle_solve(hb)
        r1 = gpu_solve(hb, pivot_rule=blp.BLP_RULE_RPC, seed=11)
        compare(hb, r1, o, strict=False, tag="rpc-" + tag)
        r2 = gpu_solve(hb, pivot_rule=blp.BLP_RULE_RPC, seed=11)
        assert np.array_equal(_bits(r1["obj"]), _bits(r2["obj"])) and np.array_equal(r1["iters"], r2["iters"])
        if tag == "cfg2":
            assert r1["iters"].mean() > o["iters"].mean()
            r3 = gpu_solve(hb, pivot_rule=blp.BLP_RULE_RPC, seed=12)
            assert not np.array_equal(r1["iters"], r3["iters"])
    rng = np.random.default_rng(17)
    lps = []
    for _ in range(300):
        m = int(rng.integers(1, 6))
        n = int(rng.integers(1, 4))
        lps.append(dict(A=rng.integers(-3, 7, size=(m, n)).astype(float), b=rng.integers(-4, 11, size=m).astype(float),
                        c=rng.integers(-2, 6, size=n).astype(float), sense=rng.integers(0, 2, size=m).astype(np.int8)))
    hb = crafted_batch(lps)
    compare(hb, gpu_solve(hb, pivot_rule=blp.BLP_RULE_RPC, seed=5), oracle_solve(hb), strict=False, tag="rpc-small")


def _host_solve(hb, chunks, fill=0.0):
    import ctypes

    import paper_1609_08114_amd as blp
    s = blp.Solver()
    K = hb.count
    st = np.zeros(K, np.int32)
    it = np.zeros(K, np.int32)
    ob = np.zeros(K)
    x = np.full(hb.c.size, fill)
    y = np.full(max(1, hb.b.size), fill)
    keep = [np.ascontiguousarray(a) for a in (hb.m, hb.n, hb.kind, hb.a_off, hb.row_off, hb.col_off)]
    P = lambda a: a.ctypes.data_as(ctypes.c_void_p)
    b = blp.blp_batch(K, 0, 0, *[P(a) for a in keep], P(hb.A), P(hb.b), P(hb.sense), P(hb.c), P(hb.l), P(hb.u))
    o = blp.blp_outputs(P(st), P(it), P(ob), P(x), P(y))
    try:
        blp.blp_solve_batch_host(s.h, b, o, chunks)
    finally:
        s.close()
    return {"status": st, "iters": it, "obj": ob, "x": x, "y": y}


@pytest.mark.parametrize("chunks", [1, 3, 7])
def test_host_resident_scattered_offsets(chunks):
    """Host-resident pieces with permuted, gapped offsets (pieces' ranges
    interleave): every LP's results at its own offsets, as the oracle solves
    them, and the gaps of the output arrays untouched."""
    hb = scattered_batch()
    SENT = 1234.5
    g = _host_solve(hb, chunks, fill=SENT)
    compare_scattered(hb, g, oracle.solve_batch(hb), tag=f"host-scattered-{chunks}")
    xw = np.zeros(hb.c.size, bool)
    yw = np.zeros(hb.b.size, bool)
    for k in range(hb.count):
        xw[hb.col_off[k]:hb.col_off[k] + hb.n[k]] = True
        yw[hb.row_off[k]:hb.row_off[k] + hb.m[k]] = True
    assert (g["x"][~xw] == SENT).all() and (g["y"][:hb.b.size][~yw] == SENT).all()


def test_device_scattered_offsets():
    hb = scattered_batch()
    compare_scattered(hb, gpu_solve(hb), oracle.solve_batch(hb), tag="device-scattered")


@pytest.mark.parametrize("chunks", [1, 3, 0])
def test_host_resident_pipeline(chunks):
    """Host arrays in, host results out, pieces on two streams: as the oracle
    solves the batch, and identical to the device-resident solve."""
    import ctypes

    import paper_1609_08114_amd as blp
    hb = lpgen.config(4, range(4000, 4150))
    ref = gpu_solve(hb)
    compare(hb, _host_solve(hb, chunks), oracle.solve_batch(hb), strict=True, tag=f"host-{chunks}")
    s = blp.Solver()
    K = hb.count
    st = np.zeros(K, np.int32)
    it = np.zeros(K, np.int32)
    ob = np.zeros(K)
    x = np.zeros(hb.c.size)
    y = np.zeros(max(1, hb.b.size))
    keep = [np.ascontiguousarray(a) for a in (hb.m, hb.n, hb.kind, hb.a_off, hb.row_off, hb.col_off)]
    P = lambda a: a.ctypes.data_as(ctypes.c_void_p)
    b = blp.blp_batch(K, 0, 0, *[P(a) for a in keep], P(hb.A), P(hb.b), P(hb.sense), P(hb.c), P(hb.l), P(hb.u))
    o = blp.blp_outputs(P(st), P(it), P(ob), P(x), P(y))
    blp.blp_solve_batch_host(s.h, b, o, chunks)
    s.close()
    assert np.array_equal(st, ref["status"]) and np.array_equal(it, ref["iters"])
    assert np.array_equal(_bits(ob), _bits(ref["obj"]))
    assert np.array_equal(_bits(x), _bits(ref["x"][:x.size]))
    assert np.array_equal(_bits(y[:hb.b.size]), _bits(ref["y"][:hb.b.size]))


def test_row_major_workspace_identical():
    """The streaming kernel on a row-major workspace (the non-coalesced
    layout of Sec. 4.3's comparison) gives the same bits as the column-major
    one."""
    import paper_1609_08114_amd as blp
    hb = lpgen.config(4, range(5000, 5060))
    a = gpu_solve(hb, variant=-2)
    b = gpu_solve(hb, variant=-2, layout=blp.BLP_LAYOUT_ROW)
    compare(hb, b, oracle.solve_batch(hb), strict=True, tag="row-major")
    for k in ("status", "iters"):
        assert np.array_equal(a[k], b[k])
    for k in ("obj", "x", "y"):
        assert np.array_equal(_bits(a[k]), _bits(b[k])), k


def test_mixed_batch_classes_run_concurrently():
    # A mixed batch of at least 2,048 LPs runs its kernel classes on forked
    # streams: every LP as the oracle solves it (all of them, m = n in
    # 20..150 over several register variants), and graph replays (the
    # captured sequence keeps the classes on one stream) identical to the
    # eager solve.
    import torch

    import oracle
    import paper_1609_08114_amd as blp
    from solve_util import compare
    hb = lpgen.config(5, range(2600), part="simplex")
    g = gpu_solve(hb)
    assert sum(1 for c in g["bins"][:-2] if c > 0) >= 3  # several classes at once
    compare(hb, g, oracle.solve_batch(hb), strict=True, tag="forked")
    db = blp.DeviceBatch.from_host(hb)
    s = blp.Solver(graph=True)
    try:
        for rep in range(3):
            out = s.solve(db)
            torch.cuda.synchronize()
            _ = torch.randn(1000, device="cuda").sum().item()  # eager work between replays
            assert np.array_equal(out["status"][:hb.count].cpu().numpy(), g["status"])
            assert np.array_equal(_bits(out["obj"][:hb.count].cpu().numpy()), _bits(g["obj"]))
            assert np.array_equal(_bits(out["x"][:hb.c.size].cpu().numpy()), _bits(g["x"][:hb.c.size]))
    finally:
        s.close()


def test_one_handle_on_two_streams():
    """A handle's calls reuse its buffers: a solve issued on a second stream
    right after one on a first stream waits for it, so both results are the
    oracle's."""
    import torch

    import paper_1609_08114_amd as blp
    h1 = lpgen.config(5, range(300), part="simplex")
    h2 = lpgen.config(4, range(300, 420))
    d1, d2 = blp.DeviceBatch.from_host(h1), blp.DeviceBatch.from_host(h2)
    s = blp.Solver()
    sa, sb = torch.cuda.Stream(), torch.cuda.Stream()
    try:
        o1 = s.solve(d1, stream=sa)
        o2 = s.solve(d2, stream=sb)  # own buffers of the handle reused at once
        g = torch.ones(h2.count, dtype=torch.float64, device="cuda")
        grads = s.backward(g, stream=sa, want=("dc",))
        torch.cuda.synchronize()
        r1 = {k: v.cpu().numpy() for k, v in o1.items()}
        r2 = {k: v.cpu().numpy() for k, v in o2.items()}
        dc = grads["dc"].cpu().numpy()
    finally:
        s.close()
    for hb, r, tag in ((h1, r1, "first"), (h2, r2, "second")):
        for k in ("status", "iters", "obj"):
            r[k] = r[k][:hb.count]
        compare(hb, r, oracle.solve_batch(hb), strict=True, tag=tag)
    ok = r2["status"] == 0
    for k in np.nonzero(ok)[0][:50]:
        co, n = h2.col_off[k], h2.n[k]
        assert np.array_equal(_bits(dc[co:co + n]), _bits(r2["x"][co:co + n])) or h2.kind[k] == 1
