"""The allocation-free entry point (blp_solve_batch_static) against
blp_solve_batch, through the C ABI: two calls in a row on one handle, the
second with a smaller batch, each bit-identical to the allocating entry point
on the same inputs; and a batch whose metadata exceeds the static scratch is
refused before any launch."""
from __future__ import annotations

import ctypes

import numpy as np
import pytest

import lpgen

pytestmark = pytest.mark.gpu


def _outputs(torch, db):
    K = db.count
    tot_m = int(db.m[0]) * K if db.uniform else int((db.row_off + db.m).max(initial=0))
    tot_n = int(db.n[0]) * K if db.uniform else int((db.col_off + db.n).max(initial=0))
    dev = torch.device("cuda")
    # filled with a marker so that anything the solve does not write shows up
    return {"status": torch.full((max(K, 1),), -7, dtype=torch.int32, device=dev),
            "iters": torch.full((max(K, 1),), -7, dtype=torch.int32, device=dev),
            "obj": torch.full((max(K, 1),), 7.5, dtype=torch.float64, device=dev),
            "x": torch.full((max(tot_n, 1),), 7.5, dtype=torch.float64, device=dev),
            "y": torch.full((max(tot_m, 1),), 7.5, dtype=torch.float64, device=dev)}


def _c_out(blp, o):
    return blp.blp_outputs(*[ctypes.c_void_p(o[k].data_ptr()) for k in ("status", "iters", "obj", "x", "y")])


def _same(a: dict, b: dict, K: int, tag: str) -> None:
    for key in ("status", "iters", "obj", "x", "y"):
        x, y = a[key].cpu().numpy(), b[key].cpu().numpy()
        if key in ("status", "iters", "obj"):
            x, y = x[:K], y[:K]
        assert np.array_equal(x.view(np.int64) if x.dtype == np.float64 else x,
                              y.view(np.int64) if y.dtype == np.float64 else y), f"{tag}: {key} differs"


def _run_pair(blp, torch, h, hb, tag):
    db = blp.DeviceBatch.from_host(hb)
    st = torch.cuda.current_stream().cuda_stream
    ref = _outputs(torch, db)
    b1 = db.c_struct()
    blp.blp_solve_batch(h, b1, _c_out(blp, ref), st)
    got = _outputs(torch, db)
    b2 = db.c_struct()
    blp.blp_solve_batch_static(h, b2, _c_out(blp, got), st)
    torch.cuda.synchronize()
    _same(ref, got, db.count, tag)
    return got


def test_static_entry_point_matches_solve_batch():
    import torch

    import paper_1609_08114_amd as blp
    assert blp.blp_static_scratch_bytes() == 64 << 20
    s = blp.Solver()
    try:
        # mixed sizes and kinds: lane, register, column-split, block and
        # streaming kernels and the hyperbox kernel, non-uniform metadata
        big = lpgen.config(4, range(240))
        small = lpgen.config(4, range(40, 100))
        _run_pair(blp, torch, s.h, big, "mixed 240")
        _run_pair(blp, torch, s.h, small, "mixed 60 after 240")
        # a uniform batch (no per-LP metadata), then a smaller one
        _run_pair(blp, torch, s.h, lpgen.config(2, range(600)), "uniform 100x100 x600")
        _run_pair(blp, torch, s.h, lpgen.config(1, range(50)), "uniform 5x5 x50")
    finally:
        s.close()


def test_static_entry_point_refuses_oversized_batch():
    import torch

    import paper_1609_08114_amd as blp
    s = blp.Solver()
    try:
        # 1.5M non-uniform 1 x 1 LPs: 48 bytes of metadata and work lists
        # each (72 MB) exceed the 64 MiB scratch; refused before any launch
        K = 1_500_000
        m = np.ones(K, np.int32)
        n = np.ones(K, np.int32)
        kind = np.zeros(K, np.int32)
        dev = torch.device("cuda")
        A = torch.ones(K, dtype=torch.float64, device=dev)
        b = torch.ones(K, dtype=torch.float64, device=dev)
        sense = torch.zeros(K, dtype=torch.int8, device=dev)
        c = torch.ones(K, dtype=torch.float64, device=dev)
        out = {"status": torch.empty(K, dtype=torch.int32, device=dev),
               "iters": torch.empty(K, dtype=torch.int32, device=dev),
               "obj": torch.empty(K, dtype=torch.float64, device=dev),
               "x": torch.empty(K, dtype=torch.float64, device=dev),
               "y": torch.empty(K, dtype=torch.float64, device=dev)}
        keep = [m, n, kind]
        P = lambda a: a.ctypes.data_as(ctypes.c_void_p)
        T = lambda t: ctypes.c_void_p(t.data_ptr())
        batch = blp.blp_batch(K, 0, 0, P(m), P(n), P(kind), None, None, None, T(A), T(b), T(sense), T(c), None,
                              None)
        with pytest.raises(blp.BlpError) as ei:
            blp.blp_solve_batch_static(s.h, batch, _c_out(blp, out), torch.cuda.current_stream().cuda_stream)
        assert ei.value.code == 5, ei.value
        del keep
        # the handle still works afterwards, on a batch that fits
        _run_pair(blp, torch, s.h, lpgen.config(1, range(10)), "after refusal")
    finally:
        s.close()
