"""Pivot trace of the 100 x 100 class's kernel (blp_pivot_trace): the pivots
it records are the oracle's, mapped to slots of the condensed tableau, and
replaying them (Steps 1 and 2 replaced by the record) reproduces the solve
bit for bit; invalid records and too small strides are reported per LP."""
import numpy as np
import pytest

import lpgen
import oracle
from solve_util import gpu_solve

pytestmark = pytest.mark.gpu


def _bits(a):
    return np.asarray(a).view(np.int64)


def _slots(m: int, n: int, pivots) -> list:
    """The oracle's pivots (row, full-tableau column) as (row, condensed slot):
    slot j < n starts with structural variable j, the slack of row i starts
    basic in row i, and a pivot's slot takes the leaving variable."""
    slot_of = {j: j for j in range(n)}
    basis = [n + i for i in range(m)]
    out = []
    for l, v in pivots:
        s = slot_of.pop(int(v))
        out.append((int(l), s))
        slot_of[basis[int(l)]] = s
        basis[int(l)] = int(v)
    return out


def test_pivot_trace_record_and_replay():
    import torch

    import paper_1609_08114_amd as blp
    K = 600
    hb = lpgen.config(2, range(5000, 5000 + K))
    db = blp.DeviceBatch.from_host(hb)
    ref = gpu_solve(hb)
    stride = 1 + 2 * 64
    tr = torch.full((K * stride,), -7, dtype=torch.int32, device="cuda")
    s = blp.Solver()
    try:
        rec = {k: v.cpu().numpy() for k, v in s.pivot_trace(db, tr, stride, replay=False).items()}
        torch.cuda.synchronize()
        # the recording run solves exactly like the normal path
        for k in ("status", "iters"):
            assert np.array_equal(rec[k][:K], ref[k]), k
        for k in ("obj", "x", "y"):
            assert np.array_equal(_bits(rec[k][:len(ref[k])]), _bits(ref[k])), k
        t = tr.cpu().numpy().reshape(K, stride)
        assert np.array_equal(t[:, 0], ref["iters"])
        # the recorded pivots are the oracle's
        m, n = int(hb.m[0]), int(hb.n[0])
        for k in range(0, K, 7):
            A = hb.A[k * m * n:(k + 1) * m * n].reshape(m, n)
            o = oracle.solve(A, hb.b[k * m:(k + 1) * m], hb.c[k * n:(k + 1) * n], hb.sense[k * m:(k + 1) * m],
                             trace=True)
            got = [(int(t[k, 1 + 2 * p]), int(t[k, 2 + 2 * p])) for p in range(int(t[k, 0]))]
            assert got == _slots(m, n, o["trace"]), k
        # replay: the same bits
        rp = {k: v.cpu().numpy() for k, v in s.pivot_trace(db, tr, stride, replay=True).items()}
        torch.cuda.synchronize()
        for k in ("status", "iters"):
            assert np.array_equal(rp[k][:K], ref[k]), k
        for k in ("obj", "x", "y"):
            assert np.array_equal(_bits(rp[k][:len(ref[k])]), _bits(ref[k])), k
        # an invalid record (a slot out of range) fails that LP only
        bad = tr.clone()
        bad[2] = n + 3
        rb = s.pivot_trace(db, bad, stride, replay=True)
        st = rb["status"][:K].cpu().numpy()
        assert st[0] == -1 and np.array_equal(st[1:], ref["status"][1:])
        assert np.array_equal(_bits(rb["obj"][1:K].cpu().numpy()), _bits(ref["obj"][1:]))
        # a stride too small for an LP's pivots records -1 for it
        small = 1 + 2 * 12
        tr2 = torch.zeros(K * small, dtype=torch.int32, device="cuda")
        s.pivot_trace(db, tr2, small, replay=False)
        cnt = tr2.cpu().numpy().reshape(K, small)[:, 0]
        assert np.array_equal(cnt, np.where(ref["iters"] <= 12, ref["iters"], -1))
        assert (cnt == -1).any() and (cnt >= 0).any()
        # and its replay fails exactly those LPs
        r3 = s.pivot_trace(db, tr2, small, replay=True)
        st3 = r3["status"][:K].cpu().numpy()
        assert np.array_equal(st3 == -1, cnt == -1)
        assert np.array_equal(_bits(r3["obj"][:K].cpu().numpy()[cnt >= 0]), _bits(ref["obj"][cnt >= 0]))
    finally:
        s.close()


def test_pivot_trace_argument_errors():
    import torch

    import paper_1609_08114_amd as blp
    tr = torch.zeros(100 * 129, dtype=torch.int32, device="cuda")
    ragged = lpgen.config(4, range(0, 20))
    big = lpgen.config(3, range(0, 4))
    ok = lpgen.config(2, range(0, 100))
    s = blp.Solver()
    r = blp.Solver(pivot_rule=blp.BLP_RULE_RPC)
    try:
        for solver, hb, stride in ((s, ragged, 129), (s, big, 129), (r, ok, 129), (s, ok, 0), (s, ok, 600)):
            with pytest.raises(blp.BlpError) as ei:
                solver.pivot_trace(blp.DeviceBatch.from_host(hb), tr, stride, replay=False)
            assert ei.value.code == 1
    finally:
        s.close()
        r.close()
