"""Adjoint of the batched LP optimum (GPU): the backward kernel against the
oracle's primal/dual solution and against central finite differences
(h = 1e-6) at non-degenerate optima."""
import numpy as np
import pytest

import lpgen
import oracle

pytestmark = pytest.mark.gpu

H = 1e-6


def nondegenerate(lp, r, tol=1e-7):
    """Unique primal and dual optimum: exactly m strictly positive basic
    variables (structural or slack) and strictly negative reduced costs for
    every nonbasic variable."""
    A, b, c = lp["A"], lp["b"], lp["c"]
    m, n = A.shape
    x, y = r["x"], r["y"]
    slack = b - A @ x
    scale = max(1.0, float(np.abs(b).max()))
    basic_x = x > tol * scale
    basic_s = slack > tol * scale
    if basic_x.sum() + basic_s.sum() != m:
        return False
    d = c - A.T @ y
    if (np.abs(d[~basic_x]) <= tol).any():
        return False
    if (np.abs(y[~basic_s]) <= tol).any():
        return False
    return True


def _solve_obj(blp, torch, hb):
    db = blp.DeviceBatch.from_host(hb)
    s = blp.Solver()
    out = s.solve(db)
    torch.cuda.synchronize()
    o = out["obj"][:hb.count].cpu().numpy().copy()
    s.close()
    return o


def test_backward_matches_oracle_duals():
    import torch

    import paper_1609_08114_amd as blp
    from paper_1609_08114_amd.autograd import batched_lp
    hb = lpgen.config(5, range(40), part="simplex")
    ref = oracle.solve_batch(hb)
    db = blp.DeviceBatch.from_host(hb)
    A = db.A.clone().requires_grad_(True)
    b = db.b.clone().requires_grad_(True)
    c = db.c.clone().requires_grad_(True)
    w = torch.from_numpy(lpgen.weights(1005, range(40))).cuda()
    obj, st = batched_lp(db, A=A, b=b, c=c)
    (obj * w).sum().backward()
    torch.cuda.synchronize()
    wn = w.cpu().numpy()
    for k in range(hb.count):
        lp = hb.lp(k)
        co, ro, ao = int(hb.col_off[k]), int(hb.row_off[k]), int(hb.a_off[k])
        m, n = lp["m"], lp["n"]
        x = ref["x"][co:co + n]
        y = ref["y"][ro:ro + m]
        assert np.array_equal(c.grad[co:co + n].cpu().numpy(), wn[k] * x)
        assert np.array_equal(b.grad[ro:ro + m].cpu().numpy(), wn[k] * y)
        dA = A.grad[ao:ao + m * n].cpu().numpy().reshape(m, n)
        assert np.allclose(dA, -np.outer(wn[k] * y, x), rtol=1e-15, atol=0)


def test_backward_central_differences():
    import torch

    import paper_1609_08114_amd as blp
    from paper_1609_08114_amd.autograd import batched_lp
    rng = np.random.default_rng(5)
    base = lpgen.config(5, range(200), part="simplex")
    ref = oracle.solve_batch(base)
    picked = []
    for k in range(base.count):
        lp = base.lp(k)
        co, ro = int(base.col_off[k]), int(base.row_off[k])
        r = {"x": ref["x"][co:co + lp["n"]], "y": ref["y"][ro:ro + lp["m"]]}
        if ref["status"][k] == 0 and nondegenerate(lp, r):
            picked.append(k)
        if len(picked) == 6:
            break
    assert len(picked) >= 3, "no non-degenerate instances found"
    for k in picked:
        one = lpgen.config(5, [k], part="simplex")
        lp = one.lp(0)
        m, n = lp["m"], lp["n"]
        db = blp.DeviceBatch.from_host(one)
        A = db.A.clone().requires_grad_(True)
        b = db.b.clone().requires_grad_(True)
        c = db.c.clone().requires_grad_(True)
        obj, _ = batched_lp(db, A=A, b=b, c=c)
        obj.sum().backward()
        gA, gb, gc = (t.grad.cpu().numpy() for t in (A, b, c))
        scale = max(1.0, float(np.abs(np.concatenate([gA, gb, gc])).max()))
        checks = []
        # random directions over all of (A, b, c), plus sampled coordinates
        for _ in range(3):
            dA = rng.normal(size=m * n)
            dbv = rng.normal(size=m)
            dc = rng.normal(size=n)
            checks.append((dA, dbv, dc))
        for idx in rng.choice(m * n, 4, replace=False):
            e = np.zeros(m * n)
            e[idx] = 1.0
            checks.append((e, np.zeros(m), np.zeros(n)))
        for idx in rng.choice(m, 2, replace=False):
            e = np.zeros(m)
            e[idx] = 1.0
            checks.append((np.zeros(m * n), e, np.zeros(n)))
        for idx in rng.choice(n, 2, replace=False):
            e = np.zeros(n)
            e[idx] = 1.0
            checks.append((np.zeros(m * n), np.zeros(m), e))
        pert = []
        for dA, dbv, dc in checks:
            for sgn in (1.0, -1.0):
                p = lpgen.config(5, [k], part="simplex")
                p.A = p.A + sgn * H * dA
                p.b = p.b + sgn * H * dbv
                p.c = p.c + sgn * H * dc
                pert.append(p)
        # solve all perturbed copies in one batch
        K = len(pert)
        big = lpgen.make_batch(1005, np.full(K, k), np.ones(K, np.int32), np.full(K, m), np.full(K, n))
        big.A = np.concatenate([p.A for p in pert])
        big.b = np.concatenate([p.b for p in pert])
        big.c = np.concatenate([p.c for p in pert])
        objs = _solve_obj(blp, torch, big)
        for q, (dA, dbv, dc) in enumerate(checks):
            fd = (objs[2 * q] - objs[2 * q + 1]) / (2 * H)
            an = float(gA @ dA + gb @ dbv + gc @ dc)
            assert abs(fd - an) <= 1e-6 * max(1.0, abs(an)), (k, q, fd, an, scale)


def test_hyperbox_backward():
    import torch

    import paper_1609_08114_amd as blp
    from paper_1609_08114_amd.autograd import batched_lp
    hb = lpgen.config(5, range(3000), part="box28")
    db = blp.DeviceBatch.from_host(hb)
    c = db.c.clone().requires_grad_(True)
    l = db.l.clone().requires_grad_(True)
    u = db.u.clone().requires_grad_(True)
    w = torch.from_numpy(lpgen.weights(1025, range(3000))).cuda()
    obj, st = batched_lp(db, c=c, l=l, u=u)
    (obj * w).sum().backward()
    cn, ln, un = hb.c, hb.l, hb.u
    wn = np.repeat(w.cpu().numpy(), 28)
    h = np.where(cn < 0, ln, un)
    assert np.array_equal(c.grad.cpu().numpy(), wn * h)
    assert np.array_equal(l.grad.cpu().numpy(), np.where(cn < 0, wn * cn, 0.0))
    assert np.array_equal(u.grad.cpu().numpy(), np.where(cn < 0, 0.0, wn * cn))
    # central differences on a few coordinates (exact: the optimum is linear in l, u, c)
    k = 7
    for i in range(28):
        p = lpgen.config(5, [k, k], part="box28")
        p.u[i] += H
        p.u[28 + i] -= H
        o = _solve_obj(blp, torch, p)
        fd = (o[0] - o[1]) / (2 * H)
        an = float(np.where(cn[k * 28 + i] < 0, 0.0, cn[k * 28 + i]))
        assert abs(fd - an) <= 1e-6 * max(1.0, abs(an))
