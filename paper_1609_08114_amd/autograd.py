"""Differentiable batched LP optimum (an extension beyond the paper).

``batched_lp(db, A=..., b=..., c=..., l=..., u=...)`` returns the optimal
objective of every LP of the batch as a tensor; its backward is the library's
adjoint kernel (``blp_backward``): for a simplex LP k with optimum x*, y*,
d obj/dc = x*, d obj/db = y*, d obj/dA = -y* x*^T; for a hyperbox LP,
d obj/dc = h, d obj/dl = min(c, 0), d obj/du = max(c, 0).  The gradient is the
true derivative only where the optimum is non-degenerate (x* and y* unique);
LPs that are not OPTIMAL get zero gradients.

Only pointers and streams go through torch; the solve and the adjoint run in
the HIP kernels.
"""
from __future__ import annotations

import torch

from . import DeviceBatch, Solver

_FIELDS = ("A", "b", "c", "l", "u")


class _BatchedLP(torch.autograd.Function):
    @staticmethod
    def forward(ctx, skeleton: DeviceBatch, solver_kw: dict, A, b, c, l, u):
        db = DeviceBatch(m=skeleton.m, n=skeleton.n, kind=skeleton.kind, a_off=skeleton.a_off,
                         row_off=skeleton.row_off, col_off=skeleton.col_off, A=A.detach(), b=b.detach(),
                         sense=skeleton.sense, c=c.detach(), l=None if l is None else l.detach(),
                         u=None if u is None else u.detach(), uniform=skeleton.uniform)
        db._count = skeleton.count
        # one handle per forward call: its backward refers to this solve
        solver = Solver(**solver_kw)
        out = solver.solve(db)
        ctx.solver = solver
        ctx.db = db
        ctx.has = [t is not None for t in (A, b, c, l, u)]
        K = skeleton.count
        obj, status = out["obj"][:K].clone(), out["status"][:K].clone()
        ctx.mark_non_differentiable(status)
        return obj, status

    @staticmethod
    def backward(ctx, g_obj, _g_status):
        solver = ctx.solver
        g = g_obj.contiguous().to(torch.float64)
        want = tuple(f for f, h, need in zip(_FIELDS, ctx.has, ctx.needs_input_grad[2:]) if h and need)
        names = {"A": "dA", "b": "db", "c": "dc", "l": "dl", "u": "du"}
        res = solver.backward(g, want=tuple(names[f] for f in want)) if want else {}
        grads = [res.get(names[f]) if f in want else None for f in _FIELDS]
        solver.close()
        ctx.solver = None
        return (None, None, *grads)


def batched_lp(db: DeviceBatch, A=None, b=None, c=None, l=None, u=None, **solver_kw):
    """Optimal objectives (and statuses) of the LPs in ``db``, differentiable
    with respect to whichever of A, b, c, l, u are given as tensors (each
    defaults to the batch's own data, not differentiated)."""
    A = db.A if A is None else A
    b = db.b if b is None else b
    c = db.c if c is None else c
    l = db.l if l is None else l
    u = db.u if u is None else u
    return _BatchedLP.apply(db, solver_kw, A, b, c, l, u)
