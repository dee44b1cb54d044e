"""Differentiable solve of -div(k grad u) = f (with optional h2 B term) behind
torch.autograd: the forward pass is libsem's PCG, the backward pass is the
hand-written adjoint of libsem (sem_adjoint): one more solve with the same
symmetric operator, dL/df = B o lam, and the fused element kernel for
dL/dk = -(D lam)^T G (D u).  Only f, k (and u unless `recompute`) are kept
for the backward pass; no iterate of either solve is stored."""
from __future__ import annotations

import torch

from .sem import Sem, SemError


class SemSolve(torch.autograd.Function):
    """u = SemSolve.apply(f, k, sem, opts, recompute)

    f, k: FP64 device L-vectors (per-copy load and coefficient; k may be None
    for k = 1).  opts: dict of sem_solve_opts fields (tol, maxit, h1, h2, ...).
    recompute: re-solve for u in backward instead of saving it."""

    @staticmethod
    def forward(ctx, f, k, sem: Sem, opts: dict, recompute: bool = False):
        b = sem.rhs(f.contiguous())
        u, st, rc = sem.solve(b, k=k, **opts)
        if rc != 0:
            raise SemError(rc, f"forward solve failed: {st}")
        ctx.sem, ctx.opts, ctx.recompute = sem, dict(opts), recompute
        ctx.has_k = k is not None
        if recompute:
            ctx.save_for_backward(f, k) if k is not None else ctx.save_for_backward(f)
        else:
            ctx.save_for_backward(f, k, u) if k is not None else ctx.save_for_backward(f, u)
        ctx.forward_stats = st
        return u

    @staticmethod
    def backward(ctx, g):
        saved = ctx.saved_tensors
        sem, opts = ctx.sem, ctx.opts
        if ctx.recompute:
            f = saved[0]
            k = saved[1] if ctx.has_k else None
            u, st, rc = sem.solve(sem.rhs(f.contiguous()), k=k, **opts)
            if rc != 0:
                raise SemError(rc, f"recomputed forward solve failed: {st}")
        else:
            if ctx.has_k:
                f, k, u = saved
            else:
                (f, u), k = saved, None
        need_k = ctx.has_k and ctx.needs_input_grad[1]
        lam, gf, gk, st, rc = sem.adjoint(u, g.contiguous(), need_grad_k=need_k, k=k, **opts)
        if rc != 0:
            raise SemError(rc, f"adjoint solve failed: {st}")
        return (gf if ctx.needs_input_grad[0] else None, gk if need_k else None, None, None, None)


def solve(f, k, sem: Sem, recompute: bool = False, **opts):
    """Functional form of SemSolve.apply."""
    return SemSolve.apply(f, k, sem, opts, recompute)
