"""torch.autograd wrappers of the contraction and the inner product.

Forward and backward both run in libqtt: the contraction backward is the
local core-by-core transpose of the contraction (qtt_contract_backward); the
inner-product backward uses left/right environment sweeps
(qtt_inner_backward), i.e. the core derivative d<A,B>/dA_k of the paper's
variational formulation (Sec. 3.3, eq. variational).  Only scalar glue
(sums of inner products) is left to torch.
"""
from __future__ import annotations

from typing import List, Sequence

import torch

from . import qtt as Q


class QttContract(torch.autograd.Function):
    """C = contract(spec, A, B) core by core; inputs and outputs are core lists."""

    @staticmethod
    def forward(ctx, spec: str, n: int, *cores):
        a, b = list(cores[:n]), list(cores[n:])
        ctx.spec, ctx.n = spec, n
        ctx.save_for_backward(*cores)
        with torch.no_grad():
            out = Q.contract(spec, [c.detach() for c in a], [c.detach() for c in b])
        return tuple(out)

    @staticmethod
    def backward(ctx, *dc):
        n, spec = ctx.n, ctx.spec
        cores = ctx.saved_tensors
        a, b = list(cores[:n]), list(cores[n:])
        need = ctx.needs_input_grad[2:]
        want_a, want_b = any(need[:n]), any(need[n:])
        ranks_c = [a[0].shape[0] * b[0].shape[0]] + [x.shape[-1] * y.shape[-1] for x, y in zip(a, b)]
        grads = []
        for k, g in enumerate(dc):
            if g is None:
                g = torch.zeros((ranks_c[k], a[k].shape[1], ranks_c[k + 1]), dtype=a[k].dtype, device=a[k].device)
            grads.append(g.contiguous())
        da, db = Q.contract_backward(spec, a, b, grads, want_a=want_a, want_b=want_b)
        da = da if da is not None else [None] * n
        db = db if db is not None else [None] * n
        return (None, None, *da, *db)


class QttInner(torch.autograd.Function):
    """<A, B> as a 0-d tensor (storage dtype of the cores)."""

    @staticmethod
    def forward(ctx, n: int, *cores):
        a, b = list(cores[:n]), list(cores[n:])
        ctx.n = n
        ctx.save_for_backward(*cores)
        with torch.no_grad():
            val = Q.inner([c.detach() for c in a], [c.detach() for c in b])
        return torch.tensor(val, dtype=a[0].dtype, device=a[0].device)

    @staticmethod
    def backward(ctx, g):
        n = ctx.n
        cores = ctx.saved_tensors
        a, b = list(cores[:n]), list(cores[n:])
        need = ctx.needs_input_grad[1:]
        want_a, want_b = any(need[:n]), any(need[n:])
        gv = float(g.item())
        da, db = Q.inner_backward(a, b, gv, want_a=want_a, want_b=want_b)
        da = da if da is not None else [None] * n
        db = db if db is not None else [None] * n
        return (None, *da, *db)


def contract(spec: str, a: Sequence[torch.Tensor], b: Sequence[torch.Tensor]) -> List[torch.Tensor]:
    return list(QttContract.apply(spec, len(a), *a, *b))


def inner(a: Sequence[torch.Tensor], b: Sequence[torch.Tensor]) -> torch.Tensor:
    return QttInner.apply(len(a), *a, *b)


def residual_loss(W: Sequence[torch.Tensor], x: Sequence[torch.Tensor], b: Sequence[torch.Tensor]) -> torch.Tensor:
    """||W x - b||^2 = <y,y> - 2<y,b> + <b,b> with y = W x (MPO applied to MPS)."""
    y = contract("ij,j->i", W, x)
    return inner(y, y) - 2.0 * inner(y, b) + inner(b, b)
