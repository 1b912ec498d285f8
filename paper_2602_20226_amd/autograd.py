"""torch.autograd wrappers of the contraction and the inner product.

Forward and backward both run in libqtt: the contraction backward is the
local core-by-core transpose of the contraction (qtt_contract_backward); the
inner-product backward uses left/right environment sweeps
(qtt_inner_backward), i.e. the core derivative d<A,B>/dA_k of the paper's
variational formulation (Sec. 3.3, eq. variational).  The residual loss
||W x - b||^2 is the squared norm of the exact difference train y - b (the
block sum of Sec. 3.1, qtt_add) taken by a QR sweep (qtt_orthogonalize), so
it carries no cancellation between <y,y>, <y,b> and <b,b>.
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


def _blocks_of_difference(dD, y, b):
    """(dL/dy_k, dL/db_k) from dL/dD_k for D = y - b as the block train
    [y_1, -b_1], diag(y_k, b_k), [y_n; b_n]: the y and b blocks of each core
    gradient, with the sign of b's first block."""
    n = len(y)
    dy, db = [], []
    for k in range(n):
        ry0, ry1 = y[k].shape[0], y[k].shape[-1]
        g = dD[k]
        if n == 1:
            gy, gb = g, -g
        elif k == 0:
            gy, gb = g[..., :ry1], -g[..., ry1:]
        elif k == n - 1:
            gy, gb = g[:ry0], g[ry0:]
        else:
            gy, gb = g[:ry0, ..., :ry1], g[ry0:, ..., ry1:]
        dy.append(gy.contiguous())
        db.append(gb.contiguous())
    return dy, db


class QttResidual(torch.autograd.Function):
    """||W x - b||^2 (W an MPO, x and b MPS), as a 0-d tensor.

    Forward: y = W x (qtt_contract), D = y - b (qtt_add), L = ||D||^2 from
    the QR sweep of D (qtt_orthogonalize, FP64; FP32 cores are widened
    exactly first).  Backward: dL/dD_k = 2 g E_{k-1} D_k F_{k+1} from the
    environment sweeps of <D, D> (qtt_inner_backward), split into the y and
    b blocks, then dL/dW, dL/dx by the contraction backward."""

    @staticmethod
    def forward(ctx, n: int, *cores):
        W, x, b = list(cores[:n]), list(cores[n:2 * n]), list(cores[2 * n:])
        ctx.n = n
        with torch.no_grad():
            y = Q.contract("ij,j->i", [c.detach() for c in W], [c.detach() for c in x])
            D = Q.add([y, [c.detach() for c in b]], [1.0, -1.0])
            D64 = D if D[0].dtype == torch.float64 else [c.double() for c in D]
            _, nrm = Q.orthogonalize(D64)
        ctx.save_for_backward(*W, *x, *b, *y, *D)
        return torch.tensor(nrm * nrm, dtype=W[0].dtype, device=W[0].device)

    @staticmethod
    def backward(ctx, g):
        n = ctx.n
        saved = ctx.saved_tensors
        W, x, b = list(saved[:n]), list(saved[n:2 * n]), list(saved[2 * n:3 * n])
        y, D = list(saved[3 * n:4 * n]), list(saved[4 * n:])
        need = ctx.needs_input_grad[1:]
        want_w, want_x, want_b = any(need[:n]), any(need[n:2 * n]), any(need[2 * n:])
        dD, _ = Q.inner_backward(D, D, 2.0 * float(g.item()), want_a=True, want_b=False)
        dy, db = _blocks_of_difference(dD, y, b)
        dW, dx = [None] * n, [None] * n
        if want_w or want_x:
            gw, gx = Q.contract_backward("ij,j->i", W, x, dy, want_a=want_w, want_b=want_x)
            dW = gw if gw is not None else dW
            dx = gx if gx is not None else dx
        return (None, *dW, *dx, *(db if want_b else [None] * n))


def residual_loss(W: Sequence[torch.Tensor], x: Sequence[torch.Tensor], b: Sequence[torch.Tensor]) -> torch.Tensor:
    """||W x - b||^2 with W an MPO applied to the MPS x (see QttResidual)."""
    return QttResidual.apply(len(x), *W, *x, *b)
