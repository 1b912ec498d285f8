"""The allocation-free contraction + rounding entry point against the one
that takes a caller workspace (same kernels, so the results must agree bit
for bit), on two calls in a row with the second input smaller, and its
rejection of a product whose workspace exceeds the fixed array."""
import ctypes as C

import numpy as np
import pytest
import torch

import oracle as O
import qtt_inputs as I
from paper_2602_20226_amd import qtt as Q

pytestmark = pytest.mark.gpu


def _case(m, rmax):
    w = I.laplacian2d_r64(seed=7, m=m, rmax=rmax)
    A = Q.to_device(w.a, "cuda:0")
    B = Q.to_device(w.b, "cuda:0")
    return w, A, B


def _out_buffers(w, A, B):
    n = len(A)
    d = [c.shape[1] for c in A]
    rc = [x * y for x, y in zip(_ranks(A), _ranks(B))]
    bnd = Q.rank_bounds(rc, d, w.max_rank)
    # filled with NaN so that a core the call fails to write shows up
    return [torch.full((bnd[k] * d[k] * bnd[k + 1],), float("nan"), dtype=torch.float64, device="cuda:0")
            for k in range(n)]


def _ranks(cores):
    return [cores[0].shape[0]] + [c.shape[-1] for c in cores]


def _workspace_bytes(w, A, B):
    L = Q.load_library()
    va, vb = Q.TTView(list(A), 2), Q.TTView(list(B), 1)
    nb = C.c_size_t()
    st = L.qtt_workspace_size(None, Q.OP_CONTRACT_ROUND, w.spec.encode(), C.byref(va.struct), C.byref(vb.struct),
                              int(w.max_rank), 0, C.byref(nb))
    assert st == 0
    return nb.value


@pytest.mark.parametrize("prec", ["fp64", "bf16x6"])
def test_noalloc_matches_workspace_entry_point_twice(prec):
    torch.cuda.synchronize()
    for m, rmax in [(10, 32), (6, 8)]:  # second call smaller than the first
        w, A, B = _case(m, rmax)
        assert _workspace_bytes(w, A, B) <= Q.NOALLOC_SCRATCH_BYTES
        ref = Q.contract_round(w.spec, A, B, w.rel_tol, w.max_rank, prec=prec)
        got = Q.contract_round_noalloc(w.spec, A, B, w.rel_tol, w.max_rank, _out_buffers(w, A, B), prec=prec)
        torch.cuda.synchronize()
        assert got.ranks == ref.ranks, (m, got.ranks, ref.ranks)
        for k, (g, r) in enumerate(zip(got.cores, ref.cores)):
            assert torch.equal(g, r), (m, k)
        assert got.err_bound == ref.err_bound and got.norm == ref.norm
        # and against the oracle, to the tolerance of the arithmetic
        want, info = O.round_tt(O.contract(w.spec, w.a, w.b), w.rel_tol, w.max_rank, return_info=True)
        assert got.ranks == info.ranks
        err = O.rel_error(Q.to_host(got.cores), want)
        assert err <= (1e-12 if prec == "fp64" else 1e-6), (m, err)


def test_noalloc_rejects_products_larger_than_its_array():
    w, A, B = _case(16, 96)
    assert _workspace_bytes(w, A, B) > Q.NOALLOC_SCRATCH_BYTES
    with pytest.raises(Q.QttError, match="WORKSPACE"):
        Q.contract_round_noalloc(w.spec, A, B, w.rel_tol, w.max_rank, _out_buffers(w, A, B))
    # the array is still usable afterwards
    w, A, B = _case(6, 8)
    ref = Q.contract_round(w.spec, A, B, w.rel_tol, w.max_rank)
    got = Q.contract_round_noalloc(w.spec, A, B, w.rel_tol, w.max_rank, _out_buffers(w, A, B))
    assert got.ranks == ref.ranks
    assert all(torch.equal(g, r) for g, r in zip(got.cores, ref.cores))
