"""Precision forms at the full 3D rank-256 size against the FP64 oracle.

The oracle rounds the exact rank-1792 product once (about half a minute of
LAPACK work); every GEMM arithmetic of the GPU path is compared with it.
"""
import math
import sys

import numpy as np
import pytest

torch = pytest.importorskip("torch")

import oracle as O
import qtt_inputs as I

pytestmark = pytest.mark.gpu

if torch.cuda.is_available():
    from paper_2602_20226_amd import qtt as Q

DEV = "cuda:0"


def log(msg):
    print(msg, flush=True)


@pytest.fixture(scope="module")
def lap3d():
    w = I.laplacian3d_r256()
    log("laplacian3d: oracle contract + round (FP64, LAPACK)")
    C = O.contract(w.spec, w.a, w.b)
    ref, info = O.round_tt(C, w.rel_tol, w.max_rank, return_info=True)
    del C
    A = Q.to_device(w.a, DEV)
    B = Q.to_device(w.b, DEV)
    return w, ref, info, A, B


def _run(lap3d, prec):
    w, ref, info, A, B = lap3d
    got = Q.contract_round(w.spec, A, B, w.rel_tol, w.max_rank, prec=prec, want_sigmas=True)
    err = O.rel_error(Q.to_host(got.cores), ref)
    sig = 0.0
    for k, s in enumerate(info.sigmas):
        g = np.array(got.sigmas[k][: len(s)])
        sig = max(sig, np.abs(g - s).max() / s[0])
    log(f"laplacian3d {prec}: rel err {err:.3e}  max sigma err/sigma1 {sig:.3e}  ranks equal {got.ranks == info.ranks}")
    return got, err, sig


@pytest.mark.timeout(900)
def test_lap3d_fp64_path(lap3d):
    got, err, sig = _run(lap3d, "fp64")
    _, _, info, _, _ = lap3d
    assert got.ranks == info.ranks
    assert sig <= 1e-12
    assert err <= 1e-12


@pytest.mark.timeout(900)
def test_lap3d_bf16x6_path(lap3d):
    got, err, sig = _run(lap3d, "bf16x6")
    _, _, info, _, _ = lap3d
    assert got.ranks == info.ranks
    assert sig <= 1e-6
    assert err <= 1e-6


@pytest.mark.timeout(900)
def test_lap3d_bf16x3_and_fp32_reported(lap3d):
    """Three-product split and FP32 GEMMs: ranks must match, errors are reported."""
    _, _, info, _, _ = lap3d
    for prec in ["bf16x3", "fp32"]:
        got, err, sig = _run(lap3d, prec)
        assert got.ranks == info.ranks
        assert err <= 1e-4


@pytest.mark.timeout(300)
def test_inner_precision_forms_rank256():
    """The environment sweep of the inner product in each GEMM arithmetic at
    the rank-256 size: <X, Y> and <X, X> of two 42-core rank-256 MPS against
    the oracle, to 1e-6 ||X|| ||Y|| for the reduced forms."""
    w = I.laplacian3d_r256()
    X = w.b
    Y = I.random_mps(len(X), 256, np.random.default_rng(13))
    nx, ny = O.norm(X), O.norm(Y)
    ref_xy, ref_xx = O.inner(X, Y), O.inner(X, X)
    dX, dY = Q.to_device(X, DEV), Q.to_device(Y, DEV)
    for prec, tol in [("fp64", 1e-13), ("bf16x6", 1e-6), ("fp32", 1e-6), ("bf16x3", 1e-4)]:
        exy = abs(Q.inner(dX, dY, prec=prec) - ref_xy) / (nx * ny)
        exx = abs(Q.inner(dX, dX, prec=prec) - ref_xx) / (nx * nx)
        log(f"inner {prec}: |err|/(|x||y|) {exy:.2e}, <x,x> {exx:.2e}")
        assert exy <= tol and exx <= tol, (prec, exy, exx)
