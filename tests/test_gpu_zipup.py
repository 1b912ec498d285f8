"""GPU parity of the decomposition (zip-up) path against the FP64 oracle's zip-up."""
import math
import sys

import numpy as np
import pytest

torch = pytest.importorskip("torch")

import oracle as O
import qtt_inputs as I
from conftest import ranks_agree

pytestmark = pytest.mark.gpu

if torch.cuda.is_available():
    from paper_2602_20226_amd import qtt as Q

DEV = "cuda:0"


def log(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def dev(cores):
    return Q.to_device(cores, DEV, torch.float64)


def host(cores):
    return Q.to_host(cores)


def rand_tt(rng, ranks, d=2):
    return [rng.standard_normal((ranks[k], d, ranks[k + 1])) for k in range(len(ranks) - 1)]


def rand_mpo(rng, ranks, d=2):
    return [rng.standard_normal((ranks[k], d, d, ranks[k + 1])) for k in range(len(ranks) - 1)]


def check_zipup(got, ref, info, tol=1e-12, sig_tol=1e-12):
    gh = host(got.cores)
    assert ranks_agree(got.ranks, info), (got.ranks, info.ranks)
    # left-orthonormal cores 1..n-1
    for c in gh[:-1]:
        M = c.reshape(-1, c.shape[-1])
        assert np.abs(M.T @ M - np.eye(M.shape[1])).max() <= 1e-13
    for b, s in enumerate(info.sigmas):
        g = np.array(got.sigmas[b][: len(s)])
        assert np.abs(g - s).max() <= sig_tol * s[0] + 1e-300, b
    for b in range(len(info.tails)):
        assert abs(got.tails[b] - info.tails[b]) <= 1e-10 * info.sigmas[b][0] + 1e-300
    assert abs(got.norm - info.norm) <= 1e-13 * info.norm
    err = O.rel_error(gh, ref)
    assert err <= tol, err
    return err


@pytest.mark.parametrize("spec", ["ij,j->i", "i,i->i"])
@pytest.mark.parametrize("N", [1, 2])
@pytest.mark.parametrize("tol,maxr", [(0.0, 0), (1e-6, 0), (1e-2, 0), (0.0, 9)])
def test_zipup_random_ragged(spec, N, tol, maxr):
    """Ragged ranks (split matrices of 2..74 rows, several Jacobi blocks and
    QR panels with tails), both products, both super-core sizes."""
    log(f"zipup random {spec} N={N} tol={tol} maxr={maxr}")
    rng = np.random.default_rng(200 + N)
    if spec == "ij,j->i":
        A = rand_mpo(rng, [1, 3, 5, 5, 5, 5, 5, 5, 5, 3, 1])
    else:
        A = rand_tt(rng, [1, 2, 3, 3, 3, 3, 3, 3, 3, 2, 1])
    B = rand_tt(rng, [1, 2, 4, 8, 16, 37, 16, 8, 4, 2, 1])
    ref, info = O.zipup(spec, A, B, tol, maxr, ncores=N, return_info=True)
    got = Q.contract_zipup(spec, dev(A), dev(B), tol, maxr, ncores=N, want_sigmas=True)
    check_zipup(got, ref, info)
    if tol == 0.0 and maxr == 0:
        assert O.rel_error(host(got.cores), O.contract(spec, A, B)) <= 1e-13


def test_zipup_identity_operator_error_is_discarded_norm():
    """I x: every split is an exact truncated SVD, so the result's error
    against x is the orthogonal sum of the discarded norms (each scaled back
    by the operator normalisation factor 2^(-q/2), q = n - 1 - b for N = 1)."""
    log("zipup identity")
    rng = np.random.default_rng(210)
    n = 12
    X = O.tt_add(rand_tt(rng, [1] + [2] * (n - 1) + [1]),
                 rand_tt(rng, [1, 2, 4, 8, 16, 24, 24, 24, 16, 8, 4, 2, 1]), 1.0, 1e-3)
    W = [np.eye(2).reshape(1, 2, 2, 1).copy() for _ in range(n)]
    got = Q.contract_zipup("ij,j->i", dev(W), dev(X), 1e-3, 0, ncores=1, want_sigmas=True)
    err = O.diff_norm(host(got.cores), X)
    expect = math.sqrt(sum((t / 2.0 ** ((n - 1 - b) / 2)) ** 2 for b, t in enumerate(got.tails)))
    nx = O.norm(X)
    assert expect > 1e-6 * nx
    assert abs(err - expect) <= 1e-10 * nx


def test_zipup_laplacian2d_against_exact_product():
    """2D Laplacian (rank 5) times a rank-64 MPS at n = 32, truncated to rank
    64: parity with the oracle's zip-up, and an error against the exact
    product close to that of TT rounding at the same rank cap (the cap, not
    the tolerance, sets the error here: 0.086 for rounding)."""
    log("zipup laplacian2d")
    w = I.laplacian2d_r64()
    C = O.contract(w.spec, w.a, w.b)
    e_round = O.rel_error(O.round_tt(C, w.rel_tol, w.max_rank), C)
    for N in (1, 2):
        ref, info = O.zipup(w.spec, w.a, w.b, w.rel_tol, w.max_rank, ncores=N, return_info=True)
        got = Q.contract_zipup(w.spec, dev(w.a), dev(w.b), w.rel_tol, w.max_rank, ncores=N, want_sigmas=True)
        err = check_zipup(got, ref, info, tol=1e-12, sig_tol=1e-12)
        exact = O.rel_error(host(got.cores), C)
        log(f"  N={N} ranks max {max(got.ranks)} vs oracle {err:.2e} vs exact {exact:.2e} (rounding {e_round:.2e})")
        assert e_round <= exact <= 1.5 * e_round


@pytest.mark.timeout(600)
@pytest.mark.parametrize("N", [1, 2])
def test_zipup_laplacian3d_r256_full_size(N):
    """The rank-256 3D workload at full size (n = 42, splits of 512 x 1792 or
    512 x 3584): ranks, per-bond singular values and the tensor against the
    oracle's zip-up."""
    log(f"zipup laplacian3d N={N}")
    w = I.laplacian3d_r256()
    ref, info = O.zipup(w.spec, w.a, w.b, w.rel_tol, w.max_rank, ncores=N, return_info=True)
    got = Q.contract_zipup(w.spec, dev(w.a), dev(w.b), w.rel_tol, w.max_rank, ncores=N, want_sigmas=True)
    err = check_zipup(got, ref, info, tol=1e-12, sig_tol=1e-12)
    log(f"  rel err vs oracle {err:.2e}, max rank {max(got.ranks)}, sweeps {got.jacobi_sweeps_max}")


def test_zipup_argument_errors():
    rng = np.random.default_rng(211)
    A = rand_mpo(rng, [1, 3, 1])
    B = rand_tt(rng, [1, 2, 1])
    with pytest.raises(Q.QttError) as e:
        Q.contract_zipup("ij,j->i", dev(A), dev(B), 1e-8, 0, ncores=3)
    assert e.value.status == -10
    with pytest.raises(Q.QttError) as e:
        Q.contract_zipup("ij,j->i", dev(A), dev(B), -1.0, 0)
    assert e.value.status == -1
    with pytest.raises(ValueError):
        Q.contract_zipup("ij->i", dev(A), dev(B), 1e-8, 0)


def test_zipup_single_core_and_zero():
    rng = np.random.default_rng(212)
    A = [rng.standard_normal((1, 2, 2, 1))]
    B = [rng.standard_normal((1, 2, 1))]
    got = Q.contract_zipup("ij,j->i", dev(A), dev(B), 1e-8, 0)
    ref = O.contract("ij,j->i", A, B)
    assert got.ranks == [1, 1]
    assert np.abs(host(got.cores)[0] - ref[0]).max() <= 1e-15 * np.abs(ref[0]).max()
    Z = [np.zeros((1, 2, 3)), np.zeros((3, 2, 3)), np.zeros((3, 2, 1))]
    got = Q.contract_zipup("i,i->i", dev(Z), dev(rand_tt(rng, [1, 2, 2, 1])), 1e-8, 0)
    assert got.ranks == [1, 1, 1, 1]
    assert np.abs(O.to_dense(host(got.cores))).max() == 0.0
