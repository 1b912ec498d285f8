"""GPU parity of the DMRG-like linear solver (Sec. 5) against the FP64
oracle's solver: the same sweeps from the same guess, one-core and two-core,
on the Dirichlet Laplacian shifted by s I (symmetric positive definite)."""
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
    sys.stdout.flush()


def dev(cores):
    return Q.to_device(cores, DEV, torch.float64)


def host(cores):
    return Q.to_host(cores)


def shifted_laplacian(m, D, s):
    return I.laplacian_mpo(m, D, diag=2.0 + s / D)


@pytest.mark.parametrize("ncores,nsweeps,cap", [(1, 1, 0), (1, 3, 0), (2, 2, 6)])
def test_solve_random_rhs_against_oracle(ncores, nsweeps, cap):
    """A 2D 2^5 x 2^5 grid (10 cores), right-hand side of rank 4, guess of
    ragged ranks: the GPU sweeps against the oracle's from the same guess."""
    log(f"solve ncores={ncores} sweeps={nsweeps} cap={cap}")
    m, D = 5, 2
    A = shifted_laplacian(m, D, 0.5)
    n = m * D
    rng = np.random.default_rng(610)
    b = I.random_mps(n, 4, rng)
    guess = I.random_mps(n, 5, rng)
    ref, info = O.solve_energy(A, b, guess, nsweeps=nsweeps, ncores=ncores, rel_tol=1e-10, max_rank=cap,
                               return_info=True)
    cores, ranks, nrm = Q.solve(dev(A), dev(b), dev(guess), nsweeps=nsweeps, ncores=ncores, rel_tol=1e-10,
                                max_rank=cap)
    assert ranks == info["ranks"], (ranks, info["ranks"])
    gh = host(cores)
    err = O.rel_error(gh, ref)
    log(f"  ranks {ranks}, rel err vs oracle {err:.2e}")
    assert err <= 1e-10
    assert abs(nrm - O.norm(ref)) <= 1e-10 * O.norm(ref)


@pytest.mark.parametrize("ncores", [1, 2])
def test_solve_eigenvector_full_size(ncores):
    """(L + s I) f = (lambda + s) f on a 2^12 x 2^12 grid (24 cores): from a
    random rank-4 guess three sweeps recover f, as in the oracle's pin."""
    log(f"solve eigenvector ncores={ncores}")
    m, D, s = 12, 2, 1.0
    N = 2 ** m
    f, lam = None, 0.0
    for a, k in enumerate([N // 3, N // 2 - 1]):
        w = math.pi * k / (N + 1)
        fa = I.trig_qtt(m, w, w, "sin")
        lam += 2.0 - 2.0 * math.cos(w)
        ea = I.embed_axis(fa, D, a)
        f = ea if f is None else O.contract("i,i->i", f, ea)
    f = O.round_tt(f, 1e-14)
    A = shifted_laplacian(m, D, s)
    b = O.tt_scale(f, lam + s)
    guess = I.random_mps(m * D, 4, np.random.default_rng(7))
    cores, ranks, nrm = Q.solve(dev(A), dev(b), dev(guess), nsweeps=3, ncores=ncores, rel_tol=1e-13, max_rank=4)
    err = O.rel_error(host(cores), f)
    log(f"  ranks {max(ranks)} max, rel err vs f {err:.2e}")
    assert err <= 1e-11


def test_solve_argument_errors():
    m, D = 3, 2
    A = dev(shifted_laplacian(m, D, 1.0))
    b = dev(I.random_mps(m * D, 2, np.random.default_rng(1)))
    with pytest.raises(Q.QttError, match="ARG"):
        Q.solve(A, b, b, ncores=3)
    with pytest.raises(Q.QttError, match="SHAPE"):
        Q.solve(A, b[:-1], b[:-1])
