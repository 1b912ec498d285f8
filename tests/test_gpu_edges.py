"""Degenerate and smallest cases of the later entry points: one- and
two-core trains, rank-1 products, a zero right-hand side, and the
stream-ordered rounding on the smallest trains, each against the oracle or
the synchronous call; the solvers on the shortest chains, and their error
on an operator that is not positive definite."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

import oracle as O
import qtt_inputs as I

pytestmark = pytest.mark.gpu

if torch.cuda.is_available():
    from paper_2602_20226_amd import qtt as Q

DEV = "cuda:0"


def dev(cores):
    return Q.to_device(cores, DEV, torch.float64)


def host(cores):
    return Q.to_host(cores)


def rand_tt(rng, ranks, d=2):
    return [rng.standard_normal((ranks[k], d, ranks[k + 1])) for k in range(len(ranks) - 1)]


def rand_mpo(rng, ranks, d=2):
    return [rng.standard_normal((ranks[k], d, d, ranks[k + 1])) for k in range(len(ranks) - 1)]


@pytest.mark.parametrize("n", [1, 2])
def test_fit2_one_and_two_cores(n):
    rng = np.random.default_rng(700 + n)
    A = rand_mpo(rng, [1] + [3] * (n - 1) + [1])
    B = rand_tt(rng, [1] + [2] * (n - 1) + [1])
    G = rand_tt(rng, [1] * (n + 1))
    ref, info = O.fit_two_core("ij,j->i", A, B, G, 1e-13, 0, 1, return_info=True)
    cores, ranks, nrm, _ = Q.fit2("ij,j->i", dev(A), dev(B), dev(G), nsweeps=1, rel_tol=1e-13)
    assert ranks == info["ranks"]
    assert O.rel_error(host(cores), ref) <= 1e-13
    # the fit of an exactly representable product is the product
    assert O.rel_error(host(cores), O.contract("ij,j->i", A, B)) <= 1e-13


def test_fit2_rank_one_product_and_loose_tolerance():
    """exp * exp is rank 1: from a rank-3 guess the two-core fit falls to rank 1."""
    n = 8
    e = I.exp_qtt(n, 0.3)
    G = rand_tt(np.random.default_rng(3), [1, 2, 3, 3, 3, 3, 3, 2, 1])
    cores, ranks, nrm, _ = Q.fit2("i,i->i", dev(e), dev(e), dev(G), nsweeps=1, rel_tol=1e-12)
    assert max(ranks) == 1
    assert O.rel_error(host(cores), O.contract("i,i->i", e, e)) <= 1e-13


def test_solve_single_core_is_the_dense_solve():
    rng = np.random.default_rng(710)
    M = rng.standard_normal((4, 4))
    W = [(M @ M.T + 4 * np.eye(4)).reshape(1, 4, 4, 1)]
    b = [rng.standard_normal((1, 4, 1))]
    x0 = [np.ones((1, 4, 1))]
    cores, ranks, nrm = Q.solve(dev(W), dev(b), dev(x0))
    want = np.linalg.solve(W[0].reshape(4, 4), b[0].reshape(4))
    assert np.abs(host(cores)[0].reshape(4) - want).max() <= 1e-13 * np.abs(want).max()


@pytest.mark.parametrize("ncores", [1, 2])
def test_solve_zero_right_hand_side_gives_zero(ncores):
    m, D = 3, 2
    W = I.laplacian_mpo(m, D, diag=3.0)
    b = [np.zeros((1, 2, 1)) for _ in range(m * D)]
    g = I.random_mps(m * D, 2, np.random.default_rng(4))
    cores, ranks, nrm = Q.solve(dev(W), dev(b), dev(g), nsweeps=1, ncores=ncores, max_rank=4)
    assert nrm == 0.0 and max(ranks) == 1
    assert float(np.abs(O.to_dense(host(cores))).max()) == 0.0


@pytest.mark.parametrize("n", [1, 2, 3])
def test_async_rounding_smallest_trains(n):
    rng = np.random.default_rng(720 + n)
    A = rand_mpo(rng, [1] + [3] * (n - 1) + [1])
    B = rand_tt(rng, [1] + [4] * (n - 1) + [1])
    dA, dB = dev(A), dev(B)
    ref = Q.contract_round("ij,j->i", dA, dB, 1e-10, 0)
    run = Q.ContractRoundAsync("ij,j->i", dA, dB, 1e-10, 0)
    run.enqueue()
    cores, ranks = run.result()
    assert ranks == ref.ranks
    assert all(torch.equal(x, y) for x, y in zip(cores, ref.cores))
    want, info = O.round_tt(O.contract("ij,j->i", A, B), 1e-10, 0, return_info=True)
    assert ranks == info.ranks
    assert O.rel_error(host(cores), want) <= 1e-13


@pytest.mark.parametrize("solver", ["dmrg1", "dmrg2", "amen"])
def test_solvers_reject_an_indefinite_operator(solver):
    """The linear solvers take W symmetric positive definite: the local
    matrices of a negative definite W have no Cholesky factor (the first
    pivot's square root is NaN), and the call ends with QTT_ERR_NONFINITE
    instead of returning a train."""
    print(f"indefinite operator, {solver}", flush=True)
    m, D = 3, 2
    W = [c.copy() for c in I.laplacian_mpo(m, D, diag=2.5)]
    W[0] = -W[0]  # -W: negative definite
    rng = np.random.default_rng(21)
    b = I.random_mps(m * D, 2, rng)
    x0 = I.random_mps(m * D, 2, rng)
    z0 = I.random_mps(m * D, 2, rng)
    with pytest.raises(Q.QttError, match="NONFINITE"):
        if solver == "amen":
            Q.solve_amen(dev(W), dev(b), dev(x0), dev(z0), nsweeps=1, max_rank=4)
        else:
            Q.solve(dev(W), dev(b), dev(x0), nsweeps=1, ncores=1 if solver == "dmrg1" else 2, max_rank=4)


@pytest.mark.parametrize("n", [2, 3])
@pytest.mark.parametrize("solver", ["dmrg1", "dmrg2", "amen"])
def test_solvers_on_the_shortest_chains(solver, n):
    """Two- and three-core chains (a shifted 1D Laplacian on 2^n points),
    where every core is an end core or next to one: both sweeps turn at
    once.  Two sweeps from a rank-2 guess (and a rank-2 residual train for
    AMEn) against the oracle's solver: ranks identical, the solution within
    1e-10 (relative), and the dense solve reached to 1e-12."""
    print(f"short chain n={n}, {solver}", flush=True)
    W = I.laplacian_mpo(n, 1, diag=2.5)
    rng = np.random.default_rng(730 + n)
    b = I.random_mps(n, 2, rng)
    x0 = I.random_mps(n, 2, rng)
    if solver == "amen":
        z0 = I.random_mps(n, 2, rng)
        ref, info = O.solve_amen(W, b, x0, z0, nsweeps=2, rel_tol=1e-12, return_info=True)
        xc, ranks, _, _, _ = Q.solve_amen(dev(W), dev(b), dev(x0), dev(z0), nsweeps=2, rel_tol=1e-12)
    else:
        nc = 1 if solver == "dmrg1" else 2
        ref, info = O.solve_energy(W, b, x0, nsweeps=2, ncores=nc, rel_tol=1e-12, return_info=True)
        xc, ranks, _ = Q.solve(dev(W), dev(b), dev(x0), nsweeps=2, ncores=nc, rel_tol=1e-12)
    assert ranks == info["ranks"], (ranks, info["ranks"])
    got = host(xc)
    assert O.rel_error(got, ref) <= 1e-10
    # rank 2 is the full rank of every bond here, so the sweeps reach the exact solution
    A = O.mpo_to_dense(W)
    xs = np.linalg.solve(A, O.to_dense(b).ravel())
    assert np.linalg.norm(O.to_dense(got).ravel() - xs) <= 1e-12 * np.linalg.norm(xs)
