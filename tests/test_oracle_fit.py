"""Pins of the oracle's variational fitting (Sec. 3.3, eq. variational), CPU only.

The checks use dense vectors on tiny grids: the updated centre core is the
exact minimiser (the dense gradient of ||C - Y||^2 with respect to it
vanishes), the error never grows from sweep to sweep, full ranks reproduce
the product exactly, and the fit improves on the decomposition algorithm's
result it starts from.  The two-core (super-core) variant: a full-rank guess
reproduces the product in one sweep with the ranks of its dense unfoldings,
a rank-1 guess grows to them in two, and under a rank cap the last pair is
the best rank-r approximation of the dense projection of the product.
"""
import numpy as np
import pytest

import oracle as O
import qtt_inputs as Q


def rand_tt(rng, ranks, d=2):
    return [rng.standard_normal((ranks[k], d, ranks[k + 1])) for k in range(len(ranks) - 1)]


def rand_mpo(rng, ranks):
    return [rng.standard_normal((ranks[k], 2, 2, ranks[k + 1])) for k in range(len(ranks) - 1)]


def dense_grad_last_core(C, y):
    """d ||C - y||^2 / d C_n, entry by entry from dense tensors."""
    r = O.to_dense(C) - y
    last = C[-1]
    g = np.zeros_like(last)
    for idx in np.ndindex(*last.shape):
        E = [c for c in C[:-1]] + [np.zeros_like(last)]
        E[-1][idx] = 1.0
        g[idx] = 2.0 * float(O.to_dense(E) @ r)
    return g


@pytest.mark.parametrize("spec", ["ij,j->i", "i,i->i"])
def test_centre_core_is_the_exact_minimiser(spec):
    rng = np.random.default_rng(80)
    X = rand_tt(rng, [1, 2, 4, 6, 6, 4, 2, 1])
    A = rand_mpo(rng, [1, 3, 3, 3, 3, 3, 3, 1]) if spec == "ij,j->i" else rand_tt(rng, [1, 2, 2, 2, 2, 2, 2, 1])
    y = O.to_dense(O.contract(spec, A, X))
    guess = rand_tt(rng, [1, 2, 3, 3, 3, 3, 2, 1])
    C = O.fit(spec, A, X, guess, nsweeps=1)
    g = dense_grad_last_core(C, y)
    assert np.abs(g).max() <= 1e-11 * np.linalg.norm(y) * np.abs(C[-1]).max()
    for c in C[:-1]:  # the others are left-orthonormal
        M = c.reshape(-1, c.shape[-1])
        assert np.abs(M.T @ M - np.eye(M.shape[1])).max() < 1e-13


def test_error_never_grows_and_full_ranks_are_exact():
    rng = np.random.default_rng(81)
    n = 8
    X = rand_tt(rng, [1, 2, 4, 8, 8, 8, 4, 2, 1])
    W = rand_mpo(rng, [1, 3, 3, 3, 3, 3, 3, 3, 1])
    Y = O.contract("ij,j->i", W, X)
    C = rand_tt(rng, [1, 2, 3, 3, 3, 3, 3, 2, 1])
    errs = []
    for _ in range(4):
        C = O.fit("ij,j->i", W, X, C, nsweeps=1)
        errs.append(O.rel_error(C, Y))
    assert all(b <= a * (1 + 1e-12) for a, b in zip(errs, errs[1:])), errs
    full = rand_tt(rng, [min(2 ** k, 2 ** (n - k)) for k in range(n + 1)])
    Z = O.fit("ij,j->i", W, X, full, nsweeps=1)
    assert O.rel_error(Z, Y) <= 1e-13


def test_fit_improves_on_the_decomposition_result():
    """Starting from the zip-up result (the guess the paper recommends), a
    sweep lowers the error, towards that of TT rounding at the same ranks."""
    W = Q.laplacian_mpo(5, 2)
    n = len(W)
    rng = np.random.default_rng(82)
    X = rand_tt(rng, [min(8, 2 ** k, 2 ** (n - k)) for k in range(n + 1)])
    Y = O.contract("ij,j->i", W, X)
    Z = O.zipup("ij,j->i", W, X, 0.0, 12, ncores=1)
    e0 = O.rel_error(Z, Y)
    C1 = O.fit("ij,j->i", W, X, Z, nsweeps=1)
    C3 = O.fit("ij,j->i", W, X, C1, nsweeps=2)
    e1, e3 = O.rel_error(C1, Y), O.rel_error(C3, Y)
    e_round = O.rel_error(O.round_tt(Y, 0.0, 12), Y)
    assert e1 < 0.5 * e0 and e3 <= e1 * (1 + 1e-12)
    assert e3 <= 1.05 * e_round


# ---------------------------------------------------------------- two-core super-cores
def _dense_ranks(y, d, n, tol=1e-12):
    """Bond ranks of a dense vector from the numerical ranks of its unfoldings."""
    out = [1]
    for k in range(1, n):
        M = y.reshape(d ** k, -1)
        s = np.linalg.svd(M, compute_uv=False)
        out.append(int(np.sum(s > tol * s[0])))
    return out + [1]


def _lap_case(seed=5):
    rng = np.random.default_rng(seed)
    W = Q.laplacian_mpo(4, 2)  # 2D Laplacian on 16 x 16, 8 cores
    X = Q.random_mps(8, 4, rng)
    return W, X, O.to_dense(O.contract("ij,j->i", W, X))


@pytest.mark.parametrize("spec", ["ij,j->i", "i,i->i"])
def test_two_core_full_rank_guess_reproduces_product(spec):
    """With a guess of full profile ranks every pair's super-core is the exact
    projection, so one sweep reproduces the product and the ranks fall to
    the product's own (the numerical ranks of its dense unfoldings)."""
    rng = np.random.default_rng(81)
    X = rand_tt(rng, [1, 2, 4, 5, 5, 4, 2, 1])
    A = rand_mpo(rng, [1, 3, 3, 3, 3, 3, 3, 1]) if spec == "ij,j->i" else rand_tt(rng, [1, 2, 2, 2, 2, 2, 2, 1])
    y = O.to_dense(O.contract(spec, A, X))
    G = rand_tt(rng, [1, 2, 4, 8, 8, 4, 2, 1])
    C, info = O.fit_two_core(spec, A, X, G, 1e-12, 0, 1, return_info=True)
    assert info["ranks"] == _dense_ranks(y, 2, 7)
    assert np.linalg.norm(O.to_dense(C) - y) <= 1e-13 * np.linalg.norm(y)


def test_two_core_grows_ranks_from_rank_one():
    """From a rank-1 guess the super-core splits raise the ranks: two sweeps
    reach the product's ranks and reproduce it."""
    W, X, y = _lap_case()
    G = Q.random_mps(8, 1, np.random.default_rng(2))
    C1, i1 = O.fit_two_core("ij,j->i", W, X, G, 1e-12, 0, 1, return_info=True)
    C2, i2 = O.fit_two_core("ij,j->i", W, X, G, 1e-12, 0, 2, return_info=True)
    want = _dense_ranks(y, 2, 8)
    assert max(i1["ranks"]) < max(want)  # one sweep is not enough from rank 1
    assert i2["ranks"] == want
    assert np.linalg.norm(O.to_dense(C2) - y) <= 1e-12 * np.linalg.norm(y)


@pytest.mark.parametrize("cap", [4, 8])
def test_two_core_rank_cap_and_final_pair_is_truncated_projection(cap):
    """Under a rank cap: ranks stay within it, the error never grows from
    sweep to sweep and is no larger than TT rounding's at the same cap, and
    the last pair equals the best rank-r approximation of the dense
    projection of the product onto the left interface of the other cores."""
    W, X, y = _lap_case()
    G = Q.random_mps(8, 64, np.random.default_rng(1))
    errs = []
    for ns in (1, 2, 3):
        C, info = O.fit_two_core("ij,j->i", W, X, G, 0.0, cap, ns, return_info=True)
        assert max(info["ranks"]) <= cap
        errs.append(np.linalg.norm(O.to_dense(C) - y) / np.linalg.norm(y))
    assert errs[1] <= errs[0] * (1 + 1e-12) and errs[2] <= errs[1] * (1 + 1e-12)
    e_round = np.linalg.norm(O.to_dense(O.round_tt(O.contract("ij,j->i", W, X), 0.0, cap)) - y) / np.linalg.norm(y)
    assert errs[2] <= e_round * (1 + 1e-12)
    # dense check of the last split (pair of cores 7, 8, right end)
    n = len(C)
    left = C[: n - 2]
    r = left[-1].shape[-1]
    # left interface: dense 2^(n-2) x r matrix of the left-orthonormal cores
    M = np.ones((1, 1))
    for c in left:
        M = np.einsum("xa,aib->xib", M, c).reshape(-1, c.shape[-1])
    assert np.allclose(M.T @ M, np.eye(r), atol=1e-12)
    # projection of the product, as the (r 2) x 2 unfolding of the pair
    S = (M.T @ y.reshape(M.shape[0], -1)).reshape(2 * r, 2)
    U, sg, Vt = np.linalg.svd(S, full_matrices=False)
    k = C[-1].shape[0]
    best = (U[:, :k] * sg[None, :k]) @ Vt[:k]
    pair = np.einsum("aib,bjc->aijc", C[-2], C[-1]).reshape(2 * r, 2)
    assert np.linalg.norm(pair - best) <= 1e-12 * np.linalg.norm(S)
