"""Pins of the oracle's variational fitting (Sec. 3.3, eq. variational), CPU only.

The checks use dense vectors on tiny grids: the updated centre core is the
exact minimiser (the dense gradient of ||C - Y||^2 with respect to it
vanishes), the error never grows from sweep to sweep, full ranks reproduce
the product exactly, and the fit improves on the decomposition algorithm's
result it starts from.
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
