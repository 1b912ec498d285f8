"""Oracle pins for general digit bases (factorised dimensions, Sec. 2), CPU only.

A dimension of size N = b_1 b_2 ... b_n is split into digits i_q < b_q with
i = sum_q c_q i_q and c_q = prod_{r>q} b_r (eq. quantization, first digit
most significant).  Every check below builds its reference from that formula
directly, not from the oracle's own flattening.
"""
import itertools
import math

import numpy as np
import pytest

import oracle as O


def rand_tt(rng, ranks, bases):
    return [rng.standard_normal((ranks[k], bases[k], ranks[k + 1])) for k in range(len(bases))]


def rand_mpo(rng, ranks, bout, bin_):
    return [rng.standard_normal((ranks[k], bout[k], bin_[k], ranks[k + 1])) for k in range(len(bout))]


def factors(bases):
    return [math.prod(bases[q + 1:]) for q in range(len(bases))]


def brute_dense(cores, bases):
    c = factors(bases)
    out = np.zeros(math.prod(bases))
    for idx in itertools.product(*[range(b) for b in bases]):
        v = np.ones((1, 1))
        for k, i in enumerate(idx):
            v = v @ cores[k][:, i, :]
        out[sum(ci * i for ci, i in zip(c, idx))] = v[0, 0]
    return out


def brute_mpo(cores, bout, bin_):
    co, ci = factors(bout), factors(bin_)
    out = np.zeros((math.prod(bout), math.prod(bin_)))
    for ii in itertools.product(*[range(b) for b in bout]):
        for jj in itertools.product(*[range(b) for b in bin_]):
            v = np.ones((1, 1))
            for k in range(len(bout)):
                v = v @ cores[k][:, ii[k], jj[k], :]
            out[sum(a * b for a, b in zip(co, ii)), sum(a * b for a, b in zip(ci, jj))] = v[0, 0]
    return out


@pytest.mark.parametrize("bases", [[2, 2, 5], [2, 5, 2], [3, 3, 2, 4]])
def test_dense_flattening_follows_the_quantization_formula(bases):
    rng = np.random.default_rng(60)
    X = rand_tt(rng, [1] + [3] * (len(bases) - 1) + [1], bases)
    np.testing.assert_allclose(O.to_dense(X), brute_dense(X, bases), rtol=1e-13, atol=1e-13)


def test_exp_on_factorised_grid_is_rank_one():
    """exp(a i) = prod_q exp(a c_q i_q): one rank-1 core per digit, here for
    20 = 2 * 2 * 5 and 20 = 2 * 5 * 2 (the two factorisations of Sec. 2)."""
    a = 0.37
    for bases in ([2, 2, 5], [2, 5, 2]):
        c = factors(bases)
        X = [np.exp(a * c[q] * np.arange(b)).reshape(1, b, 1) for q, b in enumerate(bases)]
        np.testing.assert_allclose(O.to_dense(X), np.exp(a * np.arange(20)), rtol=1e-14)


def test_rectangular_mpo_and_products_against_dense():
    rng = np.random.default_rng(61)
    bout, bin_ = [3, 2, 5], [2, 4, 3]
    W = rand_mpo(rng, [1, 2, 3, 1], bout, bin_)
    np.testing.assert_allclose(O.mpo_to_dense(W), brute_mpo(W, bout, bin_), rtol=1e-13, atol=1e-13)
    X = rand_tt(rng, [1, 3, 2, 1], bin_)
    y = O.to_dense(O.contract("ij,j->i", W, X))
    np.testing.assert_allclose(y, brute_mpo(W, bout, bin_) @ brute_dense(X, bin_), rtol=1e-12, atol=1e-12)
    A = rand_tt(rng, [1, 2, 2, 1], bout)
    B = rand_tt(rng, [1, 3, 2, 1], bout)
    h = O.to_dense(O.contract("i,i->i", A, B))
    np.testing.assert_allclose(h, brute_dense(A, bout) * brute_dense(B, bout), rtol=1e-12, atol=1e-12)


def test_round_and_zipup_on_mixed_bases_against_dense_unfoldings():
    rng = np.random.default_rng(62)
    bases = [3, 2, 5, 2, 3, 4]
    X = rand_tt(rng, [1, 3, 6, 9, 7, 4, 1], bases)
    x = brute_dense(X, bases)
    Y, info = O.round_tt(X, 0.0, 0, return_info=True)
    np.testing.assert_allclose(O.to_dense(Y), x, rtol=0, atol=1e-12 * np.abs(x).max())
    for k in range(1, len(bases)):
        sv = np.linalg.svd(x.reshape(math.prod(bases[:k]), -1), compute_uv=False)
        m = min(len(sv), len(info.sigmas[k - 1]))
        np.testing.assert_allclose(info.sigmas[k - 1][:m], sv[:m], rtol=0, atol=1e-12 * sv[0])
    W = rand_mpo(rng, [1, 2, 2, 2, 2, 2, 1], bases, bases)
    for N in (1, 2):
        Z = O.zipup("ij,j->i", W, X, 0.0, ncores=N)
        ref = O.mpo_to_dense(W) @ x  # mpo_to_dense is pinned by brute force above
        np.testing.assert_allclose(O.to_dense(Z), ref, rtol=0, atol=1e-12 * np.abs(ref).max())
