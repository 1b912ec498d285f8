"""Pins of the oracle's decomposition ("zip-up") algorithm (Sec. 3.2), CPU only.

Each property is checked against something other than the oracle itself:
dense products built with numpy on tiny grids, a direct TT-SVD of the dense
tensor written out here, and the identity operator, for which the exact right
part of the product is a scaled orthonormal map, so that the singular values
and the error follow from the dense tensor's Schmidt values.
"""
import math

import numpy as np
import pytest

import oracle as O
import qtt_inputs as Q


def rand_tt(rng, ranks, d=2):
    return [rng.standard_normal((ranks[k], d, ranks[k + 1])) for k in range(len(ranks) - 1)]


def rand_mpo(rng, ranks):
    return [rng.standard_normal((ranks[k], 2, 2, ranks[k + 1])) for k in range(len(ranks) - 1)]


def identity_mpo(n):
    return [np.eye(2).reshape(1, 2, 2, 1).copy() for _ in range(n)]


def dense_product(spec, A, B):
    if spec == "ij,j->i":
        return O.mpo_to_dense(A) @ O.to_dense(B)
    return O.to_dense(A) * O.to_dense(B)


def dense_tt_svd(x, n, rel_tol):
    """Left-to-right TT-SVD of a dense vector of 2^n entries (Oseledets 2011,
    Alg. 1): ranks and the per-bond singular values of the remainders."""
    nrm = np.linalg.norm(x)
    delta = rel_tol * nrm / math.sqrt(n - 1)
    ranks, sigmas, tails = [1], [], []
    rem = x.reshape(1, -1)
    for k in range(n - 1):
        r0 = rem.shape[0]
        M = rem.reshape(r0 * 2, -1)
        U, S, Vt = np.linalg.svd(M, full_matrices=False)
        t2 = np.concatenate([np.cumsum((S * S)[::-1])[::-1], [0.0]])
        r = next(c for c in range(1, S.size + 1) if math.sqrt(t2[c]) <= delta)
        ranks.append(r)
        sigmas.append(S)
        tails.append(math.sqrt(t2[r]))
        rem = S[:r, None] * Vt[:r]
    ranks.append(1)
    return ranks, sigmas, tails


def left_orthonormal_error(cores):
    worst = 0.0
    for c in cores[:-1]:
        M = c.reshape(-1, c.shape[-1])
        worst = max(worst, np.abs(M.T @ M - np.eye(M.shape[1])).max())
    return worst


# ---------------------------------------------------------------- right sweep
@pytest.mark.parametrize("legs", [1, 2])
def test_orthogonalize_right_invariants(legs):
    rng = np.random.default_rng(31)
    ranks = [1, 2, 4, 7, 7, 4, 2, 1] if legs == 1 else [1, 3, 5, 5, 5, 3, 1]
    X = rand_tt(rng, ranks) if legs == 1 else rand_mpo(rng, ranks)
    Y, nrm = O.orthogonalize_right(X)
    for c in Y[1:]:
        G = c.reshape(c.shape[0], -1)
        assert np.abs(G @ G.T - np.eye(G.shape[0])).max() < 1e-13
    dense = O.to_dense if legs == 1 else O.mpo_to_dense
    np.testing.assert_allclose(dense(Y), dense(X), rtol=1e-12, atol=1e-12 * np.abs(dense(X)).max())
    assert abs(nrm - np.linalg.norm(dense(X))) <= 1e-13 * nrm
    # rank after the sweep = min(r_k, P * r'_{k+1}) from the right
    P = 2 ** legs
    expect = [1]
    for k in range(len(X) - 1, 0, -1):
        expect.insert(0, min(X[k].shape[0], P * expect[0]))
    assert O.ranks_of(Y) == [1] + expect


# ---------------------------------------------------------------- zip-up
@pytest.mark.parametrize("spec", ["ij,j->i", "i,i->i"])
@pytest.mark.parametrize("N", [1, 2, 3])
def test_zipup_without_truncation_is_exact(spec, N):
    rng = np.random.default_rng(32 + N)
    X = rand_tt(rng, [1, 2, 4, 6, 6, 4, 2, 1])
    A = rand_mpo(rng, [1, 3, 3, 3, 3, 3, 3, 1]) if spec == "ij,j->i" else rand_tt(rng, [1, 2, 3, 3, 3, 3, 2, 1])
    Z, info = O.zipup(spec, A, X, 0.0, ncores=N, return_info=True)
    ref = dense_product(spec, A, X)
    np.testing.assert_allclose(O.to_dense(Z), ref, rtol=0, atol=1e-13 * np.abs(ref).max())
    assert left_orthonormal_error(Z) < 1e-13
    assert info.err_bound == 0.0
    assert info.ranks[0] == 1 and info.ranks[-1] == 1


@pytest.mark.parametrize("spec", ["ij,j->i", "i,i->i"])
def test_zipup_full_supercore_is_dense_tt_svd(spec):
    """With N = n the super-core is the whole product: the algorithm reduces to
    a left-to-right TT-SVD of the dense tensor."""
    rng = np.random.default_rng(40)
    n = 8
    X = rand_tt(rng, [1, 2, 4, 8, 8, 8, 4, 2, 1])
    A = rand_mpo(rng, [1, 3, 3, 3, 3, 3, 3, 3, 1]) if spec == "ij,j->i" else rand_tt(rng, [1, 2, 2, 2, 2, 2, 2, 2, 1])
    ref = dense_product(spec, A, X)
    nref = np.linalg.norm(ref)
    for tol in [0.0, 1e-2, 1e-1]:
        Z, info = O.zipup(spec, A, X, tol, ncores=n, return_info=True)
        ranks, sigmas, tails = dense_tt_svd(ref, n, tol)
        assert abs(info.norm - nref) <= 1e-13 * nref
        for b in range(n - 1):
            m = min(len(sigmas[b]), len(info.sigmas[b]))
            np.testing.assert_allclose(info.sigmas[b][:m], sigmas[b][:m], rtol=0, atol=1e-12 * nref)
        if tol == 0.0:
            assert all(a >= b for a, b in zip(info.ranks, ranks))
            continue
        assert info.ranks == ranks
        err = np.linalg.norm(O.to_dense(Z) - ref)
        # TT-SVD errors are orthogonal: the error norm equals the discarded norm
        assert abs(err - info.err_bound) <= 1e-10 * nref
        assert info.err_bound <= tol * nref * (1 + 1e-12)


@pytest.mark.parametrize("N", [1, 2])
def test_zipup_identity_operator_exact_error(N):
    """I x with W_k = delta_ij.  The right sweep turns every operator core but
    the first into delta_ij / sqrt(2) and moves 2^((n-1)/2) into the first, so
    the exact part of the product to the right of a split made with q cores
    not yet absorbed is 2^(-q/2) times an orthonormal map: the super-core's
    singular values are the dense tensor's Schmidt values times 2^(q/2), each
    split is an exact truncated SVD, and the error is the orthogonal sum of
    the discarded norms scaled back by 2^(-q/2).  q = max(0, n - N - b) at
    bond b."""
    rng = np.random.default_rng(41 + N)
    n = 9
    X = O.tt_add(rand_tt(rng, [1] + [2] * (n - 1) + [1]),
                 rand_tt(rng, [1, 2, 4, 8, 8, 8, 8, 4, 2, 1]), 1.0, 1e-2)
    x = O.to_dense(X)
    nx = np.linalg.norm(x)
    scale = [2.0 ** (max(0, n - N - b) / 2) for b in range(n - 1)]
    _, sig0, _ = dense_tt_svd(x, n, 0.0)
    Z0, info0 = O.zipup("ij,j->i", identity_mpo(n), X, 0.0, ncores=N, return_info=True)
    assert abs(info0.norm - nx * 2.0 ** ((n - N) / 2)) <= 1e-13 * info0.norm
    np.testing.assert_allclose(O.to_dense(Z0), x, rtol=0, atol=1e-13 * np.abs(x).max())
    for b in range(n - 1):
        m = min(len(sig0[b]), len(info0.sigmas[b]))
        np.testing.assert_allclose(info0.sigmas[b][:m], scale[b] * sig0[b][:m], rtol=0, atol=1e-12 * info0.norm)
    truncated = False
    for tol in [3e-3, 3e-2, 3e-1]:
        Z, info = O.zipup("ij,j->i", identity_mpo(n), X, tol, ncores=N, return_info=True)
        err = np.linalg.norm(O.to_dense(Z) - x)
        expect = math.sqrt(sum((t / s) ** 2 for t, s in zip(info.tails, scale)))
        assert abs(err - expect) <= 1e-10 * nx
        truncated |= err > 1e-8 * nx
        assert left_orthonormal_error(Z) < 1e-12
    assert truncated


def test_zipup_max_rank_caps_every_bond():
    rng = np.random.default_rng(45)
    X = rand_tt(rng, [1, 2, 4, 8, 8, 4, 2, 1])
    W = rand_mpo(rng, [1, 3, 3, 3, 3, 3, 3, 1])
    Z, info = O.zipup("ij,j->i", W, X, 0.0, max_rank=5, ncores=2, return_info=True)
    assert max(info.ranks) <= 5 and any(info.maxrank_hit)
    for b, hit in enumerate(info.maxrank_hit):
        if hit:
            assert info.tails[b] > 0


def test_zipup_laplacian_error_near_tolerance():
    """On the paper's structured operator (the Laplacian MPO, Sec. 4.2) the
    zip-up result stays within a small multiple of the requested tolerance of
    the exact product."""
    W = Q.laplacian_mpo(5, 2)
    rng = np.random.default_rng(46)
    n = len(W)
    X = rand_tt(rng, [min(8, 2 ** k, 2 ** (n - k)) for k in range(n + 1)])
    ref = dense_product("ij,j->i", W, X)
    nref = np.linalg.norm(ref)
    for N in (1, 2):
        for tol in (1e-3, 1e-6):
            Z, info = O.zipup("ij,j->i", W, X, tol, ncores=N, return_info=True)
            err = np.linalg.norm(O.to_dense(Z) - ref)
            assert err <= 4 * tol * nref, (N, tol, err / nref)


def test_zipup_and_fit_on_closed_form_products():
    """exp(a x) exp(b x) = exp((a+b) x) and sin(x) cos(x) = sin(2x)/2 (the
    closed forms of Sec. 4.1) through the decomposition algorithm and one
    variational sweep from its result: the closed-form values and ranks."""
    n = 12
    e1, e2 = Q.exp_qtt(n, 0.7), Q.exp_qtt(n, -1.9)
    ref = O.to_dense(Q.exp_qtt(n, 0.7 - 1.9))
    for N in (1, 2):
        Z = O.zipup("i,i->i", e1, e2, 1e-12, 0, ncores=N)
        assert max(O.ranks_of(Z)) == 1
        np.testing.assert_allclose(O.to_dense(Z), ref, rtol=1e-12)
    s = Q.trig_qtt(n, 1.3, 0.0, "sin")
    c = Q.trig_qtt(n, 1.3, 0.0, "cos")
    ref2 = 0.5 * O.to_dense(Q.trig_qtt(n, 2.6, 0.0, "sin"))
    Z = O.zipup("i,i->i", s, c, 1e-12, 0, ncores=1)
    # one-core super-cores can keep more than the minimal rank near the right
    # end (the exact right part is not orthonormal); rounding finds rank 2
    assert max(O.ranks_of(Z)) <= 4 and max(O.ranks_of(O.round_tt(Z, 1e-12))) == 2
    np.testing.assert_allclose(O.to_dense(Z), ref2, rtol=0, atol=1e-12 * np.abs(ref2).max())
    F = O.fit("i,i->i", s, c, Z, nsweeps=1)
    np.testing.assert_allclose(O.to_dense(F), ref2, rtol=0, atol=1e-12 * np.abs(ref2).max())
