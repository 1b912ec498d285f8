"""Pins of the FP64 oracle against things other than itself (CPU only).

Each test ties an oracle function to a brute-force dense computation, a
closed form the paper gives (Sec. 4) or a mathematical invariant, chosen so
that a dropped term, a wrong sign/index or a transposed operand fails one.
"""
import itertools
import math

import numpy as np
import pytest

import oracle as O
import qtt_inputs as Q


def rand_tt(rng, ranks, d=2):
    return [rng.standard_normal((ranks[k], d, ranks[k + 1])) for k in range(len(ranks) - 1)]


def brute_dense(cores):
    """Entry-by-entry product of core slices (independent of to_dense)."""
    n = len(cores)
    out = np.zeros(2 ** n)
    for idx in itertools.product(range(2), repeat=n):
        v = np.ones((1, 1))
        for k, i in enumerate(idx):
            v = v @ cores[k][:, i, :]
        flat = 0
        for i in idx:
            flat = 2 * flat + i
        out[flat] = v[0, 0]
    return out


def brute_mpo_dense(cores):
    n = len(cores)
    N = 2 ** n
    out = np.zeros((N, N))
    for ii in itertools.product(range(2), repeat=n):
        for jj in itertools.product(range(2), repeat=n):
            v = np.ones((1, 1))
            for k in range(n):
                v = v @ cores[k][:, ii[k], jj[k], :]
            fi = int("".join(map(str, ii)), 2)
            fj = int("".join(map(str, jj)), 2)
            out[fi, fj] = v[0, 0]
    return out


# ---------------------------------------------------------------- dense helpers
def test_to_dense_matches_brute_force():
    rng = np.random.default_rng(11)
    X = rand_tt(rng, [1, 2, 3, 3, 2, 1])
    np.testing.assert_allclose(O.to_dense(X), brute_dense(X), rtol=1e-13, atol=1e-13)


def test_mpo_to_dense_matches_brute_force():
    rng = np.random.default_rng(12)
    W = [rng.standard_normal((r0, 2, 2, r1)) for r0, r1 in [(1, 3), (3, 2), (2, 1)]]
    np.testing.assert_allclose(O.mpo_to_dense(W), brute_mpo_dense(W), rtol=1e-13, atol=1e-13)


# ---------------------------------------------------------------- closed forms (Sec. 4.1)
def test_sin_qtt_values_on_unit_grid():
    n = 10
    N = 2 ** n
    x = np.arange(N) / (N - 1)  # end point included (Sec. 2, uniform grid)
    f = Q.sin_unit_interval(n)
    assert O.ranks_of(f) == [1] + [2] * (n - 1) + [1]
    np.testing.assert_allclose(O.to_dense(f), np.sin(2 * np.pi * x), atol=2e-15)


@pytest.mark.parametrize("kind", ["sin", "cos"])
def test_trig_qtt_general_argument(kind):
    n = 9
    v, ph = 0.0137, 0.71
    i = np.arange(2 ** n)
    ref = np.sin(v * i + ph) if kind == "sin" else np.cos(v * i + ph)
    np.testing.assert_allclose(O.to_dense(Q.trig_qtt(n, v, ph, kind)), ref, atol=3e-15)


def test_exp_qtt_rank1_values():
    n = 8
    N = 2 ** n
    x = -1.0 + 2.0 * np.arange(N) / (N - 1)
    f = Q.exp_qtt(n, 0.7, -1.0, 1.0, 0.3)
    assert O.ranks_of(f) == [1] * (n + 1)
    np.testing.assert_allclose(O.to_dense(f), np.exp(0.7 * (x - 0.3)), rtol=1e-14)


def test_poly_qtt_values_and_rank():
    n = 8
    N = 2 ** n
    x = -1.0 + 2.0 * np.arange(N) / (N - 1)
    coeffs = [0.1, 0.0, 1.0, -0.5]
    f = Q.poly_qtt(n, coeffs, -1.0, 1.0, 0.5)
    ref = sum(c * (x - 0.5) ** s for s, c in enumerate(coeffs))
    np.testing.assert_allclose(O.to_dense(f), ref, atol=1e-13)
    assert max(O.ranks_of(f)) == len(coeffs)


# ---------------------------------------------------------------- shift / Laplacian (Sec. 4.2)
@pytest.mark.parametrize("n", [2, 3, 4])
def test_paper_shift_recursion_is_dense_shift(n):
    N = 2 ** n
    for d in range(N):
        W = O.shift_mpo_paper(n, d)
        np.testing.assert_array_equal(O.mpo_to_dense(W), O.dense_shift(N, d))


@pytest.mark.parametrize("m,D", [(4, 1), (6, 1), (3, 2), (2, 3)])
def test_laplacian_mpo_is_kronecker_sum(m, D):
    W = Q.laplacian_mpo(m, D)
    dense_tt = O.mpo_to_dense(W)
    perm = O.interleaved_index(m, D)
    ref = O.dense_laplacian(m, D)[np.ix_(perm, perm)]
    np.testing.assert_array_equal(dense_tt, ref)


@pytest.mark.parametrize("D,rank", [(1, 3), (2, 5), (3, 7)])
def test_laplacian_interior_rank(D, rank):
    W = Q.laplacian_mpo(5, D)
    r = O.ranks_of(W)
    assert max(r) == rank
    assert r[0] == r[-1] == 1


def test_laplacian_from_paper_shift_tt():
    """2I - Q_1 - Q_1^T assembled from the paper's shift TT equals the Laplacian MPO."""
    n = 5
    Qs = O.shift_mpo_paper(n, 1)
    Qt = [c.transpose(0, 2, 1, 3).copy() for c in Qs]
    eye = [np.eye(2).reshape(1, 2, 2, 1) for _ in range(n)]

    def add_mpo(A, B, a, b):
        A3 = [c.reshape(c.shape[0], 4, c.shape[-1]) for c in A]
        B3 = [c.reshape(c.shape[0], 4, c.shape[-1]) for c in B]
        S = O.tt_add(A3, B3, a, b)
        return [c.reshape(c.shape[0], 2, 2, c.shape[-1]) for c in S]

    L = add_mpo(add_mpo(eye, Qs, 2.0, -1.0), Qt, 1.0, -1.0)
    np.testing.assert_array_equal(O.mpo_to_dense(L), O.mpo_to_dense(Q.laplacian_mpo(n, 1)))


# ---------------------------------------------------------------- contraction (eq. einsum)
def test_hadamard_matches_dense_product():
    rng = np.random.default_rng(3)
    A = rand_tt(rng, [1, 2, 3, 4, 3, 2, 1])
    B = rand_tt(rng, [1, 2, 2, 3, 2, 2, 1])
    C = O.contract("i,i->i", A, B)
    assert O.ranks_of(C) == [a * b for a, b in zip(O.ranks_of(A), O.ranks_of(B))]
    np.testing.assert_allclose(O.to_dense(C), O.to_dense(A) * O.to_dense(B), rtol=1e-12, atol=1e-12)


def test_mpo_mps_matches_dense_matvec():
    rng = np.random.default_rng(4)
    W = [rng.standard_normal((r0, 2, 2, r1)) for r0, r1 in [(1, 2), (2, 3), (3, 3), (3, 2), (2, 1)]]
    X = rand_tt(rng, [1, 2, 4, 4, 2, 1])
    C = O.contract("ij,j->i", W, X)
    np.testing.assert_allclose(O.to_dense(C), O.mpo_to_dense(W) @ O.to_dense(X), rtol=1e-12, atol=1e-12)


def test_mpo_not_transposed():
    """A non-symmetric MPO (the shift) distinguishes A x from A^T x."""
    W = O.shift_mpo_paper(4, 1)
    x = np.arange(16, dtype=float)
    X = [c for c in Q.poly_qtt(4, [0.0, 15.0], 0.0, 1.0)]  # x(i) = i
    np.testing.assert_allclose(O.to_dense(X), x, atol=1e-13)
    y = O.to_dense(O.contract("ij,j->i", W, X))
    np.testing.assert_allclose(y, np.concatenate([[0.0], x[:-1]]), atol=1e-12)


# ---------------------------------------------------------------- orthogonalisation
def test_orthogonalize_invariants():
    rng = np.random.default_rng(5)
    X = rand_tt(rng, [1, 2, 4, 7, 7, 4, 2, 1])
    Y, nrm = O.orthogonalize(X)
    for c in Y[:-1]:
        M = c.reshape(-1, c.shape[-1])
        assert np.abs(M.T @ M - np.eye(M.shape[1])).max() < 1e-13
    np.testing.assert_allclose(O.to_dense(Y), O.to_dense(X), rtol=1e-12, atol=1e-12)
    assert abs(nrm - np.linalg.norm(O.to_dense(X))) <= 1e-13 * nrm
    # rank after QR = min(d * r'_{k-1}, r_k)
    expect = [1]
    for k in range(len(X)):
        expect.append(min(2 * expect[-1], X[k].shape[-1]))
    assert O.ranks_of(Y) == expect


def test_orthogonalize_rank_deficient_unfolding():
    rng = np.random.default_rng(6)
    X = rand_tt(rng, [1, 2, 2, 1])
    # duplicate a bond: core0 -> [c, c], core1 -> [c1; 0] keeps the tensor but adds a null direction
    X2 = [np.concatenate([X[0], X[0]], axis=2), np.concatenate([X[1], np.zeros_like(X[1])], axis=0), X[2]]
    Y, _ = O.orthogonalize(X2)
    M = Y[0].reshape(-1, Y[0].shape[-1])
    assert np.abs(M.T @ M - np.eye(M.shape[1])).max() < 1e-13
    np.testing.assert_allclose(O.to_dense(Y), O.to_dense(X), atol=1e-13)


# ---------------------------------------------------------------- rounding
def test_truncation_rank_by_definition():
    s = np.array([3.0, 2.0, 1.0, 0.5, 0.25])
    # tails: r=1: sqrt(4+1+.25+.0625), r=2: sqrt(1.3125), r=3: sqrt(.3125), r=4: .25, r=5: 0
    assert O.truncation_rank(s, 0.25, 0)[0] == 4            # equality truncates
    assert O.truncation_rank(s, 0.2499, 0)[0] == 5
    assert O.truncation_rank(s, math.sqrt(0.3125), 0)[0] == 3
    assert O.truncation_rank(s, 100.0, 0)[0] == 1           # never below 1
    assert O.truncation_rank(s, 0.0, 2) == (2, math.sqrt(1.3125), math.sqrt(5.3125), True)


def test_round_tol0_returns_same_tensor_and_dense_sigmas():
    rng = np.random.default_rng(7)
    X = rand_tt(rng, [1, 2, 4, 5, 4, 2, 1])
    Y, info = O.round_tt(X, 0.0, 0, return_info=True)
    np.testing.assert_allclose(O.to_dense(Y), O.to_dense(X), rtol=1e-12, atol=1e-12)
    dense = O.to_dense(X)
    n = len(X)
    for k in range(1, n):
        unf = dense.reshape(2 ** k, -1)
        sv = np.linalg.svd(unf, compute_uv=False)
        got = info.sigmas[k - 1]
        m = min(len(got), len(sv))
        np.testing.assert_allclose(got[:m], sv[:m], rtol=1e-10, atol=1e-12 * sv[0])
        # dense unfolding rank equals the untruncated rounded rank
        assert np.sum(sv > 1e-10 * sv[0]) <= info.ranks[k]


def test_round_error_bound_and_idempotence():
    rng = np.random.default_rng(8)
    A = rand_tt(rng, [1, 2, 2, 2, 2, 2, 2, 2, 1])
    B = rand_tt(rng, [1, 2, 4, 8, 8, 8, 4, 2, 1])
    X = O.tt_add(A, B, 1.0, 3e-3)
    dense = O.to_dense(X)
    nx = np.linalg.norm(dense)
    truncated = False
    for tol in [1e-1, 3e-2, 1e-3, 1e-4]:
        Y, info = O.round_tt(X, tol, 0, return_info=True)
        truncated |= info.err_bound > 0
        err = np.linalg.norm(O.to_dense(Y) - dense)
        assert err <= info.err_bound * (1 + 1e-10) + 1e-13 * nx
        assert info.err_bound <= tol * nx * (1 + 1e-12)
        Z0 = O.round_tt(Y, 0.0, 0)
        assert O.ranks_of(Z0) == info.ranks  # rounding a rounded TT keeps its ranks
        Z1, info1 = O.round_tt(Y, tol, 0, return_info=True)
        assert all(a <= b for a, b in zip(info1.ranks, info.ranks))
    assert truncated


def test_round_max_rank_is_best_rank_r_at_last_bond():
    """The first SVD of the sweep is an exact truncated SVD of the dense unfolding."""
    rng = np.random.default_rng(9)
    X = rand_tt(rng, [1, 2, 4, 8, 4, 2, 1])
    n = len(X)
    Y, info = O.round_tt(X, 0.0, 3, return_info=True)
    dense = O.to_dense(X)
    sv = np.linalg.svd(dense.reshape(2 ** (n - 1), 2), compute_uv=False)
    np.testing.assert_allclose(info.sigmas[-1], sv, rtol=1e-12)
    assert max(info.ranks) <= 3
    assert any(info.maxrank_hit)


def test_sin_noise_1d_ranks_and_dense_error():
    w = Q.sin_noise_1d()
    C = O.contract(w.spec, w.a, w.b)
    Y, info = O.round_tt(C, w.rel_tol, 0, return_info=True)
    assert info.ranks == [1, 2, 4, 8, 8, 8, 8, 8, 4, 2, 1]
    ref = O.to_dense(w.a) * O.to_dense(w.b)
    assert np.linalg.norm(O.to_dense(Y) - ref) <= 1e-14 * np.linalg.norm(ref)


def test_closed_form_products_round_to_known_ranks():
    n = 10
    N = 2 ** n
    x = np.arange(N) / (N - 1)
    v = 2 * np.pi / (N - 1)
    s = Q.trig_qtt(n, v, 0.0, "sin")
    c = Q.trig_qtt(n, v, 0.0, "cos")
    sc = O.round_tt(O.contract("i,i->i", s, c), 1e-13)
    assert max(O.ranks_of(sc)) == 2
    np.testing.assert_allclose(O.to_dense(sc), 0.5 * np.sin(4 * np.pi * x), atol=5e-15)
    ss = O.round_tt(O.contract("i,i->i", s, s), 1e-13)
    assert max(O.ranks_of(ss)) == 3
    e = Q.exp_qtt(n, 1.3)
    ee = O.round_tt(O.contract("i,i->i", e, e), 1e-13)
    assert max(O.ranks_of(ee)) == 1
    np.testing.assert_allclose(O.to_dense(ee), np.exp(2.6 * x), rtol=1e-13)
    p2 = Q.poly_qtt(n, [0.0, 0.0, 1.0])
    p3 = Q.poly_qtt(n, [0.0, 0.0, 0.0, 1.0])
    pp = O.round_tt(O.contract("i,i->i", p2, p3), 1e-13)
    assert max(O.ranks_of(pp)) == 6  # degree 5
    np.testing.assert_allclose(O.to_dense(pp), x ** 5, atol=1e-13)


def _sin_mode(m, k):
    """f(i) = sin(pi k (i+1) / (N+1)), an eigenvector of the 1D Dirichlet stencil."""
    N = 2 ** m
    w = math.pi * k / (N + 1)
    return Q.trig_qtt(m, w, w, "sin"), 2.0 - 2.0 * math.cos(w)


@pytest.mark.parametrize("m,D", [(10, 1), (16, 2), (14, 3)])
def test_laplacian_eigenvector_rounds_to_rank_2D(m, D):
    """Delta f = lambda f for a product of high-frequency sine modes, at full size."""
    N = 2 ** m
    modes = [N // 3, N // 2 - 1, N // 3 + 5][:D]
    f = None
    lam = 0.0
    for a in range(D):
        fa, la = _sin_mode(m, modes[a])
        lam += la
        ea = Q.embed_axis(fa, D, a)
        f = ea if f is None else O.contract("i,i->i", f, ea)
    W = Q.laplacian_mpo(m, D)
    y = O.round_tt(O.contract("ij,j->i", W, f), 1e-12)
    assert max(O.ranks_of(y)) == 2 ** D
    assert O.rel_error(y, O.tt_scale(f, lam)) < 1e-12


# ---------------------------------------------------------------- inner products
def test_inner_closed_forms():
    n = 12
    N = 2 ** n
    x = np.arange(N) / (N - 1)
    s = Q.sin_unit_interval(n)
    assert abs(O.inner(s, s) - np.sum(np.sin(2 * np.pi * x) ** 2)) < 1e-11
    e = Q.exp_qtt(n, 0.5)
    t = 2 * 0.5 / (N - 1)
    geo = math.expm1(t * N) / math.expm1(t)  # sum_i q^i, q = e^t, without cancellation
    assert abs(O.inner(e, e) - geo) <= 1e-13 * geo


def test_inner_matches_dense_and_norm():
    rng = np.random.default_rng(10)
    A = rand_tt(rng, [1, 2, 3, 3, 2, 1])
    B = rand_tt(rng, [1, 2, 4, 2, 2, 1])
    assert abs(O.inner(A, B) - O.to_dense(A) @ O.to_dense(B)) < 1e-12
    assert abs(O.norm(A) - math.sqrt(O.inner(A, A))) < 1e-12 * O.norm(A)
    assert abs(O.inner(A, B)) <= O.norm(A) * O.norm(B)


def test_rel_error_matches_dense():
    rng = np.random.default_rng(13)
    A = rand_tt(rng, [1, 2, 3, 2, 1])
    B = [c + 1e-9 * rng.standard_normal(c.shape) for c in A]
    d = np.linalg.norm(O.to_dense(A) - O.to_dense(B)) / np.linalg.norm(O.to_dense(B))
    assert abs(O.rel_error(A, B) - d) <= 1e-6 * d


# ---------------------------------------------------------------- gradients
def _small_grad_problem(seed=14):
    rng = np.random.default_rng(seed)
    W = Q.laplacian_mpo(2, 2)
    W[1] = W[1] + 0.3 * rng.standard_normal(W[1].shape)  # break symmetry
    x = Q.random_mps(4, 3, rng)
    b = Q.random_mps(4, 2, rng)
    return W, x, b


def test_inner_grad_dense():
    rng = np.random.default_rng(15)
    A = rand_tt(rng, [1, 2, 3, 2, 1])
    B = rand_tt(rng, [1, 2, 2, 2, 1])
    g = O.inner_grad(A, B)
    h = 1e-6
    for k in range(len(A)):
        for idx in [(0, 0, 0), tuple(s - 1 for s in A[k].shape)]:
            Ap = [c.copy() for c in A]
            Am = [c.copy() for c in A]
            Ap[k][idx] += h
            Am[k][idx] -= h
            fd = (O.inner(Ap, B) - O.inner(Am, B)) / (2 * h)
            assert abs(fd - g[k][idx]) < 1e-8 * (1 + abs(fd))


def test_grad_axb_finite_differences_and_routes():
    W, x, b = _small_grad_problem()
    g1 = O.grad_axb(W, x, b)
    g2 = O.grad_axb_sandwich(W, x, b)
    dense = O.mpo_to_dense(W)
    L0 = np.sum((dense @ O.to_dense(x) - O.to_dense(b)) ** 2)
    assert abs(O.loss_axb(W, x, b) - L0) < 1e-12 * (1 + L0)
    h = 1e-6
    for k in range(len(x)):
        np.testing.assert_allclose(g1[k], g2[k], rtol=1e-11, atol=1e-11)
        for idx in itertools.product(*[range(s) for s in x[k].shape]):
            xp = [c.copy() for c in x]
            xm = [c.copy() for c in x]
            xp[k][idx] += h
            xm[k][idx] -= h
            Lp = np.sum((dense @ O.to_dense(xp) - O.to_dense(b)) ** 2)
            Lm = np.sum((dense @ O.to_dense(xm) - O.to_dense(b)) ** 2)
            fd = (Lp - Lm) / (2 * h)
            assert abs(fd - g1[k][idx]) < 1e-7 * (1 + abs(fd))


def test_grad_euler_identity():
    W, x, b = _small_grad_problem(16)
    g = O.grad_axb(W, x, b)
    y = O.contract("ij,j->i", W, x)
    rhs = 2 * O.inner(y, y) - 2 * O.inner(y, b)
    for k in range(len(x)):
        assert abs(np.sum(g[k] * x[k]) - rhs) < 1e-11 * (1 + abs(rhs))


@pytest.mark.parametrize("spec", ["ij,j->i", "i,i->i"])
def test_contract_grad_is_the_adjoint_of_contract(spec):
    """contract_grad's dW and dX against the definition of a gradient.

    The product is bilinear in (W, X), so for any direction D the central
    difference <G, C(W + hD, X)> - <G, C(W - hD, X)> equals 2h <dW, D> with no
    truncation error, and likewise for X; C here is the contraction written
    out entry by entry from eq. einsum (independent of contract()).  A
    transposed index or a swapped operand in either output fails it."""
    rng = np.random.default_rng(41)
    if spec == "ij,j->i":
        W = [rng.standard_normal(s) for s in [(1, 2, 3, 3), (3, 2, 3, 2), (2, 3, 2, 1)]]
        X = [rng.standard_normal(s) for s in [(1, 3, 2), (2, 3, 4), (4, 2, 1)]]
    else:
        W = [rng.standard_normal(s) for s in [(1, 2, 3), (3, 3, 2), (2, 2, 1)]]
        X = [rng.standard_normal(s) for s in [(1, 2, 2), (2, 3, 4), (4, 2, 1)]]

    def core_product(w, x):
        # C[(mu,nu), i, (mu',nu')] = sum_j W[mu,i,j,mu'] X[nu,j,nu'] (or W[mu,i,mu'] X[nu,i,nu'])
        if spec == "ij,j->i":
            ra, di, dj, rb = w.shape
        else:
            ra, di, rb = w.shape
            dj = di
        rc, _, rd = x.shape
        c = np.zeros((ra * rc, di, rb * rd))
        for mu, nu, i, mu2, nu2 in itertools.product(range(ra), range(rc), range(di), range(rb), range(rd)):
            if spec == "ij,j->i":
                v = sum(w[mu, i, j, mu2] * x[nu, j, nu2] for j in range(dj))
            else:
                v = w[mu, i, mu2] * x[nu, i, nu2]
            c[mu * rc + nu, i, mu2 * rd + nu2] = v
        return c

    G = [rng.standard_normal(core_product(w, x).shape) for w, x in zip(W, X)]
    dW, dX = O.contract_grad(spec, W, X, G)
    h = 0.37  # any step: the pairing is linear in each operand
    for k in range(len(W)):
        assert dW[k].shape == W[k].shape and dX[k].shape == X[k].shape
        for _ in range(3):
            D = rng.standard_normal(W[k].shape)
            lhs = np.sum(G[k] * core_product(W[k] + h * D, X[k])) - np.sum(G[k] * core_product(W[k] - h * D, X[k]))
            assert abs(lhs - 2 * h * np.sum(dW[k] * D)) <= 1e-12 * max(1.0, abs(lhs))
            E = rng.standard_normal(X[k].shape)
            lhs = np.sum(G[k] * core_product(W[k], X[k] + h * E)) - np.sum(G[k] * core_product(W[k], X[k] - h * E))
            assert abs(lhs - 2 * h * np.sum(dX[k] * E)) <= 1e-12 * max(1.0, abs(lhs))


def _two_core_with_sigmas(rng, s, d=16):
    """X = U diag(s) V^T as a two-core train: the bond's singular values are s."""
    U, _ = np.linalg.qr(rng.standard_normal((d, len(s))))
    V, _ = np.linalg.qr(rng.standard_normal((d, len(s))))
    return [U.reshape(1, d, len(s)), (np.diag(s) @ V.T).reshape(len(s), d, 1)]


@pytest.mark.parametrize("g", [0.5, 1e-2, 1e-4])
def test_cut_gap_is_the_constructed_gap(g):
    rng = np.random.default_rng(42)
    s = np.array([1.0, 0.5, 0.5 * (1.0 - g), 0.1])
    X = _two_core_with_sigmas(rng, s)
    _, info = O.round_tt(X, 0.0, 2, return_info=True)
    assert info.ranks == [1, 2, 1]
    assert np.allclose(info.sigmas[0], s, rtol=0, atol=1e-15)
    assert abs(info.gaps[0] - g) <= 1e-12
    # nothing discarded: no cut, no gap
    _, info = O.round_tt(X, 0.0, 0, return_info=True)
    assert info.ranks == [1, 4, 1] and info.gaps == [math.inf]


def test_noise_amplification_follows_the_gap():
    """Wide gap: the rounded tensor moves by about the input change.  Narrow
    gap: the kept pair of singular vectors rotates by about eps / gap, so the
    ratio grows like 1 / gap (Wedin)."""
    rng = np.random.default_rng(43)
    wide = _two_core_with_sigmas(rng, np.array([1.0, 0.5, 0.25, 0.1]))
    amp, ratios = O.noise_amplification(wide, 0.0, 2, eps=1e-9, seed=1, trials=4)
    assert 0.3 <= min(ratios) and amp <= 3.0
    g = 1e-4
    narrow = _two_core_with_sigmas(rng, np.array([1.0, 0.5, 0.5 * (1.0 - g), 0.1]))
    amp, _ = O.noise_amplification(narrow, 0.0, 2, eps=1e-9, seed=1, trials=4)
    assert amp >= 0.01 / g
    # no truncation: rounding is the identity on the tensor, ratio 1
    amp, ratios = O.noise_amplification(wide, 0.0, 0, eps=1e-9, seed=1, trials=2)
    assert all(abs(r - 1.0) <= 1e-4 for r in ratios)
