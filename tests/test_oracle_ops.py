"""Oracle pins for exact addition of many trains and the operator product
'ij,jk->ik' (Sec. 3.1), CPU only: dense linear algebra on tiny grids and the
paper's shift matrices (Sec. 4.2), whose products are shifts again."""
import numpy as np
import pytest

import oracle as O


def rand_tt(rng, ranks, d=2):
    return [rng.standard_normal((ranks[k], d, ranks[k + 1])) for k in range(len(ranks) - 1)]


def rand_mpo(rng, ranks, dout, din):
    return [rng.standard_normal((ranks[k], dout[k], din[k], ranks[k + 1])) for k in range(len(dout))]


def test_tt_sum_is_the_dense_linear_combination():
    rng = np.random.default_rng(70)
    terms = [rand_tt(rng, r) for r in ([1, 2, 4, 3, 1], [1, 1, 1, 1, 1], [1, 2, 2, 2, 1], [1, 2, 3, 2, 1])]
    coeffs = [0.5, -2.0, 3.25, 1e-3]
    S = O.tt_sum(terms, coeffs)
    ref = sum(c * O.to_dense(t) for c, t in zip(coeffs, terms))
    np.testing.assert_allclose(O.to_dense(S), ref, rtol=0, atol=1e-14 * np.abs(ref).max())
    # interior ranks add up, the boundary ranks stay 1
    assert O.ranks_of(S) == [1, 7, 10, 8, 1]
    # one core: the plain weighted sum
    one = [[rng.standard_normal((1, 3, 1))] for _ in range(3)]
    s1 = O.tt_sum(one, [1.0, -1.0, 2.0])
    np.testing.assert_allclose(s1[0], one[0][0] - one[1][0] + 2.0 * one[2][0], rtol=1e-15)


def test_sum_then_round_recovers_a_low_rank_sum():
    """X + X - X = X: the exact sum has triple rank, rounding returns X's ranks."""
    rng = np.random.default_rng(71)
    X = rand_tt(rng, [1, 2, 4, 5, 4, 2, 1])
    S = O.tt_sum([X, X, X], [1.0, 1.0, -1.0])
    Y, info = O.round_tt(S, 1e-12, 0, return_info=True)
    assert info.ranks == O.round_tt(X, 1e-12, 0, return_info=True)[1].ranks
    assert O.rel_error(Y, X) <= 1e-12


def test_operator_product_is_the_dense_matrix_product():
    rng = np.random.default_rng(72)
    dout, dmid, din = [2, 3, 2], [3, 2, 4], [2, 2, 5]
    A = rand_mpo(rng, [1, 3, 2, 1], dout, dmid)
    B = rand_mpo(rng, [1, 2, 4, 1], dmid, din)
    C = O.contract("ij,jk->ik", A, B)
    assert [c.shape for c in C] == [(1, 2, 2, 6), (6, 3, 2, 8), (8, 2, 5, 1)]
    np.testing.assert_allclose(O.mpo_to_dense(C), O.mpo_to_dense(A) @ O.mpo_to_dense(B), rtol=1e-12, atol=1e-12)


@pytest.mark.parametrize("n,d1,d2", [(6, 1, 1), (6, 1, 3), (7, 5, 2)])
def test_shift_products_are_shifts(n, d1, d2):
    """Q^N_{d1} Q^N_{d2} = Q^N_{d1+d2} (Sec. 4.2): the operator product of the
    paper's shift trains rounds to the shift train of the summed distance."""
    N = 2 ** n
    P = O.contract("ij,jk->ik", O.shift_mpo_paper(n, d1), O.shift_mpo_paper(n, d2))
    dense = O.mpo_to_dense(P)
    np.testing.assert_array_equal(dense, O.dense_shift(N, d1 + d2))
    flat = [c.reshape(c.shape[0], 4, c.shape[-1]) for c in P]
    R = O.round_tt(flat, 1e-13, 0)
    ref = O.shift_mpo_paper(n, d1 + d2)
    ref_rank = max(O.ranks_of(O.round_tt([c.reshape(c.shape[0], 4, c.shape[-1]) for c in ref], 1e-13, 0)))
    assert max(O.ranks_of(R)) == ref_rank
    back = [c.reshape(c.shape[0], 2, 2, c.shape[-1]) for c in R]
    np.testing.assert_allclose(O.mpo_to_dense(back), O.dense_shift(N, d1 + d2), atol=1e-12)


def test_laplacian_squared_against_dense():
    import qtt_inputs as Q
    W = Q.laplacian_mpo(4, 2)
    P = O.contract("ij,jk->ik", W, W)
    perm = O.interleaved_index(4, 2)  # train index (interleaved digits) -> grid index
    L = O.dense_laplacian(4, 2)[np.ix_(perm, perm)]
    np.testing.assert_array_equal(O.mpo_to_dense(P), L @ L)


def test_tt_sum_of_operators_is_the_dense_matrix_sum():
    rng = np.random.default_rng(73)
    W1 = rand_mpo(rng, [1, 3, 2, 1], [2, 3, 2], [2, 2, 4])
    W2 = rand_mpo(rng, [1, 2, 4, 1], [2, 3, 2], [2, 2, 4])
    S = O.tt_sum([W1, W2], [2.0, -0.5])
    np.testing.assert_allclose(O.mpo_to_dense(S), 2.0 * O.mpo_to_dense(W1) - 0.5 * O.mpo_to_dense(W2),
                               rtol=0, atol=1e-13)
