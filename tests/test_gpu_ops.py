"""GPU parity for the exact sum of many trains and the operator product
'ij,jk->ik' (Sec. 3.1), each followed by rounding, against the FP64 oracle."""
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


def dev(cores, dtype=torch.float64):
    return Q.to_device(cores, DEV, dtype)


def host(cores):
    return Q.to_host(cores)


def rand_tt(rng, ranks, d=2):
    return [rng.standard_normal((ranks[k], d, ranks[k + 1])) for k in range(len(ranks) - 1)]


def rand_mpo(rng, ranks, dout, din):
    return [rng.standard_normal((ranks[k], dout[k], din[k], ranks[k + 1])) for k in range(len(dout))]


def as_mps(cores):
    return [c.reshape(c.shape[0], -1, c.shape[-1]) for c in cores]


@pytest.mark.parametrize("count", [1, 2, 5, 16])
def test_add_is_exact(count):
    """Block cores are copies and the first core one product per entry, so the
    sum matches the oracle bit for bit (ragged ranks, one- and many-core trains)."""
    log(f"add count={count}")
    rng = np.random.default_rng(400 + count)
    prof = [[1, 2, 4, 3, 5, 2, 1], [1, 1, 1, 1, 1, 1, 1], [1, 2, 3, 7, 3, 2, 1], [1, 2, 2, 2, 2, 2, 1]]
    terms = [rand_tt(rng, prof[t % 4]) for t in range(count)]
    coeffs = list(rng.standard_normal(count))
    ref = O.tt_sum(terms, coeffs)
    got = host(Q.add([dev(t) for t in terms], coeffs))
    for g, r in zip(got, ref):
        assert g.shape == r.shape
        np.testing.assert_array_equal(g, r)
    ones = [[rng.standard_normal((1, 3, 1))] for _ in range(count)]
    g1 = host(Q.add([dev(t) for t in ones], coeffs))[0]
    np.testing.assert_array_equal(g1, O.tt_sum(ones, coeffs)[0])


def test_add_mpo_and_fp32():
    rng = np.random.default_rng(410)
    W1 = rand_mpo(rng, [1, 3, 2, 1], [2, 3, 2], [2, 2, 4])
    W2 = rand_mpo(rng, [1, 2, 4, 1], [2, 3, 2], [2, 2, 4])
    ref = O.tt_sum([W1, W2], [2.0, -0.5])
    got = host(Q.add([dev(W1), dev(W2)], [2.0, -0.5]))
    for g, r in zip(got, ref):
        np.testing.assert_array_equal(g, r)
    X1 = rand_tt(rng, [1, 2, 4, 2, 1])
    X2 = rand_tt(rng, [1, 3, 3, 3, 1])
    ref32 = O.tt_sum([[c.astype(np.float32).astype(np.float64) for c in X] for X in (X1, X2)], [1.0, 3.0])
    got32 = Q.add([dev(X1, torch.float32), dev(X2, torch.float32)], [1.0, 3.0])
    for g, r in zip(got32, ref32):
        assert g.dtype == torch.float32
        assert np.abs(g.cpu().numpy().astype(np.float64) - r).max() <= 1e-6 * np.abs(r).max()


@pytest.mark.parametrize("case", ["cancel", "tol", "maxrank"])
def test_add_then_round(case):
    log(f"add+round {case}")
    rng = np.random.default_rng(411)
    X = rand_tt(rng, [1, 2, 4, 8, 16, 21, 16, 8, 4, 2, 1])
    if case == "cancel":
        terms, coeffs, tol, maxr = [X, X, X], [1.0, 1.0, -1.0], 1e-12, 0
    else:
        Y = rand_tt(rng, [1, 2, 4, 8, 9, 9, 9, 8, 4, 2, 1])
        Z = rand_tt(rng, [1, 2, 3, 3, 3, 3, 3, 3, 3, 2, 1])
        terms, coeffs = [X, Y, Z], [1.0, 1e-3, -2e-2]
        tol, maxr = (1e-4, 0) if case == "tol" else (0.0, 12)
    S = O.tt_sum(terms, coeffs)
    ref, info = O.round_tt(S, tol, maxr, return_info=True)
    summed = Q.add([dev(t) for t in terms], coeffs)
    got = Q.round_tt(summed, tol, maxr, want_sigmas=True)
    assert got.ranks == info.ranks
    assert O.rel_error(host(got.cores), ref) <= 1e-12
    for k, s in enumerate(info.sigmas):
        assert np.abs(np.array(got.sigmas[k][: len(s)]) - s).max() <= 1e-12 * s[0]
    if case == "cancel":
        assert O.rel_error(host(got.cores), X) <= 1e-12


def test_operator_product_elementwise():
    rng = np.random.default_rng(412)
    dout, dmid, din = [2, 3, 2, 5, 2], [3, 2, 4, 2, 2], [2, 2, 5, 3, 2]
    A = rand_mpo(rng, [1, 3, 2, 4, 3, 1], dout, dmid)
    B = rand_mpo(rng, [1, 2, 4, 3, 2, 1], dmid, din)
    ref = O.contract("ij,jk->ik", A, B)
    got = host(Q.contract("ij,jk->ik", dev(A), dev(B)))
    for g, r in zip(got, ref):
        assert g.shape == r.shape
        assert np.abs(g - r).max() <= 8 * 2.2e-16 * np.abs(r).max()


@pytest.mark.parametrize("d1,d2", [(1, 1), (1, 3), (5, 2)])
def test_shift_products_are_shifts(d1, d2):
    """Q^N_{d1} Q^N_{d2} = Q^N_{d1+d2} (Sec. 4.2) at N = 2^12: the operator
    product on the GPU, element-wise against the oracle and densely against
    the shift of the summed distance."""
    log(f"shift product {d1}+{d2}")
    n = 12
    A, B = O.shift_mpo_paper(n, d1), O.shift_mpo_paper(n, d2)
    got = host(Q.contract("ij,jk->ik", dev(A), dev(B)))
    for g, r in zip(got, O.contract("ij,jk->ik", A, B)):
        np.testing.assert_array_equal(g, r)
    assert np.abs(O.mpo_to_dense(got) - O.dense_shift(2 ** n, d1 + d2)).max() == 0.0


@pytest.mark.parametrize("d1,d2", [(1, 1), (1, 3), (5, 2)])
def test_shift_products_round_to_shifts(d1, d2):
    """The same products rounded on the GPU as an MPS of the combined leg:
    dense equality with the shift and the rank of the paper's shift train.
    After a truncated bond the Jacobi input holds a row that is an exact tiny
    multiple of another; it is deflated instead of rotated without end."""
    log(f"shift product rounded {d1}+{d2}")
    n = 12
    P = Q.contract("ij,jk->ik", dev(O.shift_mpo_paper(n, d1)), dev(O.shift_mpo_paper(n, d2)))
    got = Q.round_tt([c.reshape(c.shape[0], 4, c.shape[-1]) for c in P], 1e-13, 0)
    ref_rank = max(O.ranks_of(O.round_tt(as_mps(O.shift_mpo_paper(n, d1 + d2)), 1e-13, 0)))
    assert max(got.ranks) == ref_rank
    back = [c.reshape(c.shape[0], 2, 2, c.shape[-1]) for c in host(got.cores)]
    dense = O.mpo_to_dense(back)
    assert np.abs(dense - O.dense_shift(2 ** n, d1 + d2)).max() <= 1e-12


def test_laplacian3d_squared_full_size():
    """The 3D Laplacian (n = 42, rank 7) squared by the operator product and
    rounded on the GPU, against the oracle's product and rounding."""
    log("laplacian3d squared")
    W = I.laplacian_mpo(14, 3)
    ref_c = O.contract("ij,jk->ik", W, W)
    got_c = Q.contract("ij,jk->ik", dev(W), dev(W))
    for k in (0, 1, 20, 41):
        r = ref_c[k]
        assert np.abs(got_c[k].cpu().numpy() - r).max() <= 8 * 2.2e-16 * np.abs(r).max()
    ref, info = O.round_tt(as_mps(ref_c), 1e-12, 0, return_info=True)
    got = Q.round_tt([c.reshape(c.shape[0], 4, c.shape[-1]) for c in got_c], 1e-12, 0, want_sigmas=True)
    assert got.ranks == info.ranks
    assert O.rel_error(host(got.cores), ref) <= 1e-12
