"""GPU parity for general digit bases (factorised dimensions, Sec. 2): cores of
physical size 2, 3, 4 and 5 mixed in one train, and rectangular operators
(d_out != d_in), through contraction, rounding, zip-up and inner products."""
import math
import sys

import numpy as np
import pytest

torch = pytest.importorskip("torch")

import oracle as O
from conftest import ranks_agree

pytestmark = pytest.mark.gpu

if torch.cuda.is_available():
    from paper_2602_20226_amd import qtt as Q

DEV = "cuda:0"
BASES = [3, 2, 5, 2, 3, 4, 2, 5]


def log(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def dev(cores):
    return Q.to_device(cores, DEV, torch.float64)


def host(cores):
    return Q.to_host(cores)


def profile(bases, r):
    n = len(bases)
    return [min(r, math.prod(bases[:k]), math.prod(bases[k:])) for k in range(n + 1)]


def rand_tt(rng, ranks, bases):
    return [rng.standard_normal((ranks[k], bases[k], ranks[k + 1])) for k in range(len(bases))]


def rand_mpo(rng, ranks, bout, bin_):
    return [rng.standard_normal((ranks[k], bout[k], bin_[k], ranks[k + 1])) for k in range(len(bout))]


def operands(spec, seed):
    rng = np.random.default_rng(seed)
    if spec == "ij,j->i":
        bin_ = BASES
        bout = [2, 3, 2, 4, 5, 2, 3, 2]
        A = rand_mpo(rng, [1, 3, 4, 3, 4, 3, 4, 3, 1], bout, bin_)
        B = rand_tt(rng, profile(bin_, 13), bin_)
    else:
        A = rand_tt(rng, profile(BASES, 4), BASES)
        B = rand_tt(rng, profile(BASES, 11), BASES)
    return A, B


@pytest.mark.parametrize("spec", ["ij,j->i", "i,i->i"])
def test_contract_general_bases(spec):
    log(f"bases contract {spec}")
    A, B = operands(spec, 300)
    ref = O.contract(spec, A, B)
    got = host(Q.contract(spec, dev(A), dev(B)))
    for g, r in zip(got, ref):
        assert g.shape == r.shape
        assert np.abs(g - r).max() <= 8 * 2.2e-16 * np.abs(r).max()


@pytest.mark.parametrize("spec", ["ij,j->i", "i,i->i"])
@pytest.mark.parametrize("tol,maxr", [(0.0, 0), (1e-6, 0), (0.0, 7)])
def test_contract_round_general_bases(spec, tol, maxr):
    log(f"bases contract_round {spec} tol={tol} maxr={maxr}")
    A, B = operands(spec, 301)
    C = O.contract(spec, A, B)
    ref, info = O.round_tt(C, tol, maxr, return_info=True)
    got = Q.contract_round(spec, dev(A), dev(B), tol, maxr, want_sigmas=True)
    assert ranks_agree(got.ranks, info)
    gh = host(got.cores)
    assert O.rel_error(gh, ref) <= 1e-12
    for c in gh[1:]:
        M = c.reshape(c.shape[0], -1)
        assert np.abs(M @ M.T - np.eye(M.shape[0])).max() <= 1e-13
    for k, s in enumerate(info.sigmas):
        g = np.array(got.sigmas[k][: len(s)])
        assert np.abs(g - s).max() <= 1e-12 * s[0]


@pytest.mark.parametrize("spec", ["ij,j->i", "i,i->i"])
@pytest.mark.parametrize("N", [1, 2])
def test_zipup_general_bases(spec, N):
    log(f"bases zipup {spec} N={N}")
    A, B = operands(spec, 302)
    for tol, maxr in [(0.0, 0), (1e-4, 0), (0.0, 6)]:
        ref, info = O.zipup(spec, A, B, tol, maxr, ncores=N, return_info=True)
        got = Q.contract_zipup(spec, dev(A), dev(B), tol, maxr, ncores=N, want_sigmas=True)
        assert ranks_agree(got.ranks, info), (tol, maxr, got.ranks, info.ranks)
        gh = host(got.cores)
        assert O.rel_error(gh, ref) <= 1e-12
        for c in gh[:-1]:
            M = c.reshape(-1, c.shape[-1])
            assert np.abs(M.T @ M - np.eye(M.shape[1])).max() <= 1e-13
        for b, s in enumerate(info.sigmas):
            g = np.array(got.sigmas[b][: len(s)])
            assert np.abs(g - s).max() <= 1e-12 * s[0]


def test_round_and_inner_general_bases():
    """A rank-1 exponential on the factorised grid (one core per digit,
    exp(a c_q i_q), c_q = prod_{r>q} b_r) plus a small random train: rounding
    against the oracle, and inner products against the dense sum."""
    log("bases round + inner")
    rng = np.random.default_rng(303)
    c = [math.prod(BASES[q + 1:]) for q in range(len(BASES))]
    E = [np.exp(-3e-4 * c[q] * np.arange(b)).reshape(1, b, 1) for q, b in enumerate(BASES)]
    X = O.tt_add(E, rand_tt(rng, profile(BASES, 9), BASES), 1.0, 1e-3)
    for tol in (0.0, 1e-5):
        ref, info = O.round_tt(X, tol, 0, return_info=True)
        got = Q.round_tt(dev(X), tol, 0, want_sigmas=True)
        assert ranks_agree(got.ranks, info)
        assert O.rel_error(host(got.cores), ref) <= 1e-12
    Y = rand_tt(rng, profile(BASES, 6), BASES)
    dense = float(O.to_dense(X) @ O.to_dense(Y))
    g = Q.inner(dev(X), dev(Y))
    scale = np.linalg.norm(O.to_dense(X)) * np.linalg.norm(O.to_dense(Y))
    assert abs(g - dense) <= 1e-13 * scale
