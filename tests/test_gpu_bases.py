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


def spd_local_mpo(rng, bases, eps=0.1):
    """W = sum_k A_k (acting on digit k) + eps sum_k B_k B_{k+1} (adjacent
    digits): A_k random SPD with eigenvalues >= 1, B_k symmetric of norm 1,
    so W >= n - eps (n - 1) > 0.  Rank-3 MPO (states: before, coupling
    pending, done)."""
    n = len(bases)
    cores = []
    for k, d in enumerate(bases):
        G = rng.standard_normal((d, d))
        A = G @ G.T / d + np.eye(d)
        Bs = rng.standard_normal((d, d))
        Bs = (Bs + Bs.T) / 2
        Bs /= np.linalg.norm(Bs, 2)
        c = np.zeros((3, d, d, 3))
        c[0, :, :, 0] = np.eye(d)
        c[0, :, :, 2] = A
        c[0, :, :, 1] = Bs
        c[1, :, :, 2] = eps * Bs
        c[2, :, :, 2] = np.eye(d)
        if k == 0:
            c = c[:1]
        if k == n - 1:
            c = c[:, :, :, 2:]
        cores.append(c)
    return cores


@pytest.mark.parametrize("solver", ["dmrg1", "dmrg2", "amen"])
def test_solvers_mixed_bases(solver):
    """The DMRG-like solver (one and two cores) and AMEn on a symmetric
    positive definite operator over digits of bases 3, 2, 5, 2, 3, 4, 2, 5:
    against the oracle's solvers from the same guesses; with ranks that
    adapt (capped at 12, where the exact solution needs up to 60) the result
    is also within 1e-4 of the dense solve (the oracle: 6.6e-6 two-core,
    6.4e-5 AMEn)."""
    log(f"solver {solver} on mixed bases")
    rng = np.random.default_rng(77)
    W = spd_local_mpo(rng, BASES)
    b = rand_tt(rng, profile(BASES, 3), BASES)
    x0 = rand_tt(rng, profile(BASES, 2), BASES)
    z0 = rand_tt(rng, profile(BASES, 2), BASES)
    if solver == "amen":
        ref, info = O.solve_amen(W, b, x0, z0, nsweeps=2, rel_tol=1e-12, max_rank=12, return_info=True)
        xc, rx, _, _, _ = Q.solve_amen(dev(W), dev(b), dev(x0), dev(z0), nsweeps=2, rel_tol=1e-12, max_rank=12)
    else:
        nc = 1 if solver == "dmrg1" else 2
        ref, info = O.solve_energy(W, b, x0, nsweeps=2, ncores=nc, rel_tol=1e-12, max_rank=12, return_info=True)
        xc, rx, _ = Q.solve(dev(W), dev(b), dev(x0), nsweeps=2, ncores=nc, rel_tol=1e-12, max_rank=12)
    assert rx == info["ranks"], (rx, info["ranks"])
    err = O.rel_error(host(xc), ref)
    xs = np.linalg.solve(O.mpo_to_dense(W), O.to_dense(b).ravel())
    derr = float(np.linalg.norm(O.to_dense(host(xc)).ravel() - xs) / np.linalg.norm(xs))
    log(f"  ranks {rx}, rel err vs oracle {err:.2e}, vs dense solve {derr:.2e}")
    assert err <= 1e-10
    if solver != "dmrg1":
        assert derr <= 1e-4
