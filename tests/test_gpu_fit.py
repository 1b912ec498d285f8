"""GPU parity of the variational fitting (Sec. 3.3) against the FP64 oracle."""
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


def dev(cores):
    return Q.to_device(cores, DEV, torch.float64)


def host(cores):
    return Q.to_host(cores)


def rand_tt(rng, ranks, d=2):
    return [rng.standard_normal((ranks[k], d, ranks[k + 1])) for k in range(len(ranks) - 1)]


def rand_mpo(rng, ranks, d=2):
    return [rng.standard_normal((ranks[k], d, d, ranks[k + 1])) for k in range(len(ranks) - 1)]


@pytest.mark.parametrize("spec", ["ij,j->i", "i,i->i"])
@pytest.mark.parametrize("nsweeps", [0, 1, 3])
def test_fit_random_against_oracle(spec, nsweeps):
    log(f"fit {spec} sweeps={nsweeps}")
    rng = np.random.default_rng(500)
    if spec == "ij,j->i":
        A = rand_mpo(rng, [1, 3, 5, 5, 5, 5, 5, 5, 5, 3, 1])
    else:
        A = rand_tt(rng, [1, 2, 3, 3, 3, 3, 3, 3, 3, 2, 1])
    B = rand_tt(rng, [1, 2, 4, 8, 16, 37, 16, 8, 4, 2, 1])
    # guess with ragged ranks, one of them above what the left QR allows (shrinks)
    guess = rand_tt(rng, [1, 3, 4, 7, 9, 11, 9, 7, 4, 2, 1])
    ref = O.fit(spec, A, B, guess, nsweeps=nsweeps)
    cores, ranks, nrm = Q.fit(spec, dev(A), dev(B), dev(guess), nsweeps=nsweeps)
    assert ranks == O.ranks_of(ref)
    gh = host(cores)
    assert O.rel_error(gh, ref) <= 1e-12
    assert abs(nrm - O.norm(ref)) <= 1e-12 * O.norm(ref)
    for c in gh[:-1]:
        M = c.reshape(-1, c.shape[-1])
        assert np.abs(M.T @ M - np.eye(M.shape[1])).max() <= 1e-13


def test_fit_from_zipup_laplacian2d():
    """The pipeline the paper recommends on the 2D workload (n = 32): zip-up
    truncated to rank 64, then variational sweeps from it; parity with the
    oracle after each sweep and an error that falls towards TT rounding's."""
    log("fit laplacian2d from zip-up")
    w = I.laplacian2d_r64()
    C = O.contract(w.spec, w.a, w.b)
    e_round = O.rel_error(O.round_tt(C, w.rel_tol, w.max_rank), C)
    z = Q.contract_zipup(w.spec, dev(w.a), dev(w.b), w.rel_tol, w.max_rank, ncores=1)
    guess = host(z.cores)
    e_prev = O.rel_error(guess, C)
    for sweeps in (1, 2):
        ref = O.fit(w.spec, w.a, w.b, guess, nsweeps=sweeps)
        cores, ranks, _ = Q.fit(w.spec, dev(w.a), dev(w.b), dev(guess), nsweeps=sweeps)
        gh = host(cores)
        assert ranks == O.ranks_of(ref)
        assert O.rel_error(gh, ref) <= 1e-11
        e = O.rel_error(gh, C)
        log(f"  sweeps {sweeps}: error {e:.4e} (zip-up {O.rel_error(guess, C):.4e}, rounding {e_round:.4e})")
        assert e <= e_prev * (1 + 1e-12)
        e_prev = e
    assert e_prev <= 1.05 * e_round


def test_fit_argument_errors():
    rng = np.random.default_rng(501)
    A = rand_mpo(rng, [1, 3, 1])
    B = rand_tt(rng, [1, 2, 1])
    g = rand_tt(rng, [1, 2, 1])
    with pytest.raises(Q.QttError) as e:
        Q.fit("ij,j->i", dev(A), dev(B), dev(g), nsweeps=-1)
    assert e.value.status == -1
    bad = rand_tt(rng, [1, 2, 1], d=3)
    with pytest.raises(Q.QttError) as e:
        Q.fit("ij,j->i", dev(A), dev(B), dev(bad), nsweeps=1)
    assert e.value.status == -3


# ---------------------------------------------------------------- two-core super-cores
@pytest.mark.parametrize("spec", ["ij,j->i", "i,i->i"])
@pytest.mark.parametrize("tol,cap,nsweeps", [(1e-12, 0, 2), (0.0, 6, 2), (1e-3, 0, 1)])
def test_fit2_random_against_oracle(spec, tol, cap, nsweeps):
    """Two-core fitting from a ragged random guess: ranks (which grow or
    shrink), the fitted tensor and the orthonormality of the cores against the
    oracle's two-core fit, for an uncapped near-exact fit, a rank cap and a
    loose tolerance."""
    log(f"fit2 {spec} tol={tol} cap={cap} sweeps={nsweeps}")
    rng = np.random.default_rng(501)
    if spec == "ij,j->i":
        A = rand_mpo(rng, [1, 3, 5, 5, 5, 5, 5, 5, 5, 3, 1])
    else:
        A = rand_tt(rng, [1, 2, 3, 3, 3, 3, 3, 3, 3, 2, 1])
    B = rand_tt(rng, [1, 2, 4, 6, 6, 6, 6, 6, 4, 2, 1])
    guess = rand_tt(rng, [1, 2, 3, 2, 4, 5, 3, 1, 2, 2, 1])
    ref, info = O.fit_two_core(spec, A, B, guess, tol, cap, nsweeps, return_info=True)
    cores, ranks, nrm, extra = Q.fit2(spec, dev(A), dev(B), dev(guess), nsweeps=nsweeps, rel_tol=tol, max_rank=cap)
    assert ranks == info["ranks"], (ranks, info["ranks"])
    gh = host(cores)
    err = O.rel_error(gh, ref)
    log(f"  ranks {ranks}, rel err vs oracle {err:.2e}")
    assert err <= 1e-11
    assert abs(nrm - O.norm(ref)) <= 1e-12 * O.norm(ref)
    for c in gh[:-1]:
        M = c.reshape(-1, c.shape[-1])
        assert np.abs(M.T @ M - np.eye(M.shape[1])).max() <= 1e-12
    if cap:
        assert max(ranks) <= cap


def test_fit2_laplacian2d_rank64_from_zipup():
    """The 2D rank-64 workload (n = 32): the zip-up result refined by one
    two-core sweep under the same rank cap, against the oracle's two-core fit
    of the same guess; the error against the exact product is no larger than
    the guess's."""
    log("fit2 laplacian2d r64")
    w = I.laplacian2d_r64()
    A, B = dev(w.a), dev(w.b)
    Z = Q.contract_zipup(w.spec, A, B, w.rel_tol, w.max_rank, ncores=1)
    guess = host(Z.cores)
    ref, info = O.fit_two_core(w.spec, w.a, w.b, guess, w.rel_tol, w.max_rank, 1, return_info=True)
    cores, ranks, nrm, extra = Q.fit2(w.spec, A, B, Z.cores, nsweeps=1, rel_tol=w.rel_tol, max_rank=w.max_rank)
    assert ranks == info["ranks"]
    gh = host(cores)
    err = O.rel_error(gh, ref)
    C = O.contract(w.spec, w.a, w.b)
    e_fit, e_zip = O.rel_error(gh, C), O.rel_error(guess, C)
    log(f"  max rank {max(ranks)}, vs oracle {err:.2e}, vs exact {e_fit:.4e} (zip-up guess {e_zip:.4e})")
    assert err <= 1e-10
    assert e_fit <= e_zip * (1 + 1e-12)
