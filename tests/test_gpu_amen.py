"""GPU parity of the AMEn linear solver (Sec. 5: single-core sweeps with
gradient enrichment) against the FP64 oracle's solver from the same guess
and the same initial residual train, on Dirichlet Laplacians (shifted by
s I where a right-hand side is random)."""
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


def dev(cores):
    return Q.to_device(cores, DEV, torch.float64)


def host(cores):
    return Q.to_host(cores)


@pytest.mark.parametrize("nsweeps,cap,rz", [(1, 6, 3), (2, 6, 3), (2, 4, 5), (3, 8, 2)])
def test_amen_random_rhs_against_oracle(nsweeps, cap, rz):
    """A 2D 2^5 x 2^5 grid (10 cores), right-hand side of rank 4, guess of
    rank 2: x (ranks and tensor) and the residual train z against the
    oracle's."""
    log(f"amen sweeps={nsweeps} cap={cap} rz={rz}")
    m, D = 5, 2
    W = I.laplacian_mpo(m, D, diag=2.25)
    n = m * D
    rng = np.random.default_rng(620)
    b = I.random_mps(n, 4, rng)
    x0 = I.random_mps(n, 2, rng)
    z0 = I.random_mps(n, rz, rng)
    ref, info = O.solve_amen(W, b, x0, z0, nsweeps=nsweeps, rel_tol=1e-10, max_rank=cap, return_info=True)
    xc, rx, zc, rzs, nrm = Q.solve_amen(dev(W), dev(b), dev(x0), dev(z0), nsweeps=nsweeps, rel_tol=1e-10,
                                        max_rank=cap)
    assert rx == info["ranks"], (rx, info["ranks"])
    assert rzs == [1] + [c.shape[-1] for c in info["z"]]
    err = O.rel_error(host(xc), ref)
    zerr = O.diff_norm(host(zc), info["z"]) / O.norm(b)
    log(f"  ranks {rx}, x rel err {err:.2e}, z err / |b| {zerr:.2e}")
    assert err <= 1e-10
    assert zerr <= 1e-10
    assert abs(nrm - O.norm(ref)) <= 1e-10 * O.norm(ref)


def test_amen_overlapping_frames_against_oracle():
    """A 1D chain of 7 cores with a rank-3 residual train: near the ends the
    frames of x and z overlap, so the projected residual has exactly null
    directions there; both sides leave them out of the new bases and agree."""
    m = 7
    W = I.laplacian_mpo(m, 1, diag=2.25)
    rng = np.random.default_rng(620)
    b = I.random_mps(m, 2, rng)
    x0 = I.random_mps(m, 2, rng)
    z0 = I.random_mps(m, 3, rng)
    ref, info = O.solve_amen(W, b, x0, z0, nsweeps=2, rel_tol=1e-10, max_rank=12, return_info=True)
    xc, rx, zc, rzs, _ = Q.solve_amen(dev(W), dev(b), dev(x0), dev(z0), nsweeps=2, rel_tol=1e-10, max_rank=12)
    assert rx == info["ranks"] and rzs == [1] + [c.shape[-1] for c in info["z"]]
    err = O.rel_error(host(xc), ref)
    zerr = O.diff_norm(host(zc), info["z"]) / O.norm(b)
    log(f"amen overlap ranks {rx}, z ranks {rzs}, x rel err {err:.2e}, z err / |b| {zerr:.2e}")
    assert err <= 1e-10 and zerr <= 1e-10


def test_amen_poisson_closed_form():
    """tridiag(-1, 2, -1) u = 1 on 2^12 points (12 cores) from a rank-1
    guess: u_j = j (N + 1 - j) / 2 after one sweep, to the accuracy the
    operator's condition number kappa = 4 (N + 1)^2 / pi^2 allows (4 kappa u).
    (Here kappa u exceeds the enrichment cut, so rounding noise in the
    projected residual may enter the bases: a valid solve, not compared
    with the oracle's ranks.)"""
    m = 12
    N = 2 ** m
    W = I.laplacian_mpo(m, 1, diag=2.0)
    b = [np.ones((1, 2, 1)) for _ in range(m)]
    rng = np.random.default_rng(3)
    x0 = I.random_mps(m, 1, rng)
    z0 = I.random_mps(m, 3, rng)
    xc, rx, _, _, _ = Q.solve_amen(dev(W), dev(b), dev(x0), dev(z0), nsweeps=1, rel_tol=1e-12, max_rank=6)
    j = np.arange(1, N + 1, dtype=np.float64)
    u = j * (N + 1 - j) / 2.0
    xd = O.to_dense(host(xc)).ravel()
    err = float(np.linalg.norm(xd - u) / np.linalg.norm(u))
    bound = 4.0 * (4.0 * (N + 1) ** 2 / math.pi ** 2) * np.finfo(np.float64).eps
    log(f"amen poisson ranks {rx}, rel err vs closed form {err:.2e} (bound {bound:.1e})")
    assert err <= bound


def test_amen_eigenvector_full_size():
    """(L + s I) f = (lambda + s) f on a 2^12 x 2^12 grid (24 cores), f a
    product of two sines (rank 2): from a random rank-1 guess and a rank-4
    residual train, AMEn recovers f."""
    m, D, s = 12, 2, 1.0
    N = 2 ** m
    f, lam = None, 0.0
    for a, k in enumerate([N // 3, N // 2 - 1]):
        w = math.pi * k / (N + 1)
        fa = I.trig_qtt(m, w, w, "sin")
        lam += 2.0 - 2.0 * math.cos(w)
        ea = I.embed_axis(fa, D, a)
        f = ea if f is None else O.contract("i,i->i", f, ea)
    f = O.round_tt(f, 1e-14)
    W = I.laplacian_mpo(m, D, diag=2.0 + s / D)
    b = O.tt_scale(f, lam + s)
    rng = np.random.default_rng(9)
    x0 = I.random_mps(m * D, 1, rng)
    z0 = I.random_mps(m * D, 4, rng)
    xc, rx, _, _, _ = Q.solve_amen(dev(W), dev(b), dev(x0), dev(z0), nsweeps=2, rel_tol=1e-12, max_rank=4)
    err = O.rel_error(host(xc), f)
    log(f"amen eigenvector ranks {max(rx)} max, rel err vs f {err:.2e}")
    assert err <= 1e-11


def test_amen_single_core_and_zero_rhs():
    W = [np.array([[[[3.0], [0.5]], [[0.5], [2.0]]]])]
    b = [np.array([[[1.0], [-2.0]]])]
    x0 = [np.array([[[0.3], [0.1]]])]
    z0 = [np.array([[[1.0], [1.0]]])]
    xc, rx, zc, rz, _ = Q.solve_amen(dev(W), dev(b), dev(x0), dev(z0), nsweeps=1)
    xs = np.linalg.solve(np.array([[3.0, 0.5], [0.5, 2.0]]), np.array([1.0, -2.0]))
    assert np.abs(host(xc)[0].ravel() - xs).max() <= 1e-15
    assert np.abs(host(zc)[0]).max() <= 1e-15
    # zero right-hand side: zero trains of rank 1
    m, D = 3, 2
    Wl = I.laplacian_mpo(m, D, diag=2.5)
    rng = np.random.default_rng(5)
    b0 = [np.zeros_like(c) for c in I.random_mps(m * D, 2, rng)]
    xc, rx, zc, rz, nrm = Q.solve_amen(dev(Wl), dev(b0), dev(I.random_mps(m * D, 2, rng)),
                                       dev(I.random_mps(m * D, 2, rng)), nsweeps=1, max_rank=4)
    assert nrm == 0.0 and max(rx) == 1 and max(rz) == 1
    assert all(float(np.abs(c).max()) == 0.0 for c in host(xc))


def test_amen_argument_errors():
    m, D = 3, 2
    W = dev(I.laplacian_mpo(m, D, diag=2.5))
    rng = np.random.default_rng(1)
    b = dev(I.random_mps(m * D, 2, rng))
    z = dev(I.random_mps(m * D, 2, rng))
    with pytest.raises(Q.QttError, match="SHAPE"):
        Q.solve_amen(W, b, b, z[:-1])
    with pytest.raises(Q.QttError, match="ARG"):
        Q.solve_amen(W, b, b, z, nsweeps=-1)
