"""Pins of the oracle's DMRG-like linear solver (Sec. 5), CPU only.

The operator is the Dirichlet Laplacian shifted by s I (the operator of an
implicit heat step scaled by the inverse time step: symmetric positive
definite).  The checks: a full-rank guess reproduces the dense solution in
one sweep, the energy never grows from one local solve to the next and ends
at -b^T A^{-1} b, super-cores of two cores grow a rank-1 guess to the
solution's own ranks (from its dense unfoldings), and at full size a
Laplacian eigenvector, which solves (L + s I) f = (lambda + s) f, is
recovered from a guess of its rank.
"""
import math

import numpy as np
import pytest

import oracle as O
import qtt_inputs as Q


def shifted_laplacian(m, D, s):
    return Q.laplacian_mpo(m, D, diag=2.0 + s / D)


def test_operator_is_the_shifted_dense_laplacian():
    """The diagonal coefficient shifts the Laplacian MPO by s I (same
    interleaved index order), and the shifted operator is SPD."""
    A = O.mpo_to_dense(shifted_laplacian(3, 2, 0.7))
    L = O.mpo_to_dense(Q.laplacian_mpo(3, 2))
    assert np.abs(A - (L + 0.7 * np.eye(64))).max() < 1e-14
    assert np.abs(A - A.T).max() == 0.0 and np.linalg.eigvalsh(A).min() > 0.7 - 1e-12


def _dense_case(seed=3):
    m, D = 3, 2
    A = shifted_laplacian(m, D, 2.0)
    n = m * D
    b = Q.random_mps(n, 4, np.random.default_rng(seed))
    Ad, bd = O.mpo_to_dense(A), O.to_dense(b)
    return A, b, Ad, bd, np.linalg.solve(Ad, bd), n


def _dense_ranks(y, n, tol=1e-12):
    out = [1]
    for k in range(1, n):
        s = np.linalg.svd(y.reshape(2 ** k, -1), compute_uv=False)
        out.append(int(np.sum(s > tol * s[0])))
    return out + [1]


def test_full_rank_guess_solves_in_one_sweep_and_energy_decreases():
    A, b, Ad, bd, xd, n = _dense_case()
    guess = Q.random_mps(n, 64, np.random.default_rng(1))
    x, info = O.solve_energy(A, b, guess, nsweeps=1, ncores=1, return_info=True)
    assert np.linalg.norm(O.to_dense(x) - xd) <= 1e-13 * np.linalg.norm(xd)
    e = info["energies"]
    assert len(e) == 2 * n
    assert all(e[i + 1] <= e[i] + 1e-13 * abs(e[i]) for i in range(len(e) - 1))
    assert abs(e[-1] - (-bd @ xd)) <= 1e-12 * abs(bd @ xd)


def test_fixed_low_rank_energy_decreases_and_beats_rounded_guess():
    """With fixed ranks below the solution's the energy still decreases
    monotonically, and it ends below the energy of the dense solution rounded
    to the same ranks (the solver minimises J over that rank set)."""
    A, b, Ad, bd, xd, n = _dense_case()
    guess = Q.random_mps(n, 2, np.random.default_rng(5))
    x, info = O.solve_energy(A, b, guess, nsweeps=3, ncores=1, return_info=True)
    e = info["energies"]
    assert all(e[i + 1] <= e[i] + 1e-13 * abs(e[i]) for i in range(len(e) - 1))
    xv = O.to_dense(x)
    # the recorded energy is J of the final train, evaluated densely
    assert xv @ Ad @ xv - 2 * xv @ bd == pytest.approx(e[-1], rel=1e-10)
    assert e[-1] > -bd @ xd  # a rank-2 train cannot reach the exact minimum here


def test_two_core_grows_rank_one_guess_to_the_solution():
    A, b, Ad, bd, xd, n = _dense_case()
    g1 = Q.random_mps(n, 1, np.random.default_rng(2))
    x1, i1 = O.solve_energy(A, b, g1, nsweeps=1, ncores=2, rel_tol=1e-12, return_info=True)
    x2, i2 = O.solve_energy(A, b, g1, nsweeps=2, ncores=2, rel_tol=1e-12, return_info=True)
    assert np.linalg.norm(O.to_dense(x1) - xd) > 1e-6 * np.linalg.norm(xd)
    assert np.linalg.norm(O.to_dense(x2) - xd) <= 1e-12 * np.linalg.norm(xd)
    assert i2["ranks"] == _dense_ranks(xd, n)


@pytest.mark.parametrize("ncores", [1, 2])
def test_eigenvector_solution_at_full_size(ncores):
    """(L + s I) f = (lambda + s) f for a product of sine modes on a
    2^12 x 2^12 grid (24 cores): with b = (lambda + s) f the solver recovers f
    from a random guess of f's rank (4) in three sweeps."""
    m, D, s = 12, 2, 1.0
    N = 2 ** m
    f, lam = None, 0.0
    for a, k in enumerate([N // 3, N // 2 - 1]):
        w = math.pi * k / (N + 1)
        fa = Q.trig_qtt(m, w, w, "sin")
        lam += 2.0 - 2.0 * math.cos(w)
        ea = Q.embed_axis(fa, D, a)
        f = ea if f is None else O.contract("i,i->i", f, ea)
    f = O.round_tt(f, 1e-14)
    A = shifted_laplacian(m, D, s)
    b = O.tt_scale(f, lam + s)
    guess = Q.random_mps(m * D, 4, np.random.default_rng(7))
    x = O.solve_energy(A, b, guess, nsweeps=3, ncores=ncores, rel_tol=1e-13, max_rank=4)
    assert O.rel_error(x, f) <= 1e-11
