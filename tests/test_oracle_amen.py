"""Pins of the oracle's AMEn linear solver (Sec. 5: single-core sweeps with
gradient enrichment), CPU only.

The checks do not go through the oracle's other solvers:
- the 1D Dirichlet Poisson problem tridiag(-1, 2, -1) u = 1 has the closed
  form u_j = j (N + 1 - j) / 2 (QTT rank 3); AMEn reaches it from a rank-1
  guess, which one-core sweeps without enrichment cannot leave;
- on a 2D shifted Laplacian with a random right-hand side the result equals
  the dense solve, and the final energy is -b^T A^-1 b;
- the energy never grows from one local solve to the next while nothing is
  truncated;
- a guess of full unfolding ranks gives the dense solution in one sweep;
- the residual train z is the orthogonal projection of the final residual
  r = b - W x onto its frame: <z, r> = ||z||^2 <= ||r||^2, and z vanishes
  when x has converged;
- ranks stay within the cap plus the enrichment rank (and grow past the
  cap: the enrichment is kept);
- x and z are linear in b (the basis cut is relative to the residual's own
  terms);
- the enriched bases are orthonormal, span every significant direction of
  [V^T; e/s] and hold none of the exactly null directions that the overlap
  of the x and z frames near the chain ends produces.
"""
import numpy as np

import oracle as O
import qtt_inputs as Q


def _poisson_1d(m):
    N = 2 ** m
    j = np.arange(1, N + 1, dtype=np.float64)
    return Q.laplacian_mpo(m, 1, diag=2.0), [np.ones((1, 2, 1)) for _ in range(m)], j * (N + 1 - j) / 2.0


def _rel(a, b):
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


def test_poisson_closed_form_from_rank_one_guess():
    m = 10
    W, b, u = _poisson_1d(m)
    rng = np.random.default_rng(0)
    x0 = Q.random_mps(m, 1, rng)
    z0 = Q.random_mps(m, 3, rng)
    X = O.solve_amen(W, b, x0, z0, nsweeps=1, rel_tol=1e-12, max_rank=6)
    assert _rel(O.to_dense(X).ravel(), u) < 1e-10
    # without enrichment the ranks of the guess (1) cannot grow
    X1 = O.solve_energy(W, b, x0, nsweeps=3, ncores=1)
    assert _rel(O.to_dense(X1).ravel(), u) > 0.5


def _case_2d(seed=1, m=4, D=2):
    n = m * D
    W = Q.laplacian_mpo(m, D, diag=2.5)
    rng = np.random.default_rng(seed)
    b = Q.random_mps(n, 3, rng)
    x0 = Q.random_mps(n, 2, rng)
    z0 = Q.random_mps(n, 3, rng)
    A, bd = O.mpo_to_dense(W), O.to_dense(b).ravel()
    return W, b, x0, z0, A, bd, np.linalg.solve(A, bd)


def test_equals_dense_solve_and_energy():
    W, b, x0, z0, A, bd, xs = _case_2d()
    X, info = O.solve_amen(W, b, x0, z0, nsweeps=3, return_info=True)
    assert _rel(O.to_dense(X).ravel(), xs) < 1e-12
    assert abs(info["energies"][-1] + xs @ bd) < 1e-12 * abs(xs @ bd)


def test_energy_non_increasing_without_truncation():
    W, b, x0, z0, A, bd, xs = _case_2d(seed=5)
    _, info = O.solve_amen(W, b, x0, z0, nsweeps=2, return_info=True)
    en = np.array(info["energies"])
    assert len(en) == 2 * 2 * 8
    assert np.all(np.diff(en) <= 1e-13 * abs(en[-1]))
    assert en[-1] >= -(xs @ bd) * (1 + 1e-12)


def test_full_rank_guess_is_exact_in_one_sweep():
    W, b, _, z0, A, bd, xs = _case_2d(seed=7, m=3)
    n = 6
    x0 = Q.random_mps(n, 64, np.random.default_rng(8))  # full unfolding ranks
    X = O.solve_amen(W, b, x0, z0, nsweeps=1)
    assert _rel(O.to_dense(X).ravel(), xs) < 1e-12


def test_residual_train_is_a_projection_of_the_residual():
    W, b, x0, z0, A, bd, xs = _case_2d(seed=11)
    # unconverged (rank cap): z is the projection of the final residual
    X, info = O.solve_amen(W, b, x0, z0, nsweeps=1, rel_tol=1e-10, max_rank=3, return_info=True)
    r = bd - A @ O.to_dense(X).ravel()
    z = O.to_dense(info["z"]).ravel()
    assert np.linalg.norm(z) > 1e-6 * np.linalg.norm(r)
    assert abs(z @ r - z @ z) <= 1e-12 * (r @ r)
    assert z @ z <= (r @ r) * (1 + 1e-12)
    # converged: the residual and its train vanish
    X, info = O.solve_amen(W, b, x0, z0, nsweeps=3, return_info=True)
    assert np.linalg.norm(O.to_dense(info["z"]).ravel()) < 1e-10 * np.linalg.norm(bd)


def test_ranks_within_cap_plus_enrichment():
    W, b, x0, z0, A, bd, xs = _case_2d(seed=13)
    n = 8
    for cap in (2, 4):
        X, info = O.solve_amen(W, b, x0, z0, nsweeps=2, rel_tol=1e-10, max_rank=cap, return_info=True)
        zr = [1] + [c.shape[-1] for c in info["z"]]
        assert info["ranks"] == [1] + [c.shape[-1] for c in X]
        # after the left-to-right pass a bond holds at most the truncated rank
        # plus z's rank, and at most the left unfolding size (the enriched
        # basis may exceed the right unfolding: it is orthonormal, not minimal)
        assert all(info["ranks"][k] <= min(2 ** k, cap + 3) for k in range(n + 1))
        assert max(info["ranks"]) > cap
        assert all(zr[k] <= 3 for k in range(n + 1))


def test_single_core_is_the_dense_solve():
    W = [np.array([[[[3.0], [0.5]], [[0.5], [2.0]]]])]  # a 2 x 2 SPD operator, one core
    b = [np.array([[[1.0], [-2.0]]])]
    x0 = [np.array([[[0.3], [0.1]]])]
    z0 = [np.array([[[1.0], [1.0]]])]
    X, info = O.solve_amen(W, b, x0, z0, nsweeps=1, return_info=True)
    xs = np.linalg.solve(np.array([[3.0, 0.5], [0.5, 2.0]]), np.array([1.0, -2.0]))
    assert _rel(X[0].ravel(), xs) < 1e-15
    assert np.abs(info["z"][0]).max() < 1e-15


def _left_frame(cores, q):
    """prod(d_<q) x r_q matrix of the first q cores."""
    F = np.ones((1, 1))
    for c in cores[:q]:
        F = np.einsum("Ia,aib->Iib", F, c).reshape(-1, c.shape[2])
    return F


def _right_frame(cores, q):
    """r_{q+1} x prod(d_>q) matrix of the cores after q."""
    F = np.ones((1, 1))
    for c in reversed(cores[q + 1:]):
        F = np.einsum("aib,bJ->aiJ", c, F).reshape(c.shape[0], -1)
    return F


def test_enrichment_and_residual_cores_follow_their_definitions():
    """At every truncated step (the cap binds), with the frames the step
    used: the current tensor is X_<q xt X_>q, e_q is the projection of
    b - W x onto (Z_<q x I x X_>q) moving left and (X_<q x I x Z_>q) moving
    right, and z's core the projection onto (Z_<q x I x Z_>q); checked with
    dense frames."""
    W, b, x0, z0, A, bd, xs = _case_2d(seed=17, m=3)
    trace = []
    O.solve_amen(W, b, x0, z0, nsweeps=2, rel_tol=1e-10, max_rank=2, trace=trace)
    assert {t["dir"] for t in trace} == {"left", "right"} and len(trace) == 2 * 2 * 5
    truncated = 0
    for t in trace:
        q, X, Z, xt = t["q"], t["X"], t["Z"], t["xt"]
        r0, d, r1 = xt.shape
        FLx, FRx = _left_frame(X, q), _right_frame(X, q)
        FLz, FRz = _left_frame(Z, q), _right_frame(Z, q)
        x = np.einsum("Ia,aic,cJ->IiJ", FLx, xt, FRx).ravel()
        r = (bd - A @ x).reshape(FLx.shape[0], d, FRx.shape[1])
        if t["dir"] == "left":
            e_ref = np.einsum("Ia,IiJ,cJ->aic", FLz, r, FRx)
        else:
            e_ref = np.einsum("Ia,IiJ,cJ->aic", FLx, r, FRz)
        zc_ref = np.einsum("Ia,IiJ,cJ->aic", FLz, r, FRz)
        scale = np.linalg.norm(bd)
        assert np.abs(t["e"] - e_ref).max() < 1e-12 * scale
        assert np.abs(t["zc"] - zc_ref).max() < 1e-12 * scale
        sv = np.linalg.svd(xt.reshape(r0, d * r1) if t["dir"] == "left" else xt.reshape(r0 * d, r1),
                           compute_uv=False)
        truncated += int(np.sum(sv > 1e-12 * sv[0]) <= 2)
    assert truncated == len(trace)


def test_solution_is_linear_in_the_right_hand_side():
    """x(c b) = c x(b) and z(c b) = c z(b) with the same ranks: the
    enrichment cut is measured against the residual's own terms, not an
    absolute level."""
    W, b, x0, z0, A, bd, xs = _case_2d(seed=19)
    X1, i1 = O.solve_amen(W, b, x0, z0, nsweeps=2, rel_tol=1e-10, max_rank=4, return_info=True)
    for c in (1e-12, 1e12):
        bc = O.tt_scale(b, c)
        Xc, ic = O.solve_amen(W, bc, x0, z0, nsweeps=2, rel_tol=1e-10, max_rank=4, return_info=True)
        assert ic["ranks"] == i1["ranks"]
        assert O.rel_error(O.tt_scale(Xc, 1.0 / c), X1) < 1e-12
        assert O.diff_norm(O.tt_scale(ic["z"], 1.0 / c), i1["z"]) < 1e-12 * O.norm(b)


def test_enriched_bases_hold_no_null_directions():
    """Near the ends of the chain the frames of x and z overlap, so the
    residual's projection has exactly null directions there, and where the
    residual vanishes in the frames it is rounding noise.  The new bases
    are orthonormal, every row carries a direction of [V^T; e/s] (and of
    z's projection), and no significant direction is left out."""
    m = 7
    W = Q.laplacian_mpo(m, 1, diag=2.25)
    rng = np.random.default_rng(620)
    b = Q.random_mps(m, 2, rng)
    x0 = Q.random_mps(m, 2, rng)
    z0 = Q.random_mps(m, 3, rng)
    trace = []
    O.solve_amen(W, b, x0, z0, nsweeps=2, rel_tol=1e-10, max_rank=12, trace=trace)
    shrunk = 0
    for t in trace:
        B, Bz, Vt = t["B"], t["Bz"], t["Vt"]
        r0, d, r1 = t["xt"].shape
        if t["dir"] == "left":
            E = np.vstack([Vt, t["e"].reshape(t["e"].shape[0], d * r1) / t["se"]])
            Ez = t["zc"].reshape(t["zc"].shape[0], -1) / t["sz"]
        else:
            E = np.vstack([Vt, (t["e"].reshape(r0 * d, -1) / t["se"]).T])
            Ez = (t["zc"].reshape(-1, t["zc"].shape[2]) / t["sz"]).T
        for basis, M in ((B, E), (Bz, Ez)):
            k = basis.shape[0]
            assert np.abs(basis @ basis.T - np.eye(k)).max() < 1e-13
            assert np.linalg.norm(M - (M @ basis.T) @ basis) < 1e-9
            if basis is B or np.linalg.norm(M) > 1e-6:
                assert np.linalg.svd(M @ basis.T, compute_uv=False).min() > 1e-8
        shrunk += int(B.shape[0] < min(E.shape))
    assert shrunk > 0  # the overlap occurs in this case
