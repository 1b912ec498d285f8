"""GPU parity of the HIP path (through the C ABI) against the FP64 oracle."""
import math
import sys

import numpy as np
import pytest

torch = pytest.importorskip("torch")

import oracle as O
import qtt_inputs as I
from conftest import ranks_agree

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


def rand_mpo(rng, ranks, d=2):
    return [rng.standard_normal((ranks[k], d, d, ranks[k + 1])) for k in range(len(ranks) - 1)]


# ------------------------------------------------------------------ contraction (a1, a2)
@pytest.mark.parametrize("case", ["sin_noise", "ragged", "mpo_ragged"])
def test_contract_elementwise(case):
    log(f"contract {case}")
    rng = np.random.default_rng(100)
    if case == "sin_noise":
        w = I.sin_noise_1d()
        spec, A, B = w.spec, w.a, w.b
    elif case == "ragged":
        spec = "i,i->i"
        A = rand_tt(rng, [1, 2, 3, 5, 7, 3, 1])
        B = rand_tt(rng, [1, 2, 4, 3, 2, 2, 1])
    else:
        spec = "ij,j->i"
        A = rand_mpo(rng, [1, 3, 5, 2, 4, 1])
        B = rand_tt(rng, [1, 2, 3, 7, 2, 1])
    ref = O.contract(spec, A, B)
    got = host(Q.contract(spec, dev(A), dev(B)))
    for g, r in zip(got, ref):
        assert g.shape == r.shape
        assert np.abs(g - r).max() <= 2e-16 * max(np.abs(r).max(), 1e-300) * 4


def test_contract_laplacian3d_r256_sampled_cores():
    """Full-size 3D Laplacian (rank 7) times the rank-256 MPS: sampled cores, element-wise."""
    log("contract laplacian3d sampled")
    w = I.laplacian3d_r256()
    got = Q.contract(w.spec, dev(w.a), dev(w.b))
    for k in [0, 1, 9, 20, 33, 41]:
        ref = O.contract(w.spec, [w.a[k]], [w.b[k]])[0]
        g = got[k].cpu().numpy()
        assert g.shape == ref.shape
        assert np.abs(g - ref).max() <= 1e-15 * np.abs(ref).max()


def test_contract_fp32_storage():
    rng = np.random.default_rng(101)
    A = rand_mpo(rng, [1, 3, 2, 1])
    B = rand_tt(rng, [1, 2, 4, 1])
    ref = O.contract("ij,j->i", A, B)
    got = host(Q.contract("ij,j->i", dev(A, torch.float32), dev(B, torch.float32)))
    for g, r in zip(got, ref):
        assert np.abs(g - r).max() <= 1e-6 * np.abs(r).max()


# ------------------------------------------------------------------ inner (a5)
@pytest.mark.parametrize("ranks", [([1, 2, 4, 3, 1], [1, 2, 2, 5, 1]), ([1, 1], [1, 1]),
                                   ([1, 2, 4, 8, 16, 33, 16, 8, 4, 2, 1], [1, 2, 4, 8, 17, 8, 8, 8, 4, 2, 1])])
def test_inner(ranks):
    log(f"inner {ranks}")
    rng = np.random.default_rng(102)
    A = rand_tt(rng, ranks[0])
    B = rand_tt(rng, ranks[1])
    ref = O.inner(A, B)
    got = Q.inner(dev(A), dev(B))
    assert abs(got - ref) <= 1e-13 * O.norm(A) * O.norm(B)


def test_inner_closed_form_sin():
    n = 20
    N = 2 ** n
    s = I.sin_unit_interval(n)
    x = np.arange(N) / (N - 1)
    ref = np.sum(np.sin(2 * np.pi * x) ** 2)
    assert abs(Q.inner(dev(s), dev(s)) - ref) <= 1e-11 * ref


# ------------------------------------------------------------------ orthogonalisation (a3)
@pytest.mark.parametrize("ranks", [[1, 2, 4, 7, 7, 4, 2, 1], [1, 2, 4, 8, 16, 40, 16, 8, 4, 2, 1], [1, 1, 1],
                                   [1, 2, 300, 2, 1]])
def test_orthogonalize(ranks):
    log(f"orthogonalize {ranks}")
    rng = np.random.default_rng(103)
    X = rand_tt(rng, ranks)
    Y, nrm = Q.orthogonalize(dev(X))
    Yh = host(Y)
    for c in Yh[:-1]:
        M = c.reshape(-1, c.shape[-1])
        assert np.abs(M.T @ M - np.eye(M.shape[1])).max() <= 1e-13
    _, ref_norm = O.orthogonalize(X)
    assert abs(nrm - ref_norm) <= 1e-13 * ref_norm
    assert O.rel_error(Yh, X) <= 1e-13
    expect = [1]
    for k in range(len(X)):
        expect.append(min(2 * expect[-1], X[k].shape[-1]))
    assert O.ranks_of(Yh) == expect


def _rank1_probe(cores, z):
    """<T, Z> for a rank-1 TT Z given by its vectors z[k] (length d_k)."""
    v = np.ones(1)
    for c, zk in zip(cores, z):
        v = np.einsum("a,aib,i->b", v, c, zk)
    return float(v[0])


@pytest.mark.timeout(600)
def test_orthogonalize_largest_unfolding():
    """Ranks up to 2048, so the middle unfolding is 4096 x 2048: the tallest
    panel shape the QR supports.  Checks orthogonality of every core, the
    norm against the oracle, and the tensor through random rank-1 probes."""
    n = 24
    ranks = [min(2 ** k, 2048, 2 ** (n - k)) for k in range(n + 1)]
    log(f"orthogonalize largest unfolding, max rank {max(ranks)}")
    rng = np.random.default_rng(107)
    X = [rng.standard_normal((ranks[k], 2, ranks[k + 1])) / np.sqrt(2 * ranks[k + 1]) for k in range(n)]
    Y, nrm = Q.orthogonalize(dev(X))
    Yh = host(Y)
    assert max(c.shape[0] * c.shape[1] for c in Yh) == 4096
    for c in Yh[:-1]:
        M = c.reshape(-1, c.shape[-1])
        assert np.abs(M.T @ M - np.eye(M.shape[1])).max() <= 1e-13
    _, ref_norm = O.orthogonalize(X)
    assert abs(nrm - ref_norm) <= 1e-13 * ref_norm
    for _ in range(4):
        z = [rng.standard_normal(2) for _ in range(n)]
        zn = np.prod([np.linalg.norm(v) for v in z])
        assert abs(_rank1_probe(Yh, z) - _rank1_probe(X, z)) <= 1e-12 * ref_norm * zn


@pytest.mark.timeout(600)
@pytest.mark.parametrize("r1,r2", [(129, 131), (513, 64), (897, 131), (1025, 64), (1537, 131), (1793, 131)])
def test_orthogonalize_panel_configurations(r1, r2):
    """Unfoldings of 2 r1 rows on both sides of every row-count boundary at
    which the QR changes its panel shape, inner-application tile or split-K
    chunking (258 ... 3586 rows), with odd and even column counts (row
    strides that forbid and allow 16-byte accesses).  Left ranks double up to
    1024 so that every unfolding has full row rank."""
    ranks = [2 ** k for k in range(11)] + [r1, r2, 2, 1]
    log(f"orthogonalize panel configurations r1={r1} r2={r2}")
    rng = np.random.default_rng(109 + r1)
    X = [rng.standard_normal((ranks[k], 2, ranks[k + 1])) / np.sqrt(2 * ranks[k + 1]) for k in range(len(ranks) - 1)]
    Y, nrm = Q.orthogonalize(dev(X))
    Yh = host(Y)
    assert Yh[11].shape == (r1, 2, r2)
    for c in Yh[:-1]:
        M = c.reshape(-1, c.shape[-1])
        assert np.abs(M.T @ M - np.eye(M.shape[1])).max() <= 1e-13
    _, ref_norm = O.orthogonalize(X)
    assert abs(nrm - ref_norm) <= 1e-13 * ref_norm
    for _ in range(4):
        z = [rng.standard_normal(2) for _ in range(len(X))]
        zn = np.prod([np.linalg.norm(v) for v in z])
        assert abs(_rank1_probe(Yh, z) - _rank1_probe(X, z)) <= 1e-12 * ref_norm * zn


# ------------------------------------------------------------------ rounding (a3 + a4)
def check_round(got, ref_cores, ref_info, tol=1e-12, sig_tol=1e-12, ranks_exact=True):
    gh = host(got.cores)
    assert got.ranks[0] == 1 and got.ranks[-1] == 1
    if ranks_exact:
        assert ranks_agree(got.ranks, ref_info), (got.ranks, ref_info.ranks)
    err = O.rel_error(gh, ref_cores)
    assert err <= tol, err
    # right-orthonormal cores 2..n
    for c in gh[1:]:
        M = c.reshape(c.shape[0], -1)
        assert np.abs(M @ M.T - np.eye(M.shape[0])).max() <= 1e-13
    if got.sigmas is not None:
        for k, s in enumerate(ref_info.sigmas):
            g = np.array(got.sigmas[k][: len(s)])
            assert np.abs(g - s).max() <= sig_tol * s[0] + 1e-300
    return err


@pytest.mark.parametrize("case", ["tol0", "tol", "maxrank", "rankdef", "tiny", "single", "wide_tall"])
def test_round_small(case):
    log(f"round small {case}")
    rng = np.random.default_rng(104)
    tol, maxr = 0.0, 0
    if case in ("tol0", "tol", "maxrank"):
        A = rand_tt(rng, [1, 2, 2, 2, 2, 2, 2, 2, 1])
        B = rand_tt(rng, [1, 2, 4, 8, 11, 8, 4, 2, 1])
        X = O.tt_add(A, B, 1.0, 3e-3)
        if case == "tol":
            tol = 1e-3
        if case == "maxrank":
            maxr = 3
    elif case == "rankdef":
        Xa = rand_tt(rng, [1, 2, 3, 3, 2, 1])
        X = O.tt_add(Xa, Xa, 1.0, 1.0)  # duplicated blocks: exactly rank-deficient unfoldings
        tol = 1e-14
    elif case == "tiny":
        X = rand_tt(rng, [1, 2, 1])
    elif case == "single":
        X = rand_tt(rng, [1, 1])
    else:
        X = rand_tt(rng, [1, 2, 4, 8, 16, 21, 16, 8, 4, 2, 1], d=2)
        tol = 1e-2
    ref, info = O.round_tt(X, tol, maxr, return_info=True)
    got = Q.round_tt(dev(X), tol, maxr, want_sigmas=True)
    check_round(got, ref, info)
    if case == "tol0":
        assert O.rel_error(host(got.cores), X) <= 1e-13


@pytest.mark.timeout(600)
@pytest.mark.parametrize("peak,maxr", [(512, 0), (512, 400), (1024, 512)])
def test_round_longest_jacobi_rows(peak, maxr):
    """Ranks up to 512 (n = 20): the SVD sweep's matrices reach 512 rows of
    2 x 512 = 1024 entries, the longest rows the Jacobi takes (its widest LDS
    staging); untruncated and with the cap binding at 400.  With the middle
    rank 1024 and a cap of 512 (the cap keeps every row length within 1024)
    one matrix has 1024 rows of 2 x 512 entries: the most rows and the
    largest grid of the Jacobi."""
    n = 20
    ranks = [min(2 ** k, peak, 2 ** (n - k)) for k in range(n + 1)]
    log(f"round longest Jacobi rows, max rank {max(ranks)}, cap {maxr}")
    rng = np.random.default_rng(111)
    X = [rng.standard_normal((ranks[k], 2, ranks[k + 1])) / np.sqrt(2 * ranks[k + 1]) for k in range(n)]
    ref, info = O.round_tt(X, 0.0, maxr, return_info=True)
    got = Q.round_tt(dev(X), 0.0, maxr, want_sigmas=True)
    assert max(got.ranks) == (peak if maxr == 0 else maxr)
    check_round(got, ref, info)


def test_round_rejects_rows_longer_than_1024():
    """Without a cap, the core left of a rank-1024 bond splits into rows of
    2 x 1024 entries, past the Jacobi's limit: the size check refuses the
    call (QTT_ERR_UNSUPPORTED) before anything is launched."""
    n = 20
    ranks = [min(2 ** k, 1024, 2 ** (n - k)) for k in range(n + 1)]
    rng = np.random.default_rng(112)
    X = [rng.standard_normal((ranks[k], 2, ranks[k + 1])) for k in range(n)]
    with pytest.raises(Q.QttError, match="UNSUPPORTED"):
        Q.round_tt(dev(X), 0.0, 0)


def test_round_zero_tensor_is_rank1_zero():
    X = [np.zeros((1, 2, 3)), np.zeros((3, 2, 3)), np.zeros((3, 2, 1))]
    got = Q.round_tt(dev(X), 1e-8, 0)
    assert got.ranks == [1, 1, 1, 1]
    assert all(np.all(np.isfinite(c)) for c in host(got.cores))
    assert np.abs(O.to_dense(host(got.cores))).max() == 0.0


def test_round_nonfinite_rejected():
    X = [np.ones((1, 2, 2)), np.full((2, 2, 1), np.nan)]
    with pytest.raises(Q.QttError) as e:
        Q.round_tt(dev(X), 1e-8, 0)
    assert e.value.status == -8


@pytest.mark.parametrize("spec", ["i,i->i", "ij,j->i"])
def test_contract_round_random(spec):
    log(f"contract_round random {spec}")
    rng = np.random.default_rng(105)
    if spec == "i,i->i":
        A = rand_tt(rng, [1, 2, 4, 8, 13, 8, 4, 2, 1])
    else:
        A = rand_mpo(rng, [1, 3, 5, 5, 5, 5, 5, 3, 1])
    B = rand_tt(rng, [1, 2, 4, 8, 9, 8, 4, 2, 1])
    C = O.contract(spec, A, B)
    for tol, maxr in [(0.0, 0), (1e-6, 0), (0.0, 7)]:
        ref, info = O.round_tt(C, tol, maxr, return_info=True)
        got = Q.contract_round(spec, dev(A), dev(B), tol, maxr, want_sigmas=True)
        check_round(got, ref, info)


def test_sin_noise_1d_contract_round():
    log("sin_noise_1d contract_round")
    w = I.sin_noise_1d()
    C = O.contract(w.spec, w.a, w.b)
    ref, info = O.round_tt(C, w.rel_tol, 0, return_info=True)
    got = Q.contract_round(w.spec, dev(w.a), dev(w.b), w.rel_tol, 0, want_sigmas=True)
    assert got.ranks == [1, 2, 4, 8, 8, 8, 8, 8, 4, 2, 1]
    check_round(got, ref, info)
    dense = O.to_dense(w.a) * O.to_dense(w.b)
    assert np.linalg.norm(O.to_dense(host(got.cores)) - dense) <= 1e-14 * np.linalg.norm(dense)


def test_laplacian2d_r64_contract_round():
    log("laplacian2d contract_round")
    w = I.laplacian2d_r64()
    C = O.contract(w.spec, w.a, w.b)
    ref, info = O.round_tt(C, w.rel_tol, w.max_rank, return_info=True)
    got = Q.contract_round(w.spec, dev(w.a), dev(w.b), w.rel_tol, w.max_rank, want_sigmas=True)
    err = check_round(got, ref, info, tol=1e-12, sig_tol=1e-12)
    log(f"laplacian2d rel err {err:.3e} ranks {got.ranks}")


@pytest.mark.parametrize("m,D", [(16, 2), (14, 3)])
def test_laplacian_eigenvector_full_size(m, D):
    """round(Delta f) = lambda f with rank 2^D at the 2D (n=32) and 3D (n=42) sizes."""
    log(f"laplacian eigen m={m} D={D}")
    N = 2 ** m
    modes = [N // 3, N // 2 - 1, N // 3 + 5][:D]
    f, lam = None, 0.0
    for a in range(D):
        wv = math.pi * modes[a] / (N + 1)
        fa = I.trig_qtt(m, wv, wv, "sin")
        lam += 2.0 - 2.0 * math.cos(wv)
        ea = I.embed_axis(fa, D, a)
        f = ea if f is None else O.contract("i,i->i", f, ea)
    W = I.laplacian_mpo(m, D)
    got = Q.contract_round("ij,j->i", dev(W), dev(f), 1e-12, 0)
    assert max(got.ranks) == 2 ** D
    assert O.rel_error(host(got.cores), O.tt_scale(f, lam)) <= 1e-12


# ------------------------------------------------------------------ Jacobi sweep cap
def test_jacobi_sweep_cap_edge_and_noconv():
    """A rounding whose Jacobi needs s sweeps succeeds with the cap at s (it
    converges on its last allowed sweep) and fails with QTT_ERR_NOCONV at
    s - 1; the handle's cap is restored afterwards."""
    log("jacobi sweep cap")
    rng = np.random.default_rng(77)
    X = [rng.standard_normal(s) for s in [(1, 2, 8), (8, 2, 24), (24, 2, 24), (24, 2, 8), (8, 2, 1)]]
    try:
        got = Q.round_tt(dev(X), 1e-10, 0)
        s = got.jacobi_sweeps_max
        assert 2 <= s < 80
        Q.set_jacobi_max_sweeps(s)
        again = Q.round_tt(dev(X), 1e-10, 0)
        assert again.ranks == got.ranks and again.jacobi_sweeps_max == s
        Q.set_jacobi_max_sweeps(s - 1)
        with pytest.raises(Q.QttError) as ei:
            Q.round_tt(dev(X), 1e-10, 0)
        assert ei.value.status == -9
        Q.set_jacobi_max_sweeps(1)
        Y = [rng.standard_normal(s) for s in [(1, 2, 2), (2, 2, 2), (2, 2, 2), (2, 2, 2), (2, 2, 1)]]
        with pytest.raises(Q.QttError) as ei:
            Q.contract_zipup("i,i->i", dev(X), dev(Y), 1e-10, 0, ncores=1)
        assert ei.value.status == -9
    finally:
        Q.set_jacobi_max_sweeps(0)
    assert Q.round_tt(dev(X), 1e-10, 0).jacobi_sweeps_max == s
