"""C-ABI checks that need no GPU: exports, status codes, argument errors, planning."""
import ctypes as C
import os
import re

import pytest

from paper_2602_20226_amd import qtt as Q
from paper_2602_20226_amd.build import LIB

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "qtt.h")

pytestmark = pytest.mark.skipif(not os.path.exists(LIB), reason="libqtt.so not built (run __graft_entry__.build())")


def header_functions():
    txt = open(HEADER).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    return sorted(set(re.findall(r"\b(qtt_[a-z0-9_]+)\s*\(", txt)))


def test_every_declared_symbol_is_exported():
    L = C.CDLL(LIB)
    names = header_functions()
    assert len(names) >= 11
    for n in names:
        assert hasattr(L, n), n
    assert set(names) == set(Q.EXPORTS)


def test_status_strings():
    L = Q.load_library()
    for code in range(0, -11, -1):
        s = L.qtt_status_string(code).decode()
        assert s and s != "unknown status"
    assert L.qtt_status_string(-99).decode() == "unknown status"


def test_create_without_gpu_or_bad_args():
    L = Q.load_library()
    h = C.c_void_p()
    assert L.qtt_create(None, 0) == -1
    st = L.qtt_create(C.byref(h), 10_000)
    assert st == -6  # QTT_ERR_NODEVICE: no such device (none at all in the CPU container)
    assert L.qtt_destroy(None) == -1


def _fake_tt(ranks, phys, legs=1, null_core=False):
    n = len(ranks) - 1
    ph = (C.c_int32 * (n * legs))(*phys)
    rk = (C.c_int64 * (n + 1))(*ranks)
    ptrs = (C.c_void_p * n)(*([None] * n if null_core else [0x1000 + 64 * k for k in range(n)]))
    t = Q.TT(n, legs, ph, rk, ptrs, Q.F64)
    t._keep = (ph, rk, ptrs)
    return t


def test_null_handle_rejected_by_compute_calls():
    L = Q.load_library()
    a = _fake_tt([1, 2, 1], [2, 2])
    out = C.c_double()
    assert L.qtt_inner(None, C.byref(a), C.byref(a), C.byref(out), None, 0, None) == -1
    assert L.qtt_contract(None, b"i,i->i", C.byref(a), C.byref(a), C.byref(a), None, 0, None) == -1
    assert L.qtt_round(None, C.byref(a), 1e-8, 0, 0, None, None, 0, None) == -1
    assert L.qtt_set_jacobi_max_sweeps(None, 5) == -1
    assert L.qtt_inner_prec(None, C.byref(a), C.byref(a), 3, C.byref(out), None, 0, None) == -1
    assert L.qtt_contract_round_noalloc(None, b"i,i->i", C.byref(a), C.byref(a), C.byref(a), 1e-8, 0, 0,
                                        None, None) == -1


def ws(op, a, b=None, spec=None, max_rank=0, prec=0):
    L = Q.load_library()
    nb = C.c_size_t()
    st = L.qtt_workspace_size(None, op, spec, C.byref(a), C.byref(b) if b is not None else None, max_rank, prec,
                              C.byref(nb))
    return st, nb.value


def test_workspace_planning_and_shape_errors():
    a = _fake_tt([1, 2, 4, 2, 1], [2, 2, 2, 2])
    st, nb = ws(Q.OP_ROUND, a)
    assert st == 0 and nb > 0
    st, _ = ws(Q.OP_INNER, a, a)
    assert st == 0
    # boundary rank must be 1
    bad = _fake_tt([2, 2, 1], [2, 2])
    assert ws(Q.OP_ROUND, bad)[0] == -3
    # unsupported einsum string
    assert ws(Q.OP_CONTRACT_ROUND, a, a, b"ijk->i")[0] == -2
    # the operator product has no fused rounding (its result is an MPO)
    assert ws(Q.OP_CONTRACT_ROUND, a, a, b"ij,jk->ik")[0] == -10
    # MPO operand must have two legs
    assert ws(Q.OP_CONTRACT_ROUND, a, a, b"ij,j->i")[0] == -3
    # physical size mismatch in a Hadamard product
    c = _fake_tt([1, 2, 4, 2, 1], [2, 3, 2, 2])
    assert ws(Q.OP_CONTRACT_ROUND, a, c, b"i,i->i")[0] == -3
    # null core pointer
    z = _fake_tt([1, 2, 1], [2, 2], null_core=True)
    assert ws(Q.OP_ROUND, z)[0] == -1


def test_workspace_for_the_benchmark_shapes():
    import qtt_inputs as I
    from paper_2602_20226_amd.qtt import rank_bounds
    w = I.laplacian3d_r256()
    ra = [1] + [c.shape[-1] for c in w.a]
    rb = [1] + [c.shape[-1] for c in w.b]
    n = len(w.a)
    W = _fake_tt(ra, [2] * (2 * n), legs=2)
    X = _fake_tt(rb, [2] * n)
    st, nb = ws(Q.OP_CONTRACT_ROUND, W, X, b"ij,j->i", 256, 3)
    assert st == 0
    # QR-sweep factors (41 matrices up to 3584 x 1792) dominate: a few GB, well inside 288 GB HBM
    assert 1e9 < nb < 1.2e10
    bnd = rank_bounds([x * y for x, y in zip(ra, rb)], [2] * n, 256)
    assert max(bnd) == 256 and bnd[0] == bnd[-1] == 1
    # too-tall unfolding (rank 2049 * d = 4098 rows) is outside the implemented range
    big = _fake_tt([1, 2, 4096, 2, 1], [2, 2048, 2, 2])
    assert ws(Q.OP_ROUND, big)[0] in (-10, -3)


def test_rank_bounds_match_profile():
    from paper_2602_20226_amd.qtt import rank_bounds
    b = rank_bounds([1, 4, 16, 64, 16, 4, 1], [2] * 6, 0)
    assert b == [1, 2, 4, 8, 4, 2, 1]
    b = rank_bounds([1, 4, 16, 64, 16, 4, 1], [2] * 6, 3)
    assert b == [1, 2, 3, 3, 3, 2, 1]


def test_orthogonalisation_plans_the_largest_unfolding():
    """Ranks 2048 make 4096 x 2048 unfoldings: the QR supports them, the Jacobi
    of the rounding sweep (rows of length <= 1024) does not."""
    n = 24
    ranks = [min(2 ** k, 2048, 2 ** (n - k)) for k in range(n + 1)]
    a = _fake_tt(ranks, [2] * n)
    st, nb = ws(Q.OP_ORTHOGONALIZE, a)
    assert st == 0 and nb > 0
    assert ws(Q.OP_ROUND, a)[0] == -10  # QTT_ERR_UNSUPPORTED
    n2 = 26
    too_tall = _fake_tt([min(2 ** k, 4096, 2 ** (n2 - k)) for k in range(n2 + 1)], [2] * n2)  # 8192-row unfolding
    assert ws(Q.OP_ORTHOGONALIZE, too_tall)[0] == -10


@pytest.mark.parametrize("N", [1, 2])
def test_zipup_query_bounds_equal_untruncated_oracle_ranks(N):
    """Untruncated zip-up of random operands keeps every singular value, so its
    ranks equal the planned bounds exactly."""
    import numpy as np
    import oracle as O
    rng = np.random.default_rng(50 + N)
    rx = [1, 2, 4, 8, 8, 8, 8, 4, 2, 1]
    rw = [1, 3, 5, 5, 5, 5, 5, 5, 3, 1]
    X = [rng.standard_normal((rx[k], 2, rx[k + 1])) for k in range(9)]
    W = [rng.standard_normal((rw[k], 2, 2, rw[k + 1])) for k in range(9)]
    _, info = O.zipup("ij,j->i", W, X, 0.0, ncores=N, return_info=True)
    a = _fake_tt(rw, [2] * 18, legs=2)
    b = _fake_tt(rx, [2] * 9)
    bnd, nb = Q.zipup_query("ij,j->i", a, b, 0, N)
    assert bnd == info.ranks
    assert nb > 0
    bnd5, _ = Q.zipup_query("ij,j->i", a, b, 5, N)
    assert max(bnd5) <= 5 and all(x <= y for x, y in zip(bnd5, bnd))


def test_zipup_query_errors_and_benchmark_shape():
    L = Q.load_library()
    a = _fake_tt([1, 2, 1], [2, 2, 2, 2], legs=2)
    b = _fake_tt([1, 2, 1], [2, 2])
    nb = C.c_size_t()
    assert L.qtt_zipup_query(b"ij,j->i", C.byref(a), C.byref(b), 0, 3, None, C.byref(nb)) == -10
    assert L.qtt_zipup_query(b"ij,j->i", C.byref(a), C.byref(a), 0, 1, None, C.byref(nb)) == -3
    assert L.qtt_zipup_query(b"ij->i", C.byref(a), C.byref(b), 0, 1, None, C.byref(nb)) == -2
    assert L.qtt_contract_zipup(None, b"ij,j->i", C.byref(a), C.byref(b), C.byref(b), 1e-8, 0, 1, 0, None,
                                None, 0, None) == -1
    # 3D Laplacian (rank 7) x rank-256 MPS, n = 42: splits up to 512 x 3584
    n = 42
    rx = [min(256, 2 ** k, 2 ** (n - k)) for k in range(n + 1)]
    rw = [1] + [7] * (n - 1) + [1]
    a = _fake_tt(rw, [2] * (2 * n), legs=2)
    b = _fake_tt(rx, [2] * n)
    for N in (1, 2):
        bnd, nbytes = Q.zipup_query("ij,j->i", a, b, 256, N)
        assert max(bnd) == 256 and bnd[0] == bnd[-1] == 1
        assert nbytes < 2 * 1024 ** 3


def test_add_rejects_null_handle_and_arguments():
    L = Q.load_library()
    a = _fake_tt([1, 2, 1], [2, 2])
    arr = (Q.TT * 2)(a, a)
    out = _fake_tt([1, 4, 1], [2, 2])
    assert L.qtt_add(None, 2, arr, None, C.byref(out), None) == -1
    assert L.qtt_contract(None, b"ij,jk->ik", C.byref(a), C.byref(a), C.byref(a), None, 0, None) == -1


def test_fit_workspace_size_and_shape_errors():
    L = Q.load_library()
    n = 42
    rx = [min(256, 2 ** k, 2 ** (n - k)) for k in range(n + 1)]
    rw = [1] + [7] * (n - 1) + [1]
    a = _fake_tt(rw, [2] * (2 * n), legs=2)
    b = _fake_tt(rx, [2] * n)
    c = _fake_tt(rx, [2] * n)
    nb = C.c_size_t()
    assert L.qtt_fit_workspace_size(b"ij,j->i", C.byref(a), C.byref(b), C.byref(c), C.byref(nb)) == 0
    # the exactly contracted product (rank 7 x 256) alone is 1.4 GB
    assert 1.3e9 < nb.value < 3e9
    bad = _fake_tt(rx, [3] * n)
    assert L.qtt_fit_workspace_size(b"ij,j->i", C.byref(a), C.byref(b), C.byref(bad), C.byref(nb)) == -3
    assert L.qtt_fit_workspace_size(b"ij,jk->ik", C.byref(a), C.byref(b), C.byref(c), C.byref(nb)) == -10
    assert L.qtt_fit(None, b"ij,j->i", C.byref(a), C.byref(b), C.byref(c), 1, None, None, 0, None) == -1


def test_fit2_and_solve_queries_bounds_and_errors():
    """Rank capacities and workspace of the two-core fit and the linear
    solver from the shapes alone, and their argument errors."""
    L = Q.load_library()
    n = 6
    W = _fake_tt([1, 3, 5, 5, 5, 3, 1], [2] * (2 * n), legs=2)
    b = _fake_tt([1, 2, 4, 4, 4, 2, 1], [2] * n)
    x = _fake_tt([1, 2, 2, 2, 2, 2, 1], [2] * n)
    bnd = (C.c_int64 * (n + 1))()
    nb = C.c_size_t()
    # two-core fit: bounds min(left, right, product rank, cap), at least the guess's
    assert L.qtt_fit2_query(b"ij,j->i", C.byref(W), C.byref(b), C.byref(x), 0, bnd, C.byref(nb)) == 0
    assert list(bnd) == [1, 2, 4, 8, 4, 2, 1] and nb.value > 0
    assert L.qtt_fit2_query(b"ij,j->i", C.byref(W), C.byref(b), C.byref(x), 3, bnd, C.byref(nb)) == 0
    assert list(bnd) == [1, 2, 3, 3, 3, 2, 1]
    assert L.qtt_fit2_query(b"ijk->i", C.byref(W), C.byref(b), C.byref(x), 0, bnd, C.byref(nb)) == -2
    short = _fake_tt([1, 2, 2, 1], [2] * 3)
    assert L.qtt_fit2_query(b"ij,j->i", C.byref(W), C.byref(b), C.byref(short), 0, bnd, C.byref(nb)) == -3
    # linear solver: one core keeps the guess's ranks, two cores grow to the cap
    assert L.qtt_solve_query(C.byref(W), C.byref(b), C.byref(x), 1, 0, bnd, C.byref(nb)) == 0
    assert list(bnd) == [1, 2, 2, 2, 2, 2, 1]
    assert L.qtt_solve_query(C.byref(W), C.byref(b), C.byref(x), 2, 4, bnd, C.byref(nb)) == 0
    assert list(bnd) == [1, 2, 4, 4, 4, 2, 1]
    assert L.qtt_solve_query(C.byref(W), C.byref(b), C.byref(x), 3, 4, bnd, C.byref(nb)) == -1
    assert L.qtt_solve_query(C.byref(W), C.byref(b), C.byref(short), 1, 0, bnd, C.byref(nb)) == -3
    rect = _fake_tt([1, 3, 5, 5, 5, 3, 1], [2, 3] * n, legs=2)  # d_out != d_in
    assert L.qtt_solve_query(C.byref(rect), C.byref(b), C.byref(x), 1, 0, bnd, C.byref(nb)) == -3
    # two cores with no cap: local systems beyond the QR limit are refused
    big = _fake_tt([1] + [2 ** min(k, 24 - k) for k in range(1, 24)] + [1], [2] * 24)
    W24 = _fake_tt([1] + [5] * 23 + [1], [2] * 48, legs=2)
    b24 = _fake_tt([1] + [2] * 23 + [1], [2] * 24)
    bnd24 = (C.c_int64 * 25)()
    assert L.qtt_solve_query(C.byref(W24), C.byref(b24), C.byref(big), 2, 0, bnd24, C.byref(nb)) == -10
    assert L.qtt_solve(None, C.byref(W), C.byref(b), C.byref(x), 1, 1, 0.0, 0, None, None, 0, None) == -1
    # AMEn: z's bounds are its left-orthogonalised ranks; x's hold the cap
    # plus z's rank, within the larger unfolding size
    z = _fake_tt([1, 3, 3, 3, 3, 3, 1], [2] * n)
    bz = (C.c_int64 * (n + 1))()
    assert L.qtt_solve_amen_query(C.byref(W), C.byref(b), C.byref(x), C.byref(z), 4, bnd, bz, C.byref(nb)) == 0
    assert list(bz) == [1, 2, 3, 3, 3, 3, 1]
    assert list(bnd) == [1, 6, 7, 7, 7, 7, 1] and nb.value > 0
    assert L.qtt_solve_amen_query(C.byref(W), C.byref(b), C.byref(x), C.byref(z), 0, bnd, None, C.byref(nb)) == 0
    assert list(bnd) == [1, 32, 16, 8, 16, 32, 1]
    assert L.qtt_solve_amen_query(C.byref(W), C.byref(b), C.byref(x), C.byref(z), 4, None, None, None) == -1
    assert L.qtt_solve_amen_query(C.byref(W), C.byref(b), C.byref(x), C.byref(short), 4, bnd, bz,
                                  C.byref(nb)) == -3
    z24 = _fake_tt([1] + [4] * 23 + [1], [2] * 24)
    x24 = _fake_tt([1] + [2] * 23 + [1], [2] * 24)
    assert L.qtt_solve_amen_query(C.byref(W24), C.byref(b24), C.byref(x24), C.byref(z24), 0, bnd24, None,
                                  C.byref(nb)) == -10
    assert L.qtt_solve_amen_query(C.byref(W24), C.byref(b24), C.byref(x24), C.byref(z24), 32, bnd24, None,
                                  C.byref(nb)) == 0
    assert max(bnd24) == 36
    assert L.qtt_solve_amen(None, C.byref(W), C.byref(b), C.byref(x), C.byref(z), 1, 0.0, 0, None, None, 0,
                            None) == -1
    assert L.qtt_fit2(None, b"ij,j->i", C.byref(W), C.byref(b), C.byref(x), 1, 0.0, 0, None, None, 0, None) == -1
