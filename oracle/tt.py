"""FP64 oracle implementation (test infrastructure only; see package docstring).

Core layouts: MPS core [r_l, d, r_r], MPO core [r_l, d_out, d_in, r_r], all
float64 row-major.  Core 0 holds the most significant digit (Sec. 2, eq.
quantization).
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field
from typing import List, Optional, Sequence

import numpy as np

__all__ = [
    "contract",
    "tt_add",
    "tt_sum",
    "tt_scale",
    "orthogonalize",
    "orthogonalize_right",
    "round_tt",
    "zipup",
    "fit",
    "fit_two_core",
    "solve_energy",
    "solve_amen",
    "RoundInfo",
    "truncation_rank",
    "cut_gaps",
    "noise_amplification",
    "inner",
    "norm",
    "rel_error",
    "diff_norm",
    "to_dense",
    "mpo_to_dense",
    "ranks_of",
    "bond_singular_values",
    "shift_mpo_paper",
    "dense_shift",
    "dense_laplacian",
    "interleaved_index",
    "env_left",
    "env_right",
    "inner_grad",
    "contract_grad",
    "loss_axb",
    "grad_axb",
    "grad_axb_sandwich",
]


# --------------------------------------------------------------------------
# exact operations (Sec. 3.1)
# --------------------------------------------------------------------------
def contract(spec: str, A: Sequence[np.ndarray], B: Sequence[np.ndarray]):
    """Core-by-core Einstein summation (eq. einsum).

    'i,i->i':  C_k[(mu,nu), i, (mu',nu')] = A_k[mu,i,mu'] B_k[nu,i,nu']
    'ij,j->i': C_k[(mu,nu), i, (mu',nu')] = sum_j A_k[mu,i,j,mu'] B_k[nu,j,nu']
    'ij,jk->ik': C_k[(mu,nu), i, k, (mu',nu')] = sum_j A_k[mu,i,j,mu'] B_k[nu,j,k,nu']
                 (operator product, both operands MPOs)
    The flattened bond is xi = mu * r_B + nu (mu major), as in the flatten
    xi_q = overline{mu_q nu_q} of the paper.
    """
    if len(A) != len(B):
        raise ValueError("core count mismatch")
    out = []
    for a, b in zip(A, B):
        if spec == "i,i->i":
            c = np.einsum("aib,cid->acibd", a, b)
            ra, d, rb = a.shape
            rc, _, rd = b.shape
            out.append(c.reshape(ra * rc, d, rb * rd))
        elif spec == "ij,j->i":
            c = np.einsum("aijb,cjd->acibd", a, b)
            ra, di, dj, rb = a.shape
            rc, _, rd = b.shape
            out.append(c.reshape(ra * rc, di, rb * rd))
        elif spec == "ij,jk->ik":
            c = np.einsum("aijb,cjkd->acikbd", a, b)
            ra, di, dj, rb = a.shape
            rc, _, dk, rd = b.shape
            out.append(c.reshape(ra * rc, di, dk, rb * rd))
        else:
            raise ValueError(f"unsupported spec {spec!r}")
    return out


def tt_add(X, Y, alpha: float = 1.0, beta: float = 1.0):
    """alpha X + beta Y as an exact TT with block cores (Sec. 3.1, addition).

    First core [X_1 Y_1] (row), middle cores diag(X_k, Y_k), last core
    [X_n; Y_n] (column); the scalars are folded into the first core.
    """
    n = len(X)
    if n != len(Y):
        raise ValueError("core count mismatch")
    if n == 1:
        return [alpha * X[0] + beta * Y[0]]
    out = []
    for k in range(n):
        x, y = X[k], Y[k]
        rx0, rx1 = x.shape[0], x.shape[-1]
        ry0, ry1 = y.shape[0], y.shape[-1]
        mid = x.shape[1:-1]  # physical legs: one (MPS) or two (MPO)
        if k == 0:
            c = np.concatenate([alpha * x, beta * y], axis=x.ndim - 1)
        elif k == n - 1:
            c = np.concatenate([x, y], axis=0)
        else:
            c = np.zeros((rx0 + ry0,) + mid + (rx1 + ry1,))
            c[:rx0, ..., :rx1] = x
            c[rx0:, ..., rx1:] = y
        out.append(c)
    return out


def tt_sum(terms, coeffs=None):
    """sum_t c_t X_t as one exact TT (Sec. 3.1, addition of many trains).

    The block structure of tt_add taken over all terms at once: the first
    core is the row [c_1 X_1, c_2 X_2, ...], the last the column of the
    terms' last cores, the middle cores block-diagonal in term order; it
    equals folding tt_add from the left.
    """
    if coeffs is None:
        coeffs = [1.0] * len(terms)
    out = tt_scale(terms[0], coeffs[0])
    for X, c in zip(terms[1:], coeffs[1:]):
        out = tt_add(out, X, 1.0, c)
    return out


def tt_scale(X, s: float):
    out = [c.copy() for c in X]
    out[0] = out[0] * s
    return out


def ranks_of(X) -> List[int]:
    return [X[0].shape[0]] + [c.shape[-1] for c in X]


# --------------------------------------------------------------------------
# orthogonalisation (QR sweep) -- normalisation step of Sec. 3.2
# --------------------------------------------------------------------------
def orthogonalize(X):
    """Left-to-right QR sweep.  Returns (cores, norm).

    For k = 1..n-1: the (r_{k-1} d) x r_k unfolding of core k is factored
    Q R (reduced QR, signs fixed so that diag(R) >= 0); Q becomes core k and R
    is multiplied into core k+1.  A wide unfolding gives the new rank
    r_{k-1} d.  The norm of the tensor is the Frobenius norm of the last core.
    """
    cores = [np.array(c, dtype=np.float64, copy=True) for c in X]
    n = len(cores)
    for k in range(n - 1):
        c = cores[k]
        r0 = c.shape[0]
        mid = c.shape[1:-1]
        r1 = c.shape[-1]
        M = c.reshape(-1, r1)
        Q, R = np.linalg.qr(M, mode="reduced")
        s = np.sign(np.diag(R))
        s[s == 0] = 1.0
        Q = Q * s[None, :]
        R = R * s[:, None]
        q = Q.shape[1]
        cores[k] = Q.reshape((r0,) + mid + (q,))
        nxt = cores[k + 1]
        cores[k + 1] = np.tensordot(R, nxt, axes=([1], [0]))
    nrm = float(np.linalg.norm(cores[-1].ravel()))
    return cores, nrm


# --------------------------------------------------------------------------
# rounding (QR sweep + truncated SVD sweep)
# --------------------------------------------------------------------------
@dataclass
class RoundInfo:
    norm: float = 0.0
    delta: float = 0.0
    err_bound: float = 0.0
    ranks: List[int] = field(default_factory=list)
    tails: List[float] = field(default_factory=list)       # per bond 1..n-1
    margin_lo: List[float] = field(default_factory=list)   # tail(r-1)/delta
    margin_hi: List[float] = field(default_factory=list)   # tail(r)/delta
    maxrank_hit: List[bool] = field(default_factory=list)
    sigmas: List[np.ndarray] = field(default_factory=list)  # per bond 1..n-1
    gaps: List[float] = field(default_factory=list)         # per bond: (s_r - s_{r+1}) / s_r
    deltas: List[float] = field(default_factory=list)       # per bond: truncation threshold used


def truncation_rank(sig: np.ndarray, delta: float, max_rank: int):
    """Smallest r >= 1 with sqrt(sum_{i>r} sigma_i^2) <= delta, capped at max_rank.

    Returns (r, tail(r), tail(r-1), capped).  The tail sums are accumulated
    from the smallest singular value upwards.
    """
    s = np.asarray(sig, dtype=np.float64)
    m = s.size
    tail2 = np.zeros(m + 1)  # tail2[r] = sum_{i >= r} s_i^2 (0-based i)
    acc = 0.0
    for i in range(m - 1, -1, -1):
        acc += s[i] * s[i]
        tail2[i] = acc
    r = m
    for cand in range(1, m + 1):
        if math.sqrt(tail2[cand]) <= delta:
            r = cand
            break
    capped = False
    if max_rank and max_rank > 0 and r > max_rank:
        r = max_rank
        capped = True
    r = max(1, min(r, max(m, 1)))
    t_r = math.sqrt(tail2[r]) if r <= m else 0.0
    t_rm1 = math.sqrt(tail2[r - 1]) if r - 1 <= m else 0.0
    return r, t_r, t_rm1, capped


def round_tt(X, rel_tol: float, max_rank: int = 0, return_info: bool = False):
    """TT rounding: QR sweep left to right, truncated SVD sweep right to left.

    delta = rel_tol * ||X|| / sqrt(n-1).  At bond k the kept rank is the
    smallest r >= 1 whose discarded singular values have 2-norm <= delta,
    capped at max_rank (max_rank <= 0: no cap).  A zero tensor rounds to
    rank 1.
    """
    n = len(X)
    cores, nrm = orthogonalize(X)
    info = RoundInfo(norm=nrm)
    if n == 1:
        info.ranks = ranks_of(cores)
        return (cores, info) if return_info else cores
    delta = rel_tol * nrm / math.sqrt(n - 1)
    info.delta = delta
    tails = [0.0] * (n - 1)
    mlo = [0.0] * (n - 1)
    mhi = [0.0] * (n - 1)
    hit = [False] * (n - 1)
    sigs = [None] * (n - 1)
    for k in range(n - 1, 0, -1):
        c = cores[k]
        r0 = c.shape[0]
        mid = c.shape[1:-1]
        r1 = c.shape[-1]
        B = c.reshape(r0, -1)
        U, S, Vt = np.linalg.svd(B, full_matrices=False)
        r, t_r, t_rm1, capped = truncation_rank(S, delta, max_rank)
        if nrm == 0.0:
            r, t_r, t_rm1 = 1, 0.0, 0.0
        sigs[k - 1] = S.copy()
        tails[k - 1] = t_r
        hit[k - 1] = capped
        mlo[k - 1] = (t_rm1 / delta) if delta > 0 else math.inf
        mhi[k - 1] = (t_r / delta) if delta > 0 else 0.0
        cores[k] = Vt[:r].reshape((r,) + mid + (r1,))
        US = U[:, :r] * S[None, :r]
        prev = cores[k - 1]
        cores[k - 1] = np.tensordot(prev, US, axes=([prev.ndim - 1], [0]))
    info.ranks = ranks_of(cores)
    info.tails = tails
    info.margin_lo = mlo
    info.margin_hi = mhi
    info.maxrank_hit = hit
    info.sigmas = sigs
    info.gaps = cut_gaps(sigs, info.ranks)
    info.deltas = [delta] * (n - 1)
    info.err_bound = math.sqrt(sum(t * t for t in tails))
    return (cores, info) if return_info else cores


def cut_gaps(sigmas, ranks) -> List[float]:
    """Relative singular-value gap at every bond's cut: (s_r - s_{r+1}) / s_r.

    r is the kept rank at the bond and s the bond's singular values before
    truncation.  When nothing is discarded (r equals the number of singular
    values) the kept subspace is the whole space and the gap is reported as
    inf.  The rounding of a perturbed input moves the kept subspace by about
    ||perturbation|| / (s_r - s_{r+1}) (Wedin's bound for the truncated SVD),
    so a small gap marks a bond where several truncations are equally valid
    and a tiny input change is amplified.
    """
    out = []
    for b, s in enumerate(sigmas):
        s = np.asarray(s, dtype=np.float64)
        r = ranks[b + 1]
        if r >= s.size or s[r - 1] <= 0.0:
            out.append(math.inf)
        else:
            out.append(float((s[r - 1] - s[r]) / s[r - 1]))
    return out


def noise_amplification(X, rel_tol: float, max_rank: int = 0, eps: float = 1e-10, seed: int = 0,
                        trials: int = 2):
    """How much the rounding amplifies a small relative change of its input.

    Every core of X receives independent Gaussian noise of relative Frobenius
    size eps (X_k + eps ||X_k|| G / ||G||); the perturbed train is rounded with
    the same tolerance and rank cap, and the change of the rounded tensor is
    divided by the change of the input tensor, both measured exactly through
    difference trains.  Returns (largest ratio over the trials, list of
    ratios).  A ratio near 1 means the truncation decisions are stable; a
    large one means an error of a given size in any implementation's
    contraction (different rounding order, reduced-precision products) shows
    up multiplied by that factor in the rounded result.
    """
    rng = np.random.default_rng(seed)
    base = round_tt(X, rel_tol, max_rank)
    ratios = []
    for _ in range(trials):
        Xp = []
        for c in X:
            g = rng.standard_normal(c.shape)
            Xp.append(c + eps * np.linalg.norm(c) / np.linalg.norm(g) * g)
        d_in = diff_norm(Xp, X)
        out = round_tt(Xp, rel_tol, max_rank)
        d_out = diff_norm(out, base)
        ratios.append(d_out / d_in if d_in > 0 else 0.0)
    return max(ratios), ratios


def orthogonalize_right(X):
    """Right-to-left QR sweep.  Returns (cores, norm).

    Moves the normalisation centre to the left end (the preparation step of
    the decomposition algorithm, Sec. 3.2): for k = n..2 the r_{k-1} x (P r_k)
    unfolding G of core k (P = all physical legs) is factored through a
    reduced QR of its transpose, G^T = Q R with diag(R) >= 0; core k becomes
    Q^T (right-orthonormal: G G^T = I) and R^T is multiplied into core k-1
    from the right.  A tall G^T keeps the rank, a wide one gives P r_k.  The
    norm of the tensor is the Frobenius norm of the first core.
    """
    cores = [np.array(c, dtype=np.float64, copy=True) for c in X]
    n = len(cores)
    for k in range(n - 1, 0, -1):
        c = cores[k]
        r0 = c.shape[0]
        rest = c.shape[1:]
        G = c.reshape(r0, -1)
        Q, R = np.linalg.qr(G.T, mode="reduced")
        s = np.sign(np.diag(R))
        s[s == 0] = 1.0
        Q = Q * s[None, :]
        R = R * s[:, None]
        q = Q.shape[1]
        cores[k] = Q.T.reshape((q,) + rest)
        prev = cores[k - 1]
        cores[k - 1] = np.tensordot(prev, R.T, axes=([prev.ndim - 1], [0]))
    nrm = float(np.linalg.norm(cores[0].ravel()))
    return cores, nrm


def zipup(spec: str, A, B, rel_tol: float, max_rank: int = 0, ncores: int = 1, return_info: bool = False):
    """Decomposition ("zip-up") algorithm of Sec. 3.2 for contract(spec, A, B)
    with super-cores of N = ncores exact product cores.

    1. Both operands move their normalisation centre to the left end
       (orthogonalize_right).
    2. The super-core S (r x P x r_C, P = d^j for j physical legs, starting as
       [[1]]) grows by one exact local product core C_k (eq. einsum) at a time:
       S <- S C_k.
    3. Whenever S holds N physical legs and more cores remain, and until it
       holds one leg after the last core was added, S is split off one core:
       the (r d) x (rest) unfolding is factored S = U Sig V^T (SVD), the kept
       rank follows the rule of round_tt with delta = rel_tol ||S|| /
       sqrt(n-1), capped at max_rank; the next result core is U_r
       (left-orthonormal, so the normalisation stays on the remainder) and
       S <- Sig_r V_r^T.
    4. The final one-leg S is the last core.

    The paper takes the norm of the result to sit in the super-core once the
    centres are at the left end; that holds only when the exact right part
    of the product is orthonormal, which the operands' normalisation does
    not ensure (an operator normalised in the Frobenius sense carries a
    factor per core).  The norm in delta is therefore that of the super-core
    being split, which makes each decision independent of such factors;
    info.norm reports the first super-core's norm.

    The discarded singular values are reported like round_tt's, but their
    2-norm bounds the error only when the exact right part of the product is
    orthonormal (for example when one operand is the identity operator).
    """
    n = len(A)
    if len(B) != n:
        raise ValueError("core count mismatch")
    if ncores < 1:
        raise ValueError("ncores >= 1")
    N = min(ncores, n)
    A0, _ = orthogonalize_right(A)
    B0, _ = orthogonalize_right(B)
    info = RoundInfo()
    nb = max(n - 1, 0)
    tails = [0.0] * nb
    mlo = [0.0] * nb
    mhi = [0.0] * nb
    hit = [False] * nb
    sigs = [None] * nb
    deltas = [0.0] * nb
    out = []
    S = np.ones((1, 1, 1))  # [r, P, r_C]
    legs = 0
    nrm = 0.0
    delta = 0.0
    for k in range(n):
        Ck = contract(spec, [A0[k]], [B0[k]])[0]  # [r_C, d, r_C']
        r0, P, _ = S.shape
        S = np.tensordot(S, Ck, axes=([2], [0])).reshape(r0, P * Ck.shape[1], Ck.shape[2])
        legs += 1
        if legs == N and k == N - 1:
            nrm = float(np.linalg.norm(S.ravel()))
        while (legs == N and k < n - 1) or (k == n - 1 and legs > 1):
            r0, P, rc = S.shape
            delta = rel_tol * float(np.linalg.norm(S.ravel())) / math.sqrt(n - 1)
            d = Ck.shape[1] if legs == 1 else A0[len(out)].shape[1]
            U, Sig, Vt = np.linalg.svd(S.reshape(r0 * d, (P // d) * rc), full_matrices=False)
            b = len(out)  # bond between result cores b and b+1
            r, t_r, t_rm1, capped = truncation_rank(Sig, delta, max_rank)
            if nrm == 0.0:
                r, t_r, t_rm1 = 1, 0.0, 0.0
            sigs[b] = Sig.copy()
            deltas[b] = delta
            tails[b] = t_r
            hit[b] = capped
            mlo[b] = (t_rm1 / delta) if delta > 0 else math.inf
            mhi[b] = (t_r / delta) if delta > 0 else 0.0
            out.append(U[:, :r].reshape(r0, d, r))
            S = (Sig[:r, None] * Vt[:r]).reshape(r, P // d, rc)
            legs -= 1
    out.append(S)
    info.norm = nrm
    info.delta = delta
    info.ranks = ranks_of(out)
    info.tails = tails
    info.margin_lo = mlo
    info.margin_hi = mhi
    info.maxrank_hit = hit
    info.sigmas = sigs
    info.deltas = deltas
    info.gaps = cut_gaps(sigs, info.ranks)
    info.err_bound = math.sqrt(sum(t * t for t in tails))
    return (out, info) if return_info else out


def _qr_pos(M):
    """Reduced QR with diag(R) >= 0."""
    Qm, R = np.linalg.qr(M, mode="reduced")
    s = np.sign(np.diag(R))
    s[s == 0] = 1.0
    return Qm * s[None, :], R * s[:, None]


def fit(spec: str, A, B, C0, nsweeps: int = 1):
    """Variational fitting of C to the product Y = contract(spec, A, B)
    (Sec. 3.3, eq. variational), one core at a time with the ranks of C.

    With every core left of q left-orthonormal and every core right of q
    right-orthonormal, the core that minimises ||C - Y|| is the derivative
    d<C|Y>/dC_q^* = L_{q-1} Y_q R_{q+1}, where L and R are the left and right
    environments of <C|Y> (Y's cores are contracted exactly).  The guess is
    first orthogonalised from the left (centre at core n, as the
    decomposition algorithm leaves it).  A sweep then updates the cores from
    right to left -- each updated core except the first is replaced by Q^T
    from a QR of its transposed unfolding, so that the centre moves left --
    and back from left to right with a QR of each updated core except the
    last.  Ranks never grow (a QR may shrink one).  Returns the cores.
    """
    Y = [_mat(c) for c in contract(spec, A, B)]
    C, _ = orthogonalize(C0)
    C = [_mat(c).copy() for c in C]
    n = len(C)
    one = np.ones((1, 1))
    for _ in range(nsweeps):
        L = [one]
        for q in range(n - 1):
            L.append(np.einsum("ab,aic,bid->cd", L[q], C[q], Y[q], optimize=True))
        F = [None] * (n + 1)
        F[n] = one
        for q in range(n - 1, -1, -1):
            P = np.einsum("ab,bid,cd->aic", L[q], Y[q], F[q + 1], optimize=True)
            r0, d, r1 = P.shape
            if q > 0:
                Qm, _ = _qr_pos(P.reshape(r0, d * r1).T)
                C[q] = Qm.T.reshape(Qm.shape[1], d, r1)
            else:
                C[q] = P
            F[q] = np.einsum("aic,bid,cd->ab", C[q], Y[q], F[q + 1], optimize=True)
        L = [one]
        for q in range(n):
            P = np.einsum("ab,bid,cd->aic", L[q], Y[q], F[q + 1], optimize=True)
            r0, d, r1 = P.shape
            if q < n - 1:
                Qm, _ = _qr_pos(P.reshape(r0 * d, r1))
                C[q] = Qm.reshape(r0, d, Qm.shape[1])
            else:
                C[q] = P
            L.append(np.einsum("ab,aic,bid->cd", L[q], C[q], Y[q], optimize=True))
    return C


def fit_two_core(spec: str, A, B, C0, rel_tol: float = 0.0, max_rank: int = 0, nsweeps: int = 1,
                 return_info: bool = False):
    """Variational fitting with super-cores of two adjacent cores (Sec. 3.3,
    multi-core strategy): the ranks of C adapt to the product
    Y = contract(spec, A, B).

    With the cores left of the pair (q, q+1) left-orthonormal and those right
    of it right-orthonormal, the best super-core is the derivative of <C|Y>
    with respect to it (eq. variational applied to the fused pair):
    S[a, i, j, c] = sum L_{q-1}[a, b] Y_q[b, i, d] Y_{q+1}[d, j, e] R_{q+2}[c, e].
    S is then decomposed again by a truncated SVD of its (r_a i) x (j r_c)
    unfolding, keeping the smallest rank r whose discarded singular values
    have 2-norm <= delta = rel_tol * ||S||_F / sqrt(n-1), capped at max_rank.
    The guess is first orthogonalised from the left (centre at core n), so
    a sweep runs over the pairs from the right end to the left -- core q+1
    becomes V^T, core q takes U Sigma -- and back from the left, core q
    becoming U and core q+1 Sigma V^T.  Returns the cores (and, with
    return_info, the ranks and the discarded tail of each split)."""
    Y = [_mat(c) for c in contract(spec, A, B)]
    C, _ = orthogonalize(C0)
    C = [_mat(c).copy() for c in C]
    n = len(C)
    if n == 1:
        out = [Y[0].copy()]
        return (out, {"ranks": [1, 1], "tails": []}) if return_info else out
    one = np.ones((1, 1))
    tails = []

    def split(S, q, left_orthonormal):
        a, i, j, c = S.shape
        U, sg, Vt = np.linalg.svd(S.reshape(a * i, j * c), full_matrices=False)
        delta = rel_tol * float(np.linalg.norm(sg)) / math.sqrt(n - 1)
        r, t_r, _, _ = truncation_rank(sg, delta, max_rank)
        tails.append(t_r)
        if left_orthonormal:
            C[q] = U[:, :r].reshape(a, i, r)
            C[q + 1] = (sg[:r, None] * Vt[:r]).reshape(r, j, c)
        else:
            C[q] = (U[:, :r] * sg[None, :r]).reshape(a, i, r)
            C[q + 1] = Vt[:r].reshape(r, j, c)

    def supercore(Lq, q, Rq2):
        return np.einsum("ab,bid,dje,ce->aijc", Lq, Y[q], Y[q + 1], Rq2, optimize=True)

    def left_env(Lq, q):
        return np.einsum("ab,aic,bid->cd", Lq, C[q], Y[q], optimize=True)

    def right_env(Rq1, q):
        return np.einsum("aic,bid,cd->ab", C[q], Y[q], Rq1, optimize=True)

    for _ in range(nsweeps):
        L = [one]
        for q in range(n - 2):
            L.append(left_env(L[q], q))
        R = [None] * (n + 1)
        R[n] = one
        for q in range(n - 2, -1, -1):  # pairs (q, q+1) from the right end
            split(supercore(L[q], q, R[q + 2]), q, left_orthonormal=False)
            R[q + 1] = right_env(R[q + 2], q + 1)
        L = [one]
        for q in range(n - 1):  # and back from the left end
            split(supercore(L[q], q, R[q + 2]), q, left_orthonormal=True)
            L.append(left_env(L[q], q))
    ranks = [1] + [c.shape[-1] for c in C]
    if return_info:
        return C, {"ranks": ranks, "tails": tails}
    return C


def solve_energy(W, b, x0, nsweeps: int = 1, ncores: int = 1, rel_tol: float = 0.0, max_rank: int = 0,
                 return_info: bool = False):
    """Solution of W x = b for a symmetric positive definite operator W (an
    MPO) by the DMRG-like strategy of Sec. 5: the energy
    J(x) = <x, W x> - 2 <x, b> is minimised core by core (ncores = 1, ranks
    fixed) or over super-cores of two cores (ncores = 2, ranks adapt).

    With every core outside the current block orthonormal (left of it
    left-orthonormal, right of it right-orthonormal), J restricted to the
    block is the quadratic form of the local matrix
      A_loc[(a,i,c),(a',j,c')] = sum LW[a,al,a'] W[al,i,j,be] RW[c,be,c']
    (LW, RW the three-layer environments of <x|W|x>; for two cores W is the
    product of the two operator cores) and the local right-hand side
      b_loc[a,i,c] = sum Lb[a,e] b[e,i,f] Rb[c,f]
    (the environments of <x|b>); its minimiser solves A_loc x_loc = b_loc
    (a dense solve here).  The guess is left-orthogonalised first; a sweep
    runs from the right end to the left and back, as the variational
    fitting does: one-core blocks move the centre by a QR of the solved core
    (of its transpose on the way left), two-core blocks are split by the
    truncated SVD of the fitting (delta = rel_tol ||S||_F / sqrt(n-1), capped
    at max_rank).  Returns the cores (and, with return_info, the ranks and
    the energy after every local solve)."""
    if ncores not in (1, 2):
        raise ValueError("ncores must be 1 or 2")
    Wm = [np.asarray(w, dtype=np.float64) for w in W]
    Bm = [_mat(c) for c in b]
    x, _ = orthogonalize(x0)
    X = [_mat(c).copy() for c in x]
    n = len(X)
    energies = []
    one3 = np.ones((1, 1, 1))
    one2 = np.ones((1, 1))

    def lw_next(LW, q):
        return np.einsum("aAx,aic,AijB,xjy->cBy", LW, X[q], Wm[q], X[q], optimize=True)

    def rw_prev(RW, q):
        return np.einsum("aic,AijB,xjy,cBy->aAx", X[q], Wm[q], X[q], RW, optimize=True)

    def lb_next(Lb, q):
        return np.einsum("ae,aic,eif->cf", Lb, X[q], Bm[q], optimize=True)

    def rb_prev(Rb, q):
        return np.einsum("aic,eif,cf->ae", X[q], Bm[q], Rb, optimize=True)

    def local_solve(q, LW, RW, Lb, Rb):
        if ncores == 1:
            A = np.einsum("aAx,AijB,cBy->aicxjy", LW, Wm[q], RW, optimize=True)
            rhs = np.einsum("ae,eif,cf->aic", Lb, Bm[q], Rb, optimize=True)
        else:
            A = np.einsum("aAx,AikB,BjlC,cCy->aijcxkly", LW, Wm[q], Wm[q + 1], RW, optimize=True)
            rhs = np.einsum("ae,eif,fjg,cg->aijc", Lb, Bm[q], Bm[q + 1], Rb, optimize=True)
        shp = rhs.shape
        N = rhs.size
        sol = np.linalg.solve(A.reshape(N, N), rhs.reshape(N))
        energies.append(-float(sol @ rhs.reshape(N)))
        return sol.reshape(shp)

    def split(S, q, left_orthonormal):
        a, i, j, c = S.shape
        U, sg, Vt = np.linalg.svd(S.reshape(a * i, j * c), full_matrices=False)
        delta = rel_tol * float(np.linalg.norm(sg)) / math.sqrt(max(n - 1, 1))
        r, _, _, _ = truncation_rank(sg, delta, max_rank)
        if left_orthonormal:
            X[q] = U[:, :r].reshape(a, i, r)
            X[q + 1] = (sg[:r, None] * Vt[:r]).reshape(r, j, c)
        else:
            X[q] = (U[:, :r] * sg[None, :r]).reshape(a, i, r)
            X[q + 1] = Vt[:r].reshape(r, j, c)

    for _ in range(nsweeps):
        LW, Lb = [one3], [one2]
        for q in range(n - 1):
            LW.append(lw_next(LW[q], q))
            Lb.append(lb_next(Lb[q], q))
        RW, Rb = [None] * (n + 1), [None] * (n + 1)
        RW[n], Rb[n] = one3, one2
        if ncores == 1 or n == 1:
            for q in range(n - 1, -1, -1):  # right to left
                sol = local_solve(q, LW[q], RW[q + 1], Lb[q], Rb[q + 1])
                r0, d, r1 = sol.shape
                if q > 0:
                    Qm, Rr = _qr_pos(sol.reshape(r0, d * r1).T)
                    X[q] = Qm.T.reshape(Qm.shape[1], d, r1)
                    X[q - 1] = np.einsum("aib,bc->aic", X[q - 1], Rr.T)
                else:
                    X[q] = sol
                RW[q] = rw_prev(RW[q + 1], q)
                Rb[q] = rb_prev(Rb[q + 1], q)
            LW, Lb = [one3], [one2]
            for q in range(n):  # and back
                sol = local_solve(q, LW[q], RW[q + 1], Lb[q], Rb[q + 1])
                r0, d, r1 = sol.shape
                if q < n - 1:
                    Qm, Rr = _qr_pos(sol.reshape(r0 * d, r1))
                    X[q] = Qm.reshape(r0, d, Qm.shape[1])
                    X[q + 1] = np.einsum("ab,bic->aic", Rr, X[q + 1])
                else:
                    X[q] = sol
                LW.append(lw_next(LW[q], q))
                Lb.append(lb_next(Lb[q], q))
        else:
            for q in range(n - 2, -1, -1):  # pairs from the right end
                split(local_solve(q, LW[q], RW[q + 2], Lb[q], Rb[q + 2]), q, left_orthonormal=False)
                RW[q + 1] = rw_prev(RW[q + 2], q + 1)
                Rb[q + 1] = rb_prev(Rb[q + 2], q + 1)
            LW, Lb = [one3], [one2]
            for q in range(n - 1):  # and back from the left end
                split(local_solve(q, LW[q], RW[q + 2], Lb[q], Rb[q + 2]), q, left_orthonormal=True)
                LW.append(lw_next(LW[q], q))
                Lb.append(lb_next(Lb[q], q))
    ranks = [1] + [c.shape[-1] for c in X]
    if return_info:
        return X, {"ranks": ranks, "energies": energies}
    return X


def solve_amen(W, b, x0, z0, nsweeps: int = 1, rel_tol: float = 0.0, max_rank: int = 0,
               span_tol: float = 1e-10, return_info: bool = False, trace: Optional[list] = None):
    """Solution of W x = b (W symmetric positive definite) by the AMEn solver
    named in Sec. 5: one-core energy minimisation as in solve_energy,
    followed at every step by a truncation of the solved core and a gradient
    (residual) enrichment of its basis, after Dolgov and Savostyanov's
    alternating minimal energy method.

    Besides x the method carries a second train z (ranks never grow) that
    approximates the residual r = b - W x.  A step at core q of a sweep
    moving left (moving right is the mirror image):
      1. the local system of solve_energy gives the core x_q (frames of x
         orthonormal around q);
      2. x_q's unfolding (r_q) x (d r_{q+1}) is truncated by an SVD,
         keeping the smallest rank whose discarded singular values have
         2-norm <= rel_tol ||x_q||_F / sqrt(n-1), capped at max_rank:
         x_q ~= (U S) V^T;
      3. z's core is built from the projection of r (with the truncated
         core) onto z's own left and right frames,
         z_q = (Z_<q x I x Z_>q)^T r, as the orthonormal rows spanning its
         rows (below);
      4. the enrichment core is the projection of r onto z's left frame and
         x's right frame, e_q = (Z_<q x I x X_>q)^T r;
      5. x's core becomes the orthonormal rows spanning the rows of
         [V^T; e_q / s] (rank up to r + r_z), and x_{q-1} takes the
         coefficients of U S V^T in that basis (the tensor x is the
         truncated one, now in a larger basis that contains the residual
         direction).
    "Orthonormal rows spanning the rows of M" are the right singular vectors
    of M whose discarded singular values have 2-norm <= span_tol (at least
    one; a zero row where the kept singular value is zero), with M scaled
    by s = ||projection of b|| + ||projection of W x|| (the two terms of the
    projected residual).  A QR would span the same space when M has full
    row rank; where it has not -- the frames of x and z overlap near the
    ends of the chain, and a converged residual is rounding noise -- its
    extra rows are arbitrary, and the next local solve would search along
    them.  The cut leaves out directions below span_tol relative to the
    residual's own terms, so the result does not depend on how the basis is
    completed.
    The end cores of a pass take the solved core itself, and z's end core
    the projection.  (The factor absorbed into the neighbour in step 5 keeps
    x a valid train between steps; the next local solve replaces that core,
    so the result does not depend on it.)  The guess x and the initial
    residual train z (its random numbers are an input) are orthogonalised
    from the left first; each sweep runs from the right end to the left and
    back.  Returns x's cores (and, with return_info, z's cores, the ranks of
    x and the energy -x_loc . b_loc after every local solve).  trace
    (tests): a list that receives, per truncated step, the direction, q,
    the truncated core, e_q, z's projected core, their scales s, copies of
    the cores of x and z the projections used as frames, the kept singular
    vectors and the new bases of x and z (as rows)."""
    Wm = [np.asarray(w, dtype=np.float64) for w in W]
    Bm = [_mat(c) for c in b]
    x, _ = orthogonalize(x0)
    X = [_mat(c).copy() for c in x]
    z, _ = orthogonalize(z0)
    Z = [_mat(c).copy() for c in z]
    n = len(X)
    if len(Z) != n:
        raise ValueError("x0 and z0 must have the same number of cores")
    energies = []
    one3 = np.ones((1, 1, 1))
    one2 = np.ones((1, 1))

    def w_left(LW, U, q, V):  # <U|W|V> environment, one core to the right
        return np.einsum("aAx,aic,AijB,xjy->cBy", LW, U, Wm[q], V, optimize=True)

    def w_right(RW, U, q, V):
        return np.einsum("aic,AijB,xjy,cBy->aAx", U, Wm[q], V, RW, optimize=True)

    def b_left(Lb, U, q):  # <U|b> environment
        return np.einsum("ae,aic,eif->cf", Lb, U, Bm[q], optimize=True)

    def b_right(Rb, U, q):
        return np.einsum("aic,eif,cf->ae", U, Bm[q], Rb, optimize=True)

    def project(q, LW, RW, Lb, Rb, xq):
        """(frame_left x I x frame_right)^T (b - W x) with x's core q = xq, and
        the scale ||projection of b|| + ||projection of W x||."""
        pb = np.einsum("ae,eif,cf->aic", Lb, Bm[q], Rb, optimize=True)
        pw = np.einsum("aAx,AijB,xjy,cBy->aic", LW, Wm[q], xq, RW, optimize=True)
        return pb - pw, float(np.linalg.norm(pb) + np.linalg.norm(pw))

    def span_rows(M):
        _, sg, Vt = np.linalg.svd(M, full_matrices=False)
        k = truncation_rank(sg, span_tol, 0)[0]
        out = Vt[:k].copy()
        out[sg[:k] == 0.0] = 0.0
        return out

    def unit(M, s):
        return M / s if s > 0.0 else M

    def local_solve(q, LW, RW, Lb, Rb):
        A = np.einsum("aAx,AijB,cBy->aicxjy", LW, Wm[q], RW, optimize=True)
        rhs = np.einsum("ae,eif,cf->aic", Lb, Bm[q], Rb, optimize=True)
        N = rhs.size
        sol = np.linalg.solve(A.reshape(N, N), rhs.reshape(N))
        energies.append(-float(sol @ rhs.reshape(N)))
        return sol.reshape(rhs.shape)

    def truncate(M):
        U, sg, Vt = np.linalg.svd(M, full_matrices=False)
        delta = rel_tol * float(np.linalg.norm(sg)) / math.sqrt(max(n - 1, 1))
        r = max(truncation_rank(sg, delta, max_rank)[0], 1)
        return U[:, :r], sg[:r], Vt[:r]

    LW, Lb, LzW, Lzb = [one3], [one2], [one3], [one2]
    for q in range(n - 1):
        LW.append(w_left(LW[q], X[q], q, X[q]))
        Lb.append(b_left(Lb[q], X[q], q))
        LzW.append(w_left(LzW[q], Z[q], q, X[q]))
        Lzb.append(b_left(Lzb[q], Z[q], q))
    RW, Rb, RzW, Rzb = ([None] * (n + 1) for _ in range(4))
    RW[n], Rb[n], RzW[n], Rzb[n] = one3, one2, one3, one2
    for _ in range(nsweeps):
        for q in range(n - 1, -1, -1):  # right to left
            sol = local_solve(q, LW[q], RW[q + 1], Lb[q], Rb[q + 1])
            if q == 0:
                X[0] = sol
                Z[0] = project(0, LzW[0], RzW[1], Lzb[0], Rzb[1], sol)[0]
                break
            r0, d, r1 = sol.shape
            U, sg, Vt = truncate(sol.reshape(r0, d * r1))
            US = U * sg[None, :]
            xt = (US @ Vt).reshape(r0, d, r1)
            zc, sz = project(q, LzW[q], RzW[q + 1], Lzb[q], Rzb[q + 1], xt)
            e, se = project(q, LzW[q], RW[q + 1], Lzb[q], Rb[q + 1], xt)
            if trace is not None:
                trace.append({"dir": "left", "q": q, "xt": xt, "e": e, "zc": zc, "se": se, "sz": sz,
                              "X": [c.copy() for c in X], "Z": [c.copy() for c in Z]})
            B = span_rows(np.vstack([Vt, unit(e.reshape(e.shape[0], d * r1), se)]))
            X[q] = B.reshape(B.shape[0], d, r1)
            X[q - 1] = np.einsum("aib,bc->aic", X[q - 1], US @ (Vt @ B.T))
            Bz = span_rows(unit(zc.reshape(zc.shape[0], d * zc.shape[2]), sz))
            Z[q] = Bz.reshape(Bz.shape[0], d, zc.shape[2])
            if trace is not None:
                trace[-1].update({"Vt": Vt, "B": B, "Bz": Bz})
            RW[q] = w_right(RW[q + 1], X[q], q, X[q])
            Rb[q] = b_right(Rb[q + 1], X[q], q)
            RzW[q] = w_right(RzW[q + 1], Z[q], q, X[q])
            Rzb[q] = b_right(Rzb[q + 1], Z[q], q)
        LW, Lb, LzW, Lzb = [one3], [one2], [one3], [one2]
        for q in range(n):  # and back
            sol = local_solve(q, LW[q], RW[q + 1], Lb[q], Rb[q + 1])
            if q == n - 1:
                X[q] = sol
                Z[q] = project(q, LzW[q], RzW[q + 1], Lzb[q], Rzb[q + 1], sol)[0]
                break
            r0, d, r1 = sol.shape
            U, sg, Vt = truncate(sol.reshape(r0 * d, r1))
            SVt = sg[:, None] * Vt
            xt = (U @ SVt).reshape(r0, d, r1)
            zc, sz = project(q, LzW[q], RzW[q + 1], Lzb[q], Rzb[q + 1], xt)
            e, se = project(q, LW[q], RzW[q + 1], Lb[q], Rzb[q + 1], xt)
            if trace is not None:
                trace.append({"dir": "right", "q": q, "xt": xt, "e": e, "zc": zc, "se": se, "sz": sz,
                              "X": [c.copy() for c in X], "Z": [c.copy() for c in Z]})
            B = span_rows(np.vstack([U.T, unit(e.reshape(r0 * d, e.shape[2]), se).T]))
            X[q] = B.T.reshape(r0, d, B.shape[0])
            X[q + 1] = np.einsum("ab,bic->aic", (B @ U) @ SVt, X[q + 1])
            Bz = span_rows(unit(zc.reshape(zc.shape[0] * d, zc.shape[2]), sz).T)
            Z[q] = Bz.T.reshape(zc.shape[0], d, Bz.shape[0])
            if trace is not None:
                trace[-1].update({"Vt": U.T, "B": B, "Bz": Bz})
            LW.append(w_left(LW[q], X[q], q, X[q]))
            Lb.append(b_left(Lb[q], X[q], q))
            LzW.append(w_left(LzW[q], Z[q], q, X[q]))
            Lzb.append(b_left(Lzb[q], Z[q], q))
    ranks = [1] + [c.shape[-1] for c in X]
    if return_info:
        return X, {"z": Z, "ranks": ranks, "energies": energies}
    return X


def bond_singular_values(X):
    """Singular values of every bond unfolding (QR sweep, then untruncated SVD sweep)."""
    _, info = round_tt(X, 0.0, 0, return_info=True)
    return info.sigmas


# --------------------------------------------------------------------------
# inner products and norms (Sec. 3.3, <C|C>-type contractions)
# --------------------------------------------------------------------------
def _mat(core):
    """[r_l, phys..., r_r] -> (r_l, P, r_r) with the physical legs flattened."""
    return core.reshape(core.shape[0], -1, core.shape[-1])


def inner(A, B) -> float:
    """<A, B> = E_n with E_0 = [[1]], E_k = sum_i A_k(i)^T E_{k-1} B_k(i)."""
    E = np.ones((1, 1))
    for a, b in zip(A, B):
        a3, b3 = _mat(a), _mat(b)
        E = sum(a3[:, i, :].T @ E @ b3[:, i, :] for i in range(a3.shape[1]))
    return float(E[0, 0])


def norm(X) -> float:
    return orthogonalize(X)[1]


def diff_norm(X, Y) -> float:
    """||X - Y||_F via the exact difference TT and a QR sweep (no cancellation)."""
    D = tt_add(X, Y, 1.0, -1.0)
    return orthogonalize(D)[1]


def rel_error(X, Y) -> float:
    """||X - Y|| / ||Y|| (Frobenius), computed without Gram cancellation."""
    ny = norm(Y)
    dn = diff_norm(X, Y)
    return dn / ny if ny > 0 else dn


# --------------------------------------------------------------------------
# dense helpers (tiny grids only)
# --------------------------------------------------------------------------
def to_dense(X) -> np.ndarray:
    """Full tensor as a flat vector, core 0 = most significant digit."""
    T = np.ones((1, 1))
    for c in X:
        c3 = _mat(c)
        T = np.einsum("pa,aib->pib", T, c3).reshape(-1, c3.shape[-1])
    return T[:, 0]


def mpo_to_dense(W) -> np.ndarray:
    """Dense matrix A(i, j) of an MPO with cores [r, d_out, d_in, r']."""
    T = np.ones((1, 1, 1))
    for c in W:
        T = np.einsum("pqa,aijb->piqjb", T, c)
        s = T.shape
        T = T.reshape(s[0] * s[1], s[2] * s[3], s[4])
    return T[:, :, 0]


def interleaved_index(m: int, D: int) -> np.ndarray:
    """Map flat TT index (interleaved digits) -> row-major grid index (x_0, .., x_{D-1}).

    Core k = q*D + a holds bit q (MSB first) of axis a.
    """
    n = m * D
    flat = np.arange(2 ** n)
    coords = np.zeros((D, flat.size), dtype=np.int64)
    for k in range(n):
        bit = (flat >> (n - 1 - k)) & 1
        q, a = divmod(k, D)
        coords[a] |= bit << (m - 1 - q)
    grid = np.zeros(flat.size, dtype=np.int64)
    for a in range(D):
        grid = grid * (2 ** m) + coords[a]
    return grid


def dense_shift(N: int, d: int) -> np.ndarray:
    """Q^N_d(i, j) = 1 iff i - j = d (Sec. 4.2); zero if d > N."""
    Q = np.zeros((N, N))
    for j in range(N):
        i = j + d
        if 0 <= i < N:
            Q[i, j] = 1.0
    return Q


def dense_laplacian(m: int, D: int) -> np.ndarray:
    """Kronecker sum of the 1D Dirichlet stencil 2I - S - S^T on (2^m)^D points."""
    N = 2 ** m
    S = dense_shift(N, 1)
    L1 = 2.0 * np.eye(N) - S - S.T
    out = np.zeros((N ** D, N ** D))
    for a in range(D):
        term = np.ones((1, 1))
        for b in range(D):
            term = np.kron(term, L1 if b == a else np.eye(N))
        out += term
    return out


def shift_mpo_paper(n: int, dshift: int):
    """TT of (Q^N_d; R^N_d) by the paper's recursion (eq. shif_dec), N = 2^n.

    Each core is the 2x2 block [[Q^2_{d_q}, Q^2_{d_q+1}], [R^2_{d_q},
    R^2_{d_q+1}]] of 2x2 shift matrices, the last core the column (Q^2_{d_n};
    R^2_{d_n}); the digits d_q of d are taken MSB first.  Q is selected by the
    row vector (1, 0) from the left.  Uses R^N_d = (Q^N_{N-d})^T and Q^N_d = 0
    for d >= N.  Returns MPO cores for Q^N_d.
    """
    def Q2(dd):
        return dense_shift(2, dd) if dd < 2 else np.zeros((2, 2))

    def R2(dd):
        return Q2(2 - dd).T if 0 <= 2 - dd else np.zeros((2, 2))

    digits = [(dshift >> (n - 1 - q)) & 1 for q in range(n)]
    cores = []
    for q in range(n):
        dq = digits[q]
        if q < n - 1:
            c = np.zeros((2, 2, 2, 2))
            c[0, :, :, 0] = Q2(dq)
            c[0, :, :, 1] = Q2(dq + 1)
            c[1, :, :, 0] = R2(dq)
            c[1, :, :, 1] = R2(dq + 1)
        else:
            c = np.zeros((2, 2, 2, 1))
            c[0, :, :, 0] = Q2(dq)
            c[1, :, :, 0] = R2(dq)
        cores.append(c)
    sel = np.array([1.0, 0.0])
    cores[0] = np.einsum("a,aijb->ijb", sel, cores[0])[None]
    return cores


# --------------------------------------------------------------------------
# gradients (variational derivative, Sec. 3.3)
# --------------------------------------------------------------------------
def env_left(A, B) -> List[np.ndarray]:
    """E[k] = left environment before core k of <A,B>; E[0] = [[1]]."""
    E = [np.ones((1, 1))]
    for a, b in zip(A, B):
        E.append(np.einsum("ab,aic,bid->cd", E[-1], _mat(a), _mat(b)))
    return E


def env_right(A, B) -> List[np.ndarray]:
    """F[k] = right environment after core k-1 of <A,B>; F[n] = [[1]]."""
    n = len(A)
    F = [None] * (n + 1)
    F[n] = np.ones((1, 1))
    for k in range(n - 1, -1, -1):
        F[k] = np.einsum("aic,bid,cd->ab", _mat(A[k]), _mat(B[k]), F[k + 1])
    return F


def inner_grad(A, B) -> List[np.ndarray]:
    """d<A,B>/dA_k = E_{k-1} B_k(i) F_{k+1}^T for every core k."""
    E, F = env_left(A, B), env_right(A, B)
    out = []
    for k in range(len(A)):
        g = np.einsum("ab,bid,cd->aic", E[k], _mat(B[k]), F[k + 1])
        out.append(g.reshape(A[k].shape))
    return out


def contract_grad(spec: str, W, X, dC):
    """Local backward of contract(): (dW, dX) from dC, core by core."""
    dW, dX = [], []
    for w, x, dc in zip(W, X, dC):
        if spec == "ij,j->i":
            ra, di, dj, rb = w.shape
            rc, _, rd = x.shape
            g = dc.reshape(ra, rc, di, rb, rd)
            dX.append(np.einsum("aijb,acibd->cjd", w, g))
            dW.append(np.einsum("cjd,acibd->aijb", x, g))
        elif spec == "i,i->i":
            ra, d, rb = w.shape
            rc, _, rd = x.shape
            g = dc.reshape(ra, rc, d, rb, rd)
            dX.append(np.einsum("aib,acibd->cid", w, g))
            dW.append(np.einsum("cid,acibd->aib", x, g))
        else:
            raise ValueError(spec)
    return dW, dX


def loss_axb(W, x, b) -> float:
    """L = ||W x - b||^2 via the exact difference TT (no cancellation)."""
    y = contract("ij,j->i", W, x)
    return diff_norm(y, b) ** 2


def grad_axb(W, x, b) -> List[np.ndarray]:
    """dL/dx_k for L = ||W x - b||^2 (route 1: through y = W x).

    L = <y,y> - 2<y,b> + <b,b>, so dL/dy_k = 2 E^{yy} y_k F^{yy} -
    2 E^{yb} b_k F^{yb} (environments of the two inner products); the local
    contraction backward then maps dL/dy_k to dL/dx_k.
    """
    y = contract("ij,j->i", W, x)
    gyy = inner_grad(y, y)      # one slot of <y,y>; both slots give 2 * gyy
    gyb = inner_grad(y, b)
    dy = [2.0 * g1 - 2.0 * g2 for g1, g2 in zip(gyy, gyb)]
    _, dx = contract_grad("ij,j->i", W, x, dy)
    return dx


def grad_axb_sandwich(W, x, b) -> List[np.ndarray]:
    """dL/dx_k (route 2): three-layer environments of <x|W^T W|x> and <b|W|x>.

    L = <x, W^T W x> - 2 <b, W x> + <b, b>; no contracted TT is formed.
    """
    n = len(x)
    # left environments of x^T W^T W x : tensors [r_x, r_w, r_w, r_x]
    EL = [np.ones((1, 1, 1, 1))]
    for k in range(n - 1):
        EL.append(np.einsum("pabq,pjx,aijc,bikd,qky->xcdy",
                            EL[-1], x[k], W[k], W[k], x[k]))
    ER = [None] * (n + 1)
    ER[n] = np.ones((1, 1, 1, 1))
    for k in range(n - 1, 0, -1):
        ER[k] = np.einsum("pjx,aijc,bikd,qky,xcdy->pabq",
                          x[k], W[k], W[k], x[k], ER[k + 1])
    # left/right environments of <b, W x>: [r_b, r_w, r_x]
    GL = [np.ones((1, 1, 1))]
    for k in range(n - 1):
        GL.append(np.einsum("pab,piq,aijc,bjd->qcd", GL[-1], b[k], W[k], x[k]))
    GR = [None] * (n + 1)
    GR[n] = np.ones((1, 1, 1))
    for k in range(n - 1, 0, -1):
        GR[k] = np.einsum("piq,aijc,bjd,qcd->pab", b[k], W[k], x[k], GR[k + 1])
    out = []
    for k in range(n):
        # <Wx, Wx> with x_k removed from one slot; both slots give 2 * g1
        g1 = np.einsum("pabq,aijc,bikd,qky,xcdy->pjx",
                       EL[k], W[k], W[k], x[k], ER[k + 1])
        g2 = np.einsum("pab,piq,aijc,qcd->bjd", GL[k], b[k], W[k], GR[k + 1])
        out.append(2.0 * g1 - 2.0 * g2)
    return out
