"""Seeded synthetic inputs shared by the oracle tests, the GPU tests and the bench.

This module only *builds operands*: it draws random cores and writes down
closed-form tensor trains that the paper gives (or that follow directly from
its definitions).  It performs none of the method's arithmetic -- no
contraction, orthogonalisation, rounding or inner product -- so that the
oracle and the HIP path can share it without sharing any step they are
compared on.

Conventions (paper, Sec. 2 "Notation", eq. quantization / vector_dec):
  * a dimension of size 2**m is split into m binary digits, digit 1 (core 0
    here) being the most significant one;
  * digit values are 0-based;
  * an MPS core is stored as a float64 array [r_left, d, r_right] and an MPO
    core as [r_left, d_out, d_in, r_right] (row-major); the MPO acts as
    y(i) = sum_j A(i, j) x(j) (Sec. 3.1, eq. quant_sum);
  * multi-dimensional grids use one digit per core with the axes interleaved
    (x1, y1, x2, y2, ... most significant first), i.e. the explicit digit
    grouping of the user guide's TrainShape with one digit per core.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field
from typing import List, Optional, Sequence

import numpy as np

__all__ = [
    "rank_profile",
    "random_mps",
    "random_mpo",
    "trig_qtt",
    "sin_unit_interval",
    "exp_qtt",
    "poly_qtt",
    "laplacian_mpo",
    "embed_axis",
    "Workload",
    "sin_noise_1d",
    "laplacian2d_r64",
    "hadamard_batch",
    "laplacian3d_r256",
    "residual_grad_2d",
    "sum4_n42_r128",
]


# --------------------------------------------------------------------------
# random operands
# --------------------------------------------------------------------------
def rank_profile(n: int, rmax: int, d: int = 2) -> List[int]:
    """Bond ranks r_0..r_n of a generic TT with n cores of physical size d.

    r_k = min(rmax, d**k, d**(n-k)): the largest rank an unfolding of a
    d**n tensor can have, capped at rmax.  A flat rmax at the boundary bonds
    would be structurally rank deficient.
    """
    out = []
    for k in range(n + 1):
        r = rmax
        r = min(r, d ** min(k, 62))
        r = min(r, d ** min(n - k, 62))
        out.append(int(max(r, 1)))
    return out


def random_mps(n: int, rmax: int, rng: np.random.Generator, d: int = 2,
               scale: str = "variance", ranks: Optional[Sequence[int]] = None):
    """Gaussian MPS cores [r_k, d, r_{k+1}], drawn in core order, C order.

    scale="raw":      entries N(0, 1).
    scale="variance": core k is scaled by 1/sqrt(d * r_{k+1}), which makes
                      E||X||_F^2 = 1 exactly (each core then contributes a
                      factor d * r_{k+1} * s_k^2 = 1 to the expected norm).
    """
    rk = list(ranks) if ranks is not None else rank_profile(n, rmax, d)
    cores = []
    for k in range(n):
        c = rng.standard_normal((rk[k], d, rk[k + 1]))
        if scale == "variance":
            c *= 1.0 / math.sqrt(d * rk[k + 1])
        elif scale != "raw":
            raise ValueError(scale)
        cores.append(c)
    return cores


def random_mpo(n: int, rmax: int, rng: np.random.Generator, d: int = 2,
               scale: str = "variance"):
    """Gaussian MPO cores [r_k, d, d, r_{k+1}] with the profile min(rmax, d^2k, ...)."""
    rk = rank_profile(n, rmax, d * d)
    cores = []
    for k in range(n):
        c = rng.standard_normal((rk[k], d, d, rk[k + 1]))
        if scale == "variance":
            c *= 1.0 / math.sqrt(d * rk[k + 1])
        cores.append(c)
    return cores


# --------------------------------------------------------------------------
# closed forms of Sec. 4.1 ("Construction of basic functions")
# --------------------------------------------------------------------------
def _rot(t: float) -> np.ndarray:
    c, s = math.cos(t), math.sin(t)
    return np.array([[c, -s], [s, c]])


def trig_qtt(n: int, v: float, phase: float = 0.0, kind: str = "cos"):
    """Rank-2 real QTT of f(i) = cos(v*i + phase) or sin(v*i + phase), i in [0, 2^n).

    Sec. 4.1 ("Trigonometric functions"): with theta_q = v*2^(n-q)*i_q +
    phase/n the argument splits into a sum over digits, and
        cos(sum_q theta_q) = 1/2 (1, 1) R(theta_1) ... R(theta_n) (1, 1)^T
    with R the 2x2 rotation; the first core absorbs (1,1)/2, the last (1,1)^T.
    The sine follows from the shift by pi/2 (sin y = cos(y - pi/2)).
    """
    if kind == "sin":
        phase = phase - math.pi / 2.0
    elif kind != "cos":
        raise ValueError(kind)
    cores = []
    for q in range(n):
        core = np.zeros((2, 2, 2))
        for iq in range(2):
            theta = v * float(2 ** (n - 1 - q)) * iq + phase / n
            core[:, iq, :] = _rot(theta)
        cores.append(core)
    first = np.einsum("a,aib->ib", np.array([0.5, 0.5]), cores[0])[None]
    last = np.einsum("aib,b->ai", cores[-1], np.array([1.0, 1.0]))[..., None]
    if n == 1:
        only = np.einsum("a,aib,b->i", np.array([0.5, 0.5]), cores[0],
                         np.array([1.0, 1.0]))
        return [only.reshape(1, 2, 1)]
    cores[0] = first
    cores[-1] = last
    return cores


def sin_unit_interval(n: int, freq: float = 2.0 * math.pi):
    """sin(freq * x) on the uniform grid x_i = i / (2^n - 1) of [0, 1].

    The grid includes both end points (Sec. 2, x(i) = (b-a)/(dim-1) i + a).
    """
    N = 2 ** n
    return trig_qtt(n, freq / (N - 1), 0.0, "sin")


def exp_qtt(n: int, v: float, a: float = 0.0, b: float = 1.0, x0: float = 0.0):
    """Rank-1 QTT of exp(v (x - x0)) on the uniform grid of [a, b] (eq. exp_dec)."""
    N = 2 ** n
    h = (b - a) / (N - 1)
    cores = []
    for q in range(n):
        c = np.array([math.exp(v * h * 2 ** (n - 1 - q) * iq) for iq in range(2)])
        cores.append(c.reshape(1, 2, 1))
    cores[0] = cores[0] * math.exp(v * (a - x0))
    return cores


def poly_qtt(n: int, coeffs: Sequence[float], a: float = 0.0, b: float = 1.0,
             x0: float = 0.0):
    """QTT of sum_s coeffs[s] (x - x0)^s, rank p+1 (Sec. 4.1 "Polynomials").

    With xt_q = c_q x_q + (a - x0)/n the polynomial of sum_q xt_q expands by
    the binomial theorem.  Bond state s stands for the factor
    (xt_{q+1} + ... + xt_n)^s: the first core is the row
        C_1^{s} = sum_{t>=s} a_t binom(t, s) xt_1^(t-s),
    the last core the column (1, xt_n, ..., xt_n^p)^T, and a middle core
    expands (xt_q + rest)^s, C_q^{st} = binom(s, t) xt_q^(s-t) for t <= s.
    (The paper prints the middle core with s and t exchanged; with its own
    first and last cores only this orientation reproduces the polynomial.)
    """
    p = len(coeffs) - 1
    N = 2 ** n
    h = (b - a) / (N - 1)
    shift = (a - x0) / n

    def xt(q, iq):
        return h * 2 ** (n - 1 - q) * iq + shift

    cores = []
    for q in range(n):
        if q == 0:
            c = np.zeros((1, 2, p + 1))
            for iq in range(2):
                x = xt(q, iq)
                for s in range(p + 1):
                    c[0, iq, s] = sum(coeffs[t] * math.comb(t, s) * x ** (t - s)
                                      for t in range(s, p + 1))
        elif q == n - 1:
            c = np.zeros((p + 1, 2, 1))
            for iq in range(2):
                x = xt(q, iq)
                for s in range(p + 1):
                    c[s, iq, 0] = x ** s
        else:
            c = np.zeros((p + 1, 2, p + 1))
            for iq in range(2):
                x = xt(q, iq)
                for s in range(p + 1):
                    for t in range(0, s + 1):
                        c[s, iq, t] = math.comb(s, t) * x ** (s - t)
        cores.append(c)
    if n == 1:
        raise ValueError("poly_qtt needs n >= 2")
    return cores


# --------------------------------------------------------------------------
# finite-difference Laplacian as an MPO
# --------------------------------------------------------------------------
def laplacian_mpo(m: int, D: int = 1, diag: float = 2.0):
    """Unscaled Dirichlet Laplacian sum_a (2 I - S_a - S_a^T) on a (2^m)^D grid
    (with diag != 2: sum_a (diag I - S_a - S_a^T), the Laplacian shifted by
    D (diag - 2) I, e.g. the operator of an implicit heat step scaled by the
    inverse time step).

    S is the shift Q^N_1 of Sec. 4.2 (S(i, j) = 1 iff i - j = 1), values
    outside the grid are zero (no wrap-around).  Cores are interleaved: core
    k = q*D + a carries bit q (0 = most significant) of axis a.

    The cores are written down from the binary carry of "j + 1": reading the
    digits from the least significant end, each term of the sum is in one of
    the states
        A   -- finished, every remaining digit is the identity;
        N   -- not started: the axis of this term lies wholly to the left;
        Q_a -- shift of axis a with a carry still to be absorbed on the left;
        P_a -- transposed shift of axis a with a carry still pending.
    At a least significant digit the shift contributes E10 (no carry) or E01
    (carry out), the transposed shift E01 / E10; a carry is absorbed by E10
    (shift) / E01 (transpose) or passed on by E01 / E10.  A carry out of the
    most significant digit leaves the grid and is dropped.  The interior
    bond rank is 2D+1 (1, 3, 5, 7 ... states), the boundary bonds are smaller.
    """
    n = m * D
    I2 = np.eye(2)
    E10 = np.array([[0.0, 0.0], [1.0, 0.0]])  # row i=1, column j=0
    E01 = np.array([[0.0, 1.0], [0.0, 0.0]])  # row i=0, column j=1

    def lsb_core(a):
        return (m - 1) * D + a

    def states(b):
        # state list of bond b (right part = cores b..n-1)
        started = [a for a in range(D) if lsb_core(a) >= b]
        st = []
        if started:
            st.append(("A",))
        if len(started) < D:
            st.append(("N",))
        for a in started:
            if a < b:  # axis a still has digits on the left
                st.append(("Q", a))
                st.append(("P", a))
        return st

    bond_states = [states(b) for b in range(n + 1)]
    cores = []
    for k in range(n):
        alpha, q = k % D, k // D
        L, R = bond_states[k], bond_states[k + 1]
        li = {s: i for i, s in enumerate(L)}
        core = np.zeros((len(L), 2, 2, len(R)))

        def put(sl, sr, mat):
            if sl in li:
                core[li[sl], :, :, R.index(sr)] += mat

        for sr in R:
            if sr == ("A",):
                put(("A",), sr, I2)
            elif sr == ("N",):
                put(("N",), sr, I2)  # still not started (if other axes remain)
                if k == lsb_core(alpha):
                    put(("A",), sr, diag * I2 - E10 - E01)
                    put(("Q", alpha), sr, -E01)
                    put(("P", alpha), sr, -E10)
            else:
                kind, a = sr
                if a != alpha:
                    put(sr, sr, I2)
                elif kind == "Q":
                    put(("A",), sr, E10)
                    if q > 0:
                        put(sr, sr, E01)
                else:
                    put(("A",), sr, E01)
                    if q > 0:
                        put(sr, sr, E10)
        cores.append(core)
    return cores


def embed_axis(cores_1d, D: int, axis: int, kind: str = "mps"):
    """Place a 1D QTT on one axis of an interleaved D-dimensional layout.

    The digits of the other axes get all-ones MPS cores (the function is
    constant along them), with the bond carried through unchanged.
    """
    m = len(cores_1d)
    out = []
    rank_in = 1
    for q in range(m):
        for a in range(D):
            if a == axis:
                c = cores_1d[q]
                out.append(c.copy())
                rank_in = c.shape[-1]
            else:
                r = rank_in
                c = np.zeros((r, 2, r))
                for i in range(2):
                    c[:, i, :] = np.eye(r)
                out.append(c)
    return out


# --------------------------------------------------------------------------
# the five benchmark workloads
# --------------------------------------------------------------------------
@dataclass
class Workload:
    name: str
    spec: str                      # "i,i->i" (Hadamard) or "ij,j->i" (MPO.MPS)
    a: list = field(default_factory=list)          # first operand cores
    b: list = field(default_factory=list)          # second operand cores
    rel_tol: float = 0.0
    max_rank: int = 0              # <= 0: none
    extra: dict = field(default_factory=dict)


def sin_noise_1d() -> Workload:
    """1D, L=10: sin(2 pi x) (rank 2) times a raw Gaussian rank-4 QTT (seed 0)."""
    rng = np.random.default_rng(0)
    f = sin_unit_interval(10)
    g = random_mps(10, 4, rng, scale="raw")
    return Workload("sin_noise_1d_L10_r4", "i,i->i", f, g, 1e-12, 0)


def laplacian2d_r64(seed: int = 1, m: int = 16, rmax: int = 64) -> Workload:
    """2D 2^16 x 2^16 grid (32 cores): Laplacian MPO times a rank-64 MPS."""
    rng = np.random.default_rng(seed)
    W = laplacian_mpo(m, 2)
    X = random_mps(2 * m, rmax, rng)
    return Workload("laplacian2d_n32_r64", "ij,j->i", W, X, 1e-10, rmax)


def hadamard_batch(count: int = 512, L: int = 24, seed: int = 2,
                   rlo: int = 8, rhi: int = 128) -> Workload:
    """512 independent 1D Hadamard products; rank_A ~ U{8..128}, rank_B = 2.

    All instance ranks are drawn first, then A_i and B_i per instance.
    """
    rng = np.random.default_rng(seed)
    ranks = rng.integers(rlo, rhi + 1, size=count)
    A, B = [], []
    for i in range(count):
        A.append(random_mps(L, int(ranks[i]), rng))
        B.append(random_mps(L, 2, rng))
    return Workload("hadamard_batch512_L24_r8to128", "i,i->i", A, B, 1e-8, 0,
                    {"ranks": [int(r) for r in ranks]})


def laplacian3d_r256(seed: int = 3, m: int = 14, rmax: int = 256) -> Workload:
    """3D 2^14 per axis (42 cores): Laplacian MPO (rank 7) times a rank-256 MPS."""
    rng = np.random.default_rng(seed)
    W = laplacian_mpo(m, 3)
    X = random_mps(3 * m, rmax, rng)
    return Workload("laplacian3d_n42_r256", "ij,j->i", W, X, 1e-8, rmax)


def residual_grad_2d(seed: int = 4, m: int = 12, rx: int = 32, rb: int = 16) -> Workload:
    """2D 2^12 x 2^12 (24 cores): loss ||A x - b||^2, x rank 32, b rank 16."""
    rng = np.random.default_rng(seed)
    W = laplacian_mpo(m, 2)
    x = random_mps(2 * m, rx, rng)
    b = random_mps(2 * m, rb, rng)
    return Workload("residual_grad2d_n24_r32", "ij,j->i", W, x, 0.0, 0, {"rhs": b})


def sum4_n42_r128(seed: int = 5, n: int = 42, rmax: int = 128) -> Workload:
    """Four Gaussian rank-128 MPS on the 42-core grid (drawn in order), to be
    summed with coefficients (1, -0.5, 0.25, 2) and rounded to rank 256 at
    1e-8 (exact sum of rank 512, then truncation)."""
    rng = np.random.default_rng(seed)
    terms = [random_mps(n, rmax, rng) for _ in range(4)]
    return Workload("sum4_n42_r128", "sum", terms, [], 1e-8, 256, {"coeffs": [1.0, -0.5, 0.25, 2.0]})
