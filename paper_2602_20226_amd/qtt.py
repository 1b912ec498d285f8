"""Python binding of libqtt (ctypes).

Argument marshalling only: every step of the contraction, rounding and
inner-product path runs in the HIP kernels of libqtt.so.  PyTorch provides
device buffers (torch.empty on a ROCm device) and the current stream.
The names follow include/qtt.h.
"""
from __future__ import annotations

import atexit
import ctypes as C
import math
import os
import weakref
from dataclasses import dataclass, field
from typing import List, Optional, Sequence

import torch

HERE = os.path.dirname(os.path.abspath(__file__))
# QTT_LIBRARY names another build of the same library (the host-sanitizer
# build of the CPU tests); by default the in-tree libqtt.so
LIB_PATH = os.environ.get("QTT_LIBRARY") or os.path.join(HERE, "libqtt.so")

QTT_OK = 0
STATUS = {
    0: "QTT_OK", -1: "QTT_ERR_ARG", -2: "QTT_ERR_SPEC", -3: "QTT_ERR_SHAPE", -4: "QTT_ERR_DTYPE",
    -5: "QTT_ERR_WORKSPACE", -6: "QTT_ERR_NODEVICE", -7: "QTT_ERR_HIP", -8: "QTT_ERR_NONFINITE",
    -9: "QTT_ERR_NOCONV", -10: "QTT_ERR_UNSUPPORTED",
}
F64, F32 = 0, 1
PREC = {"fp64": 0, "fp32": 1, "bf16x3": 2, "bf16x6": 3}
OP_CONTRACT, OP_ORTHOGONALIZE, OP_ROUND, OP_CONTRACT_ROUND, OP_INNER, OP_INNER_BACKWARD, OP_CONTRACT_BACKWARD = range(7)

EXPORTS = [
    "qtt_create", "qtt_destroy", "qtt_status_string", "qtt_workspace_size", "qtt_contract",
    "qtt_orthogonalize", "qtt_round", "qtt_contract_round", "qtt_inner", "qtt_inner_backward",
    "qtt_contract_backward", "qtt_profile_start", "qtt_profile_stop", "qtt_batch_workspace_size",
    "qtt_batch_plan_create", "qtt_batch_plan_launch", "qtt_batch_plan_results", "qtt_batch_plan_info",
    "qtt_batch_plan_destroy", "qtt_contract_zipup", "qtt_zipup_query", "qtt_add",
    "qtt_fit", "qtt_fit_workspace_size", "qtt_set_jacobi_max_sweeps", "qtt_contract_round_noalloc",
    "qtt_inner_prec", "qtt_batch_plan_tiles", "qtt_contract_round_async", "qtt_fit2", "qtt_fit2_query",
    "qtt_solve", "qtt_solve_query", "qtt_solve_amen", "qtt_solve_amen_query",
]
# size of the fixed device array behind qtt_contract_round_noalloc
NOALLOC_SCRATCH_BYTES = 64 << 20


class QttError(RuntimeError):
    def __init__(self, status: int, where: str):
        self.status = status
        super().__init__(f"{where}: {STATUS.get(status, status)} ({_status_string(status)})")


class TT(C.Structure):
    _fields_ = [
        ("n", C.c_int32),
        ("legs", C.c_int32),
        ("phys", C.POINTER(C.c_int32)),
        ("ranks", C.POINTER(C.c_int64)),
        ("cores", C.POINTER(C.c_void_p)),
        ("dtype", C.c_int32),
    ]


class RoundInfoC(C.Structure):
    _fields_ = [
        ("norm", C.c_double),
        ("delta", C.c_double),
        ("err_bound", C.c_double),
        ("tail", C.POINTER(C.c_double)),
        ("margin_lo", C.POINTER(C.c_double)),
        ("margin_hi", C.POINTER(C.c_double)),
        ("maxrank_hit", C.POINTER(C.c_uint8)),
        ("sigma", C.POINTER(C.c_double)),
        ("sigma_ld", C.c_int64),
        ("jacobi_sweeps_max", C.c_int32),
    ]


_lib = None


def lib_available() -> bool:
    return os.path.exists(LIB_PATH)


def load_library():
    """Load libqtt.so; raises if it has not been built (no fallback exists)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"libqtt.so not built at {LIB_PATH}; run paper_2602_20226_amd.build.build()")
    L = C.CDLL(LIB_PATH)
    vp = C.c_void_p
    P = C.POINTER
    L.qtt_create.argtypes = [P(vp), C.c_int]
    L.qtt_destroy.argtypes = [vp]
    L.qtt_status_string.argtypes = [C.c_int]
    L.qtt_status_string.restype = C.c_char_p
    L.qtt_workspace_size.argtypes = [vp, C.c_int, C.c_char_p, P(TT), P(TT), C.c_int64, C.c_int, P(C.c_size_t)]
    L.qtt_contract.argtypes = [vp, C.c_char_p, P(TT), P(TT), P(TT), vp, C.c_size_t, vp]
    L.qtt_orthogonalize.argtypes = [vp, P(TT), P(C.c_double), vp, C.c_size_t, vp]
    L.qtt_round.argtypes = [vp, P(TT), C.c_double, C.c_int64, C.c_int, P(RoundInfoC), vp, C.c_size_t, vp]
    L.qtt_contract_round.argtypes = [vp, C.c_char_p, P(TT), P(TT), P(TT), C.c_double, C.c_int64, C.c_int,
                                     P(RoundInfoC), vp, C.c_size_t, vp]
    L.qtt_contract_round_async.argtypes = [vp, C.c_char_p, P(TT), P(TT), P(TT), C.c_double, C.c_int64, C.c_int,
                                           vp, vp, vp, C.c_size_t, vp]
    L.qtt_contract_round_noalloc.argtypes = [vp, C.c_char_p, P(TT), P(TT), P(TT), C.c_double, C.c_int64, C.c_int,
                                             P(RoundInfoC), vp]
    L.qtt_inner.argtypes = [vp, P(TT), P(TT), P(C.c_double), vp, C.c_size_t, vp]
    L.qtt_inner_prec.argtypes = [vp, P(TT), P(TT), C.c_int, P(C.c_double), vp, C.c_size_t, vp]
    L.qtt_inner_backward.argtypes = [vp, P(TT), P(TT), C.c_double, P(TT), P(TT), vp, C.c_size_t, vp]
    L.qtt_contract_backward.argtypes = [vp, C.c_char_p, P(TT), P(TT), P(TT), P(TT), P(TT), vp, C.c_size_t, vp]
    L.qtt_batch_workspace_size.argtypes = [vp, C.c_char_p, C.c_int32, P(TT), P(TT), C.c_int64, P(C.c_size_t)]
    L.qtt_batch_plan_create.argtypes = [vp, C.c_char_p, C.c_int32, P(TT), P(TT), P(TT), C.c_double, C.c_int64,
                                        C.c_int, vp, C.c_size_t, vp, P(vp)]
    L.qtt_batch_plan_launch.argtypes = [vp, vp]
    L.qtt_batch_plan_results.argtypes = [vp, P(C.c_int64), P(C.c_double), vp]
    L.qtt_batch_plan_info.argtypes = [vp, P(C.c_int32), P(C.c_int32), P(C.c_float)]
    L.qtt_batch_plan_destroy.argtypes = [vp]
    L.qtt_batch_plan_tiles.argtypes = [vp, P(C.c_uint8), P(C.c_int32), P(C.c_float)]
    L.qtt_contract_zipup.argtypes = [vp, C.c_char_p, P(TT), P(TT), P(TT), C.c_double, C.c_int64, C.c_int32, C.c_int,
                                     P(RoundInfoC), vp, C.c_size_t, vp]
    L.qtt_fit.argtypes = [vp, C.c_char_p, P(TT), P(TT), P(TT), C.c_int32, P(C.c_double), vp, C.c_size_t, vp]
    L.qtt_fit_workspace_size.argtypes = [C.c_char_p, P(TT), P(TT), P(TT), P(C.c_size_t)]
    L.qtt_fit2.argtypes = [vp, C.c_char_p, P(TT), P(TT), P(TT), C.c_int32, C.c_double, C.c_int64, P(RoundInfoC),
                           vp, C.c_size_t, vp]
    L.qtt_solve.argtypes = [vp, P(TT), P(TT), P(TT), C.c_int32, C.c_int32, C.c_double, C.c_int64, P(RoundInfoC),
                            vp, C.c_size_t, vp]
    L.qtt_solve_query.argtypes = [P(TT), P(TT), P(TT), C.c_int32, C.c_int64, P(C.c_int64), P(C.c_size_t)]
    L.qtt_solve_amen.argtypes = [vp, P(TT), P(TT), P(TT), P(TT), C.c_int32, C.c_double, C.c_int64,
                                 P(RoundInfoC), vp, C.c_size_t, vp]
    L.qtt_solve_amen_query.argtypes = [P(TT), P(TT), P(TT), P(TT), C.c_int64, P(C.c_int64), P(C.c_int64),
                                       P(C.c_size_t)]
    L.qtt_fit2_query.argtypes = [C.c_char_p, P(TT), P(TT), P(TT), C.c_int64, P(C.c_int64), P(C.c_size_t)]
    L.qtt_add.argtypes = [vp, C.c_int32, P(TT), P(C.c_double), P(TT), vp]
    L.qtt_zipup_query.argtypes = [C.c_char_p, P(TT), P(TT), C.c_int64, C.c_int32, P(C.c_int64), P(C.c_size_t)]
    L.qtt_set_jacobi_max_sweeps.argtypes = [vp, C.c_int32]
    L.qtt_profile_start.argtypes = [vp, C.c_int, C.c_int]
    L.qtt_profile_stop.argtypes = [vp, P(C.c_int64), P(C.c_double), P(C.c_double), P(C.c_double)]
    for name in EXPORTS:
        if name != "qtt_status_string":
            getattr(L, name).restype = C.c_int
    _lib = L
    atexit.register(_release_all)
    return L


_plans = weakref.WeakSet()


def _release_all():
    """Destroy batch plans, then handles, at interpreter exit while the HIP
    runtime is still alive (instead of leaving it to __del__ during module
    teardown, whose order is unspecified)."""
    for p in list(_plans):
        try:
            p.close()
        except Exception:
            pass
    for h in list(_handles.values()):
        try:
            h.close()
        except Exception:
            pass
    _handles.clear()


def _status_string(st: int) -> str:
    try:
        return load_library().qtt_status_string(st).decode()
    except Exception:
        return ""


def _check(st: int, where: str):
    if st != QTT_OK:
        raise QttError(st, where)


class Handle:
    """Owns a qtt_handle bound to one gfx950 device."""

    def __init__(self, device: int = 0):
        L = load_library()
        self._h = C.c_void_p()
        _check(L.qtt_create(C.byref(self._h), device), "qtt_create")
        self.device = device

    @property
    def ptr(self):
        return self._h

    def close(self):
        if self._h:
            load_library().qtt_destroy(self._h)
            self._h = C.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


_handles = {}


def handle(device: Optional[int] = None) -> Handle:
    if device is None:
        device = torch.cuda.current_device()
    h = _handles.get(device)
    if h is None:
        h = Handle(device)
        _handles[device] = h
    return h


def set_jacobi_max_sweeps(max_sweeps: int, device: Optional[int] = None):
    """Sweep cap of the Jacobi SVD for this device's handle (0: default)."""
    _check(load_library().qtt_set_jacobi_max_sweeps(handle(device).ptr, int(max_sweeps)),
           "qtt_set_jacobi_max_sweeps")


@dataclass
class TTView:
    """ctypes view of a list of device core tensors (kept alive by this object)."""
    cores: List[torch.Tensor]
    legs: int
    ranks_override: Optional[Sequence[int]] = None
    phys_override: Optional[Sequence[int]] = None
    struct: TT = field(init=False)

    def __post_init__(self):
        n = len(self.cores)
        self._phys = (C.c_int32 * (n * self.legs))()
        self._ranks = (C.c_int64 * (n + 1))()
        self._ptrs = (C.c_void_p * n)()
        dt = self.cores[0].dtype
        for k, c in enumerate(self.cores):
            if c.device.type != "cuda":
                raise ValueError("cores must be device tensors")
            if c.dtype != dt:
                raise ValueError("mixed core dtypes")
            if not c.is_contiguous():
                raise ValueError("cores must be contiguous")
            if self.phys_override is not None:
                self._phys[k] = int(self.phys_override[k])
            elif self.legs == 1:
                self._phys[k] = c.shape[1]
            else:
                self._phys[2 * k] = c.shape[1]
                self._phys[2 * k + 1] = c.shape[2]
            self._ptrs[k] = c.data_ptr()
        if self.ranks_override is not None:
            for k, r in enumerate(self.ranks_override):
                self._ranks[k] = int(r)
        else:
            self._ranks[0] = self.cores[0].shape[0]
            for k, c in enumerate(self.cores):
                self._ranks[k + 1] = c.shape[-1]
        dtype = F64 if dt == torch.float64 else F32 if dt == torch.float32 else None
        if dtype is None:
            raise ValueError(f"unsupported dtype {dt}")
        self.struct = TT(n, self.legs, self._phys, self._ranks, self._ptrs, dtype)

    def ranks(self) -> List[int]:
        return [int(self._ranks[k]) for k in range(len(self.cores) + 1)]


def _stream_ptr():
    return C.c_void_p(torch.cuda.current_stream().cuda_stream)


def _workspace(nbytes: int, device) -> torch.Tensor:
    return torch.empty(max(int(nbytes), 256), dtype=torch.uint8, device=device)


def _legs(spec: str) -> int:
    s = spec.replace(" ", "")
    if s == "i,i->i":
        return 1
    if s == "ij,j->i":
        return 2
    raise ValueError(f"unsupported spec {spec!r}")


def contract(spec: str, a: Sequence[torch.Tensor], b: Sequence[torch.Tensor]) -> List[torch.Tensor]:
    """Exact core-by-core einsum; returns the contracted cores (device tensors).
    "ij,jk->ik" multiplies two MPOs and returns MPO cores."""
    L = load_library()
    h = handle(a[0].device.index)
    opop = spec.replace(" ", "") == "ij,jk->ik"
    va, vb = TTView(list(a), 2 if opop else _legs(spec)), TTView(list(b), 2 if opop else 1)
    dev = a[0].device
    out = []
    for ca, cb in zip(a, b):
        if opop:
            shp = (ca.shape[0] * cb.shape[0], ca.shape[1], cb.shape[2], ca.shape[-1] * cb.shape[-1])
        else:
            shp = (ca.shape[0] * cb.shape[0], ca.shape[1], ca.shape[-1] * cb.shape[-1])
        out.append(torch.empty(shp, dtype=ca.dtype, device=dev))
    vc = TTView(out, 2 if opop else 1)
    _check(L.qtt_contract(h.ptr, spec.encode(), C.byref(va.struct), C.byref(vb.struct), C.byref(vc.struct),
                          None, 0, _stream_ptr()), "qtt_contract")
    return out


def add(terms: Sequence[Sequence[torch.Tensor]], coeffs: Optional[Sequence[float]] = None) -> List[torch.Tensor]:
    """Exact sum of trains (MPS cores [r, d, r'] or MPO cores [r, d_out, d_in, r'])
    with block cores; returns the summed cores (device tensors)."""
    L = load_library()
    h = handle(terms[0][0].device.index)
    legs = terms[0][0].dim() - 2
    views = [TTView(list(t), legs) for t in terms]
    arr = (TT * len(terms))(*[v.struct for v in views])
    n = len(terms[0])
    ranks = [1] * (n + 1)
    for k in range(1, n):
        ranks[k] = sum(v.ranks()[k] for v in views)
    dev = terms[0][0].device
    out = []
    for k in range(n):
        shp = (ranks[k],) + tuple(terms[0][k].shape[1:-1]) + (ranks[k + 1],)
        out.append(torch.empty(shp, dtype=terms[0][0].dtype, device=dev))
    vo = TTView(out, legs)
    cf = None
    if coeffs is not None:
        cf = (C.c_double * len(terms))(*[float(c) for c in coeffs])
    _check(L.qtt_add(h.ptr, len(terms), arr, cf, C.byref(vo.struct), _stream_ptr()), "qtt_add")
    return out


def inner(a: Sequence[torch.Tensor], b: Sequence[torch.Tensor], prec: str = "fp64") -> float:
    """<a, b> by the environment sweep; `prec` selects the GEMM arithmetic."""
    L = load_library()
    h = handle(a[0].device.index)
    va, vb = TTView(list(a), 1), TTView(list(b), 1)
    nb = C.c_size_t()
    _check(L.qtt_workspace_size(h.ptr, OP_INNER, None, C.byref(va.struct), C.byref(vb.struct), 0, 0,
                                C.byref(nb)), "qtt_workspace_size")
    ws = _workspace(nb.value, a[0].device)
    out = C.c_double()
    if prec == "fp64":
        _check(L.qtt_inner(h.ptr, C.byref(va.struct), C.byref(vb.struct), C.byref(out), C.c_void_p(ws.data_ptr()),
                           ws.numel(), _stream_ptr()), "qtt_inner")
    else:
        _check(L.qtt_inner_prec(h.ptr, C.byref(va.struct), C.byref(vb.struct), PREC[prec], C.byref(out),
                                C.c_void_p(ws.data_ptr()), ws.numel(), _stream_ptr()), "qtt_inner_prec")
    return out.value


def inner_backward(a, b, g: float = 1.0, want_a: bool = True, want_b: bool = False):
    L = load_library()
    h = handle(a[0].device.index)
    va, vb = TTView(list(a), 1), TTView(list(b), 1)
    da = [torch.empty_like(c) for c in a] if want_a else None
    db = [torch.empty_like(c) for c in b] if want_b else None
    vda = TTView(da, 1) if da else None
    vdb = TTView(db, 1) if db else None
    nb = C.c_size_t()
    _check(L.qtt_workspace_size(h.ptr, OP_INNER_BACKWARD, None, C.byref(va.struct), C.byref(vb.struct), 0, 0,
                                C.byref(nb)), "qtt_workspace_size")
    ws = _workspace(nb.value, a[0].device)
    _check(L.qtt_inner_backward(h.ptr, C.byref(va.struct), C.byref(vb.struct), float(g),
                                C.byref(vda.struct) if vda else None, C.byref(vdb.struct) if vdb else None,
                                C.c_void_p(ws.data_ptr()), ws.numel(), _stream_ptr()), "qtt_inner_backward")
    return da, db


def contract_backward(spec: str, a, b, dc, want_a: bool = False, want_b: bool = True):
    L = load_library()
    h = handle(a[0].device.index)
    va, vb, vdc = TTView(list(a), _legs(spec)), TTView(list(b), 1), TTView(list(dc), 1)
    da = [torch.empty_like(c) for c in a] if want_a else None
    db = [torch.empty_like(c) for c in b] if want_b else None
    vda = TTView(da, _legs(spec)) if da else None
    vdb = TTView(db, 1) if db else None
    _check(L.qtt_contract_backward(h.ptr, spec.encode(), C.byref(va.struct), C.byref(vb.struct),
                                   C.byref(vdc.struct), C.byref(vda.struct) if vda else None,
                                   C.byref(vdb.struct) if vdb else None, None, 0, _stream_ptr()),
           "qtt_contract_backward")
    return da, db


@dataclass
class RoundResult:
    cores: List[torch.Tensor]
    ranks: List[int]
    norm: float
    delta: float
    err_bound: float
    tails: List[float]
    margin_lo: List[float]
    margin_hi: List[float]
    maxrank_hit: List[bool]
    sigmas: Optional[List[List[float]]]
    jacobi_sweeps_max: int


def rank_bounds(rc: Sequence[int], d: Sequence[int], max_rank: int) -> List[int]:
    """Upper bounds of the rounded ranks (what output buffers must hold)."""
    n = len(d)
    rho = [1] * (n + 1)
    for k in range(n - 1):
        rho[k + 1] = min(rho[k] * d[k], rc[k + 1])
    out = [1] * (n + 1)
    right = 1
    for k in range(n - 1, 0, -1):
        right = min(right * d[k], 1 << 40)
        bnd = min(rho[k], right)
        if max_rank and max_rank > 0:
            bnd = min(bnd, max_rank)
        out[k] = max(bnd, 1)
    return out


class _Info:
    def __init__(self, n: int, sigma_ld: int = 0):
        m = max(n - 1, 1)
        self.tail = (C.c_double * m)()
        self.mlo = (C.c_double * m)()
        self.mhi = (C.c_double * m)()
        self.hit = (C.c_uint8 * m)()
        self.sigma_ld = sigma_ld
        self.sigma = (C.c_double * (m * sigma_ld))() if sigma_ld > 0 else None
        self.c = RoundInfoC()
        self.c.tail = self.tail
        self.c.margin_lo = self.mlo
        self.c.margin_hi = self.mhi
        self.c.maxrank_hit = self.hit
        self.c.sigma = self.sigma if self.sigma is not None else None
        self.c.sigma_ld = sigma_ld

    def result(self, cores, ranks, n):
        m = n - 1
        sig = None
        if self.sigma is not None:
            sig = [[self.sigma[k * self.sigma_ld + i] for i in range(self.sigma_ld)] for k in range(m)]
        return RoundResult(cores, ranks, self.c.norm, self.c.delta, self.c.err_bound,
                           [self.tail[k] for k in range(m)], [self.mlo[k] for k in range(m)],
                           [self.mhi[k] for k in range(m)], [bool(self.hit[k]) for k in range(m)], sig,
                           self.c.jacobi_sweeps_max)


def _views_of_compact(buffers: List[torch.Tensor], ranks: Sequence[int], d: Sequence[int]):
    out = []
    for k, buf in enumerate(buffers):
        cnt = ranks[k] * d[k] * ranks[k + 1]
        out.append(buf.reshape(-1)[:cnt].view(ranks[k], d[k], ranks[k + 1]))
    return out


def contract_round(spec: str, a, b, rel_tol: float, max_rank: int = 0, prec: str = "fp64",
                   want_sigmas: bool = False, out_buffers: Optional[List[torch.Tensor]] = None,
                   workspace: Optional[torch.Tensor] = None) -> RoundResult:
    """Contraction + TT rounding without materialising the contracted cores."""
    L = load_library()
    h = handle(a[0].device.index)
    legs = _legs(spec)
    va, vb = TTView(list(a), legs), TTView(list(b), 1)
    n = len(a)
    d = [c.shape[1] for c in a]
    rc = [x * y for x, y in zip(va.ranks(), vb.ranks())]
    bnd = rank_bounds(rc, d, max_rank)
    dev = a[0].device
    if out_buffers is None:
        out_buffers = [torch.empty(bnd[k] * d[k] * bnd[k + 1], dtype=torch.float64, device=dev) for k in range(n)]
    vo = TTView([x.reshape(-1) for x in out_buffers], 1, ranks_override=bnd, phys_override=d)
    nb = C.c_size_t()
    _check(L.qtt_workspace_size(h.ptr, OP_CONTRACT_ROUND, spec.encode(), C.byref(va.struct), C.byref(vb.struct),
                                int(max_rank), PREC[prec], C.byref(nb)), "qtt_workspace_size")
    if workspace is None or workspace.numel() < nb.value:
        workspace = _workspace(nb.value, dev)
    sig_ld = max(bnd) * 2 if want_sigmas else 0
    if want_sigmas:
        sig_ld = max(rc) if max(rc) < 8192 else 8192
    info = _Info(n, sig_ld)
    _check(L.qtt_contract_round(h.ptr, spec.encode(), C.byref(va.struct), C.byref(vb.struct), C.byref(vo.struct),
                                float(rel_tol), int(max_rank), PREC[prec], C.byref(info.c),
                                C.c_void_p(workspace.data_ptr()), workspace.numel(), _stream_ptr()),
           "qtt_contract_round")
    ranks = vo.ranks()
    cores = _views_of_compact(out_buffers, ranks, d)
    return info.result(cores, ranks, n)


class ContractRoundAsync:
    """Stream-ordered contract + round (qtt_contract_round_async) with its
    buffers allocated once: output cores at the rank bounds, the workspace,
    and the device rank / status record.  `enqueue()` only enqueues work on
    the current stream (so it can be captured in a CUDA/HIP graph);
    `result()` reads the record after synchronising."""

    def __init__(self, spec: str, a, b, rel_tol: float, max_rank: int = 0, prec: str = "fp64"):
        L = load_library()
        self.spec, self.rel_tol, self.max_rank, self.prec = spec, float(rel_tol), int(max_rank), prec
        self.h = handle(a[0].device.index)
        self.va, self.vb = TTView(list(a), _legs(spec)), TTView(list(b), 1)
        n = len(a)
        self.n = n
        self.d = [c.shape[1] for c in a]
        rc = [x * y for x, y in zip(self.va.ranks(), self.vb.ranks())]
        bnd = rank_bounds(rc, self.d, max_rank)
        dev = a[0].device
        self.out_buffers = [torch.zeros(bnd[k] * self.d[k] * bnd[k + 1], dtype=torch.float64, device=dev)
                            for k in range(n)]
        self.vo = TTView(self.out_buffers, 1, ranks_override=bnd, phys_override=self.d)
        nb = C.c_size_t()
        _check(L.qtt_workspace_size(self.h.ptr, OP_CONTRACT_ROUND, spec.encode(), C.byref(self.va.struct),
                                    C.byref(self.vb.struct), self.max_rank, PREC[prec], C.byref(nb)),
               "qtt_workspace_size")
        self.ws = _workspace(nb.value, dev)
        self.ranks_dev = torch.zeros(n + 1, dtype=torch.int64, device=dev)
        self.status_dev = torch.zeros(1, dtype=torch.int32, device=dev)

    def enqueue(self):
        _check(load_library().qtt_contract_round_async(
            self.h.ptr, self.spec.encode(), C.byref(self.va.struct), C.byref(self.vb.struct),
            C.byref(self.vo.struct), self.rel_tol, self.max_rank, PREC[self.prec],
            C.c_void_p(self.ranks_dev.data_ptr()), C.c_void_p(self.status_dev.data_ptr()),
            C.c_void_p(self.ws.data_ptr()), self.ws.numel(), _stream_ptr()), "qtt_contract_round_async")

    def result(self):
        torch.cuda.synchronize()
        st = int(self.status_dev.item())
        if st != QTT_OK:
            raise QttError(st, "qtt_contract_round_async")
        ranks = [int(x) for x in self.ranks_dev.tolist()]
        return _views_of_compact(self.out_buffers, ranks, self.d), ranks


def contract_round_noalloc(spec: str, a, b, rel_tol: float, max_rank: int, out_buffers: List[torch.Tensor],
                           prec: str = "fp64") -> RoundResult:
    """contract_round through the allocation-free entry point.

    The caller passes the output buffers (each large enough for the rank
    bounds of `rank_bounds`); the library's fixed device array is the
    workspace, so nothing is allocated on the device by this call.
    """
    L = load_library()
    h = handle(a[0].device.index)
    va, vb = TTView(list(a), _legs(spec)), TTView(list(b), 1)
    n = len(a)
    d = [c.shape[1] for c in a]
    rc = [x * y for x, y in zip(va.ranks(), vb.ranks())]
    bnd = rank_bounds(rc, d, max_rank)
    if len(out_buffers) != n:
        raise ValueError("one output buffer per core")
    for k in range(n):
        if out_buffers[k].numel() < bnd[k] * d[k] * bnd[k + 1]:
            raise ValueError(f"output buffer {k} smaller than its rank bound")
    vo = TTView([x.reshape(-1) for x in out_buffers], 1, ranks_override=bnd, phys_override=d)
    info = _Info(n)
    _check(L.qtt_contract_round_noalloc(h.ptr, spec.encode(), C.byref(va.struct), C.byref(vb.struct),
                                        C.byref(vo.struct), float(rel_tol), int(max_rank), PREC[prec],
                                        C.byref(info.c), _stream_ptr()),
           "qtt_contract_round_noalloc")
    ranks = vo.ranks()
    return info.result(_views_of_compact(out_buffers, ranks, d), ranks, n)


def zipup_query(spec: str, a_struct: TT, b_struct: TT, max_rank: int = 0, ncores: int = 1):
    """(rank bounds of the zip-up result, workspace bytes) from the shapes alone."""
    L = load_library()
    n = a_struct.n
    bounds = (C.c_int64 * (n + 1))()
    nb = C.c_size_t()
    _check(L.qtt_zipup_query(spec.encode(), C.byref(a_struct), C.byref(b_struct), int(max_rank), int(ncores),
                             bounds, C.byref(nb)), "qtt_zipup_query")
    return [int(bounds[k]) for k in range(n + 1)], nb.value


def contract_zipup(spec: str, a, b, rel_tol: float, max_rank: int = 0, ncores: int = 1, prec: str = "fp64",
                   want_sigmas: bool = False, out_buffers: Optional[List[torch.Tensor]] = None,
                   workspace: Optional[torch.Tensor] = None) -> RoundResult:
    """Contraction by the decomposition (zip-up) algorithm: operands normalised
    to the left end, super-cores of `ncores` product cores split off one
    truncated SVD at a time; the contracted train is never formed."""
    L = load_library()
    h = handle(a[0].device.index)
    legs = _legs(spec)
    va, vb = TTView(list(a), legs), TTView(list(b), 1)
    n = len(a)
    d = [c.shape[1] for c in a]
    bnd, nbytes = zipup_query(spec, va.struct, vb.struct, max_rank, ncores)
    dev = a[0].device
    if out_buffers is None:
        out_buffers = [torch.empty(bnd[k] * d[k] * bnd[k + 1], dtype=torch.float64, device=dev) for k in range(n)]
    vo = TTView([x.reshape(-1) for x in out_buffers], 1, ranks_override=bnd, phys_override=d)
    if workspace is None or workspace.numel() < nbytes:
        workspace = _workspace(nbytes, dev)
    sig_ld = 0
    if want_sigmas:
        sig_ld = max(bnd) * max(d)  # singular values per split <= r d
    info = _Info(n, sig_ld)
    _check(L.qtt_contract_zipup(h.ptr, spec.encode(), C.byref(va.struct), C.byref(vb.struct), C.byref(vo.struct),
                                float(rel_tol), int(max_rank), int(ncores), PREC[prec], C.byref(info.c),
                                C.c_void_p(workspace.data_ptr()), workspace.numel(), _stream_ptr()),
           "qtt_contract_zipup")
    ranks = vo.ranks()
    return info.result(_views_of_compact(out_buffers, ranks, d), ranks, n)


def fit(spec: str, a, b, guess, nsweeps: int = 1, workspace: Optional[torch.Tensor] = None):
    """Variational fitting of a copy of `guess` (FP64 MPS cores) to the product
    of a and b; returns (cores, ranks, norm)."""
    L = load_library()
    h = handle(a[0].device.index)
    legs = _legs(spec)
    va, vb = TTView(list(a), legs), TTView(list(b), 1)
    bufs = [g.detach().clone().reshape(-1) for g in guess]
    d = [g.shape[1] for g in guess]
    vc = TTView(bufs, 1, ranks_override=[guess[0].shape[0]] + [g.shape[-1] for g in guess], phys_override=d)
    nb = C.c_size_t()
    _check(L.qtt_fit_workspace_size(spec.encode(), C.byref(va.struct), C.byref(vb.struct), C.byref(vc.struct),
                                    C.byref(nb)), "qtt_fit_workspace_size")
    if workspace is None or workspace.numel() < nb.value:
        workspace = _workspace(nb.value, a[0].device)
    nrm = C.c_double()
    _check(L.qtt_fit(h.ptr, spec.encode(), C.byref(va.struct), C.byref(vb.struct), C.byref(vc.struct), int(nsweeps),
                     C.byref(nrm), C.c_void_p(workspace.data_ptr()), workspace.numel(), _stream_ptr()), "qtt_fit")
    ranks = vc.ranks()
    return _views_of_compact(bufs, ranks, d), ranks, nrm.value


def fit2(spec: str, a, b, guess, nsweeps: int = 1, rel_tol: float = 0.0, max_rank: int = 0,
         workspace: Optional[torch.Tensor] = None):
    """Two-core variational fitting (qtt_fit2) of a copy of `guess` to the
    product of a and b: the ranks adapt under rel_tol / max_rank.  Returns
    (cores, ranks, norm, info dict with the last sweep's discarded tails)."""
    L = load_library()
    h = handle(a[0].device.index)
    legs = _legs(spec)
    va, vb = TTView(list(a), legs), TTView(list(b), 1)
    n = len(guess)
    d = [g.shape[1] for g in guess]
    r_in = [guess[0].shape[0]] + [g.shape[-1] for g in guess]
    probe = TTView([g.detach().reshape(-1) for g in guess], 1, ranks_override=r_in, phys_override=d)
    bnd = (C.c_int64 * (n + 1))()
    nb = C.c_size_t()
    _check(L.qtt_fit2_query(spec.encode(), C.byref(va.struct), C.byref(vb.struct), C.byref(probe.struct),
                            int(max_rank), bnd, C.byref(nb)), "qtt_fit2_query")
    bounds = [int(bnd[k]) for k in range(n + 1)]
    dev = a[0].device
    bufs = []
    for k, g in enumerate(guess):
        buf = torch.zeros(bounds[k] * d[k] * bounds[k + 1], dtype=torch.float64, device=dev)
        buf[: g.numel()] = g.detach().reshape(-1)
        bufs.append(buf)
    vc = TTView(bufs, 1, ranks_override=r_in, phys_override=d)
    if workspace is None or workspace.numel() < nb.value:
        workspace = _workspace(nb.value, dev)
    info = _Info(n)
    _check(L.qtt_fit2(h.ptr, spec.encode(), C.byref(va.struct), C.byref(vb.struct), C.byref(vc.struct),
                      int(nsweeps), float(rel_tol), int(max_rank), C.byref(info.c),
                      C.c_void_p(workspace.data_ptr()), workspace.numel(), _stream_ptr()), "qtt_fit2")
    ranks = vc.ranks()
    extra = {"tails": [info.tail[k] for k in range(n - 1)], "jacobi_sweeps_max": info.c.jacobi_sweeps_max}
    return _views_of_compact(bufs, ranks, d), ranks, info.c.norm, extra


def solve(w, b, guess, nsweeps: int = 1, ncores: int = 1, rel_tol: float = 0.0, max_rank: int = 0,
          workspace: Optional[torch.Tensor] = None):
    """DMRG-like solution of w x = b (qtt_solve) starting from a copy of
    `guess`.  Returns (cores, ranks, norm)."""
    L = load_library()
    h = handle(b[0].device.index)
    vw, vb = TTView(list(w), 2), TTView(list(b), 1)
    n = len(guess)
    d = [g.shape[1] for g in guess]
    r_in = [guess[0].shape[0]] + [g.shape[-1] for g in guess]
    probe = TTView([g.detach().reshape(-1) for g in guess], 1, ranks_override=r_in, phys_override=d)
    bnd = (C.c_int64 * (n + 1))()
    nb = C.c_size_t()
    _check(L.qtt_solve_query(C.byref(vw.struct), C.byref(vb.struct), C.byref(probe.struct), int(ncores),
                             int(max_rank), bnd, C.byref(nb)), "qtt_solve_query")
    bounds = [int(bnd[k]) for k in range(n + 1)]
    dev = b[0].device
    bufs = []
    for k, g in enumerate(guess):
        buf = torch.zeros(max(bounds[k] * d[k] * bounds[k + 1], g.numel()), dtype=torch.float64, device=dev)
        buf[: g.numel()] = g.detach().reshape(-1)
        bufs.append(buf)
    vx = TTView(bufs, 1, ranks_override=r_in, phys_override=d)
    if workspace is None or workspace.numel() < nb.value:
        workspace = _workspace(nb.value, dev)
    info = _Info(n)
    _check(L.qtt_solve(h.ptr, C.byref(vw.struct), C.byref(vb.struct), C.byref(vx.struct), int(nsweeps), int(ncores),
                       float(rel_tol), int(max_rank), C.byref(info.c), C.c_void_p(workspace.data_ptr()),
                       workspace.numel(), _stream_ptr()), "qtt_solve")
    ranks = vx.ranks()
    return _views_of_compact(bufs, ranks, d), ranks, info.c.norm


def solve_amen(w, b, guess, residual_guess, nsweeps: int = 1, rel_tol: float = 0.0, max_rank: int = 0,
               workspace: Optional[torch.Tensor] = None):
    """AMEn solution of w x = b (qtt_solve_amen) starting from copies of
    `guess` and of `residual_guess` (the initial residual train z).
    Returns (x cores, x ranks, z cores, z ranks, norm)."""
    L = load_library()
    h = handle(b[0].device.index)
    vw, vb = TTView(list(w), 2), TTView(list(b), 1)
    n = len(guess)
    d = [g.shape[1] for g in guess]
    rx_in = [guess[0].shape[0]] + [g.shape[-1] for g in guess]
    rz_in = [residual_guess[0].shape[0]] + [g.shape[-1] for g in residual_guess]
    px = TTView([g.detach().reshape(-1) for g in guess], 1, ranks_override=rx_in, phys_override=d)
    pz = TTView([g.detach().reshape(-1) for g in residual_guess], 1, ranks_override=rz_in, phys_override=d)
    bx, bz = (C.c_int64 * (n + 1))(), (C.c_int64 * (n + 1))()
    nb = C.c_size_t()
    _check(L.qtt_solve_amen_query(C.byref(vw.struct), C.byref(vb.struct), C.byref(px.struct), C.byref(pz.struct),
                                  int(max_rank), bx, bz, C.byref(nb)), "qtt_solve_amen_query")
    dev = b[0].device

    def buffers(cores, bounds):
        out = []
        for k, g in enumerate(cores):
            buf = torch.zeros(max(bounds[k] * d[k] * bounds[k + 1], g.numel()), dtype=torch.float64, device=dev)
            buf[: g.numel()] = g.detach().reshape(-1)
            out.append(buf)
        return out

    xb = buffers(guess, [int(bx[k]) for k in range(n + 1)])
    zb = buffers(residual_guess, [int(bz[k]) for k in range(n + 1)])
    vx = TTView(xb, 1, ranks_override=rx_in, phys_override=d)
    vz = TTView(zb, 1, ranks_override=rz_in, phys_override=d)
    if workspace is None or workspace.numel() < nb.value:
        workspace = _workspace(nb.value, dev)
    info = _Info(n)
    _check(L.qtt_solve_amen(h.ptr, C.byref(vw.struct), C.byref(vb.struct), C.byref(vx.struct), C.byref(vz.struct),
                            int(nsweeps), float(rel_tol), int(max_rank), C.byref(info.c),
                            C.c_void_p(workspace.data_ptr()), workspace.numel(), _stream_ptr()), "qtt_solve_amen")
    rx, rz = vx.ranks(), vz.ranks()
    return _views_of_compact(xb, rx, d), rx, _views_of_compact(zb, rz, d), rz, info.c.norm


def round_tt(cores, rel_tol: float, max_rank: int = 0, prec: str = "fp64", want_sigmas: bool = False,
             inplace: bool = False) -> RoundResult:
    """TT rounding of an FP64 MPS (copied unless inplace)."""
    L = load_library()
    h = handle(cores[0].device.index)
    bufs = [c if inplace else c.clone() for c in cores]
    d = [c.shape[1] for c in cores]
    flat = [b.reshape(-1) for b in bufs]
    v = TTView(flat, 1, ranks_override=[cores[0].shape[0]] + [c.shape[-1] for c in cores], phys_override=d)
    nb = C.c_size_t()
    _check(L.qtt_workspace_size(h.ptr, OP_ROUND, None, C.byref(v.struct), None, int(max_rank), PREC[prec],
                                C.byref(nb)), "qtt_workspace_size")
    ws = _workspace(nb.value, cores[0].device)
    n = len(cores)
    sig_ld = max(v.ranks()) if want_sigmas else 0
    info = _Info(n, sig_ld)
    _check(L.qtt_round(h.ptr, C.byref(v.struct), float(rel_tol), int(max_rank), PREC[prec], C.byref(info.c),
                       C.c_void_p(ws.data_ptr()), ws.numel(), _stream_ptr()), "qtt_round")
    ranks = v.ranks()
    return info.result(_views_of_compact(flat, ranks, d), ranks, n)


def orthogonalize(cores, inplace: bool = False):
    L = load_library()
    h = handle(cores[0].device.index)
    bufs = [c if inplace else c.clone() for c in cores]
    d = [c.shape[1] for c in cores]
    flat = [b.reshape(-1) for b in bufs]
    v = TTView(flat, 1, ranks_override=[cores[0].shape[0]] + [c.shape[-1] for c in cores], phys_override=d)
    nb = C.c_size_t()
    _check(L.qtt_workspace_size(h.ptr, OP_ORTHOGONALIZE, None, C.byref(v.struct), None, 0, 0, C.byref(nb)),
           "qtt_workspace_size")
    ws = _workspace(nb.value, cores[0].device)
    nrm = C.c_double()
    _check(L.qtt_orthogonalize(h.ptr, C.byref(v.struct), C.byref(nrm), C.c_void_p(ws.data_ptr()), ws.numel(),
                               _stream_ptr()), "qtt_orthogonalize")
    ranks = v.ranks()
    return _views_of_compact(flat, ranks, d), nrm.value


class BatchPlan:
    """Batched contract+round of many independent problems in one persistent launch.

    The plan owns the output buffers (sized by the rank bounds), the workspace
    and a captured hipGraph; launch() replays it, results() reads the ranks.
    """

    def __init__(self, spec: str, A: Sequence[Sequence[torch.Tensor]], B: Sequence[Sequence[torch.Tensor]],
                 rel_tol: float, max_rank: int = 0, tune: bool = True):
        L = load_library()
        self.spec = spec
        self.count = len(A)
        legs = _legs(spec)
        dev = A[0][0].device
        self.h = handle(dev.index)
        self.va = [TTView(list(a), legs) for a in A]
        self.vb = [TTView(list(b), 1) for b in B]
        self.d = [[c.shape[1] for c in a] for a in A]
        self.bounds, self.out_buffers, self.vo = [], [], []
        for i in range(self.count):
            rc = [x * y for x, y in zip(self.va[i].ranks(), self.vb[i].ranks())]
            bnd = rank_bounds(rc, self.d[i], max_rank)
            bufs = [torch.empty(bnd[k] * self.d[i][k] * bnd[k + 1], dtype=torch.float64, device=dev)
                    for k in range(len(self.d[i]))]
            self.bounds.append(bnd)
            self.out_buffers.append(bufs)
            self.vo.append(TTView(bufs, 1, ranks_override=bnd, phys_override=self.d[i]))
        ta = (TT * self.count)(*[v.struct for v in self.va])
        tb = (TT * self.count)(*[v.struct for v in self.vb])
        to = (TT * self.count)(*[v.struct for v in self.vo])
        self._arrays = (ta, tb, to)
        nb = C.c_size_t()
        _check(L.qtt_batch_workspace_size(self.h.ptr, spec.encode(), self.count, ta, tb, int(max_rank), C.byref(nb)),
               "qtt_batch_workspace_size")
        self.ws = _workspace(nb.value + 256, dev)
        self._plan = C.c_void_p()
        _check(L.qtt_batch_plan_create(self.h.ptr, spec.encode(), self.count, ta, tb, to, float(rel_tol),
                                       int(max_rank), 1 if tune else 0, C.c_void_p(self.ws.data_ptr()),
                                       self.ws.numel(), _stream_ptr(), C.byref(self._plan)), "qtt_batch_plan_create")
        _plans.add(self)

    def launch(self):
        _check(load_library().qtt_batch_plan_launch(self._plan, _stream_ptr()), "qtt_batch_plan_launch")

    def results(self):
        """(ranks per problem, tails per problem) after the last launch."""
        tot = sum(len(d) + 1 for d in self.d)
        tt = sum(max(len(d) - 1, 0) for d in self.d)
        r = (C.c_int64 * tot)()
        t = (C.c_double * max(tt, 1))()
        _check(load_library().qtt_batch_plan_results(self._plan, r, t, _stream_ptr()), "qtt_batch_plan_results")
        ranks, tails, o, ot = [], [], 0, 0
        for d in self.d:
            ranks.append([int(r[o + k]) for k in range(len(d) + 1)])
            tails.append([t[ot + k] for k in range(len(d) - 1)])
            o += len(d) + 1
            ot += max(len(d) - 1, 0)
        self.ranks = ranks
        return ranks, tails

    def info(self):
        v, g = C.c_int32(), C.c_int32()
        ms = (C.c_float * 4)()
        _check(load_library().qtt_batch_plan_info(self._plan, C.byref(v), C.byref(g), ms), "qtt_batch_plan_info")
        tiles = (C.c_uint8 * 8)()
        shapes = (C.c_int32 * 24)()
        pms = (C.c_float * 32)()
        _check(load_library().qtt_batch_plan_tiles(self._plan, tiles, shapes, pms), "qtt_batch_plan_tiles")
        names = ["64x64", "64x32", "32x64", "32x32"]
        gemm = {b: {"shape": [shapes[3 * b + c] for c in range(3)], "tile": names[tiles[b]],
                    "probe_ms": [pms[4 * b + v] for v in range(4)]}
                for b in range(8) if shapes[3 * b] > 0}
        return {"variant": v.value, "grid": g.value, "tuned_ms": [ms[i] for i in range(4)], "gemm_tiles": gemm}

    def cores(self, i: int) -> List[torch.Tensor]:
        return _views_of_compact(self.out_buffers[i], self.ranks[i], self.d[i])

    def close(self):
        if self._plan:
            load_library().qtt_batch_plan_destroy(self._plan)
            self._plan = C.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


PROFILE_CLASSES = {"apply_panel": 0, "jacobi": 1, "qr_panel": 2, "block_vty": 3, "block_upd": 4, "chol_block": 5,
                   "chol_update": 6, "chol_solve": 7}


def profile_start(kernel_class: str, max_launches: int = 100000, device: Optional[int] = None):
    L = load_library()
    _check(L.qtt_profile_start(handle(device).ptr, PROFILE_CLASSES[kernel_class], max_launches), "qtt_profile_start")


def profile_stop(device: Optional[int] = None):
    """Returns (launches, total_ms, algorithmic_bytes, algorithmic_flops)."""
    L = load_library()
    n = C.c_int64()
    ms, b, f = C.c_double(), C.c_double(), C.c_double()
    _check(L.qtt_profile_stop(handle(device).ptr, C.byref(n), C.byref(ms), C.byref(b), C.byref(f)),
           "qtt_profile_stop")
    return n.value, ms.value, b.value, f.value


def to_device(cores, device="cuda", dtype=torch.float64):
    return [torch.as_tensor(c, dtype=dtype).contiguous().to(device) for c in cores]


def to_host(cores):
    return [c.detach().to("cpu").double().numpy() for c in cores]
