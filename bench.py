"""Benchmark: QTT contract + round on one MI355X.

Workload: 3D finite-difference Laplacian MPO (interleaved, 42 cores of
physical size 2, interior rank 7) applied to a Gaussian rank-256 MPS
(seed 3, variance-normalised), rounded back to max rank 256 at relative
tolerance 1e-8.  A step is one call of the fused contract+round (QR sweep
with BF16x6 bond GEMMs, FP64 Householder QR, FP64 Jacobi SVD sweep); the
inputs are resident in HBM before the timed region.

Prints one JSON line: metric, value, roofline of the kernel class that
takes the most time, and the oracle's CPU baseline on the same workload.
`--workload hadamard_batch` measures the batched form instead (512 uneven 1D
Hadamard products in one graph-replayed persistent launch), and
`--workload laplacian3d_n42_r256_zipup` the same product computed by the
decomposition ("zip-up") algorithm of Sec. 3.2 (`--ncores` product cores per
super-core), whose FLOP are counted under the same conventions for the work
that algorithm does; `--workload sum4_n42_r128_round` the exact sum of four
rank-128 trains followed by rounding, and `--workload
laplacian2d_n32_r64_zipup_fit` a zip-up guess followed by one variational
sweep (Sec. 3.3); `--workload heat2d_n24_solve` and `heat2d_n24_amen` the
DMRG-like and AMEn linear solvers (Sec. 5) on an implicit heat step of a 2D
2^12 x 2^12 grid.
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)


def geqrf_flops(m, n):
    if m >= n:
        return 2.0 * m * n * n - 2.0 * n ** 3 / 3.0
    return 2.0 * n * m * m - 2.0 * m ** 3 / 3.0


def ormqr_flops(m, k, c):
    """Apply k Householder reflectors of an m-row Q to an m x c matrix."""
    return 4.0 * m * k * c - 2.0 * k * k * c


def svd_nominal_flops(m, n):
    """Nominal SVD count of an m x n matrix (fixed sweep count, not measured)."""
    if m < n:
        m, n = n, m
    return geqrf_flops(m, n) + 8 * 9.0 * n ** 3 + 2.0 * m * n * n


def contract_round_flops(ra, rb, d, dj, ranks_out, mpo=True):
    """Algorithmic FLOP of contract + round under fixed conventions.

    QR sweep: factored bond product R X_k (K = r_b) then the MPO core
    (K = r_a d_in); Householder QR of the (rho d) x r_C unfolding.
    SVD sweep: Q_k applied to [U Sigma; 0], nominal SVD of the
    rho x (d r'') unfolding, U Sigma = F V product.
    """
    n = len(d)
    rc = [x * y for x, y in zip(ra, rb)]
    rho = [1] * (n + 1)
    f = 0.0
    for k in range(n):
        m_rows = rho[k] * d[k]
        cols = rc[k + 1]
        # bond product
        f += 2.0 * (rho[k] * ra[k]) * (dj[k] * rb[k + 1]) * rb[k]
        f += 2.0 * (rho[k] * d[k]) * (ra[k + 1] * rb[k + 1]) * (ra[k] * dj[k]) if mpo else \
            2.0 * rho[k] * d[k] * ra[k + 1] * rb[k + 1] * ra[k]
        if k < n - 1:
            f += geqrf_flops(m_rows, cols)
            rho[k + 1] = min(m_rows, cols)
    rnext = 1
    for k in range(n - 1, 0, -1):
        rows = rho[k]
        D = d[k] * rnext
        if k < n - 1:
            f += ormqr_flops(rho[k] * d[k], rho[k + 1], rnext)
        f += svd_nominal_flops(rows, D)
        r = ranks_out[k]
        f += 2.0 * min(rows, D) * r * D
        rnext = r
    f += ormqr_flops(d[0], rho[1], rnext)
    return f


def round_flops(ranks, d, ranks_out):
    """Algorithmic FLOP of qtt_round on a train with bond ranks `ranks`
    (same conventions): QR sweep (R C_k product, Householder QR of the
    (rho d) x r unfolding), then the SVD sweep of contract_round_flops."""
    n = len(d)
    rho = [1] * (n + 1)
    f = 0.0
    for k in range(n - 1):
        if k > 0:
            f += 2.0 * rho[k] * ranks[k] * d[k] * ranks[k + 1]
        f += geqrf_flops(rho[k] * d[k], ranks[k + 1])
        rho[k + 1] = min(rho[k] * d[k], ranks[k + 1])
    f += 2.0 * rho[n - 1] * ranks[n - 1] * d[n - 1]
    rnext = 1
    for k in range(n - 1, 0, -1):
        rows = rho[k]
        D = d[k] * rnext
        if k < n - 1:
            f += ormqr_flops(rho[k] * d[k], rho[k + 1], rnext)
        f += svd_nominal_flops(rows, D)
        r = ranks_out[k]
        f += 2.0 * min(rows, D) * r * D
        rnext = r
    f += ormqr_flops(d[0], rho[1], rnext)
    return f


def zipup_flops(ra, rb, d, dj, ranks_out, ncores, mpo=True):
    """Algorithmic FLOP of the decomposition (zip-up) path under the same
    conventions: right-to-left QR sweeps of both operands (Householder QR of
    the transposed unfoldings, explicit Q, R^T into the left neighbour), the
    factored bond products S C_k, and per split of an m x c super-core the
    nominal SVD of m x c, U Sigma = F V and the Q application."""
    n = len(d)
    Pa = [d[k] * dj[k] for k in range(n)] if mpo else list(d)
    Pb = list(dj) if mpo else list(d)
    f = 0.0

    def right(r, P):
        nonlocal f
        rho = [1] * (n + 1)
        for k in range(n - 1, 0, -1):
            m, c = P[k] * rho[k + 1], r[k]
            q = min(m, c)
            rho[k] = q
            f += geqrf_flops(m, c) + ormqr_flops(m, q, q) + 2.0 * r[k - 1] * P[k - 1] * q * c
        return rho

    sa, sb = right(ra, Pa), right(rb, Pb)
    N = min(ncores, n)
    r, Pleg, legs, outc = 1, 1, 0, 0
    for k in range(n):
        rho0 = r * Pleg
        f += 2.0 * (rho0 * sa[k]) * (dj[k] * sb[k + 1]) * sb[k]
        f += 2.0 * (rho0 * d[k]) * (sa[k + 1] * sb[k + 1]) * (sa[k] * (dj[k] if mpo else 1))
        Pleg *= d[k]
        rcs = sa[k + 1] * sb[k + 1]
        legs += 1
        while (legs == N and k < n - 1) or (k == n - 1 and legs > 1):
            db = d[outc]
            m, c = r * db, (Pleg // db) * rcs
            rn = ranks_out[outc + 1]
            p = min(m, c)
            f += svd_nominal_flops(m, c) + 2.0 * p * rn * m
            if c >= m:
                f += ormqr_flops(c, p, rn)
            outc += 1
            r, Pleg, legs = rn, Pleg // db, legs - 1
    return f


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--prec", default="bf16x6", choices=["fp64", "fp32", "bf16x3", "bf16x6"])
    ap.add_argument("--no-fp64-leg", action="store_true")
    ap.add_argument("--no-cpu-baseline", action="store_true",
                    help="skip the oracle (its timing and the error of the timed result against it)")
    ap.add_argument("--no-amplification", action="store_true",
                    help="skip the oracle's noise-amplification estimate of the rounding")
    ap.add_argument("--no-kernel-breakdown", action="store_true",
                    help="skip the per-class profiled steps (and the roofline object)")
    ap.add_argument("--calib-copy-mb", type=int, default=0,
                    help="after the measurement, run one plain device copy of this many MiB")
    ap.add_argument("--workload", default="laplacian3d_n42_r256",
                    choices=["laplacian3d_n42_r256", "laplacian3d_n42_r256_zipup", "hadamard_batch",
                             "sum4_n42_r128_round", "laplacian2d_n32_r64_zipup_fit", "heat2d_n24_solve",
                             "heat2d_n24_amen"],
                    help="hadamard_batch: the batched form (512 uneven 1D Hadamard products, one graph launch); "
                         "laplacian3d_n42_r256_zipup: the same product by the decomposition (zip-up) algorithm")
    ap.add_argument("--ncores", type=int, default=2, choices=[1, 2],
                    help="zip-up super-core size (exact product cores per split)")
    ap.add_argument("--traffic-record", nargs=2, metavar=("FETCH_CSV", "WRITE_CSV"),
                    help="write profiles/traffic_k_jacobi.json from the counter CSVs of two rocprofv3 --pmc passes "
                         "(FETCH_SIZE, WRITE_SIZE) over this workload's step run with --calib-copy-mb; no GPU work")
    ap.add_argument("--traffic-command", action="append", default=[],
                    help="with --traffic-record: the profiling commands, stored in the record")
    args = ap.parse_args()
    if args.traffic_record:
        return traffic_record("k_jacobi", args.workload, args.traffic_record[0], args.traffic_record[1],
                              args.calib_copy_mb, args.traffic_command)
    if args.gpus != 1:
        print(f"bench.py measures one GPU only (got --gpus {args.gpus}); the single-chain rounding "
              f"sweep carries a core-to-core dependency and is not sharded across GPUs", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    import qtt_inputs as I
    from paper_2602_20226_amd import qtt as Q

    Q.load_library()
    dev = "cuda:0"
    if args.workload == "hadamard_batch":
        return bench_batch(args, I, Q, torch, dev)
    if args.workload == "sum4_n42_r128_round":
        return bench_sum(args, I, Q, torch, dev)
    if args.workload == "laplacian2d_n32_r64_zipup_fit":
        return bench_fit(args, I, Q, torch, dev)
    if args.workload == "heat2d_n24_solve":
        return bench_solve(args, I, Q, torch, dev)
    if args.workload == "heat2d_n24_amen":
        return bench_amen(args, I, Q, torch, dev)
    zipup = args.workload.endswith("_zipup")
    w = I.laplacian3d_r256()
    A = Q.to_device(w.a, dev)
    B = Q.to_device(w.b, dev)
    ra = [1] + [c.shape[-1] for c in w.a]
    rb = [1] + [c.shape[-1] for c in w.b]
    d = [c.shape[1] for c in w.a]
    dj = [c.shape[2] for c in w.a]
    L = Q.load_library()
    import ctypes as C
    va, vb = Q.TTView(A, 2), Q.TTView(B, 1)
    if zipup:
        bnd, nbytes = Q.zipup_query(w.spec, va.struct, vb.struct, w.max_rank, args.ncores)
    else:
        bnd = Q.rank_bounds([x * y for x, y in zip(ra, rb)], d, w.max_rank)
        nb = C.c_size_t()
        Q._check(L.qtt_workspace_size(None, Q.OP_CONTRACT_ROUND, w.spec.encode(), C.byref(va.struct),
                                      C.byref(vb.struct), w.max_rank, Q.PREC[args.prec], C.byref(nb)), "ws")
        nbytes = nb.value
    # output cores and workspace allocated once, outside the timed region
    outs = [torch.empty(bnd[k] * d[k] * bnd[k + 1], dtype=torch.float64, device=dev) for k in range(len(d))]
    ws = torch.empty(nbytes, dtype=torch.uint8, device=dev)

    def step(prec):
        if zipup:
            return Q.contract_zipup(w.spec, A, B, w.rel_tol, w.max_rank, ncores=args.ncores, prec=prec,
                                    out_buffers=outs, workspace=ws)
        return Q.contract_round(w.spec, A, B, w.rel_tol, w.max_rank, prec=prec, out_buffers=outs, workspace=ws)

    def timed(prec, steps, warmup):
        res = None
        for _ in range(warmup):
            res = step(prec)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(steps):
            res = step(prec)
        torch.cuda.synchronize()
        return (time.perf_counter() - t0) / steps, res

    sec, res = timed(args.prec, args.steps, args.warmup)
    # host copies of the timed results (the output buffers are reused below)
    got = (Q.to_host(res.cores), list(res.ranks))
    if zipup:
        flops = zipup_flops(ra, rb, d, dj, res.ranks, args.ncores)
        metric = ("QTT contract+truncate by zip-up TFLOP/s (3D Laplacian MPO x rank-256 MPS, n=42, "
                  "truncated to rank 256 at 1e-8)")
    else:
        flops = contract_round_flops(ra, rb, d, dj, res.ranks)
        metric = "QTT contract+round TFLOP/s (3D Laplacian MPO x rank-256 MPS, n=42, round to rank 256 at 1e-8)"
    out = {
        "metric": metric,
        "value": flops / sec / 1e12,
        "unit": "TFLOP/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": sec * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": f"{args.prec}+f64",
        "data": "synthetic",
        "config": {"workload": args.workload, "cores": len(d), "mps_rank": 256, "mpo_rank": 7, "max_rank": w.max_rank,
                   "rel_tol": w.rel_tol, "gemm": args.prec, "factorisations": "fp64"},
        "algorithmic_gflop_per_step": flops / 1e9,
        "ranks_out_max": max(res.ranks),
        "jacobi_sweeps_max": res.jacobi_sweeps_max,
    }
    got64 = None
    if not args.no_fp64_leg and args.prec != "fp64":
        sec64, res64 = timed("fp64", max(1, args.steps // 2), 1)
        got64 = (Q.to_host(res64.cores), list(res64.ranks))
        out["fp64_ms_per_step"] = sec64 * 1e3
        out["speedup_vs_fp64_path"] = sec64 / sec

    # Per-class kernel time: one extra step per class with every launch of
    # that class bracketed by HIP events on its launch stream inside libqtt.
    # The roofline is reported for the class that takes the most time.
    kernels = {} if args.no_kernel_breakdown else kernel_breakdown(Q, lambda: step(args.prec))
    if kernels:
        add_roofline(out, kernels, sec)
    if args.calib_copy_mb > 0:
        # one plain elementwise pass of known size (read n doubles, write n
        # doubles), for scaling the hardware byte counters taken on this run
        n = int(args.calib_copy_mb) * (1 << 20) // 8
        src_t = torch.empty(n, dtype=torch.float64, device=dev).uniform_()
        dst_t = torch.mul(src_t, 1.5)
        torch.cuda.synchronize()
        del src_t, dst_t

    if not args.no_cpu_baseline:
        base, ref, ref_info, C_exact = cpu_baseline(w, ra, rb, d, dj, args.ncores if zipup else 0)
        out["cpu_baseline"] = base
        # the timed results against the oracle's result of the same workload
        import oracle as O
        out["rel_err_vs_oracle"] = O.rel_error(got[0], ref)
        out["ranks_identical"] = got[1] == ref_info.ranks
        if got64 is not None:
            out["fp64_rel_err_vs_oracle"] = O.rel_error(got64[0], ref)
            out["fp64_ranks_identical"] = got64[1] == ref_info.ranks
        gaps = [g for g in ref_info.gaps if math.isfinite(g)]
        out["oracle_min_cut_gap"] = min(gaps) if gaps else None
        if C_exact is not None and not args.no_amplification:
            # how much the rounding magnifies a relative input change of 1e-7
            # (the size of the reduced-precision GEMM error): one perturbed
            # oracle rounding of the exact product
            amp, _ = O.noise_amplification(C_exact, w.rel_tol, w.max_rank, eps=1e-7, seed=5, trials=1)
            out["oracle_amplification"] = amp
    print(json.dumps(out), flush=True)


def bench_batch(args, I, Q, torch, dev):
    """The batched form: 512 independent 1D Hadamard products (L = 24, ranks
    U{8..128} times rank 2), each contracted and rounded at 1e-8, in one
    persistent launch replayed from a hipGraph.  A step is one replay; the
    launch is the only kernel, so it is also the roofline kernel."""
    w = I.hadamard_batch()
    A = [Q.to_device(a, dev) for a in w.a]
    B = [Q.to_device(b, dev) for b in w.b]
    plan = Q.BatchPlan(w.spec, A, B, w.rel_tol, w.max_rank, tune=True)
    for _ in range(args.warmup):
        plan.launch()
    torch.cuda.synchronize()
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(2 * args.steps)]
    t0 = time.perf_counter()
    for i in range(args.steps):
        ev[2 * i].record()
        plan.launch()
        ev[2 * i + 1].record()
    torch.cuda.synchronize()
    sec = (time.perf_counter() - t0) / args.steps
    launch_ms = sum(ev[2 * i].elapsed_time(ev[2 * i + 1]) for i in range(args.steps)) / args.steps
    ranks, _ = plan.results()
    flops = []
    for i in range(len(w.a)):
        ra = [1] + [c.shape[-1] for c in w.a[i]]
        rb = [1] + [c.shape[-1] for c in w.b[i]]
        d = [c.shape[1] for c in w.a[i]]
        flops.append(contract_round_flops(ra, rb, d, d, ranks[i], mpo=False))
    total = sum(flops)
    achieved = total / (launch_ms * 1e-3) / 1e12
    out = {
        "metric": "QTT batched contract+round TFLOP/s (512 uneven 1D Hadamard products, L=24, one graph launch)",
        "value": total / sec / 1e12, "unit": "TFLOP/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": sec * 1e3, "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "bf16x6+f64", "data": "synthetic",
        "config": {"workload": w.name, "problems": len(w.a), "cores": 24, "rank_a": "U{8..128}", "rank_b": 2,
                   "rel_tol": w.rel_tol, "gemm": "bf16x6 split, FP32 accumulation per 32-deep step",
                   "factorisations": "fp64"},
        "algorithmic_gflop_per_step": total / 1e9,
        "plan": plan.info(),
        "roofline": {"bound": "alu", "achieved": achieved, "peak": 78.6, "unit": "TFLOP/s", "frac": achieved / 78.6,
                     "traffic": None, "kernel": "k_batched", "launches": 1, "avg_us": launch_ms * 1e3,
                     "share_of_step": launch_ms / (sec * 1e3), "alg_flop_per_launch": total},
    }
    if not args.no_cpu_baseline:
        import oracle as O
        try:
            from threadpoolctl import threadpool_info
            threads = max([i.get("num_threads", 1) for i in threadpool_info()] or [os.cpu_count() or 1])
        except Exception:
            threads = os.cpu_count() or 1
        sample = list(range(0, len(w.a), 8))
        refs = {}
        t0 = time.perf_counter()
        for i in sample:
            refs[i] = O.round_tt(O.contract(w.spec, w.a[i], w.b[i]), w.rel_tol, w.max_rank, return_info=True)
        dt = time.perf_counter() - t0
        # the timed result against the oracle on the same problems
        out["rel_err_vs_oracle"] = max(O.rel_error(Q.to_host(plan.cores(i)), refs[i][0]) for i in sample)
        out["ranks_identical"] = all(ranks[i] == refs[i][1].ranks for i in sample)
        out["oracle_checked_problems"] = len(sample)
        out["cpu_baseline"] = {"value": sum(flops[i] for i in sample) / dt / 1e12, "unit": "TFLOP/s",
                               "cores": threads, "kind": "oracle",
                               "sample": f"every 8th problem ({len(sample)} of {len(w.a)}), NumPy FP64 + LAPACK",
                               "seconds": dt}
    print(json.dumps(out), flush=True)


KERNEL_CLASSES = {
    # class: (bound, peak, unit, kernels, source file of the kernel)
    "jacobi": ("alu", 78600.0, "GFLOP/s", "k_jacobi", "svd.hip"),
    "qr_panel": ("alu", 78600.0, "GFLOP/s", "k_qr_panel", "qr.hip"),
    "apply_panel": ("hbm", 8000.0, "GB/s", "k_apply1", "qr.hip"),
    "block_vty": ("mfma", 78600.0, "GFLOP/s", "k_vty", "qr.hip"),
    "block_upd": ("mfma", 78600.0, "GFLOP/s", "k_vupd", "qr.hip"),
    "chol_block": ("alu", 78600.0, "GFLOP/s", "k_potrf_inv", "solve.hip"),
    "chol_update": ("mfma", 78600.0, "GFLOP/s", "k_syrk_k64", "gemm.hip"),
    "chol_solve": ("hbm", 8000.0, "GB/s", "k_chol_bwd", "solve.hip"),
}
ROUNDING_CLASSES = ("jacobi", "qr_panel", "apply_panel", "block_vty", "block_upd")


def kernel_breakdown(Q, step, classes=ROUNDING_CLASSES):
    """One extra step per kernel class, every launch of the class bracketed by
    HIP events on its launch stream inside libqtt."""
    kernels = {}
    for cls in classes:
        bound, peak, unit, kname, src = KERNEL_CLASSES[cls]
        Q.profile_start(cls, 20000)
        step()
        launches, kms, kbytes, kflops = Q.profile_stop()
        work = kbytes if bound == "hbm" else kflops
        achieved = work / (kms * 1e-3) / 1e9 if kms > 0 else 0.0
        kernels[cls] = {
            "kernel": kname, "bound": bound, "launches": launches, "ms_per_step": kms,
            "avg_us": 1e3 * kms / max(launches, 1), "achieved": achieved, "peak": peak, "unit": unit,
            "frac": achieved / peak, "alg_bytes_per_launch": kbytes / max(launches, 1),
            "alg_flop_per_launch": kflops / max(launches, 1), "source": src,
        }
    return kernels


def bench_sum(args, I, Q, torch, dev):
    """Exact sum of four rank-128 trains (42 cores) followed by rounding to rank
    256 at 1e-8: one qtt_add into preallocated cores of the summed ranks, then
    qtt_round in place on them (workspace preallocated)."""
    import ctypes as C
    w = I.sum4_n42_r128()
    coeffs = w.extra["coeffs"]
    nt = len(w.a)
    terms = [Q.to_device(t, dev) for t in w.a]
    n = len(w.a[0])
    d = [c.shape[1] for c in w.a[0]]
    rsum = [1] + [sum(t[k].shape[0] for t in w.a) for k in range(1, n)] + [1]
    bufs = [torch.empty(rsum[k] * d[k] * rsum[k + 1], dtype=torch.float64, device=dev) for k in range(n)]
    L = Q.load_library()
    h = Q.handle(0)
    views = [Q.TTView(t, 1) for t in terms]
    arr = (Q.TT * nt)(*[v.struct for v in views])
    cf = (C.c_double * nt)(*coeffs)
    vo = Q.TTView(bufs, 1, ranks_override=rsum, phys_override=d)
    nb = C.c_size_t()
    Q._check(L.qtt_workspace_size(None, Q.OP_ROUND, None, C.byref(vo.struct), None, w.max_rank, 0, C.byref(nb)),
             "qtt_workspace_size")
    ws = torch.empty(nb.value, dtype=torch.uint8, device=dev)
    info = Q._Info(n)

    def step():
        for k in range(n + 1):  # qtt_round rewrote the host ranks of the previous step
            vo._ranks[k] = rsum[k]
        Q._check(L.qtt_add(h.ptr, nt, arr, cf, C.byref(vo.struct), Q._stream_ptr()), "qtt_add")
        Q._check(L.qtt_round(h.ptr, C.byref(vo.struct), float(w.rel_tol), int(w.max_rank), 0, C.byref(info.c),
                             C.c_void_p(ws.data_ptr()), ws.numel(), Q._stream_ptr()), "qtt_round")
        return vo.ranks()

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        ranks_out = step()
    torch.cuda.synchronize()
    sec = (time.perf_counter() - t0) / args.steps
    flops = round_flops(rsum, d, ranks_out)
    out = {
        "metric": "QTT add+round TFLOP/s (sum of four rank-128 MPS, n=42, rounded to rank 256 at 1e-8)",
        "value": flops / sec / 1e12, "unit": "TFLOP/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": sec * 1e3, "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f64", "data": "synthetic",
        "config": {"workload": args.workload, "cores": n, "terms": nt, "term_rank": 128, "sum_rank": max(rsum),
                   "max_rank": w.max_rank, "rel_tol": w.rel_tol},
        "algorithmic_gflop_per_step": flops / 1e9,
        "ranks_out_max": max(ranks_out),
        "jacobi_sweeps_max": info.c.jacobi_sweeps_max,
    }
    if not args.no_kernel_breakdown:
        add_roofline(out, kernel_breakdown(Q, step), sec)
    if not args.no_cpu_baseline:
        import oracle as O
        try:
            from threadpoolctl import threadpool_info
            threads = max([i.get("num_threads", 1) for i in threadpool_info()] or [os.cpu_count() or 1])
        except Exception:
            threads = os.cpu_count() or 1
        reps = 0
        t0 = time.perf_counter()
        while reps == 0 or time.perf_counter() - t0 < 10.0:  # ~10 s of CPU work
            Y, oinfo = O.round_tt(O.tt_sum(w.a, coeffs), w.rel_tol, w.max_rank, return_info=True)
            reps += 1
        dt = time.perf_counter() - t0
        out["cpu_baseline"] = {"value": reps * round_flops(rsum, d, oinfo.ranks) / dt / 1e12, "unit": "TFLOP/s",
                               "cores": threads, "kind": "oracle",
                               "sample": f"{reps} full sum + rounding runs of the same workload (NumPy FP64, "
                                         f"LAPACK QR/SVD)", "seconds": dt}
    print(json.dumps(out), flush=True)


def fit_flops(ry, rc, d, dj, nsweeps, mpo=True):
    """Algorithmic FLOP of qtt_fit (same conventions): the exactly contracted
    product, the initial left environments, and per sweep and core one
    projection L Y_q R^T, one QR with explicit Q and one environment step,
    twice (down and up); rc are the ranks of the fitted train."""
    n = len(d)
    f = 0.0
    for k in range(n):
        f += 2.0 * (dj[k] if mpo else 1) * ry[k] * d[k] * ry[k + 1]
    env = lambda k: 2.0 * rc[k] * ry[k] * d[k] * ry[k + 1] + 2.0 * rc[k + 1] * rc[k] * d[k] * ry[k + 1]
    f += sum(env(k) for k in range(n - 1))
    for _ in range(nsweeps):
        for k in range(n):
            proj = 2.0 * rc[k] * ry[k] * d[k] * ry[k + 1] + 2.0 * rc[k] * d[k] * rc[k + 1] * ry[k + 1]
            m, c = rc[k] * d[k], rc[k + 1]
            q = min(m, c)
            f += 2.0 * (proj + env(k)) + 2.0 * (geqrf_flops(m, c) + ormqr_flops(m, q, q))
    return f


def bench_fit(args, I, Q, torch, dev):
    """The pipeline the paper recommends for a product: the decomposition
    (zip-up, super-cores of one core) result truncated to rank 64 as the
    guess, then one variational sweep (Sec. 3.3), on the 2D Laplacian x
    rank-64 MPS workload (n = 32).  A step is zip-up + fit."""
    import ctypes as C
    w = I.laplacian2d_r64()
    A = Q.to_device(w.a, dev)
    B = Q.to_device(w.b, dev)
    nsweeps = 1
    va, vb = Q.TTView(A, 2), Q.TTView(B, 1)
    bnd, nbytes = Q.zipup_query(w.spec, va.struct, vb.struct, w.max_rank, 1)
    d = [c.shape[1] for c in w.a]
    dj = [c.shape[2] for c in w.a]
    outs = [torch.empty(bnd[k] * d[k] * bnd[k + 1], dtype=torch.float64, device=dev) for k in range(len(d))]
    ws = torch.empty(nbytes, dtype=torch.uint8, device=dev)
    z = Q.contract_zipup(w.spec, A, B, w.rel_tol, w.max_rank, ncores=1, out_buffers=outs, workspace=ws)
    L = Q.load_library()
    vc = Q.TTView([o.reshape(-1) for o in outs], 1, ranks_override=z.ranks, phys_override=d)
    nb = C.c_size_t()
    Q._check(L.qtt_fit_workspace_size(w.spec.encode(), C.byref(va.struct), C.byref(vb.struct), C.byref(vc.struct),
                                      C.byref(nb)), "qtt_fit_workspace_size")
    fws = torch.empty(nb.value, dtype=torch.uint8, device=dev)
    h = Q.handle(0)
    nrm = C.c_double()

    def step():
        r = Q.contract_zipup(w.spec, A, B, w.rel_tol, w.max_rank, ncores=1, out_buffers=outs, workspace=ws)
        for k, x in enumerate(r.ranks):
            vc._ranks[k] = x
        Q._check(L.qtt_fit(h.ptr, w.spec.encode(), C.byref(va.struct), C.byref(vb.struct), C.byref(vc.struct),
                           nsweeps, C.byref(nrm), C.c_void_p(fws.data_ptr()), fws.numel(), Q._stream_ptr()),
                 "qtt_fit")
        return r.ranks, vc.ranks()

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        zr, fr = step()
    torch.cuda.synchronize()
    sec = (time.perf_counter() - t0) / args.steps
    ra = [1] + [c.shape[-1] for c in w.a]
    rb = [1] + [c.shape[-1] for c in w.b]
    ry = [x * y for x, y in zip(ra, rb)]
    flops = zipup_flops(ra, rb, d, dj, zr, 1) + fit_flops(ry, zr, d, dj, nsweeps)
    out = {
        "metric": "QTT zip-up + variational sweep TFLOP/s (2D Laplacian MPO x rank-64 MPS, n=32, rank 64)",
        "value": flops / sec / 1e12, "unit": "TFLOP/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": sec * 1e3, "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f64", "data": "synthetic",
        "config": {"workload": args.workload, "cores": len(d), "mps_rank": 64, "mpo_rank": 5, "max_rank": w.max_rank,
                   "rel_tol": w.rel_tol, "zipup_ncores": 1, "fit_sweeps": nsweeps},
        "algorithmic_gflop_per_step": flops / 1e9,
        "ranks_out_max": max(fr),
    }
    if not args.no_kernel_breakdown:
        add_roofline(out, kernel_breakdown(Q, step), sec)
    if not args.no_cpu_baseline:
        import oracle as O
        try:
            from threadpoolctl import threadpool_info
            threads = max([i.get("num_threads", 1) for i in threadpool_info()] or [os.cpu_count() or 1])
        except Exception:
            threads = os.cpu_count() or 1
        reps = 0
        t0 = time.perf_counter()
        while reps == 0 or time.perf_counter() - t0 < 10.0:  # ~10 s of CPU work
            Z, zinfo = O.zipup(w.spec, w.a, w.b, w.rel_tol, w.max_rank, ncores=1, return_info=True)
            O.fit(w.spec, w.a, w.b, Z, nsweeps=nsweeps)
            reps += 1
        dt = time.perf_counter() - t0
        of = zipup_flops(ra, rb, d, dj, zinfo.ranks, 1) + fit_flops(ry, zinfo.ranks, d, dj, nsweeps)
        out["cpu_baseline"] = {"value": reps * of / dt / 1e12, "unit": "TFLOP/s", "cores": threads, "kind": "oracle",
                               "sample": f"{reps} full zip-up + variational sweep runs of the same workload "
                                         f"(NumPy FP64)", "seconds": dt}
    print(json.dumps(out), flush=True)


def solve_flops(ranks, d, rw, rb, nsweeps):
    """Algorithmic FLOP of the one-core linear solver (same conventions):
    per local solve of N = r0 d r1 unknowns the local matrix (N^2 rw0 rw1
    products of 2 FLOP), its Cholesky factorisation (N^3 / 3) and the two
    triangular solves (2 N^2), the right-hand side
    (2 r0 rb0 d rb1 + 2 r0 d rb1 r1), the QR that moves the centre (geqrf of
    the core's unfolding) and the environment steps (three-layer:
    2 r0 rw0 r0 d r1 + 2 r0 d rw1 r1 rw0 d + 2 r1 r0 d rw1 r1; two-layer:
    2 r0 rb0 d rb1 + 2 r1 r0 d rb1); two local solves per core per sweep."""
    n = len(d)
    f = 0.0
    for k in range(n):
        r0, r1, w0, w1, b0, b1, dk = ranks[k], ranks[k + 1], rw[k], rw[k + 1], rb[k], rb[k + 1], d[k]
        N = r0 * dk * r1
        local = 2.0 * N * N * w0 * w1 + N ** 3 / 3.0 + 2.0 * N * N
        local += 2.0 * r0 * b0 * dk * b1 + 2.0 * r0 * dk * b1 * r1
        move = geqrf_flops(r0 * dk, r1)
        env = 2.0 * r0 * w0 * r0 * dk * r1 + 2.0 * r0 * dk * w1 * r1 * w0 * dk + 2.0 * r1 * r0 * dk * w1 * r1
        env += 2.0 * r0 * b0 * dk * b1 + 2.0 * r1 * r0 * dk * b1
        f += 2.0 * (local + move + env)
    return f * nsweeps


def bench_solve(args, I, Q, torch, dev):
    """The DMRG-like linear solver (Sec. 5) on an implicit heat step of the 2D
    2^12 x 2^12 grid (24 cores): (L + s I) x = b with L the Dirichlet
    Laplacian MPO (rank 5), s = 1, b the rank-16 right-hand side of the 2D
    gradient workload (seed 4) and its rank-32 x as the guess; one-core
    sweeps (ranks 32), two sweeps per step.  A step is one qtt_solve call."""
    import ctypes as C
    w = I.residual_grad_2d()
    m, D, s, nsweeps = 12, 2, 1.0, 2
    Wc = I.laplacian_mpo(m, D, diag=2.0 + s / D)
    A = Q.to_device(Wc, dev)
    rhs, guess = w.extra["rhs"], w.b  # the workload's b (rank 16) and x (rank 32)
    b = Q.to_device(rhs, dev)
    g = Q.to_device(guess, dev)
    n = len(g)
    d = [c.shape[1] for c in g]
    L = Q.load_library()
    h = Q.handle(0)
    vw, vb = Q.TTView(A, 2), Q.TTView(b, 1)
    r_in = [g[0].shape[0]] + [c.shape[-1] for c in g]
    vg = Q.TTView([c.reshape(-1) for c in g], 1, ranks_override=r_in, phys_override=d)
    bnd = (C.c_int64 * (n + 1))()
    nb = C.c_size_t()
    Q._check(L.qtt_solve_query(C.byref(vw.struct), C.byref(vb.struct), C.byref(vg.struct), 1, 0, bnd, C.byref(nb)),
             "qtt_solve_query")
    bufs = [torch.zeros(int(bnd[k]) * d[k] * int(bnd[k + 1]), dtype=torch.float64, device=dev) for k in range(n)]
    ws = torch.empty(nb.value, dtype=torch.uint8, device=dev)
    vx = Q.TTView(bufs, 1, ranks_override=r_in, phys_override=d)
    info = Q._Info(n)

    def step():
        for k in range(n):  # restart from the guess
            bufs[k][: g[k].numel()] = g[k].reshape(-1)
        for k in range(n + 1):
            vx._ranks[k] = r_in[k]
        Q._check(L.qtt_solve(h.ptr, C.byref(vw.struct), C.byref(vb.struct), C.byref(vx.struct), nsweeps, 1, 0.0, 0,
                             C.byref(info.c), C.c_void_p(ws.data_ptr()), ws.numel(), Q._stream_ptr()), "qtt_solve")
        return vx.ranks()

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        ranks = step()
    torch.cuda.synchronize()
    sec = (time.perf_counter() - t0) / args.steps
    rw = [1] + [c.shape[-1] for c in Wc]
    rbr = [1] + [c.shape[-1] for c in rhs]
    flops = solve_flops(ranks, d, rw, rbr, nsweeps)
    out = {
        "metric": "QTT DMRG-like linear solve TFLOP/s (implicit heat step, 2D 2^12 x 2^12 grid, rank 32, 2 sweeps)",
        "value": flops / sec / 1e12, "unit": "TFLOP/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": sec * 1e3, "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f64", "data": "synthetic",
        "config": {"workload": args.workload, "cores": n, "operator": "Laplacian + I (MPO rank 5)", "rhs_rank": max(rbr),
                   "x_rank": max(ranks), "sweeps": nsweeps, "local_solver": "blocked Cholesky + two triangular solves"},
        "algorithmic_gflop_per_step": flops / 1e9,
    }
    if not args.no_kernel_breakdown:
        add_roofline(out, kernel_breakdown(Q, step, tuple(KERNEL_CLASSES)), sec)
    if not args.no_cpu_baseline:
        import oracle as O
        threads = _blas_threads()
        # bounded sample: one sweep of the same solve (the timed step runs two), on the host and on
        # the GPU from the same guess, for the baseline and for the error of the GPU result
        t0 = time.perf_counter()
        ref = O.solve_energy(Wc, rhs, guess, nsweeps=1, ncores=1)
        dt = time.perf_counter() - t0
        cores, r1, _ = Q.solve(A, b, g, nsweeps=1, ncores=1)
        out["rel_err_vs_oracle"] = O.rel_error(Q.to_host(cores), ref)
        out["ranks_identical"] = O.ranks_of(ref) == r1
        out["cpu_baseline"] = {"value": solve_flops(r1, d, rw, rbr, 1) / dt / 1e12, "unit": "TFLOP/s",
                               "cores": threads, "kind": "oracle",
                               "sample": "one sweep of the same solve from the same guess (NumPy FP64, dense local "
                                         "solves); the GPU result of that sweep gives rel_err_vs_oracle",
                               "seconds": dt}
    print(json.dumps(out), flush=True)


def amen_flops(ranks, zranks, d, rw, rb):
    """Algorithmic FLOP of one AMEn sweep (two passes) at fixed ranks of x
    and z: per core and pass the local solve of solve_flops (Cholesky), the nominal
    SVD of the solved core's unfolding and the product U S V^T, two residual
    projections (right-hand side part 2 a rb0 d rb1 + 2 a d rb1 c; operator
    part 2 r0 d c rw1 r1 + 2 d c rw0 r0 d rw1 + 2 a d c rw0 r0, with a x c
    the frame ranks: z x z and z x x), the nominal SVDs of the enriched
    basis ((r + rz) x d r) and of z's projection, and the environment steps
    of x and of z against x and b."""
    n = len(d)
    f = 0.0
    for k in range(n):
        r0, r1, z0, z1, w0, w1, b0, b1, dk = (ranks[k], ranks[k + 1], zranks[k], zranks[k + 1], rw[k], rw[k + 1],
                                              rb[k], rb[k + 1], d[k])
        N = r0 * dk * r1
        local = 2.0 * N * N * w0 * w1 + N ** 3 / 3.0 + 2.0 * N * N
        local += 2.0 * r0 * b0 * dk * b1 + 2.0 * r0 * dk * b1 * r1
        trunc = svd_nominal_flops(r0, dk * r1) + 2.0 * N * min(r0, dk * r1)

        def proj(a, c):
            return (2.0 * a * b0 * dk * b1 + 2.0 * a * dk * b1 * c + 2.0 * r0 * dk * c * w1 * r1
                    + 2.0 * dk * c * w0 * r0 * dk * w1 + 2.0 * a * dk * c * w0 * r0)

        projs = proj(z0, z1) + proj(z0, r1)
        bases = svd_nominal_flops(min(r0, dk * r1) + z0, dk * r1) + svd_nominal_flops(z0, dk * z1)

        def env3(a):
            return 2.0 * a * w0 * r0 * dk * r1 + 2.0 * a * dk * w1 * r1 * w0 * dk + 2.0 * r1 * a * dk * w1 * r1

        env = env3(r0) + env3(z0) + 2.0 * (r0 + z0) * b0 * dk * b1 + 2.0 * (r1 + z1) * (r0 + z0) * dk * b1
        f += 2.0 * (local + trunc + projs + bases + env)
    return f


def bench_amen(args, I, Q, torch, dev):
    """The AMEn linear solver (Sec. 5) on the implicit heat step of
    bench_solve ((L + s I) x = b on the 2D 2^12 x 2^12 grid, 24 cores, b of
    rank 16): from a random rank-4 guess and a rank-4 residual train (seed
    31), ranks capped at 24 (plus the enrichment), rel_tol 1e-8, two sweeps
    per step.  A step is one qtt_solve_amen call."""
    import ctypes as C
    import numpy as np
    w = I.residual_grad_2d()
    m, D, s, nsweeps, cap, tol = 12, 2, 1.0, 2, 24, 1e-8
    Wc = I.laplacian_mpo(m, D, diag=2.0 + s / D)
    A = Q.to_device(Wc, dev)
    rhs = w.extra["rhs"]
    b = Q.to_device(rhs, dev)
    rng = np.random.default_rng(31)
    guess = I.random_mps(m * D, 4, rng)
    zguess = I.random_mps(m * D, 4, rng)
    g, zg = Q.to_device(guess, dev), Q.to_device(zguess, dev)
    n = len(g)
    d = [c.shape[1] for c in g]
    L = Q.load_library()
    h = Q.handle(0)
    vw, vb = Q.TTView(A, 2), Q.TTView(b, 1)
    rx_in = [1] + [c.shape[-1] for c in g]
    rz_in = [1] + [c.shape[-1] for c in zg]
    px = Q.TTView([c.reshape(-1) for c in g], 1, ranks_override=rx_in, phys_override=d)
    pz = Q.TTView([c.reshape(-1) for c in zg], 1, ranks_override=rz_in, phys_override=d)
    bx, bz = (C.c_int64 * (n + 1))(), (C.c_int64 * (n + 1))()
    nb = C.c_size_t()
    Q._check(L.qtt_solve_amen_query(C.byref(vw.struct), C.byref(vb.struct), C.byref(px.struct), C.byref(pz.struct),
                                    cap, bx, bz, C.byref(nb)), "qtt_solve_amen_query")
    xb = [torch.zeros(int(bx[k]) * d[k] * int(bx[k + 1]), dtype=torch.float64, device=dev) for k in range(n)]
    zb = [torch.zeros(int(bz[k]) * d[k] * int(bz[k + 1]), dtype=torch.float64, device=dev) for k in range(n)]
    ws = torch.empty(nb.value, dtype=torch.uint8, device=dev)
    vx = Q.TTView(xb, 1, ranks_override=rx_in, phys_override=d)
    vz = Q.TTView(zb, 1, ranks_override=rz_in, phys_override=d)
    info = Q._Info(n)

    def step(sweeps=nsweeps):
        for k in range(n):  # restart from the guesses
            xb[k][: g[k].numel()] = g[k].reshape(-1)
            zb[k][: zg[k].numel()] = zg[k].reshape(-1)
        for k in range(n + 1):
            vx._ranks[k] = rx_in[k]
            vz._ranks[k] = rz_in[k]
        Q._check(L.qtt_solve_amen(h.ptr, C.byref(vw.struct), C.byref(vb.struct), C.byref(vx.struct),
                                  C.byref(vz.struct), sweeps, tol, cap, C.byref(info.c), C.c_void_p(ws.data_ptr()),
                                  ws.numel(), Q._stream_ptr()), "qtt_solve_amen")
        return vx.ranks(), vz.ranks()

    # ranks at the start of each sweep (untimed): the orthogonalised guesses, then after one sweep
    start = [step(0), step(1)]
    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        ranks, zranks = step()
    torch.cuda.synchronize()
    sec = (time.perf_counter() - t0) / args.steps
    rw = [1] + [c.shape[-1] for c in Wc]
    rbr = [1] + [c.shape[-1] for c in rhs]
    flops = sum(amen_flops(rx, rz, d, rw, rbr) for rx, rz in start)
    out = {
        "metric": "QTT AMEn linear solve TFLOP/s (implicit heat step, 2D 2^12 x 2^12 grid, rank cap 24 + 4, 2 sweeps)",
        "value": flops / sec / 1e12, "unit": "TFLOP/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": sec * 1e3, "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f64", "data": "synthetic",
        "config": {"workload": args.workload, "cores": n, "operator": "Laplacian + I (MPO rank 5)", "rhs_rank": max(rbr),
                   "guess_rank": 4, "residual_rank": 4, "max_rank": cap, "rel_tol": tol, "x_rank": max(ranks),
                   "sweeps": nsweeps},
        "algorithmic_gflop_per_step": flops / 1e9,
        "flop_ranks": "each sweep counted at the ranks it starts from (the guess's, then those after one sweep)",
    }
    if not args.no_kernel_breakdown:
        add_roofline(out, kernel_breakdown(Q, step, tuple(KERNEL_CLASSES)), sec)
    if not args.no_cpu_baseline:
        import oracle as O
        threads = _blas_threads()
        # the whole solve (two sweeps, about 10 s on the host) from the same guesses; the timed
        # step's own result gives the error against it
        gpu_x = Q.to_host(Q._views_of_compact(xb, ranks, d))
        t0 = time.perf_counter()
        ref, rinfo = O.solve_amen(Wc, rhs, guess, zguess, nsweeps=nsweeps, rel_tol=tol, max_rank=cap,
                                  return_info=True)
        dt = time.perf_counter() - t0
        out["rel_err_vs_oracle"] = O.rel_error(gpu_x, ref)
        out["ranks_identical"] = rinfo["ranks"] == ranks
        out["cpu_baseline"] = {"value": flops / dt / 1e12, "unit": "TFLOP/s", "cores": threads, "kind": "oracle",
                               "sample": "the same solve (both sweeps) from the same guesses (NumPy FP64, dense "
                                         "local solves); the timed step's result gives rel_err_vs_oracle",
                               "seconds": dt}
    print(json.dumps(out), flush=True)


def add_roofline(out, kernels, sec):
    top = max(kernels, key=lambda c: kernels[c]["ms_per_step"])
    k = kernels[top]
    scale = 1e-3 if k["unit"] == "GFLOP/s" else 1.0  # report TFLOP/s or GB/s
    out["roofline"] = {
        "bound": k["bound"], "achieved": k["achieved"] * scale, "peak": k["peak"] * scale,
        "unit": "TFLOP/s" if k["unit"] == "GFLOP/s" else "GB/s", "frac": k["frac"],
        "traffic": measured_traffic(k["kernel"], out["config"]["workload"]),
        "kernel": k["kernel"], "launches": k["launches"], "avg_us": k["avg_us"],
        "share_of_step": k["ms_per_step"] / (sec * 1e3),
        "alg_bytes_per_launch": k["alg_bytes_per_launch"], "alg_flop_per_launch": k["alg_flop_per_launch"],
    }
    out["kernels"] = {c: {key: v[key] for key in ("kernel", "bound", "launches", "ms_per_step", "avg_us", "achieved",
                                                   "unit", "frac")} for c, v in kernels.items()}


TRAFFIC_SOURCES = {"k_jacobi": ["paper_2602_20226_amd/csrc/svd.hip", "paper_2602_20226_amd/csrc/qtt_device.hpp"]}


def _sources_sha(names):
    import hashlib
    h = hashlib.sha256()
    for name in names:
        with open(os.path.join(ROOT, name), "rb") as f:
            h.update(f.read())
    return h.hexdigest()


def measured_traffic(kernel, workload):
    """Measured HBM bytes per launch of `kernel` on `workload`: the committed
    hardware-counter record (FETCH_SIZE + WRITE_SIZE of every launch of the
    kernel in one bench.py step, each scaled by the counter's reading for a
    plain copy of known size, averaged over the launches); None unless the
    record was taken on this workload and on the current source of the kernel."""
    path = os.path.join(ROOT, "profiles", f"traffic_{kernel}.json")
    try:
        with open(path) as f:
            rec = json.load(f)
        sha = _sources_sha(rec.get("sources", []))
    except (OSError, ValueError):
        return None
    if rec.get("source_sha256") != sha or rec.get("workload") != workload:
        return None
    return rec.get("measured_bytes_per_launch")


def traffic_record(kernel, workload, fetch_csv, write_csv, copy_mib, commands, path=None):
    """Builds profiles/traffic_<kernel>.json from the counter CSVs of two
    rocprofv3 --pmc passes (FETCH_SIZE, WRITE_SIZE; KiB per dispatch) over
    one bench.py step of `workload` that ends with a plain copy of copy_mib
    MiB (--calib-copy-mb): the copy's readings give the scale factors."""
    import csv

    def read(path, counter):
        per = {}
        with open(path) as f:
            for row in csv.DictReader(f):
                if row.get("Counter_Name") != counter:
                    continue
                key = (int(row["Dispatch_Id"]), row["Kernel_Name"])
                per[key] = per.get(key, 0.0) + float(row["Counter_Value"])
        return per

    fetch, write = read(fetch_csv, "FETCH_SIZE"), read(write_csv, "WRITE_SIZE")
    expect_kib = copy_mib * 1024.0

    def split(per):
        kern = [v for (i, n), v in sorted(per.items()) if kernel in n]
        copy = [v for (i, n), v in sorted(per.items()) if kernel not in n and v > 0.25 * expect_kib]
        return kern, copy

    kf, cf = split(fetch)
    kw, cw = split(write)
    if not kf or len(kf) != len(kw) or not cf or not cw:
        raise SystemExit(f"counter files do not hold matching {kernel} launches and a copy of {copy_mib} MiB")
    ff, fw = expect_kib / cf[-1], expect_kib / cw[-1]
    fetch_b = sum(kf) / len(kf) * ff * 1024.0
    write_b = sum(kw) / len(kw) * fw * 1024.0
    rec = {
        "kernel": kernel, "workload": workload, "sources": TRAFFIC_SOURCES[kernel],
        "source_sha256": _sources_sha(TRAFFIC_SOURCES[kernel]), "launches": len(kf),
        "fetch_kib_per_launch": sum(kf) / len(kf), "write_kib_per_launch": sum(kw) / len(kw),
        "calibration": {"kernel": f"plain elementwise copy of {copy_mib} MiB", "fetch_kib": cf[-1],
                        "write_kib": cw[-1], "fetch_factor": ff, "write_factor": fw},
        "measured_bytes_per_launch": fetch_b + write_b,
        "commands": commands,
    }
    path = path or os.path.join(ROOT, "profiles", f"traffic_{kernel}.json")
    with open(path, "w") as f:
        json.dump(rec, f, indent=1)
        f.write("\n")
    print(json.dumps(rec))


def _blas_threads():
    try:
        from threadpoolctl import threadpool_info
        return max([i.get("num_threads", 1) for i in threadpool_info()] or [os.cpu_count() or 1])
    except Exception:
        return os.cpu_count() or 1


def cpu_baseline(w, ra, rb, d, dj, zipup_ncores=0):
    """The FP64 oracle (NumPy + LAPACK) on this host's cores.

    value: one full contract+round (or zip-up with super-cores of
    zipup_ncores cores) of the workload with every BLAS thread; its result
    is returned as the reference for the GPU result.  Beside it, a bounded
    sample timed with all threads and with one (median of 3 each): the
    oracle's QR-sweep step on one interior bond of the workload (reduced
    Householder QR of the (2 r_C) x r_C unfolding of the contracted core
    C_21, R into the next core).  Returns (record, reference cores,
    reference info, exact contracted train or None)."""
    import numpy as np

    import oracle as O
    threads = _blas_threads()
    C = None
    t0 = time.perf_counter()
    if zipup_ncores:
        Y, info = O.zipup(w.spec, w.a, w.b, w.rel_tol, w.max_rank, ncores=zipup_ncores, return_info=True)
        dt = time.perf_counter() - t0
        flops = zipup_flops(ra, rb, d, dj, info.ranks, zipup_ncores)
        what = f"one full zip-up (super-cores of {zipup_ncores})"
    else:
        C = O.contract(w.spec, w.a, w.b)
        Y, info = O.round_tt(C, w.rel_tol, w.max_rank, return_info=True)
        dt = time.perf_counter() - t0
        flops = contract_round_flops(ra, rb, d, dj, info.ranks)
        what = "one full contract+round"
    rec = {"value": flops / dt / 1e12, "unit": "TFLOP/s", "cores": threads, "kind": "oracle",
           "sample": f"{what} of the same 42-core workload (NumPy FP64, LAPACK QR/SVD), all BLAS threads",
           "seconds": dt}
    # bounded sample, all threads and one thread, median of 3
    k = len(d) // 2
    Ck = C[k] if C is not None else O.contract(w.spec, [w.a[k]], [w.b[k]])[0]
    nxt = C[k + 1] if C is not None else O.contract(w.spec, [w.a[k + 1]], [w.b[k + 1]])[0]
    sample = [Ck.reshape(1, -1, Ck.shape[-1]), nxt[:, :, :1]]  # the unfolding as a one-row core, then R C_{k+1}
    m, c = Ck.shape[0] * Ck.shape[1], Ck.shape[-1]
    q = min(m, c)
    sflops = geqrf_flops(m, c) + (2.0 * m * q * q - 2.0 * q ** 3 / 3.0) + 2.0 * q * c * nxt.shape[1]  # geqrf+orgqr+R C

    def med3():
        ts = []
        for _ in range(3):
            t = time.perf_counter()
            O.orthogonalize(sample)
            ts.append(time.perf_counter() - t)
        return sorted(ts)[1]

    t_all = med3()
    try:
        from threadpoolctl import threadpool_limits
        with threadpool_limits(limits=1):
            t_one = med3()
        one = {"value": sflops / t_one / 1e12, "seconds_median": t_one, "cores": 1}
    except Exception:
        one = None
    rec["bond_sample"] = {"what": f"QR-sweep step of one interior bond: QR of the {m} x {c} unfolding of C_{k + 1}, "
                                  f"R into the next core (oracle.orthogonalize), median of 3",
                          "gflop": sflops / 1e9,
                          "all_threads": {"value": sflops / t_all / 1e12, "seconds_median": t_all, "cores": threads},
                          "one_thread": one, "unit": "TFLOP/s"}
    return rec, Y, info, C


if __name__ == "__main__":
    main()
