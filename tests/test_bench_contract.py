"""bench.py's command-line contract and its measurement bookkeeping (no GPU needed)."""
import json
import os
import subprocess
import sys

import pytest

import bench

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_more_than_one_gpu_is_refused_with_a_message():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr


def _counter_csv(path, counter, rows):
    with open(path, "w") as f:
        f.write("Dispatch_Id,Kernel_Name,Counter_Name,Counter_Value\n")
        for did, name, v in rows:
            f.write(f'{did},"{name}",{counter},{v}\n')


def test_traffic_record_from_counter_files(tmp_path):
    """The byte-counter record: per-launch averages of the kernel's FETCH_SIZE
    and WRITE_SIZE (KiB), each scaled by what the counter reads for the plain
    copy of known size, and applied only for the same workload and kernel
    sources."""
    k = "void qtt::(anonymous namespace)::k_jacobi<8>(double*, int)"
    cp = "at::elementwise_kernel<mul>"
    _counter_csv(tmp_path / "f.csv", "FETCH_SIZE", [(1, k, 100.0), (2, k, 300.0), (3, cp, 131072.0)])
    _counter_csv(tmp_path / "w.csv", "WRITE_SIZE", [(1, k, 50.0), (2, k, 150.0), (3, cp, 262144.0)])
    out = tmp_path / "rec.json"
    bench.traffic_record("k_jacobi", "wl", str(tmp_path / "f.csv"), str(tmp_path / "w.csv"), 256, ["cmd"], str(out))
    rec = json.load(open(out))
    assert rec["launches"] == 2
    assert rec["calibration"]["fetch_factor"] == 2.0 and rec["calibration"]["write_factor"] == 1.0
    # (200 KiB * 2 + 100 KiB * 1) per launch
    assert abs(rec["measured_bytes_per_launch"] - 500.0 * 1024) < 1e-9
    assert rec["source_sha256"] == bench._sources_sha(bench.TRAFFIC_SOURCES["k_jacobi"])


def test_committed_traffic_record_applies_only_to_its_workload_and_sources():
    path = os.path.join(ROOT, "profiles", "traffic_k_jacobi.json")
    if not os.path.exists(path):
        pytest.skip("no byte-counter record committed")
    rec = json.load(open(path))
    assert bench.measured_traffic("k_jacobi", rec["workload"] + "_other") is None
    got = bench.measured_traffic("k_jacobi", rec["workload"])
    if got is None:
        pytest.skip("the record was taken on other kernel sources: bench.py reports traffic null until re-measured")
    assert got == rec["measured_bytes_per_launch"]


def test_flop_model_reduces_to_textbook_counts():
    # Householder QR of an m x n matrix (m >= n): 2 m n^2 - 2 n^3 / 3
    assert bench.geqrf_flops(100, 10) == 2 * 100 * 100 - 2 * 1000 / 3
    assert bench.geqrf_flops(10, 100) == bench.geqrf_flops(100, 10)
    # applying k reflectors of an m-row Q to c columns: 4 m k c - 2 k^2 c
    assert bench.ormqr_flops(50, 5, 3) == 4 * 50 * 5 * 3 - 2 * 25 * 3
    # a rank-1 single-core train has no QR and no SVD: only the bond products
    f = bench.contract_round_flops([1, 1], [1, 1], [2], [2], [1, 1], mpo=True)
    assert f == 2.0 * 1 * 2 * 1 + 2.0 * 2 * 1 * 2 + bench.ormqr_flops(2, 1, 1)


def test_round_flop_model_on_two_cores():
    """qtt_round of [1, 3, 1] with d = 2, kept rank 2: QR of the 2 x 3 first
    unfolding, R times the last core, nominal SVD of the 2 x 2 centre, the
    U Sigma product and one Q application."""
    f = bench.round_flops([1, 3, 1], [2, 2], [1, 2, 1])
    expect = (bench.geqrf_flops(2, 3) + 2.0 * 2 * 3 * 2 + bench.svd_nominal_flops(2, 2) + 2.0 * 2 * 2 * 2
              + bench.ormqr_flops(2, 2, 2))
    assert f == expect


def test_zipup_and_fit_flop_models():
    import qtt_inputs as I
    w = I.laplacian3d_r256()
    ra = [1] + [c.shape[-1] for c in w.a]
    rb = [1] + [c.shape[-1] for c in w.b]
    d = [c.shape[1] for c in w.a]
    dj = [c.shape[2] for c in w.a]
    n = len(d)
    out = [min(256, 2 ** k, 2 ** (n - k)) for k in range(n + 1)]
    full = bench.contract_round_flops(ra, rb, d, dj, out)
    z1 = bench.zipup_flops(ra, rb, d, dj, out, 1)
    z2 = bench.zipup_flops(ra, rb, d, dj, out, 2)
    # the decomposition algorithm never factors the 3584 x 1792 unfoldings
    assert 0 < z1 < z2 < full
    # no sweep: the product and the first left environments only
    ry, rc, dd = [1, 4, 1], [1, 2, 1], [2, 2]
    f0 = bench.fit_flops(ry, rc, dd, dd, 0)
    prod = sum(2.0 * dd[k] * ry[k] * dd[k] * ry[k + 1] for k in range(2))
    env0 = 2.0 * rc[0] * ry[0] * dd[0] * ry[1] + 2.0 * rc[1] * rc[0] * dd[0] * ry[1]
    assert f0 == prod + env0
    assert bench.fit_flops(ry, rc, dd, dd, 2) > bench.fit_flops(ry, rc, dd, dd, 1) > f0
