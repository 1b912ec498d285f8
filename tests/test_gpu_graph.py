"""The rounding sweep with device-resident ranks: qtt_contract_round_async
enqueues the whole contraction + rounding with no host synchronisation, so it
can be captured in a HIP graph.  Its eager result must equal the synchronous
entry point's bit for bit, and every replay of the captured graph (with eager
work, synchronisations and poisoned output buffers in between) must reproduce
it bit for bit."""
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


def _workloads():
    # the 2D rank-64 workload (ranks capped at the bound) and the 1D Hadamard
    # product whose tolerance cuts ranks below their bounds
    return [I.laplacian2d_r64(), I.sin_noise_1d()]


@pytest.mark.parametrize("widx", [0, 1])
@pytest.mark.parametrize("prec", ["fp64", "bf16x6"])
def test_async_equals_sync_and_graph_replays(widx, prec):
    w = _workloads()[widx]
    log(f"graph capture: {w.name} {prec}")
    A = Q.to_device(w.a, DEV)
    B = Q.to_device(w.b, DEV)
    ref = Q.contract_round(w.spec, A, B, w.rel_tol, w.max_rank, prec=prec)
    run = Q.ContractRoundAsync(w.spec, A, B, w.rel_tol, w.max_rank, prec=prec)
    run.enqueue()
    cores, ranks = run.result()
    assert ranks == ref.ranks, (ranks, ref.ranks)
    for k, (g, r) in enumerate(zip(cores, ref.cores)):
        assert torch.equal(g, r), k
    # and the oracle, to the arithmetic's tolerance
    want, info = O.round_tt(O.contract(w.spec, w.a, w.b), w.rel_tol, w.max_rank, return_info=True)
    assert ranks == info.ranks
    err = O.rel_error(Q.to_host(cores), want)
    assert err <= (1e-12 if prec == "fp64" else 1e-6), err
    eager = [c.clone() for c in cores]
    # capture
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g, capture_error_mode="thread_local"):
        run.enqueue()
    torch.cuda.synchronize()
    for rep in range(4):
        for buf in run.out_buffers:
            buf.fill_(float("nan"))
        run.ranks_dev.fill_(-1)
        run.status_dev.fill_(12345)
        _ = (torch.ones(4096, device=DEV) * 3).sum().item()
        torch.cuda.synchronize()
        g.replay()
        c2, r2 = run.result()
        assert r2 == ranks, (rep, r2, ranks)
        for k, (x, y) in enumerate(zip(c2, eager)):
            assert torch.equal(x, y), (rep, k)
    log(f"  ranks {max(ranks)} max, err vs oracle {err:.2e}; 4 graph replays bit-identical")
