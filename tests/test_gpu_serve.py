"""Continuous batching on the GPU: requests arriving while others run are
admitted into free slots (each slot its own HIP stream and workspace), and
every result is byte-identical alone and in the mix, with captured batch
graphs (device-side planning), with graphs that keep level 0 decoded, and
with host-planned batched seeks."""
import numpy as np
import pytest

import gen

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


@pytest.mark.parametrize("keep,host", [(None, False), (1, False), (None, True)],
                         ids=["graphs", "graphs-kept-level-0", "host-planned"])
def test_results_same_alone_and_in_mix(orc, keep, host):
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2606_24531_amd import Archive, encode
    from paper_2606_24531_amd.serve import GpuBackend, Server, latency_report, poisson_run
    xs = {"genome": gen.genome(3 << 20, 51), "fastq": gen.fastq(2 << 20, 52),
          "text": gen.text(2 << 20, 53)}
    arcs = {k: Archive(encode(v, block_size=16384, interleave=32, min_match=16, hash_len=16,
                              max_level=8), device="cuda:0") for k, v in xs.items()}
    backend = GpuBackend(arcs, slots=3, keep_levels=keep, max_batch=64, batch_bytes=8 << 20, host_planned=host)
    # the consumer copies each result out as it completes and releases it,
    # which returns its bytes to the budget
    got = {}
    srv = Server(backend, budget_bytes=8 << 20, slots=3, max_batch=64,
                 on_done=lambda r: got.__setitem__(r.rid, r.result.cpu().numpy().tobytes()),
                 auto_release=True)
    reqs, wall = poisson_run(srv, list(xs), {k: len(v) for k, v in xs.items()}, rate=3000.0,
                             count=400, seed=5, min_len=16, max_len=1 << 20)
    rep = latency_report(reqs, wall)
    assert rep["requests"] == 400
    assert srv.peak_used <= 8 << 20
    assert srv.batches < 400  # requests were actually batched
    # workspaces were all allocated up front
    assert backend.device_bytes()["workspaces"] > 0
    torch.cuda.synchronize()
    assert srv.used == 0 and all(r.released for r in reqs)
    rng = np.random.default_rng(0)
    for r in reqs:
        assert got[r.rid] == xs[r.archive][r.lo:r.hi], r.rid
    for r in rng.choice(reqs, size=20, replace=False):
        solo = arcs[r.archive].seek(r.lo, r.hi, tuning=dict(mode=1))
        arcs[r.archive].check()
        assert solo.cpu().numpy().tobytes() == got[r.rid]
