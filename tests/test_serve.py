"""Scheduling logic of the continuous-batching server, on the CPU.

A fake backend stands in for the GPU: it decodes each batch with the oracle
and reports completion after a simulated device time, so admission by the
output budget, slot reuse, grouping by archive and result routing are
tested without a device."""
import time

import numpy as np
import pytest

import gen
from paper_2606_24531_amd.serve import Server, latency_report, limiter, poisson_run


class FakeBackend:
    def __init__(self, orc, archives, device_s=0.002):
        self.orc = orc
        self.archives = archives
        self.device_s = device_s
        self.launched = []

    def launch(self, slot, name, reqs):
        a = self.archives[name]
        views = [self.orc.seek(a, r.lo, r.hi) for r in reqs]
        self.launched.append((slot, name, len(reqs)))
        return (time.perf_counter() + self.device_s, views)

    def poll(self, h):
        return time.perf_counter() >= h[0]

    def finish(self, h):
        return h[1]


@pytest.fixture(scope="module")
def corpus(orc):
    xs = {"genome": gen.genome(600_000, 1), "text": gen.text(400_000, 2)}
    arcs = {k: orc.encode(v, block_size=16384, interleave=32, min_match=16, hash_len=16,
                          max_level=8) for k, v in xs.items()}
    return xs, arcs


def test_results_budget_and_slots(orc, corpus):
    xs, arcs = corpus
    be = FakeBackend(orc, arcs)
    budget = 300_000
    # the consumer checks and releases each result as it completes, so the
    # budget comes back
    bad = []
    srv = Server(be, budget_bytes=budget, slots=3, max_batch=16,
                 on_done=lambda r: r.result == xs[r.archive][r.lo:r.hi] or bad.append(r.rid),
                 auto_release=True)
    rng = np.random.default_rng(0)
    reqs = []
    for i in range(200):
        name = ["genome", "text"][i % 2]
        n = len(xs[name])
        ln = int(rng.integers(1, 60_000))
        lo = int(rng.integers(0, n - ln))
        reqs.append(srv.submit(name, lo, lo + ln))
        srv.step()
    srv.drain(timeout=60)
    assert srv.peak_used <= budget
    assert srv.used == 0 and not bad
    for r in reqs:
        assert r.done.is_set() and r.released and r.result is None
    assert max(s for s, _, _ in be.launched) <= 2
    assert all(k <= 16 for _, _, k in be.launched)
    # batches are per archive
    assert {name for _, name, _ in be.launched} == {"genome", "text"}


def test_oversized_request_rejected(orc, corpus):
    xs, arcs = corpus
    srv = Server(FakeBackend(orc, arcs), budget_bytes=1000, slots=1)
    with pytest.raises(ValueError):
        srv.submit("genome", 0, 5000)


def test_poisson_driver_reports(orc, corpus):
    xs, arcs = corpus
    got = {}
    srv = Server(FakeBackend(orc, arcs, device_s=0.001), budget_bytes=1 << 20, slots=2,
                 on_done=lambda r: got.__setitem__(r.rid, r.result), auto_release=True)
    reqs, wall = poisson_run(srv, ["genome", "text"], {k: len(v) for k, v in xs.items()},
                             rate=2000.0, count=300, seed=3, min_len=16, max_len=50_000)
    rep = latency_report(reqs, wall)
    assert rep["requests"] == 300 and rep["p99_ms"] >= rep["p50_ms"] > 0
    for r in reqs:
        assert got[r.rid] == xs[r.archive][r.lo:r.hi]
    assert srv.used == 0
    lim = limiter(srv)
    # the fake backend decodes on the host inside launch: host time is counted
    assert lim["passes"] > 0 and lim["host_share"] > 0
    assert lim["limiter"] in ("host", "slots", "budget", "arrivals")


def test_held_results_keep_their_budget(orc, corpus):
    """Results the consumer still holds stay charged: later requests wait for
    budget until a release, and the bytes come back per batch once every
    request of the batch is released."""
    xs, arcs = corpus
    srv = Server(FakeBackend(orc, arcs, device_s=0.0), budget_bytes=100_000, slots=2, max_batch=4)
    a = [srv.submit("genome", 0, 40_000), srv.submit("genome", 50_000, 90_000)]
    srv.drain(timeout=10)
    assert all(r.done.is_set() for r in a) and srv.used == 80_000
    b = srv.submit("text", 0, 30_000)
    for _ in range(50):
        srv.step()
    assert not b.done.is_set() and srv.used == 80_000  # waits for budget
    batches = {id(r.batch) for r in a}
    srv.release(a[0])
    srv.step()
    if len(batches) == 1:  # one batch: its bytes return with its last request
        assert srv.used == 80_000 and not b.done.is_set()
    srv.release(a[1])
    srv.drain(timeout=10)
    assert b.done.is_set() and b.result == xs["text"][0:30_000]
    srv.release(b)
    srv.release(b)  # a second release is a no-op
    assert srv.used == 0 and srv.peak_used <= 100_000
