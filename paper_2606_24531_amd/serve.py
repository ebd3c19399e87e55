"""Continuous-batching seek server over resident archives.

Archives stay compressed in HBM (the paper's keep -> seek -> keep pattern,
Section 9).  Requests name an archive and an absolute byte range.  A request
is admitted once its output bytes fit the output budget; admitted requests
are grouped per archive into a batch as soon as one of K in-flight slots is
free; each slot owns a HIP stream and a workspace, so batches on different
slots overlap on the device.  A batch is one seek_batch call (one
dependency-ordered decode of the union of the requests' closures, then one
gather), or, with keep_levels, one replay of a captured batch graph per
(slot, archive) whose lowest dependency levels stay decoded (ace_batch_pin),
so closures stop there.  Latency is measured from a request's scheduled arrival to the
completion of its batch, so queueing is included.

The device work goes through a backend object so the scheduling logic can
be exercised without a GPU; GpuBackend is the real one.
"""
from __future__ import annotations

import collections
import threading
import time
from dataclasses import dataclass, field

import numpy as np


@dataclass
class Request:
    rid: int
    archive: str
    lo: int
    hi: int
    t_arrival: float                 # scheduled arrival (perf_counter seconds)
    t_done: float = 0.0
    result: object = None            # device tensor view (or host bytes) of [lo, hi)
    done: threading.Event = field(default_factory=threading.Event)

    @property
    def nbytes(self) -> int:
        return self.hi - self.lo


class GpuBackend:
    """Slots on HIP streams, decoding with libaceseek's batched seek."""

    def __init__(self, archives: dict, slots: int, device="cuda:0", keep_levels=None, max_batch: int = 4096):
        import torch
        self.torch = torch
        self.archives = archives
        self.device = torch.device(device)
        self.streams = [torch.cuda.Stream(device=self.device) for _ in range(slots)]
        self.ws = [None] * slots
        # kept levels: a batch graph per (slot, archive), its lowest levels decoded once
        self.batches = {}
        if keep_levels is not None:
            for slot in range(slots):
                for name, arc in archives.items():
                    bt = arc.batch(max_batch, stream=self.streams[slot])
                    bt.pin(min(int(keep_levels), arc.depth))
                    self.batches[(slot, name)] = bt

    def launch(self, slot: int, name: str, reqs):
        torch = self.torch
        arc = self.archives[name]
        lo = np.array([r.lo for r in reqs], dtype=np.uint64)
        hi = np.array([r.hi for r in reqs], dtype=np.uint64)
        lens = (hi - lo).astype(np.int64)
        offs = np.concatenate([[0], np.cumsum(lens)[:-1]]).astype(np.uint64)
        s = self.streams[slot]
        bt = self.batches.get((slot, name))
        with torch.cuda.stream(s):
            out = torch.empty(max(int(lens.sum()), 1), dtype=torch.uint8, device=self.device)
            if bt is not None:
                bt.run((lo, hi), out, offs)
            else:
                need = arc.workspace_bytes((lo, hi))
                if self.ws[slot] is None or self.ws[slot].numel() < need:
                    self.ws[slot] = torch.zeros(max(need, 256), dtype=torch.uint8, device=self.device)
                arc.seek_batch((lo, hi), out=out, out_offsets=offs, ws=self.ws[slot], stream=s)
            ev = torch.cuda.Event()
            ev.record(s)
        views = [out[int(o):int(o) + int(n)] for o, n in zip(offs, lens)]
        return (ev, views, slot, name)

    def poll(self, handle) -> bool:
        return handle[0].query()

    def finish(self, handle):
        ev, views, slot, name = handle
        bt = self.batches.get((slot, name))
        if bt is not None:
            bt.check()
        else:
            self.archives[name].check(ws=self.ws[slot], stream=self.streams[slot])
        return views


class Server:
    def __init__(self, backend, budget_bytes: int, slots: int, max_batch: int = 4096):
        self.backend = backend
        self.budget = budget_bytes
        self.used = 0
        self.slots = slots
        self.max_batch = max_batch
        self.pending = collections.deque()  # arrived, not yet admitted
        self.admitted = collections.defaultdict(collections.deque)  # archive -> requests
        self.inflight = {}  # slot -> (handle, requests, bytes)
        self.done = []
        self.lock = threading.Lock()
        self.rid = 0
        self.peak_used = 0
        self.batches = 0

    def submit(self, archive: str, lo: int, hi: int, t_arrival: float = None) -> Request:
        with self.lock:
            r = Request(self.rid, archive, int(lo), int(hi),
                        time.perf_counter() if t_arrival is None else t_arrival)
            self.rid += 1
            if r.nbytes > self.budget:
                raise ValueError("request of %d bytes exceeds the output budget" % r.nbytes)
            self.pending.append(r)
        return r

    def _admit(self):
        # FIFO admission by output bytes
        while self.pending and self.used + self.pending[0].nbytes <= self.budget:
            r = self.pending.popleft()
            self.used += r.nbytes
            self.peak_used = max(self.peak_used, self.used)
            self.admitted[r.archive].append(r)

    def step(self) -> bool:
        """One scheduling pass; returns True if anything is still in progress."""
        with self.lock:
            # completions free slots and budget
            for slot, (h, reqs, nb) in list(self.inflight.items()):
                if self.backend.poll(h):
                    views = self.backend.finish(h)
                    t = time.perf_counter()
                    for r, v in zip(reqs, views):
                        r.result, r.t_done = v, t
                        r.done.set()
                    self.used -= nb
                    self.done.extend(reqs)
                    del self.inflight[slot]
            self._admit()
            # fill free slots with the oldest archive's admitted requests
            free = [s for s in range(self.slots) if s not in self.inflight]
            for slot in free:
                names = [n for n, q in self.admitted.items() if q]
                if not names:
                    break
                name = min(names, key=lambda n: self.admitted[n][0].t_arrival)
                q = self.admitted[name]
                reqs = [q.popleft() for _ in range(min(len(q), self.max_batch))]
                h = self.backend.launch(slot, name, reqs)
                self.inflight[slot] = (h, reqs, sum(r.nbytes for r in reqs))
                self.batches += 1
            busy = bool(self.inflight or self.pending or any(self.admitted.values()))
        return busy

    def drain(self, timeout: float = 600.0):
        t_end = time.perf_counter() + timeout
        while self.step():
            if time.perf_counter() > t_end:
                raise TimeoutError("server did not drain")
            time.sleep(0.0002)


def poisson_run(server: Server, names, n_total: dict, rate: float, count: int, seed: int,
                min_len: int = 16, max_len: int = 16 << 20):
    """Open-loop driver: Poisson arrivals at `rate` requests/s, archive uniform,
    length log-uniform in [min_len, max_len], offset uniform.  Submits each
    request at its scheduled time while scheduling continuously; returns the
    requests and the wall time of the run."""
    rng = np.random.default_rng(seed)
    gaps = rng.exponential(1.0 / rate, size=count)
    which = rng.integers(0, len(names), size=count)
    ln = np.floor(np.exp(rng.uniform(np.log(min_len), np.log(max_len), size=count))).astype(np.int64)
    u = rng.random(count)
    t0 = time.perf_counter()
    due = t0 + np.cumsum(gaps)
    reqs = []
    i = 0
    while i < count or server.step():
        now = time.perf_counter()
        while i < count and due[i] <= now:
            name = names[which[i]]
            n = n_total[name]
            L = int(min(ln[i], n))
            lo = int(u[i] * (n - L + 1))
            reqs.append(server.submit(name, lo, lo + L, t_arrival=float(due[i])))
            i += 1
        if i < count and due[i] > time.perf_counter():
            server.step()
    return reqs, time.perf_counter() - t0


def latency_report(reqs, wall: float) -> dict:
    lat = np.array([r.t_done - r.t_arrival for r in reqs]) * 1e3
    nbytes = sum(r.nbytes for r in reqs)
    return {
        "requests": len(reqs),
        "p50_ms": round(float(np.percentile(lat, 50)), 4),
        "p99_ms": round(float(np.percentile(lat, 99)), 4),
        "req_per_s": round(len(reqs) / wall, 1),
        "GB_per_s": round(nbytes / wall / 1e9, 3),
    }
