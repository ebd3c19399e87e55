"""Continuous-batching seek server over resident archives.

Archives stay compressed in HBM (the paper's keep -> seek -> keep pattern,
Section 9).  Requests name an archive and an absolute byte range.  A request
is admitted once its output bytes fit the output budget; admitted requests
are grouped per archive into a batch as soon as one of K in-flight slots is
free; each slot owns a HIP stream and a workspace, so batches on different
slots overlap on the device.  A batch is one replay of a captured batch
graph per (slot, archive): the union of the requests' closures is planned on
the device, decoded level by level, and gathered; with keep_levels the
graph's lowest dependency levels stay decoded (ace_batch_pin), so closures
stop there.  A host-planned backend runs one seek_batch call per batch
instead.  Latency is measured from a request's scheduled
arrival to the completion of its batch, so queueing is included.

Device memory is bounded up front.  A result is a view of its batch's output
buffer; the batch's bytes stay charged to the output budget until the
consumer has released every request of the batch (Server.release, or
auto_release after an on_done callback), so outputs never hold more than the
budget.  Every workspace is allocated when the backend is built (one
captured batch graph per slot and archive; or, host-planned, one workspace
per slot sized by the library's bound for a batch of max_batch requests
filling the budget) and reported by device_bytes().

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
    result: object = None            # device tensor view (or host bytes) of [lo, hi), until released
    done: threading.Event = field(default_factory=threading.Event)
    batch: object = None             # the _Batch whose output holds the result
    released: bool = False

    @property
    def nbytes(self) -> int:
        return self.hi - self.lo


@dataclass
class _Batch:
    nbytes: int      # output bytes charged to the budget
    open: int        # requests not yet released


class GpuBackend:
    """Slots on HIP streams.  Every workspace is allocated here.  By default
    each (slot, archive) owns a captured batch graph (device-side planning,
    one replay per batch), whose lowest keep_levels levels stay decoded when
    keep_levels is given; with host_planned, each slot instead owns one
    workspace sized by the library's bound for max_batch ranges of at most
    batch_bytes in all, and a batch is one host-planned seek_batch call."""

    def __init__(self, archives: dict, slots: int, device="cuda:0", keep_levels=None, max_batch: int = 4096,
                 batch_bytes: int = 1 << 30, host_planned: bool = False):
        import torch
        self.torch = torch
        self.archives = archives
        self.device = torch.device(device)
        self.streams = [torch.cuda.Stream(device=self.device) for _ in range(slots)]
        self.ws = [None] * slots
        self.batches = {}
        if not host_planned:
            for slot in range(slots):
                for name, arc in archives.items():
                    bt = arc.batch(max_batch, stream=self.streams[slot])
                    if keep_levels:
                        bt.pin(min(int(keep_levels), arc.depth))
                    self.batches[(slot, name)] = bt
        else:
            need = max(arc.workspace_bound(max_batch, batch_bytes) for arc in archives.values())
            self.ws = [torch.zeros(max(need, 256), dtype=torch.uint8, device=self.device) for _ in range(slots)]

    def device_bytes(self) -> dict:
        """Device memory held by the backend: workspaces (or batch graphs) and
        the compressed archives."""
        ws = sum(t.numel() for t in self.ws if t is not None) + sum(bt.ws.numel() for bt in self.batches.values())
        arch = sum(arc.d_arch.numel() + (arc.d_plan.numel() if arc.d_plan is not None else 0)
                   for arc in self.archives.values())
        return {"workspaces": int(ws), "archives_and_plans": int(arch)}

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
                # the slot's workspace is sized by the bound: no allocation here
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
    """on_done(request) runs at each completion (under the server's lock);
    with auto_release the request is released right after it."""

    def __init__(self, backend, budget_bytes: int, slots: int, max_batch: int = 4096, on_done=None,
                 auto_release: bool = False):
        self.backend = backend
        self.budget = budget_bytes
        self.on_done = on_done
        self.auto_release = auto_release
        self.used = 0  # output bytes admitted and not yet released
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
        # scheduling passes, and those that found every slot busy or the
        # oldest pending request not fitting the budget; host seconds spent
        # launching and finishing batches (what limits a run)
        self.passes = self.passes_slots_full = self.passes_budget_full = 0
        self.host_s = 0.0
        self.t_first = None

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
            # completions free slots; budget comes back as results are released
            if self.t_first is None:
                self.t_first = time.perf_counter()
            for slot, (h, reqs, nb) in list(self.inflight.items()):
                if self.backend.poll(h):
                    t_h = time.perf_counter()
                    views = self.backend.finish(h)
                    self.host_s += time.perf_counter() - t_h
                    t = time.perf_counter()
                    batch = _Batch(nb, len(reqs))
                    for r, v in zip(reqs, views):
                        r.result, r.t_done, r.batch = v, t, batch
                        r.done.set()
                    self.done.extend(reqs)
                    del self.inflight[slot]
                    for r in reqs:
                        if self.on_done is not None:
                            self.on_done(r)
                        if self.auto_release:
                            self._release(r)
            self._admit()
            self.passes += 1
            if self.pending:
                self.passes_budget_full += 1
            # fill free slots with the oldest archive's admitted requests
            free = [s for s in range(self.slots) if s not in self.inflight]
            if not free and any(self.admitted.values()):
                self.passes_slots_full += 1
            for slot in free:
                names = [n for n, q in self.admitted.items() if q]
                if not names:
                    break
                name = min(names, key=lambda n: self.admitted[n][0].t_arrival)
                q = self.admitted[name]
                reqs = [q.popleft() for _ in range(min(len(q), self.max_batch))]
                t_h = time.perf_counter()
                h = self.backend.launch(slot, name, reqs)
                self.host_s += time.perf_counter() - t_h
                self.inflight[slot] = (h, reqs, sum(r.nbytes for r in reqs))
                self.batches += 1
            busy = bool(self.inflight or self.pending or any(self.admitted.values()))
        return busy

    def release(self, r: Request):
        """The consumer is done with r's result: drops it, and returns its
        batch's bytes to the budget once every request of the batch is
        released."""
        with self.lock:
            self._release(r)

    def _release(self, r: Request):
        if r.released or r.batch is None:
            return
        r.released = True
        r.result = None
        r.batch.open -= 1
        if r.batch.open == 0:
            self.used -= r.batch.nbytes

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


def limiter(server: Server) -> dict:
    """What held a run back: the share of wall time the scheduler spent in
    the host part of launching and finishing batches (host-bound), and the
    shares of scheduling passes that found admitted work waiting for a slot
    (device-bound) or arrived work waiting for budget (memory-bound)."""
    n = max(server.passes, 1)
    slots, budget = server.passes_slots_full / n, server.passes_budget_full / n
    wall = time.perf_counter() - server.t_first if server.t_first else 0.0
    host = server.host_s / wall if wall > 0 else 0.0
    if host > 0.5:
        name = "host"
    elif slots >= budget and slots > 0.05:
        name = "slots"
    else:
        name = "budget" if budget > 0.05 else "arrivals"
    return {"passes": server.passes, "host_share": round(host, 4), "slots_full_share": round(slots, 4),
            "budget_full_share": round(budget, 4), "limiter": name}


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
