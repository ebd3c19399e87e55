"""Autotuner for the decode launch shape (the analogue of the paper's parser
granularity sweep, Section 7 and its Table 3).

Whole-archive decode (`tune`): searches, on a sample of the workload,
  * the interleave width W (32 or 64; the sample is re-encoded, since W is an
    archive parameter),
  * entropy streams per wavefront (1, or 2 when W <= 32),
  * wavefronts per block of the match expansion (0 = the library's choice per
    launch by the level's size, 2 or 4),
  * the decode mode (1: one expansion launch per dependency level; 3: the
    same, with the later levels' entropy decode on a second stream beside
    the first levels' expansion; 2: one persistent launch for all levels)
    and, for mode 2, the grid (every workgroup the device holds at once, or
    half of them).
The launch shape alone (`tune_archive`): the same candidates timed on a
resident archive of the workload itself (no re-encoding).
Batched seeks (`tune_batch`): the same launch-shape space for a replayed batch
graph, timed on a sample batch of requests.

Every candidate is timed with HIP events and its output compared with the
expected bytes; a candidate that decodes anything else raises instead of
being ranked.  The fastest is returned and cached as JSON keyed by (GPU
architecture, block size, profile).
"""
from __future__ import annotations

import json
import os
import time

DEFAULT_CACHE = os.path.join(os.path.expanduser("~"), ".cache", "aceseek", "tune.json")


def _arch(torch) -> str:
    try:
        return torch.cuda.get_device_properties(0).gcnArchName.split(":")[0]
    except Exception:
        return "unknown"


def _grid_full(torch) -> int:
    """Workgroups of the persistent kernel the device holds at once (an
    estimate from the CU count: ten 128-thread workgroups per CU)."""
    try:
        return 10 * torch.cuda.get_device_properties(0).multi_processor_count
    except Exception:
        return 0


def candidates(W: int, grid_full: int):
    per_wave = (1, 2) if W <= 32 else (1,)
    out = []
    for p in per_wave:
        for w in (0, 2, 4):
            out.append(dict(mode=1, waves_per_block=w, blocks_per_wg=p, grid_wgs=0))
        out.append(dict(mode=3, waves_per_block=0, blocks_per_wg=p, grid_wgs=0))
        out.append(dict(mode=2, waves_per_block=0, blocks_per_wg=p, grid_wgs=0))
        if grid_full:
            out.append(dict(mode=2, waves_per_block=0, blocks_per_wg=p, grid_wgs=grid_full // 2))
    return out


def _time_decode(arc, tuning, reps: int, torch, expect) -> float:
    out = torch.empty(arc.n_total, dtype=torch.uint8, device=arc.device)
    ws = arc.workspace(arc.workspace_bytes())
    arc.decode_all(out=out, ws=ws, tuning=tuning)
    arc.check(ws)
    if not torch.equal(out, expect):
        raise RuntimeError("autotune: candidate %r decodes wrong bytes" % (tuning,))
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    ev0.record()
    for _ in range(reps):
        arc.decode_all(out=out, ws=ws, tuning=tuning)
    ev1.record()
    torch.cuda.synchronize()
    arc.check(ws)
    return ev0.elapsed_time(ev1) / reps


def _store(cache_path: str, key: str, entry: dict):
    try:
        os.makedirs(os.path.dirname(cache_path), exist_ok=True)
        db = json.load(open(cache_path)) if os.path.exists(cache_path) else {}
        db[key] = entry
        json.dump(db, open(cache_path, "w"), indent=1)
    except (OSError, ValueError):
        pass


def tune(sample: bytes, profile: str, block_size: int = 16384, min_match: int = 20,
         max_level: int = 16, widths=(32, 64), reps: int = 5,
         cache_path: str = DEFAULT_CACHE, log=None) -> dict:
    """Returns the best {"interleave", "mode", "waves_per_block",
    "blocks_per_wg", "grid_wgs", "ms", ...} for whole-archive decodes of the
    sample, with every candidate's time under "all" of the cached entry."""
    import numpy as np
    import torch

    from .aceseek import Archive, encode

    arch = _arch(torch)
    key = "%s/B%d/%s" % (arch, block_size, profile)
    expect = torch.from_numpy(np.frombuffer(sample, dtype=np.uint8).copy()).to("cuda")
    grid_full = _grid_full(torch)
    results = []
    for W in widths:
        a = encode(sample, block_size=block_size, interleave=W, min_match=min_match,
                   hash_len=min_match, max_chain=32, max_level=max_level)
        arc = Archive(a)
        for c in candidates(W, grid_full):
            ms = _time_decode(arc, c, reps, torch, expect)
            results.append(dict(interleave=W, ms=ms, gbs=len(sample) / ms / 1e6,
                                ratio=len(sample) / len(a), **c))
            if log:
                log("tune W=%d mode=%d waves/block=%d streams/wave=%d grid=%d: %.3f ms" % (
                    W, c["mode"], c["waves_per_block"], c["blocks_per_wg"], c["grid_wgs"], ms))
        arc.close()
    best = min(results, key=lambda r: r["ms"])
    _store(cache_path, key, {"best": best, "all": results, "time": time.time(),
                             "sample_bytes": len(sample)})
    return best


def tune_archive(arc, expect, reps: int = 5, log=None) -> dict:
    """The fastest launch shape (mode, waves per block, streams per wave,
    grid) for whole-archive decodes of an archive already resident, timed on
    the archive itself; expect is the original bytes on the device.  Every
    candidate's output is compared with it before it is ranked."""
    import torch

    grid_full = _grid_full(torch)
    W = arc.interleave or 64
    results = []
    for c in candidates(W, grid_full):
        ms = _time_decode(arc, c, reps, torch, expect)
        results.append(dict(ms=ms, **c))
        if log:
            log("tune on the archive: mode=%d waves/block=%d streams/wave=%d grid=%d: %.3f ms" % (
                c["mode"], c["waves_per_block"], c["blocks_per_wg"], c["grid_wgs"], ms))
    best = dict(min(results, key=lambda r: r["ms"]))
    best["all"] = results
    return best


def tune_batch(arc, x_dev, lo, hi, reps: int = 3, log=None) -> dict:
    """The fastest launch shape for one replayed batch graph of the requests
    [lo_i, hi_i) on a resident archive (every output compared with x_dev)."""
    import numpy as np
    import torch

    ln = (hi - lo).astype(np.int64)
    offs = np.concatenate([[0], np.cumsum(ln)[:-1]]).astype(np.uint64)
    out = torch.empty(max(int(ln.sum()), 1), dtype=torch.uint8, device=arc.device)
    grid_full = _grid_full(torch)
    W = arc.interleave if hasattr(arc, "interleave") else 64
    results = []
    for c in candidates(W, grid_full):
        bt = arc.batch(len(lo), tuning=c)
        bt.run((lo, hi), out, offs)
        torch.cuda.synchronize()
        bt.check()
        for i in range(len(lo)):
            if not torch.equal(out[int(offs[i]):int(offs[i]) + int(ln[i])], x_dev[int(lo[i]):int(hi[i])]):
                bt.close()
                raise RuntimeError("autotune: batch candidate %r returns wrong bytes" % (c,))
        times = []
        for _ in range(reps):
            t = time.perf_counter()
            bt.run((lo, hi), out, offs)
            torch.cuda.synchronize()
            times.append(time.perf_counter() - t)
        bt.close()
        ms = 1e3 * float(np.median(times))
        results.append(dict(ms=ms, **c))
        if log:
            log("tune batch of %d mode=%d waves/block=%d streams/wave=%d grid=%d: %.3f ms" % (
                len(lo), c["mode"], c["waves_per_block"], c["blocks_per_wg"], c["grid_wgs"], ms))
    best = dict(min(results, key=lambda r: r["ms"]))
    best["all"] = results
    return best


def cached(profile: str, block_size: int = 16384, cache_path: str = DEFAULT_CACHE):
    import torch
    key = "%s/B%d/%s" % (_arch(torch), block_size, profile)
    try:
        return json.load(open(cache_path))[key]["best"]
    except (OSError, KeyError, ValueError):
        return None
