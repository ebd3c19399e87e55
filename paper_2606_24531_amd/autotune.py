"""Autotuner for the decode launch shape.

Searches, on a sample of the workload, the interleave width W (32 or 64;
the sample is re-encoded, since W is an archive parameter) and the entropy
streams per wavefront.  The wavefronts per block of the match expansion are
left to the library's per-launch choice by default (0), which depends on
each level's size: a sample's levels are smaller than the whole workload's,
so a fixed count tuned on it would be biased toward large workgroups.
Each candidate is timed as whole-archive decodes of the sample with HIP
events; the fastest is cached as JSON keyed by (GPU architecture, block
size, profile).
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


def _time_decode(arc, tuning, reps: int, torch) -> float:
    out = torch.empty(arc.n_total, dtype=torch.uint8, device=arc.device)
    ws = arc.workspace(arc.workspace_bytes())
    arc.decode_all(out=out, ws=ws, tuning=tuning)
    torch.cuda.synchronize()
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    ev0.record()
    for _ in range(reps):
        arc.decode_all(out=out, ws=ws, tuning=tuning)
    ev1.record()
    torch.cuda.synchronize()
    arc.check(ws)
    return ev0.elapsed_time(ev1) / reps


def tune(sample: bytes, profile: str, block_size: int = 16384, min_match: int = 20,
         max_level: int = 16, widths=(32, 64), waves=(0,), reps: int = 5,
         cache_path: str = DEFAULT_CACHE, log=None) -> dict:
    """Returns the best {"interleave", "waves_per_block", "blocks_per_wg",
    "mode"} (with its time) and caches it."""
    import torch

    from .aceseek import Archive, encode

    arch = _arch(torch)
    key = "%s/B%d/%s" % (arch, block_size, profile)
    results = []
    for W in widths:
        a = encode(sample, block_size=block_size, interleave=W, min_match=min_match,
                   hash_len=min_match, max_chain=32, max_level=max_level)
        arc = Archive(a)
        per_wave = (1, 2) if W <= 32 else (1,)
        cands = [dict(mode=1, waves_per_block=w, blocks_per_wg=p) for w in waves for p in per_wave]
        for c in cands:
            ms = _time_decode(arc, c, reps, torch)
            results.append(dict(interleave=W, ms=ms, gbs=len(sample) / ms / 1e6,
                                ratio=len(sample) / len(a), **c))
            if log:
                log("tune W=%d waves/block=%d streams/wave=%d: %.3f ms" % (
                    W, c["waves_per_block"], c["blocks_per_wg"], ms))
        arc.close()
    best = min(results, key=lambda r: r["ms"])
    entry = {"best": best, "all": results, "time": time.time(), "sample_bytes": len(sample)}
    try:
        os.makedirs(os.path.dirname(cache_path), exist_ok=True)
        db = json.load(open(cache_path)) if os.path.exists(cache_path) else {}
        db[key] = entry
        json.dump(db, open(cache_path, "w"), indent=1)
    except OSError:
        pass
    return best


def cached(profile: str, block_size: int = 16384, cache_path: str = DEFAULT_CACHE):
    import torch
    key = "%s/B%d/%s" % (_arch(torch), block_size, profile)
    try:
        return json.load(open(cache_path))[key]["best"]
    except (OSError, KeyError, ValueError):
        return None
