"""Benchmark: two-layer (rANS + absolute-offset match) full-archive decode.

Default workload: 1 GiB of the seeded synthetic mixed corpus (64 KiB chunks of
the genome, FASTQ-like, text and random profiles in shuffled order), 16 KiB
blocks, level cap 16, interleaved rANS with 12-bit frequencies (the interleave
width W and the launch shape picked by the autotuner on a 32 MiB sample
unless given), encoded on the host by the library encoder; the archive is
resident in HBM before timing starts.  One step = one whole-archive decode
through both layers (every step of the hot path).  Prints one JSON line.

Also reported on the same line: the decode's bytes against the MI355X HBM
roofline (algorithmic bytes = archive + output + match bytes read from
earlier blocks), per kernel and for the whole path; the same corpus at 64 KiB
blocks and uncapped; 100,000 seeks (length log-uniform 1 B..4 MiB) decoded as
one replayed batch graph against one seek call per request; a range decode of
blocks 0..1000 from the resident archive and out of core (archive in host
memory); and the CPU oracle's decode rate on this host's cores.
"""
import argparse
import json
import os
import platform
import subprocess
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0


def _log(msg):
    print("[bench] " + msg, file=sys.stderr, flush=True)


PROFILES_DIR = os.path.join(ROOT, "profiles")
KERNEL_SRC = os.path.join(ROOT, "paper_2606_24531_amd", "csrc", "kernels.hip")


def kernel_source_sha256() -> str:
    import hashlib
    with open(KERNEL_SRC, "rb") as f:
        return hashlib.sha256(f.read()).hexdigest()


def measured_traffic(kernel: str, workload: str):
    """HBM bytes per step moved by `kernel`'s launches, from the committed
    FETCH_SIZE / WRITE_SIZE counter summary of this workload (scaled by the
    calibration kernels recorded there), or None when no summary was taken on
    this workload with the kernel source built now."""
    if not os.path.isdir(PROFILES_DIR):
        return None
    sha = kernel_source_sha256()
    for fn in sorted(os.listdir(PROFILES_DIR)):
        if not fn.endswith("_hbm_counters.txt"):
            continue
        kv = {}
        for ln in open(os.path.join(PROFILES_DIR, fn)).read().splitlines():
            if ln.startswith("@ ") and ":" in ln:
                k, v = ln[2:].split(":", 1)
                kv[k.strip()] = v.strip()
        if kv.get("kernel_source_sha256") == sha and kv.get("workload") == workload:
            v = kv.get("hbm_bytes_per_step " + kernel)
            return int(v) if v is not None else None
    return None


def cpu_facts() -> dict:
    model = ""
    try:
        for ln in open("/proc/cpuinfo"):
            if ln.startswith("model name"):
                model = ln.split(":", 1)[1].strip()
                break
    except OSError:
        pass
    try:
        cc = subprocess.run(["gcc", "--version"], capture_output=True, text=True).stdout.splitlines()[0]
    except (OSError, IndexError):
        cc = "gcc"
    return {"cpu_model": model or platform.processor(), "host_threads": os.cpu_count(), "compiler": cc}


def cached_bytes(args, key, make):
    """make(), kept in args.cache_dir (when given) under key."""
    if not args.cache_dir:
        return make()
    path = os.path.join(args.cache_dir, key + ".bin")
    if os.path.exists(path):
        with open(path, "rb") as f:
            return f.read()
    b = make()
    os.makedirs(args.cache_dir, exist_ok=True)
    with open(path + ".tmp", "wb") as f:
        f.write(b)
    os.replace(path + ".tmp", path)
    return b


def cached_archive(args, x, block, cap, enc):
    from paper_2606_24531_amd import encode
    key = "archive-%s-%d-%d-B%d-cap%d-W%d-mm%d" % (args.profile, args.size, args.seed, block, cap,
                                                   enc["interleave"], enc["min_match"])
    return cached_bytes(args, key, lambda: encode(x, block_size=block, max_level=cap, **enc))


def _time_steps(fn, steps, warmup, stream):
    import torch
    for _ in range(warmup):
        fn()
    torch.cuda.synchronize()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    for _ in range(steps):
        fn()
    e1.record(stream)
    torch.cuda.synchronize()
    return e0.elapsed_time(e1) / steps


def decode_entry(arc, a, x_dev, tuning, steps, warmup, label):
    """Decode timing and facts of one archive (checked against the original
    bytes on the device first)."""
    import torch
    from paper_2606_24531_amd import aceseek as ace
    out = torch.empty(arc.n_total, dtype=torch.uint8, device=arc.device)
    ws = arc.workspace(arc.workspace_bytes())
    stream = torch.cuda.current_stream()
    arc.read_counters(ws)
    arc.decode_all(out=out, ws=ws, tuning=tuning)
    arc.check(ws)
    ext = arc.read_counters(ws)["ext_src_bytes"]
    ok = bool(torch.equal(out, x_dev))
    if not ok:
        _log("%s: DECODE MISMATCH" % label)
        sys.exit(1)
    ms = _time_steps(lambda: arc.decode_all(out=out, ws=ws, tuning=tuning), steps, warmup, stream)
    arc.check(ws)
    facts = ace.archive_facts(a)
    st = ace.stream_table(a)
    raw_in_place = sum(v["raw"] - v["rans_raw"] for v in st.values())   # streams stored raw
    coded = sum(v["rans_stored"] for v in st.values())
    return dict(ms=ms, ext=ext, ok=ok, facts=facts, raw_in_place=raw_in_place, coded=coded,
                rans_decoded=sum(v["rans_raw"] for v in st.values()), out=out, ws=ws)


def gather_calibration(dev) -> dict:
    """The rate HBM serves scattered whole 128-byte lines, the access pattern
    of match sources in earlier blocks: 8 Mi rows at uniform random indices
    of a 4 GiB buffer, read only (folded per thread) and copied out
    contiguously, by the calibration library's gather kernel; the best grid
    of a small sweep, each timed over 5 launches with events on the stream
    the launches run on."""
    import ctypes
    import torch
    path = os.path.join(ROOT, "paper_2606_24531_amd", "libacecalib.so")
    if not os.path.exists(path):
        raise RuntimeError("%s is not built (run __graft_entry__.build())" % path)
    cl = ctypes.CDLL(path)
    cl.acecalib_gather_lines.argtypes = [ctypes.c_void_p, ctypes.c_uint64, ctypes.c_void_p, ctypes.c_uint64,
                                         ctypes.c_void_p, ctypes.c_int, ctypes.c_uint32, ctypes.c_void_p]
    cl.acecalib_gather_lines.restype = ctypes.c_int
    cl.acecalib_threads.argtypes = [ctypes.c_uint32]
    cl.acecalib_threads.restype = ctypes.c_uint64
    src_rows, n = 32 << 20, 8 << 20
    src = torch.empty(src_rows * 128, dtype=torch.uint8, device=dev)
    src.fill_(5)
    g = torch.Generator(device="cpu").manual_seed(7)
    idx = torch.randint(0, src_rows, (n,), generator=g, dtype=torch.int64).to(torch.int32).to(dev)
    grids = (1024, 2048, 4096, 8192)
    dst = torch.empty(max(n * 128, int(cl.acecalib_threads(max(grids))) * 16), dtype=torch.uint8, device=dev)
    stream = torch.cuda.current_stream()
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(2)]
    out = {"rows": n, "row_bytes": 128, "buffer_bytes": src_rows * 128}
    for read_only, key in ((1, "read_only_GBs"), (0, "copy_GBs")):
        best = 0.0
        for grid in grids:
            def launch():
                rc = cl.acecalib_gather_lines(src.data_ptr(), src_rows, idx.data_ptr(), n, dst.data_ptr(),
                                              read_only, grid, stream.cuda_stream)
                if rc:
                    raise RuntimeError("gather calibration launch failed: HIP error %d" % rc)
            launch()
            torch.cuda.synchronize()
            ev[0].record(stream)
            for _ in range(5):
                launch()
            ev[1].record(stream)
            torch.cuda.synchronize()
            sec = ev[0].elapsed_time(ev[1]) * 1e-3 / 5
            moved = n * 128 * (1 if read_only else 2)
            best = max(best, moved / sec / 1e9)
        out[key] = round(best, 1)
    del src, idx, dst
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--profile", default="mixed")
    ap.add_argument("--size", type=int, default=1 << 30)
    ap.add_argument("--seed", type=int, default=3)
    ap.add_argument("--block", type=int, default=16384)
    ap.add_argument("--interleave", type=int, default=0,
                    help="rANS interleave width W; 0 = pick W and the launch shape with the "
                         "autotuner on a 32 MiB sample of the workload")
    ap.add_argument("--min-match", type=int, default=16)
    ap.add_argument("--max-level", type=int, default=16)
    ap.add_argument("--mode", type=int, default=0,
                    help="0: the autotuner's choice (1 when W is given); 1: entropy decode of all "
                         "blocks, then one expansion launch per level; 2: entropy decode, then one "
                         "persistent expansion launch for every level; 3: entropy decode per level "
                         "group on a second stream beside the per-level expansion")
    ap.add_argument("--grid", type=int, default=-1,
                    help="mode 2: persistent workgroups (0 = all the device holds; -1 = tuned or 0)")
    ap.add_argument("--waves-per-block", type=int, default=0,
                    help="wavefronts per block in the match expansion (1, 2, 4, 8; 0 = chosen per launch by its size)")
    ap.add_argument("--per-wave", type=int, default=0,
                    help="entropy streams per wavefront (1, or 2 when W <= 32; 0 = library default)")
    ap.add_argument("--seek-requests", type=int, default=100_000)
    ap.add_argument("--plain-requests", type=int, default=2000,
                    help="requests timed one seek call each (the first ones of the same list)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-seek", action="store_true")
    ap.add_argument("--no-extras", action="store_true",
                    help="skip the 64 KiB-block and uncapped archives of the same corpus")
    ap.add_argument("--serve", action="store_true",
                    help="instead of the decode benchmark, run the serving loop: resident "
                         "genome/FASTQ/text/mixed archives, Poisson arrivals swept over rates")
    ap.add_argument("--serve-scale", type=float, default=1.0 / 16,
                    help="archive sizes as a fraction of 4/2/1/1 GiB")
    ap.add_argument("--serve-rates", default="1000,5000,20000,100000")
    ap.add_argument("--serve-count", type=int, default=3000)
    ap.add_argument("--serve-keep", default="-1",
                    help="serving: keep this many of each archive's lowest dependency levels "
                         "decoded per slot in its batch graphs (-1: none); 'host': host-planned "
                         "batched seeks instead of graphs; a comma-separated list runs each "
                         "setting in turn on the same archives")
    ap.add_argument("--suite", default="",
                    help="instead of the headline decode, run the other workloads and print one "
                         "JSON line each: genome1m (1 MiB genome, decode + every block sought with "
                         "the three-phase check), fastq256 (256 MiB FASTQ, 16 KiB blocks, cap 16)")
    ap.add_argument("--cache-dir", default="",
                    help="keep the generated input and the encoded archives in this folder and "
                         "reuse them when the same workload is asked for again (profiling runs)")
    ap.add_argument("--calib", action="store_true",
                    help="also run the calibration kernels after the decode: for the byte counters a "
                         "256 MiB fill, 64-bit sum and copy; for the scattered-line rate a gather of "
                         "8 Mi random 128-byte rows (reported under 'calibration')")
    args = ap.parse_args()

    if args.gpus != 1:
        print("bench.py measures one GPU only: the decode path runs on a single MI355X; "
              "run with --gpus 1.", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    import gen
    from paper_2606_24531_amd import Archive, encode
    from paper_2606_24531_amd import aceseek as ace

    dev = torch.device("cuda:0")
    if args.serve:
        return serve_main(args)
    if args.suite:
        return suite_main(args)
    os.environ.setdefault("ACESEEK_ENCODE_PROGRESS", "0")
    t0 = time.time()
    x = cached_bytes(args, "input-%s-%d-%d" % (args.profile, args.size, args.seed),
                     lambda: gen.by_name(args.profile, args.size, args.seed))
    _log("generated %d bytes of %s in %.1fs" % (len(x), args.profile, time.time() - t0))
    x_dev = torch.from_numpy(np.frombuffer(x, dtype=np.uint8).copy()).to(dev)
    tuned = None
    # the launch shape is tuned on the encoded archive itself unless given
    shape_given = bool(args.mode or args.waves_per_block or args.per_wave or args.grid >= 0)
    if args.interleave == 0:
        # the interleave width is an archive parameter: picked on a 32 MiB
        # sample, re-encoded per candidate
        from paper_2606_24531_amd.autotune import tune
        t0 = time.time()
        tuned = tune(x[:min(len(x), 32 << 20)], args.profile, block_size=args.block,
                     min_match=args.min_match, max_level=args.max_level, log=_log)
        args.interleave = tuned["interleave"]
        _log("autotune (%.1fs): W=%d on the sample" % (time.time() - t0, args.interleave))
    enc = dict(interleave=args.interleave, min_match=args.min_match, hash_len=args.min_match, max_chain=32)
    t0 = time.time()
    a = cached_archive(args, x, args.block, args.max_level, enc)
    enc_s = time.time() - t0
    _log("encoded to %d bytes (ratio %.3f) in %.1fs" % (len(a), len(x) / len(a), enc_s))
    arc = Archive(a, device=dev)
    shape_tuned = None
    if not shape_given and tuned is not None:
        from paper_2606_24531_amd.autotune import tune_archive
        t0 = time.time()
        shape_tuned = tune_archive(arc, x_dev, reps=5, log=_log)
        args.mode, args.waves_per_block = shape_tuned["mode"], shape_tuned["waves_per_block"]
        args.per_wave, args.grid = shape_tuned["blocks_per_wg"], shape_tuned["grid_wgs"]
        _log("autotune on the archive (%.1fs): mode %d, %s waves per block, %d streams per wave, grid %s" % (
            time.time() - t0, args.mode, args.waves_per_block or "auto", args.per_wave,
            args.grid if args.grid > 0 else "full"))
    if not args.mode:
        args.mode = 1
    args.grid = max(args.grid, 0)
    tuning = dict(mode=args.mode, waves_per_block=args.waves_per_block, blocks_per_wg=args.per_wave,
                  grid_wgs=args.grid)
    stream = torch.cuda.current_stream()
    d = decode_entry(arc, a, x_dev, tuning, args.steps, args.warmup, "headline")
    ms, ext = d["ms"], d["ext"]
    gbs = len(x) / (ms * 1e-3) / 1e9
    alg_bytes = len(a) + len(x) + ext
    achieved = alg_bytes / (ms * 1e-3) / 1e9
    _log("parity ok; depth %d, %d blocks, external source bytes %d" % (arc.depth, arc.n_blocks, ext))
    _log("decode %.3f ms/step, %.1f GB/s decompressed, %.1f GB/s of algorithmic bytes (%.1f%% of HBM peak)" % (
        ms, gbs, achieved, 100 * achieved / HBM_PEAK_GBS))

    # per-kernel durations from HIP events the library records on this stream
    # around the entropy launch and the expansion launches
    ace.set_timing(True)
    t_ent, t_mat = [], []
    for _ in range(args.steps):
        arc.decode_all(out=d["out"], ws=d["ws"], tuning=tuning)
        e, m = ace.last_timings()
        t_ent.append(e)
        t_mat.append(m)
    ace.set_timing(False)
    ms_ent, ms_mat = float(np.mean(t_ent)), float(np.mean(t_mat))
    tok = d["facts"]["token_bytes"]
    # Each kernel's share of the decode's algorithmic bytes: k_rans reads the
    # rANS-coded streams; k_expand writes the output, reads the match bytes of
    # earlier blocks and the streams stored raw (in place).  The decoded
    # streams k_rans writes and k_expand reads back are an intermediate of
    # this design, counted apart as overhead.
    share_exp = len(x) + ext + d["raw_in_place"]
    share_ent = d["coded"]
    phase = {
        "entropy": {"kernel": "k_rans", "launches_per_step": 2 if args.mode == 3 else 1,
                    "ms": round(ms_ent, 4), "alg_bytes": share_ent,
                    "achieved_GBs": round(share_ent / (ms_ent * 1e-3) / 1e9, 2),
                    "overhead_bytes_written": d["rans_decoded"]},
        "match": {"kernel": "k_persist" if args.mode == 2 else "k_expand",
                  "launches_per_step": 1 if args.mode == 2 else arc.depth, "ms": round(ms_mat, 4),
                  "alg_bytes": share_exp,
                  "achieved_GBs": round(share_exp / (ms_mat * 1e-3) / 1e9, 2),
                  "overhead_bytes_read": d["rans_decoded"]},
    }
    dom = max(phase, key=lambda k: phase[k]["ms"])
    _log("phases: entropy %.3f ms, match %.3f ms (dominant: %s)" % (ms_ent, ms_mat, dom))

    result_calib = None
    if args.calib:
        # counter calibration, each a kernel of its own with known bytes:
        # a fill (256 MiB written with 16-byte stores), a sum over 64-bit
        # words (256 MiB read), a copy (256 MiB read and 256 MiB written)
        src = torch.empty(256 << 20, dtype=torch.uint8, device=dev)
        src.fill_(1)
        torch.cuda.synchronize()
        _ = src.view(torch.int64).sum()
        torch.cuda.synchronize()
        dst = src.clone()
        torch.cuda.synchronize()
        del dst
        _log("calibration fill, sum and copy of 256 MiB done")
        result_calib = gather_calibration(dev)
        _log("calibration gather of random 128-byte rows: read only %.0f GB/s, "
             "copy %.0f GB/s (reads + writes)" % (result_calib["read_only_GBs"], result_calib["copy_GBs"]))

    workload = "%s %d MiB, %d KiB blocks, %d-way rANS, level cap %d" % (
        args.profile, args.size >> 20, args.block >> 10, args.interleave, args.max_level)
    dk = phase[dom]
    traffic = measured_traffic(dk["kernel"], workload)
    result = {
        "metric": "2-layer decode GB/s (full archive)",
        "value": round(gbs, 2),
        "unit": "GB/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "u8",
        "data": "synthetic",
        "config": {
            "workload": workload,
            "n_total": len(x), "archive_bytes": len(a), "ratio": round(len(x) / len(a), 4),
            "block_size": args.block, "interleave": args.interleave,
            "max_level": args.max_level, "depth": arc.depth, "n_blocks": arc.n_blocks,
            "waves_per_block": args.waves_per_block or "auto",
            "streams_per_wave": args.per_wave or (2 if args.interleave <= 32 else 1),
            "autotuned": tuned is not None, "encode_s": round(enc_s, 1),
            "autotune": None if tuned is None else {
                "interleave_on_sample": {"chosen": tuned["interleave"], "sample_bytes": min(len(x), 32 << 20)},
                "shape_on_archive": None if shape_tuned is None else {
                    "chosen": {k: shape_tuned[k] for k in ("mode", "waves_per_block", "blocks_per_wg", "grid_wgs")},
                    "candidates_ms": [{k: r[k] for k in ("mode", "waves_per_block", "blocks_per_wg", "grid_wgs", "ms")}
                                      for r in shape_tuned["all"]]}},
            "dag": _dag_facts(a),
            "mode": {1: "entropy launch, then one expansion launch per level, one stream",
                     2: "entropy launch, then one persistent expansion launch for every level",
                     3: "per-level launches, entropy overlapped on a second stream"}[args.mode],
            "grid_wgs": args.grid if args.mode == 2 else None,
        },
        "roofline": {
            "bound": "hbm", "kernel": dk["kernel"],
            "achieved": dk["achieved_GBs"], "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": round(dk["achieved_GBs"] / HBM_PEAK_GBS, 4),
            "traffic": traffic,
            "traffic_unit": "HBM bytes per step (all launches of the kernel)",
            "traffic_GBs": None if traffic is None else round(traffic / (dk["ms"] * 1e-3) / 1e9, 1),
            "traffic_frac": None if traffic is None else round(traffic / (dk["ms"] * 1e-3) / 1e9 / HBM_PEAK_GBS, 4),
            "alg_bytes_per_step": dk["alg_bytes"],
            "phases": phase,
            "path": {"alg_bytes_per_step": alg_bytes, "achieved": round(achieved, 2),
                     "frac": round(achieved / HBM_PEAK_GBS, 4),
                     "archive_bytes": len(a), "output_bytes": len(x), "ext_src_bytes": ext,
                     "token_bytes": tok},
        },
    }

    if result_calib is not None:
        result["calibration"] = result_calib
    return finish(args, result, x, x_dev, a, arc, tuning, enc, d)


def encode_leg(x, enc) -> dict:
    """The encoder's entropy step on the host and on the device, on the first
    64 MiB of the workload: encode wall time with every stream left raw (the
    parse and layout alone), with the host's rANS step and with the device's
    (ENC_DEVICE_ENTROPY), median of 3 each; the two coded archives must be
    equal.  Entropy time = coded encode - raw encode."""
    import numpy as np
    from paper_2606_24531_amd import aceseek
    sample = x[:64 << 20]
    kw = dict(enc)
    flags = kw.pop("flags", 0) & ~3

    def t(f):
        ts, out = [], None
        for _ in range(3):
            t0 = time.perf_counter()
            out = aceseek.encode(sample, flags=f, **kw)
            ts.append(time.perf_counter() - t0)
        return float(np.median(ts)), out

    t_raw, _ = t(flags | 2)
    t_host, a_host = t(flags)
    t_dev, a_dev = t(flags | aceseek.ENC_DEVICE_ENTROPY)
    res = {"sample_bytes": len(sample), "raw_s": round(t_raw, 3), "host_entropy_s": round(t_host, 3),
           "device_entropy_s": round(t_dev, 3), "entropy_host_s": round(t_host - t_raw, 3),
           "entropy_device_s": round(t_dev - t_raw, 3), "archives_equal": a_host == a_dev}
    _log("encode of 64 MiB: parse and layout %.2f s; rANS step on the host %.2f s, on the device %.2f s "
         "(archives equal: %s)" % (t_raw, t_host - t_raw, t_dev - t_raw, res["archives_equal"]))
    return res


def range_decode_leg(a, arc, x_dev, tuning) -> dict:
    """Range decode of blocks 0..1000 (the paper's at-scale range), from the
    resident archive and out of core (the archive in host memory, the
    range's closure staged per call), and single-block out-of-core seeks;
    every output compared with the original.  Wall clock around calls that
    are waited on, median of 5 (single blocks: 200 uniform blocks, seed 6)."""
    import numpy as np
    import torch
    from paper_2606_24531_amd import OutOfCoreArchive
    B = arc.block_size
    lo, hi = 0, min(arc.n_total, 1001 * B)
    dev = x_dev.device
    out = torch.empty(hi - lo, dtype=torch.uint8, device=dev)
    ws = torch.zeros(max(arc.seek_device_bytes(), arc.workspace_bytes([lo, hi])), dtype=torch.uint8, device=dev)

    def timed(fn, reps=5):
        fn()
        torch.cuda.synchronize()
        t = []
        for _ in range(reps):
            t0 = time.perf_counter()
            fn()
            torch.cuda.synchronize()
            t.append(time.perf_counter() - t0)
        return float(np.median(t))

    res = {"range": [lo, hi], "blocks": (hi - lo + B - 1) // B}
    t_res = timed(lambda: arc.seek(lo, hi, out=out, ws=ws, tuning=tuning, plan="host"))
    arc.check(ws)
    res["resident_ms"] = round(1e3 * t_res, 4)
    res["resident_equal"] = bool(torch.equal(out, x_dev[lo:hi]))
    ooc = OutOfCoreArchive(a, device=dev)
    t_ooc = timed(lambda: ooc.seek(lo, hi, out=out, tuning=tuning))
    ooc.check()
    res["ooc_ms"] = round(1e3 * t_ooc, 4)
    res["ooc_equal"] = bool(torch.equal(out, x_dev[lo:hi]))
    res["ooc_workspace_bytes"] = ooc.workspace_bytes(lo, hi)
    rng = np.random.default_rng(6)
    lat, ok, staged = [], True, []
    for b in rng.integers(0, arc.n_blocks, 200):
        l0, h0 = int(b) * B, min(arc.n_total, (int(b) + 1) * B)
        t0 = time.perf_counter()
        r = ooc.seek(l0, h0, out=out[:h0 - l0], tuning=tuning)
        lat.append(time.perf_counter() - t0)
        ok = ok and bool(torch.equal(r, x_dev[l0:h0]))
        staged.append(ooc.workspace_bytes(l0, h0))
    ooc.check()
    ooc.close()
    res["ooc_single_block"] = {"p50_ms": round(1e3 * float(np.percentile(lat, 50)), 4),
                               "p99_ms": round(1e3 * float(np.percentile(lat, 99)), 4),
                               "workspace_bytes_p50": int(np.median(staged)), "outputs_equal_original": ok}
    _log("range decode of blocks 0..1000: resident %.3f ms, out of core %.3f ms (workspace %.1f MB, equal %s/%s); "
         "out-of-core single blocks p50 %.3f ms p99 %.3f ms" % (
             res["resident_ms"], res["ooc_ms"], res["ooc_workspace_bytes"] / 1e6, res["resident_equal"],
             res["ooc_equal"], res["ooc_single_block"]["p50_ms"], res["ooc_single_block"]["p99_ms"]))
    del out, ws
    torch.cuda.empty_cache()
    return res


def finish(args, result, x, x_dev, a, arc, tuning, enc, d):
    """The rest of the default line: the same corpus at 64 KiB blocks and
    uncapped, the batched-vs-plain seeks, and the CPU oracle baseline."""
    import numpy as np
    import torch

    import gen
    from paper_2606_24531_amd import Archive, encode
    from paper_2606_24531_amd import aceseek as ace

    dev = x_dev.device
    if not args.no_extras:
        extras = {}
        for key, B, cap, steps in (("blocks_64k", 65536, args.max_level, args.steps),
                                   ("uncapped", args.block, 0, 3)):
            t0 = time.time()
            ax = cached_archive(args, x, B, cap, enc)
            enc_s = time.time() - t0
            arcx = Archive(ax, device=dev)
            e = decode_entry(arcx, ax, x_dev, tuning, steps, 1, key)
            algx = len(ax) + len(x) + e["ext"]
            extras[key] = {
                "workload": "%s %d MiB, %d KiB blocks, %d-way rANS, %s" % (
                    args.profile, len(x) >> 20, B >> 10, args.interleave,
                    "level cap %d" % cap if cap else "uncapped"),
                "ms_per_step": round(e["ms"], 4), "steps": steps,
                "value": round(len(x) / (e["ms"] * 1e-3) / 1e9, 2), "unit": "GB/s",
                "ratio": round(len(x) / len(ax), 4), "depth": arcx.depth, "n_blocks": arcx.n_blocks,
                "path_frac": round(algx / (e["ms"] * 1e-3) / 1e9 / HBM_PEAK_GBS, 4),
                "ext_src_bytes": e["ext"], "encode_s": round(enc_s, 1), "parity": e["ok"],
                "dag": _dag_facts(ax)}
            _log("%s: ratio %.3f, depth %d, decode %.3f ms (%.1f GB/s)" % (
                key, len(x) / len(ax), arcx.depth, e["ms"], len(x) / e["ms"] / 1e6))
            del e
            arcx.close()
            del ax
            torch.cuda.empty_cache()
        result["extras"] = extras

    if not args.no_seek:
        n_req = args.seek_requests
        lo, hi = gen.seek_requests(len(x), n_req, 4, max_len=4 << 20)
        ln = (hi - lo).astype(np.int64)
        offs = np.concatenate([[0], np.cumsum(ln)[:-1]]).astype(np.uint64)
        total = int(ln.sum())
        out = torch.empty(total, dtype=torch.uint8, device=dev)
        # batched: every request in one replay of the captured batch graph
        bt = arc.batch(n_req, tuning=tuning)
        bt.run((lo, hi), out, offs)
        torch.cuda.synchronize()
        bt.check()
        good = all(bool(torch.equal(out[int(offs[i]):int(offs[i]) + int(ln[i])], x_dev[int(lo[i]):int(hi[i])]))
                   for i in range(n_req))
        times = []
        for _ in range(3):
            t = time.perf_counter()
            bt.run((lo, hi), out, offs)
            torch.cuda.synchronize()
            times.append(time.perf_counter() - t)
        bt.check()
        bt.close()
        tb = float(np.median(times))
        # plain: one seek call (its own plan and launches) per request, waited
        # on; the first plain_requests requests of the same list.  Planned on
        # the device (the archive's plan resident, a workspace of
        # seek_device_bytes) and, as before, on the host (closure walk).
        n_plain = min(args.plain_requests, n_req)
        ws = torch.zeros(max(arc.seek_device_bytes(), arc.workspace_bytes([0, len(x)])), dtype=torch.uint8,
                         device=dev)

        def plain(planner):
            lat = []
            for i in range(n_plain):
                t = time.perf_counter()
                arc.seek(int(lo[i]), int(hi[i]), out=out[int(offs[i]):], ws=ws, tuning=tuning, plan=planner)
                torch.cuda.synchronize()
                lat.append(time.perf_counter() - t)
            arc.check(ws)
            ok = all(bool(torch.equal(out[int(offs[i]):int(offs[i]) + int(ln[i])], x_dev[int(lo[i]):int(hi[i])]))
                     for i in range(n_plain))
            # where the time goes, on the first requests again: host planning
            # and enqueueing (library clocks), device phases (events)
            ace.set_timing(True)
            plan_us, enq_us, dev_ms = [], [], []
            for i in range(min(n_plain, 300)):
                arc.seek(int(lo[i]), int(hi[i]), out=out[int(offs[i]):], ws=ws, tuning=tuning, plan=planner)
                torch.cuda.synchronize()
                p_us, e_us = ace.last_host_times()
                e_ms, m_ms = ace.last_timings()
                plan_us.append(p_us)
                enq_us.append(e_us)
                dev_ms.append(e_ms + m_ms)
            ace.set_timing(False)
            p50 = float(np.percentile(lat, 50))
            return {
                "p50_ms": round(1e3 * p50, 4), "p99_ms": round(1e3 * float(np.percentile(lat, 99)), 4),
                "req_per_s": round(n_plain / sum(lat), 1), "outputs_equal_original": ok,
                "host_plan_us_p50": round(float(np.median(plan_us)), 1),
                "host_enqueue_us_p50": round(float(np.median(enq_us)), 1),
                "device_decode_ms_p50": round(float(np.median(dev_ms)), 4),
                "plan_share_of_p50": round(float(np.median(plan_us)) * 1e-6 / p50, 4),
            }

        pd = plain("device")
        ph = plain("host")
        result["seek"] = {
            "workload": "%d seeks on the resident archive, length log-uniform 1 B..4 MiB, uniform "
                        "offsets (seed 4)" % n_req,
            "requests": n_req, "output_bytes": total,
            "batched_latency_ms": round(1e3 * tb, 4), "batched_req_per_s": round(n_req / tb, 1),
            "batched_out_GBs": round(total / tb / 1e9, 2), "batched_outputs_equal_original": good,
            "plain_requests_timed": n_plain,
            "plain_p50_ms": pd["p50_ms"], "plain_p99_ms": pd["p99_ms"], "plain_req_per_s": pd["req_per_s"],
            "batched_vs_plain_throughput": round((n_req / tb) / pd["req_per_s"], 1),
            "plain_device_planned": pd, "plain_host_planned": ph,
        }
        _log("seek: batch of %d in %.3f ms (%.0f req/s, all outputs equal: %s)" % (n_req, 1e3 * tb, n_req / tb, good))
        for name, r in (("device", pd), ("host", ph)):
            _log("plain %s-planned: p50 %.3f ms p99 %.3f ms (%.0f req/s, equal %s); host planning p50 %.1f us "
                 "(%.1f%% of p50), enqueue %.1f us, device decode %.3f ms" % (
                     name, r["p50_ms"], r["p99_ms"], r["req_per_s"], r["outputs_equal_original"],
                     r["host_plan_us_p50"], 100 * r["plan_share_of_p50"], r["host_enqueue_us_p50"],
                     r["device_decode_ms_p50"]))
        del out
        torch.cuda.empty_cache()
        result["range_decode"] = range_decode_leg(a, arc, x_dev, tuning)
        result["encode"] = encode_leg(x, dict(enc, block_size=args.block, max_level=args.max_level))

    if not args.no_cpu_baseline:
        import oracle
        oracle.build()
        t = time.perf_counter()
        y, used = oracle.decode_levels(a, 0)
        t_all = time.perf_counter() - t
        assert y == x
        del y
        # one core: the sequential decoder on the first quarter of the
        # archive's blocks would need a second archive; it decodes the whole
        # archive once instead (bounded: about 5 s at 0.2 GB/s)
        t = time.perf_counter()
        y1 = oracle.decode(a)
        t_one = time.perf_counter() - t
        assert y1 == x
        del y1
        # single seeks on one core: the oracle's seek (its closure, decoded in
        # order) on the first requests of the seek list, bounded to ~10 s
        lo_s, hi_s = gen.seek_requests(len(x), 200, 4, max_len=4 << 20)
        seek_ms = []
        t_end = time.perf_counter() + 10.0
        for i in range(len(lo_s)):
            if seek_ms and time.perf_counter() > t_end:
                break
            t = time.perf_counter()
            got = oracle.seek(a, int(lo_s[i]), int(hi_s[i]))
            seek_ms.append(1e3 * (time.perf_counter() - t))
            assert got == x[int(lo_s[i]):int(hi_s[i])]
        result["cpu_baseline"] = dict({
            "value": round(len(x) / t_all / 1e9, 4), "unit": "GB/s", "cores": used, "kind": "oracle",
            "sample": "one full decode of the same archive, the blocks of each dependency level "
                      "decoded in parallel (OpenMP)",
            "one_core_GBs": round(len(x) / t_one / 1e9, 4),
            "one_core_seek_p50_ms": round(float(np.percentile(seek_ms, 50)), 3),
            "one_core_seek_p99_ms": round(float(np.percentile(seek_ms, 99)), 3),
            "seek_sample": "the first %d requests of the seek list (seed 4), oracle seek on one core"
                           % len(seek_ms),
            "oracle_flags": " ".join(oracle.CFLAGS)}, **cpu_facts())
        _log("cpu oracle: %.3f GB/s on %d threads, %.3f GB/s on one; one-core seek p50 %.1f ms over %d" % (
            result["cpu_baseline"]["value"], used, result["cpu_baseline"]["one_core_GBs"],
            result["cpu_baseline"]["one_core_seek_p50_ms"], len(seek_ms)))

    print(json.dumps(result), flush=True)


def serve_main(args):
    """Serving loop: four resident archives (genome, FASTQ, text, mixed), Poisson
    seek arrivals at each rate, lengths log-uniform in 16 B..16 MiB, a 32 GiB
    output budget, K in-flight slots on their own streams."""
    import numpy as np
    import torch

    import gen
    from paper_2606_24531_amd import Archive, encode
    from paper_2606_24531_amd.serve import GpuBackend, Server, latency_report, limiter, poisson_run

    sizes = {"genome": 4 << 30, "fastq": 2 << 30, "text": 1 << 30, "mixed": 1 << 30}
    seeds = {"genome": 51, "fastq": 52, "text": 53, "mixed": 3}
    mm = {"genome": 20, "fastq": 20, "text": 16, "mixed": 16}
    arcs, n_total = {}, {}
    for name, full in sizes.items():
        n = int(full * args.serve_scale)
        t0 = time.time()
        _log("%s: generating %d bytes" % (name, n))
        x = gen.by_name(name, n, seeds[name])
        a = encode(x, block_size=args.block, interleave=args.interleave or 64, min_match=mm[name],
                   hash_len=mm[name], max_chain=32, max_level=args.max_level)
        arcs[name] = Archive(a, device="cuda:0")
        n_total[name] = n
        _log("%s: %d bytes, ratio %.3f, %.1fs" % (name, n, n / len(a), time.time() - t0))
        del x
    rates = [float(r) for r in args.serve_rates.split(",")]
    budget = 32 << 30
    for keep_arg in str(args.serve_keep).split(","):
        host = keep_arg.strip() == "host"
        keep = None if host or int(keep_arg) < 0 else int(keep_arg)
        runs = []
        backend = GpuBackend(arcs, slots=4, keep_levels=keep, max_batch=4096, batch_bytes=budget,
                             host_planned=host)
        dev_bytes = backend.device_bytes()
        _log("%s, kept levels %s: device memory held by the server %s, output budget %d" % (
            "host-planned batches" if host else "batch graphs", keep, dev_bytes, budget))
        for rate in rates:
            # every 97th result is compared with a solo seek of the same range
            # after the run; results are released as they complete, which
            # returns their bytes to the budget
            sample = {}
            srv = Server(backend, budget_bytes=budget, slots=4, max_batch=4096, auto_release=True,
                         on_done=lambda r: r.rid % 97 == 0 and sample.__setitem__(r.rid, r.result.cpu()))
            reqs, wall = poisson_run(srv, list(arcs), n_total, rate=rate, count=args.serve_count,
                                     seed=int(rate), min_len=16, max_len=16 << 20)
            torch.cuda.synchronize()
            rep = latency_report(reqs, wall)
            ok = True
            for r in reqs:
                if r.rid in sample:
                    solo = arcs[r.archive].seek(r.lo, r.hi)
                    ok = ok and bool(torch.equal(solo.cpu(), sample[r.rid]))
            rep.update(offered_req_per_s=rate, batches=srv.batches, peak_out_bytes=srv.peak_used,
                       sampled_results_equal_solo_seek=ok, n_sampled=len(sample), **limiter(srv))
            runs.append(rep)
            _log("rate %.0f/s: p50 %.3f ms p99 %.3f ms, %.0f req/s, limiter %s" % (
                rate, rep["p50_ms"], rep["p99_ms"], rep["req_per_s"], rep["limiter"]))
        print(json.dumps({
            "metric": "seek latency p50/p99 vs throughput (serving loop)", "unit": "ms",
            "n_gpus": 1, "data": "synthetic", "higher_is_better": False,
            "config": {"workload": "resident genome/fastq/text/mixed archives at %.4g of 4/2/1/1 GiB, "
                                   "Poisson arrivals, 16 B..16 MiB log-uniform, 32 GiB budget, 4 slots"
                                   % args.serve_scale,
                       "planning": "host" if host else "device (batch graphs)",
                       "kept_levels": keep, "output_budget_bytes": budget, "device_bytes": dev_bytes},
            "runs": runs}), flush=True)
        del backend
        torch.cuda.empty_cache()


def _dag_facts(a: bytes) -> dict:
    """Depth, level sizes, dependency out-degree and single-block closure
    sizes, read from an archive's index (closures by a frontier walk over the
    dependency lists, which always point to lower levels)."""
    import struct

    import numpy as np
    nb = struct.unpack_from("<I", a, 24)[0]
    depth = struct.unpack_from("<I", a, 28)[0]
    n_deps = struct.unpack_from("<I", a, 36)[0]
    ent = np.frombuffer(a, dtype=np.uint32, count=8 * nb, offset=64).reshape(nb, 8)
    level, dep_off, dep_cnt = ent[:, 4], ent[:, 5].astype(np.int64), ent[:, 6].astype(np.int64)
    deps = np.frombuffer(a, dtype=np.uint32, count=n_deps, offset=64 + 32 * nb)

    def closure(b):
        need = np.zeros(nb, dtype=bool)
        need[b] = True
        front = np.array([b], dtype=np.int64)
        while front.size:
            cnt, off = dep_cnt[front], dep_off[front]
            if not cnt.sum():
                break
            start = np.repeat(off - (np.cumsum(cnt) - cnt), cnt)
            d = deps[start + np.arange(cnt.sum())].astype(np.int64)
            d = np.unique(d[~need[d]])
            need[d] = True
            front = d
        return int(need.sum())

    rng = np.random.default_rng(7)
    clos = [closure(int(b)) for b in rng.integers(0, nb, 100)]
    return {"depth": int(depth), "n_blocks": int(nb),
            "level_sizes": np.bincount(level, minlength=depth).tolist()[:64],
            "deps_per_block_mean": round(float(dep_cnt.mean()), 2), "deps_per_block_max": int(dep_cnt.max()),
            "closure_single_block_p50": float(np.median(clos)), "closure_single_block_max": int(max(clos))}


def _time_decode(arc, x_dev, tuning, steps):
    import torch
    out = torch.empty(arc.n_total, dtype=torch.uint8, device=arc.device)
    ws = arc.workspace(arc.workspace_bytes())
    arc.decode_all(out=out, ws=ws, tuning=tuning)
    arc.check(ws)
    ok = bool(torch.equal(out, x_dev))
    for _ in range(3):
        arc.decode_all(out=out, ws=ws, tuning=tuning)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(steps):
        arc.decode_all(out=out, ws=ws, tuning=tuning)
    e1.record()
    torch.cuda.synchronize()
    arc.check(ws)
    return e0.elapsed_time(e1) / steps, ok


def suite_main(args):
    import numpy as np
    import torch

    import gen
    from paper_2606_24531_amd import Archive, encode
    from paper_2606_24531_amd.autotune import tune

    dev = torch.device("cuda:0")
    which = set(args.suite.split(","))
    os.environ.setdefault("ACESEEK_ENCODE_PROGRESS", "1")  # 1 GiB encodes take a while

    def emit(d):
        d.update(n_gpus=1, data="synthetic", dtype="u8")
        print(json.dumps(d), flush=True)

    if "genome1m" in which:
        x = gen.genome(1 << 20, 1)
        a = encode(x, block_size=16384, interleave=32, min_match=20, hash_len=20, max_chain=32)
        arc = Archive(a, device=dev)
        xd = torch.frombuffer(bytearray(x), dtype=torch.uint8).to(dev)
        ms, ok = _time_decode(arc, xd, dict(mode=1), 20)
        lat, good = [], True
        for b in range(arc.n_blocks):
            lo, hi = b * 16384, min(len(x), (b + 1) * 16384)
            # the paper's three-phase check on the device: a seeded sentinel
            # everywhere, the region differs before, equals the original
            # after, and nothing outside it moved (the seek alone is timed)
            g = torch.Generator(device=dev)
            g.manual_seed(1000 + b)
            buf = torch.randint(0, 256, (len(x),), dtype=torch.uint8, device=dev, generator=g)
            before = buf.clone()
            phase1 = not torch.equal(buf[lo:hi], xd[lo:hi])
            torch.cuda.synchronize()
            t = time.perf_counter()
            arc.seek(lo, hi, out=buf[lo:], tuning=dict(mode=1))
            torch.cuda.synchronize()
            lat.append(time.perf_counter() - t)
            arc.check()
            good = good and phase1 and torch.equal(buf[lo:hi], xd[lo:hi]) and \
                torch.equal(buf[:lo], before[:lo]) and torch.equal(buf[hi:], before[hi:])
        _log("genome1m: decode %.4f ms, %d block seeks, three-phase %s" % (ms, arc.n_blocks, good))
        emit({"metric": "2-layer decode GB/s (full archive); single-block seek latency",
              "config": {"workload": "genome 1 MiB, 16 KiB blocks, 32-way rANS, uncapped",
                         "ratio": round(len(x) / len(a), 4), "depth": arc.depth},
              "value": round(len(x) / ms / 1e6, 3), "unit": "GB/s", "ms_per_step": round(ms, 4),
              "parity": ok, "seek_p50_ms": round(1e3 * float(np.median(lat)), 4),
              "seek_p99_ms": round(1e3 * float(np.percentile(lat, 99)), 4),
              "three_phase_all_blocks": good})
    if "fastq256" in which:
        # 256 MiB FASTQ-like records, 16 KiB blocks, cap 16 (the FASTQ profile alone)
        x = gen.fastq(256 << 20, 2)
        tuned = tune(x[:32 << 20], "fastq", block_size=16384, min_match=20, max_level=16)
        a = encode(x, block_size=16384, interleave=tuned["interleave"], min_match=20, hash_len=20,
                   max_chain=32, max_level=16)
        arc = Archive(a, device=dev)
        xd = torch.from_numpy(np.frombuffer(x, dtype=np.uint8).copy()).to(dev)
        shape = dict(mode=tuned["mode"], waves_per_block=tuned["waves_per_block"],
                     blocks_per_wg=tuned["blocks_per_wg"], grid_wgs=tuned["grid_wgs"])
        ms, ok = _time_decode(arc, xd, shape, 20)
        _log("fastq256: ratio %.3f, depth %d, decode %.3f ms (%.1f GB/s), parity %s" % (
            len(x) / len(a), arc.depth, ms, len(x) / ms / 1e6, ok))
        emit({"metric": "2-layer decode GB/s (full archive)",
              "config": {"workload": "fastq 256 MiB, 16 KiB blocks, %d-way rANS, level cap 16" % tuned["interleave"],
                         "ratio": round(len(x) / len(a), 4), "depth": arc.depth},
              "value": round(len(x) / ms / 1e6, 2), "unit": "GB/s", "ms_per_step": round(ms, 4),
              "parity": ok, "tuning": shape})


if __name__ == "__main__":
    main()
