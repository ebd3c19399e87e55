"""The library's own HIP kernels and host code, built for the CPU (tests/simt)
and executed lane by lane, against the oracle.  No GPU: this checks the
kernels' logic (cross-lane operations, barriers, LDS tables, every array
index bounds-checked) on the host before any device run.  Each case runs in
a child process, because a bounds violation stops the process that hits it."""
import os
import subprocess
import sys

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)

CASES = [
    # profile, n, B, W, cap, flags, min_match, mode
    ("genome", 1 << 20, 16384, 32, 0, 0, 20, 1),      # the small workload: 64 blocks, 27 levels
    ("fastq", 600_000, 16384, 64, 16, 0, 20, 1),
    ("text", 300_000, 4096, 32, 8, 1, 16, 3),
    ("mixed", 700_001, 16384, 64, 0, 4, 16, 1),        # 8-byte offsets
    ("genome", 200_003, 1000, 7, 0, 2, 20, 1),         # non-power-of-two blocks, raw streams
    ("genome", 8_000_000, 4096, 32, 0, 0, 10, 1),      # up to ~330 dependencies per block
    # the persistent level-by-level kernel (one launch, device-side counters)
    ("genome", 1 << 20, 16384, 32, 0, 0, 20, 2),
    ("mixed", 3_000_001, 16384, 32, 0, 0, 16, 2),      # uncapped: 50+ levels
    ("fastq", 600_000, 16384, 64, 16, 0, 20, 2),
    ("text", 300_000, 4096, 32, 8, 1, 16, 2),
    ("genome", 200_003, 1000, 7, 0, 2, 20, 2),
    ("text", 40_000, 37, 3, 0, 0, 4, 2),                # tiny blocks: a thousand of them
]

_WORKER = r"""
import sys
sys.path.insert(0, %(root)r); sys.path.insert(0, %(tests)r)
import gen, oracle, simt_lib
name, n, B, W, cap, flags, mm, mode = %(case)r
from paper_2606_24531_amd import encode
x = gen.by_name(name, n, 31)
a = encode(x, block_size=B, interleave=W, min_match=mm, hash_len=min(mm, 16), max_level=cap, flags=flags)
arc = simt_lib.Archive(a)
got = arc.decode_all(dict(mode=mode))
assert got == x, "decode differs from the original"
lo, hi = n // 3, n // 3 + 2 * B + 17
assert arc.seek(lo, hi, dict(mode=mode)) == x[lo:hi], "seek differs from the original"
if n <= (4 << 20):
    assert oracle.decode(a) == x, "the oracle disagrees"
    # a captured batch graph (device-side planning, strided launches), replayed
    lo_r, hi_r = gen.seek_requests(n, 9, 3, max_len=3 * B)
    got_b = simt_lib.seek_batch_graph(arc, lo_r, hi_r, dict(mode=mode if mode != 3 else 1))
    assert all(g == x[int(l):int(h)] for g, l, h in zip(got_b, lo_r, hi_r)), "batch graph differs"
    # single seeks planned on the device (the plan attached)
    for l, h in list(zip(lo_r, hi_r))[:4] + [(0, n), (n - 1, n)]:
        assert arc.seek_device(int(l), int(h), dict(mode=mode)) == x[int(l):int(h)], "device-planned seek differs"
print("OK", arc.n_blocks, arc.depth)
"""


@pytest.fixture(scope="module", autouse=True)
def built():
    sys.path.insert(0, os.path.join(HERE, "simt"))
    import build as simt_build
    simt_build.build()
    import oracle
    oracle.build()


@pytest.mark.parametrize("case", CASES, ids=lambda c: "%s-n%d-B%d-W%d-cap%d-f%d-mode%d" % (c[:6] + c[7:]))
def test_cpu_build_of_kernels_matches_oracle(case):
    code = _WORKER % {"root": ROOT, "tests": HERE, "case": case}
    # persistent-kernel cases run with few and with many concurrent workgroups
    for resident in (("3", "16") if case[7] == 2 else ("8",)):
        r = subprocess.run([sys.executable, "-c", code], capture_output=True, text=True, timeout=600,
                           env=dict(os.environ, SIMT_RESIDENT=resident))
        assert r.returncode == 0 and "OK" in r.stdout, (resident, r.returncode, r.stdout[-2000:], r.stderr[-2000:])


def _ext_bytes_reference(orc, a: bytes) -> int:
    """Match bytes whose origin, followed back through this block's own
    literals and matches, lies in an earlier block (the decode's reads from
    earlier blocks, with every block expanded as one tile)."""
    import numpy as np
    info = orc.info(a)
    B, nb = info["block_size"], info["n_blocks"]
    total = 0
    for b in range(nb):
        lit, L, M, O = orc.block_tokens(a, b)
        L, M, O = L.astype(np.int64), M.astype(np.int64), O.astype(np.int64)
        bs = b * B
        start = np.concatenate([[0], np.cumsum(L + M)[:-1]])
        mstart = bs + start + L  # absolute start of each match
        d = mstart - O
        k = np.repeat(np.arange(len(M)), M)  # every match byte: its sequence
        i = np.arange(len(k)) - np.repeat(np.cumsum(M) - M, M)
        src = O[k] + i % d[k]
        live = np.ones(len(k), dtype=bool)
        while live.any():
            ext = live & (src < bs)
            total += int(ext.sum())
            live &= ~ext
            q = src[live] - bs
            s = np.searchsorted(start, q, side="right") - 1
            r = q - start[s]
            in_match = r >= L[s]
            idx = np.where(live)[0]
            live[idx[~in_match]] = False  # a literal: not from an earlier block
            idx = idx[in_match]
            s, r = s[in_match], r[in_match]
            ii = r - L[s]
            src[idx] = O[s] + ii % d[s]
    return total


@pytest.mark.parametrize("name,n,B,mm", [("genome", 6 << 20, 16384, 20), ("mixed", 2_000_001, 16384, 16),
                                         ("text", 500_000, 4096, 12)])
def test_ext_counter_matches_origin_count(orc, name, n, B, mm):
    """The workspace counter of match bytes read from earlier blocks (the
    S_ext term of the algorithmic bytes) equals the count of match bytes
    whose origin lies in an earlier block, with 512-thread workgroups (one
    tile per block for these archives)."""
    code = r"""
import sys
sys.path.insert(0, %(root)r); sys.path.insert(0, %(tests)r)
import gen, simt_lib
from paper_2606_24531_amd import encode
x = gen.by_name(%(name)r, %(n)d, 41)
a = encode(x, block_size=%(B)d, interleave=32, min_match=%(mm)d, hash_len=%(mm)d, max_level=8)
open(%(path)r, "wb").write(a)
arc = simt_lib.Archive(a)
y, ext = simt_lib.decode_all_ext(arc, dict(mode=1, waves_per_block=8))
assert y == x
print("EXT", ext)
"""
    import tempfile
    with tempfile.TemporaryDirectory() as td:
        path = os.path.join(td, "a.bin")
        r = subprocess.run([sys.executable, "-c", code % dict(root=ROOT, tests=HERE, name=name, n=n, B=B, mm=mm,
                                                              path=path)],
                           capture_output=True, text=True, timeout=600)
        assert r.returncode == 0, r.stderr[-2000:]
        ext = int(r.stdout.split("EXT")[1].split()[0])
        a = open(path, "rb").read()
    info = orc.info(a)
    assert max(orc.block_facts(a)[1]) <= 1024  # one tile per block
    assert ext == _ext_bytes_reference(orc, a)


def test_short_period_slow_matches(orc):
    """Short-period matches whose span lies in the previous match (their
    bytes resolved in the slow pass, period wrap by period wrap) decode to
    the original bytes, and the earlier-block byte counter still equals the
    origin count."""
    import numpy as np
    import gen
    x = gen.by_name("tandem", 3_000_000, 5)
    code = r"""
import sys
sys.path.insert(0, %(root)r); sys.path.insert(0, %(tests)r)
import simt_lib
x = open(%(xpath)r, "rb").read()
from paper_2606_24531_amd import encode
a = encode(x, block_size=16384, interleave=32, min_match=16, hash_len=16, max_level=8)
open(%(path)r, "wb").write(a)
arc = simt_lib.Archive(a)
y, ext = simt_lib.decode_all_ext(arc, dict(mode=1, waves_per_block=8))
assert y == x
assert arc.decode_all(dict(mode=1, waves_per_block=2)) == x
print("EXT", ext)
"""
    import tempfile
    with tempfile.TemporaryDirectory() as td:
        path, xpath = os.path.join(td, "a.bin"), os.path.join(td, "x.bin")
        open(xpath, "wb").write(x)
        r = subprocess.run([sys.executable, "-c", code % dict(root=ROOT, tests=HERE, path=path, xpath=xpath)],
                           capture_output=True, text=True, timeout=600)
        assert r.returncode == 0, r.stderr[-2000:]
        ext = int(r.stdout.split("EXT")[1].split()[0])
        a = open(path, "rb").read()
    # the premise: many matches with a period under 16 whose span reaches
    # back past their own literals into the sequence before
    info = orc.info(a)
    n_short = 0
    for b in range(info["n_blocks"]):
        lit, L, M, O = orc.block_tokens(a, b)
        L, M, O = L.astype(np.int64), M.astype(np.int64), O.astype(np.int64)
        mstart = b * info["block_size"] + np.concatenate([[0], np.cumsum(L + M)[:-1]]) + L
        d = mstart - O
        n_short += int(((M > d) & (d < 16) & (L < d)).sum())
    assert n_short > 1000
    assert max(orc.block_facts(a)[1]) <= 1024  # one tile per block at 512 threads
    assert ext == _ext_bytes_reference(orc, a)


@pytest.mark.parametrize("case", [("genome", 1 << 20, 16384, 32, 0, 0, 20), ("mixed", 700_001, 16384, 64, 0, 4, 16),
                                  ("genome", 200_003, 1000, 7, 0, 2, 20), ("text", 40_000, 37, 3, 0, 0, 4),
                                  ("tandem", 500_000, 4096, 32, 8, 0, 16)],
                         ids=lambda c: "%s-n%d-B%d-W%d-f%d" % (c[0], c[1], c[2], c[3], c[5]))
def test_out_of_core_seeks(case):
    """Seeks on an archive opened out of core (only each range's dependency
    closure staged into the workspace) equal the original bytes, for every
    mode; the calls that need a resident archive refuse such a handle."""
    name, n, B, W, cap, flags, mm = case
    code = r"""
import sys
sys.path.insert(0, %(root)r); sys.path.insert(0, %(tests)r)
import numpy as np, gen, simt_lib
from paper_2606_24531_amd import encode
name, n, B, W, cap, flags, mm = %(case)r
x = gen.by_name(name, n, 23)
a = encode(x, block_size=B, interleave=W, min_match=mm, hash_len=min(mm, 16), max_level=cap, flags=flags)
arc = simt_lib.OocArchive(a)
rng = np.random.default_rng(3)
ranges = [(0, n), (n - 1, n), (B - 1, B + 1), (0, 1)]
for _ in range(6):
    lo = int(rng.integers(0, n))
    ranges.append((lo, min(n, lo + int(rng.integers(1, 3 * B)))))
for i, (lo, hi) in enumerate(ranges):
    mode = (1, 2, 3)[i %% 3]
    assert arc.seek(lo, hi, dict(mode=mode)) == x[lo:hi], (lo, hi, mode)
assert arc.workspace_bytes(5, 5) == 0
L = simt_lib.lib()
out = np.zeros(n, dtype=np.uint8); ws = np.zeros(1 << 20, dtype=np.uint8)
rc = L.ace_decode_all(arc._h, simt_lib._p(out), n, simt_lib._p(ws), ws.size, None, None)
assert rc == simt_lib.ACE_E_ARG and b"out of core" in L.ace_last_error(), rc
rc = L.ace_seek(arc._h, 0, 1, simt_lib._p(out), simt_lib._p(ws), ws.size, None, None)
assert rc == simt_lib.ACE_E_ARG, rc
print("OK")
"""
    r = subprocess.run([sys.executable, "-c", code % {"root": ROOT, "tests": HERE, "case": case}],
                       capture_output=True, text=True, timeout=600)
    assert r.returncode == 0 and "OK" in r.stdout, (r.stdout[-2000:], r.stderr[-2000:])


@pytest.mark.parametrize("case", [("genome", 1 << 20, 16384, 32, 0, 0), ("text", 300_000, 4096, 64, 8, 1),
                                  ("mixed", 700_001, 16384, 7, 0, 4), ("fastq", 200_000, 16384, 64, 0, 2),
                                  ("tandem", 400_000, 4096, 1, 8, 0), ("text", 40_000, 37, 3, 0, 0)],
                         ids=lambda c: "%s-n%d-B%d-W%d-f%d" % (c[0], c[1], c[2], c[3], c[5]))
def test_device_entropy_coding_matches_host(orc, case):
    """The encoder's rANS step run by the device kernel (the CPU build of
    it) gives the same archive bytes as the host's and the oracle's
    encoder, for every stream-mode policy."""
    name, n, B, W, cap, flags = case
    code = r"""
import sys
sys.path.insert(0, %(root)r); sys.path.insert(0, %(tests)r)
import ctypes as C, numpy as np, gen, simt_lib
from paper_2606_24531_amd import aceseek
name, n, B, W, cap, flags = %(case)r
x = gen.by_name(name, n, 29)
L = simt_lib.lib()
p = aceseek.EncodeParams(B, W, 16 if name != "genome" else 20, 16, 32, cap, flags | 8, 0)
L.ace_encode_bound.argtypes = [C.c_uint64, C.POINTER(aceseek.EncodeParams), C.POINTER(C.c_uint64)]
L.ace_encode_archive.argtypes = [C.c_void_p, C.c_uint64, C.POINTER(aceseek.EncodeParams), C.c_void_p,
                                 C.c_uint64, C.POINTER(C.c_uint64)]
b = C.c_uint64(0)
assert L.ace_encode_bound(n, C.byref(p), C.byref(b)) == 0
src = np.frombuffer(x, dtype=np.uint8)
out = np.zeros(b.value, dtype=np.uint8)
ln = C.c_uint64(0)
rc = L.ace_encode_archive(src.ctypes.data_as(C.c_void_p), n, C.byref(p), out.ctypes.data_as(C.c_void_p),
                          out.size, C.byref(ln))
assert rc == 0, (rc, L.ace_last_error())
open(%(path)r, "wb").write(out[:ln.value].tobytes())
print("OK")
"""
    import tempfile
    with tempfile.TemporaryDirectory() as td:
        path = os.path.join(td, "a.bin")
        r = subprocess.run([sys.executable, "-c", code % {"root": ROOT, "tests": HERE, "case": case, "path": path}],
                           capture_output=True, text=True, timeout=600)
        assert r.returncode == 0 and "OK" in r.stdout, (r.stdout[-2000:], r.stderr[-2000:])
        got = open(path, "rb").read()
    import gen
    x = gen.by_name(name, n, 29)
    mm = 16 if name != "genome" else 20
    want = orc.encode(x, block_size=B, interleave=W, min_match=mm, hash_len=16, max_chain=32, max_level=cap,
                      flags=flags)
    assert got == want
