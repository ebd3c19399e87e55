"""Shared test helpers: the three-phase seek check and archive field access.

The three-phase check follows the paper's Section 5: (1) before the seek the
output region must not already hold the original bytes, (2) after the seek
it must equal them, and (3) everything outside the region must be untouched.
Here the whole output buffer is filled with a seeded pseudo-random sentinel,
which is a stricter form of the paper's "neighbours are zero" check.
"""
import struct

import numpy as np


def sentinel(n: int, seed: int) -> np.ndarray:
    return np.random.default_rng(seed).integers(0, 256, size=n, dtype=np.uint8)


def three_phase(run_seek, x: bytes, lo: int, hi: int, seed: int = 0, fnv=None):
    """run_seek(buf, lo, hi) must write decode[lo:hi] into buf[lo:hi] (buf is a
    host numpy uint8 array of len(x) bytes, or whatever the caller maps it
    to).  Returns the region's hash before and after when fnv is given."""
    want = np.frombuffer(x, dtype=np.uint8)
    s = seed
    buf = sentinel(len(x), s)
    while hi > lo and np.array_equal(buf[lo:hi], want[lo:hi]):
        s += 1
        buf = sentinel(len(x), s)
    before = buf.copy()
    # phase 1: the region does not hold the original before the seek
    assert hi == lo or not np.array_equal(buf[lo:hi], want[lo:hi])
    h_before = fnv(buf[lo:hi].tobytes()) if fnv else None
    out = run_seek(buf, lo, hi)
    if out is not None:
        buf = out
    # phase 2: the region equals the original
    assert np.array_equal(buf[lo:hi], want[lo:hi]), "seek [%d,%d) differs from the original" % (lo, hi)
    # phase 3: nothing outside the region was written
    assert np.array_equal(buf[:lo], before[:lo]), "bytes before %d were written" % lo
    assert np.array_equal(buf[hi:], before[hi:]), "bytes after %d were written" % hi
    if fnv:
        h_after = fnv(buf[lo:hi].tobytes())
        assert h_after == fnv(x[lo:hi]) and (hi == lo or h_before != h_after)
        return h_before, h_after
    return None


# --- archive field access (byte format: 64-byte header, 32-byte block entries)
HDR, BLK, SDESC = 64, 32, 16


def header(a: bytes) -> dict:
    (magic, ver, flags, B, W, pbits, ow, n, nb, depth, max_level, n_deps, index_off,
     pay_off, fnv) = struct.unpack_from("<IHHIHBBQIIIIQQQ", a, 0)
    return dict(magic=magic, version=ver, block_size=B, interleave=W, prob_bits=pbits,
                off_width=ow, n_total=n, n_blocks=nb, depth=depth, max_level=max_level,
                n_deps=n_deps, index_off=index_off, payload_off=pay_off, fnv=fnv)


def block_entry(a: bytes, b: int) -> dict:
    pay, plen, nseq, level, dep_off, dep_cnt, res = struct.unpack_from("<QIIIIII", a, HDR + BLK * b)
    return dict(payload_off=pay, payload_len=plen, n_seq=nseq, level=level, dep_off=dep_off,
                dep_cnt=dep_cnt, reserved=res)


def stream_desc(a: bytes, b: int, t: int) -> dict:
    e = block_entry(a, b)
    mode, n_sym, clen, off = struct.unpack_from("<B3xIII", a, e["payload_off"] + SDESC * t)
    return dict(mode=mode, n_sym=n_sym, comp_len=clen, data_at=e["payload_off"] + off)
