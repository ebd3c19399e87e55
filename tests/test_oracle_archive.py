"""Oracle archive-level pins: round trips on every profile, seek and its
closure, the three-phase check, FNV test vectors and corruption handling."""
import struct

import numpy as np
import pytest

import gen
from harness import block_entry, header, stream_desc, three_phase

PROFILES = [("genome", 20), ("fastq", 20), ("text", 16), ("random", 16), ("mixed", 16), ("tandem", 16)]


def test_fnv1a64_published_vectors(orc):
    # test vectors of the FNV-1a 64-bit hash from its specification
    assert orc.fnv1a64(b"") == 0xCBF29CE484222325
    assert orc.fnv1a64(b"a") == 0xAF63DC4C8601EC8C
    assert orc.fnv1a64(b"foobar") == 0x85944171F73967E8


@pytest.mark.parametrize("name,mm", PROFILES)
@pytest.mark.parametrize("B,W,cap", [(16384, 32, 0), (4096, 64, 4), (65536, 32, 0), (1000, 7, 2)])
def test_round_trip_profiles(orc, name, mm, B, W, cap):
    x = gen.by_name(name, 300_001, 17)
    a = orc.encode(x, block_size=B, interleave=W, min_match=mm, hash_len=mm, max_level=cap)
    h = header(a)
    assert h["n_blocks"] == -(-len(x) // B) and h["n_total"] == len(x)
    assert h["fnv"] == orc.fnv1a64(x)
    assert orc.decode(a) == x
    level, _, _ = orc.block_facts(a)
    assert h["depth"] == level.max() + 1
    if cap:
        assert level.max() < cap


@pytest.mark.parametrize("flags", [1, 2])
def test_forced_stream_modes(orc, flags):
    x = gen.fastq(100_000, 3)
    a = orc.encode(x, block_size=8192, interleave=32, flags=flags)
    _, _, modes = orc.block_facts(a)
    assert np.all(modes == (1 if flags == 1 else 0))
    assert orc.decode(a) == x


@pytest.mark.parametrize("policy", [0, 1, 2])
def test_wide_offsets(orc, policy):
    """8-byte offsets (the width an output above 4 GiB needs) forced on a
    small input: the parse is the same, every stored offset is the 4-byte
    one zero-extended, and the archive decodes to the input."""
    x = gen.mixed(600_000, 9)
    kw = dict(block_size=16384, interleave=32, min_match=16, hash_len=16, max_level=8)
    a4 = orc.encode(x, flags=policy, **kw)
    a8 = orc.encode(x, flags=policy | orc.WIDE_OFFSETS, **kw)
    assert header(a4)["off_width"] == 4 and header(a8)["off_width"] == 8
    assert orc.decode(a8) == x
    nb = header(a8)["n_blocks"]
    for b in range(nb):
        t4, t8 = orc.block_tokens(a4, b), orc.block_tokens(a8, b)
        assert all(np.array_equal(u, v) for u, v in zip(t4, t8))
        if policy == 2:  # raw streams: the stored bytes themselves
            d4, d8 = stream_desc(a4, b, 2), stream_desc(a8, b, 2)
            o4 = np.frombuffer(a4, np.uint8, d4["n_sym"], d4["data_at"]).reshape(-1, 4)
            o8 = np.frombuffer(a8, np.uint8, d8["n_sym"], d8["data_at"]).reshape(-1, 8)
            assert np.array_equal(o8[:, :4], o4) and not o8[:, 4:].any()
    for lo, hi in [(0, len(x)), (123_457, 345_679), (len(x) - 10, len(x))]:
        assert orc.seek(a8, lo, hi) == x[lo:hi]


def test_seek_equals_slice_and_three_phase_every_block(orc):
    # the paper's core experiment, on the small genome workload: every block
    # sought singly, checked in three phases
    x = gen.genome(1 << 20, 1)
    a = orc.encode(x, block_size=16384, interleave=32, min_match=20, hash_len=20, max_chain=32)
    B = 16384

    def run(buf, lo, hi):
        buf[lo:hi] = np.frombuffer(orc.seek(a, lo, hi), dtype=np.uint8)

    for b in range(64):
        three_phase(run, x, b * B, (b + 1) * B, seed=b, fnv=orc.fnv1a64)
    rng = np.random.default_rng(0)
    for _ in range(50):
        lo = int(rng.integers(0, len(x)))
        hi = int(rng.integers(lo, min(len(x), lo + 200_000) + 1))
        assert orc.seek(a, lo, hi) == x[lo:hi]


def test_seek_errors(orc):
    x = gen.text(10_000, 1)
    a = orc.encode(x, block_size=1024, interleave=8, min_match=8, hash_len=8)
    with pytest.raises(orc.OracleError) as e:
        orc.seek(a, 10, 10_001)
    assert e.value.code == orc.E_RANGE
    with pytest.raises(orc.OracleError) as e:
        orc.seek(a, 11, 10)
    assert e.value.code == orc.E_ARG
    assert orc.seek(a, 500, 500) == b""


def test_closure_is_dependency_closed(orc):
    x = gen.fastq(1 << 19, 9)
    B = 4096
    a = orc.encode(x, block_size=B, interleave=32)
    nb = header(a)["n_blocks"]
    deps = []
    raw = np.frombuffer(a, dtype=np.uint8)
    dep_at = 64 + 32 * nb
    for b in range(nb):
        e = block_entry(a, b)
        deps.append([int(v) for v in raw[dep_at + 4 * e["dep_off"]:dep_at + 4 * (e["dep_off"] + e["dep_cnt"])]
                     .view("<u4")])
    for lo, hi in [(0, 1), (B * 50 + 7, B * 53 + 1), (len(x) - 1, len(x))]:
        c = set(orc.closure(a, lo, hi).tolist())
        targets = set(range(lo // B, (hi - 1) // B + 1))
        assert targets <= c
        for b in c:
            assert set(deps[b]) <= c
        # minimal: every member is a target or reachable from one
        seen, stack = set(), list(targets)
        while stack:
            b = stack.pop()
            if b in seen:
                continue
            seen.add(b)
            stack.extend(deps[b])
        assert seen == c


# ---------------------------------------------------------------- corruption
@pytest.fixture(scope="module")
def raw_archive(orc):
    x = gen.genome(1 << 17, 5)
    a = orc.encode(x, block_size=4096, interleave=16, min_match=20, hash_len=20, flags=2)
    return x, a


def _patch(a, at, fmt, value):
    b = bytearray(a)
    struct.pack_into(fmt, b, at, value)
    return bytes(b)


def _first_match(a, orc):
    h = header(a)
    for b in range(1, h["n_blocks"]):
        _, L, M, O = orc.block_tokens(a, b)
        for k in range(len(M)):
            if M[k]:
                return b, k, L, M, O
    raise AssertionError("no match found")


def test_corruptions_are_reported(orc, raw_archive):
    x, a = raw_archive
    assert orc.decode(a) == x
    E = orc.E_CORRUPT
    h = header(a)
    cases = {}
    cases["magic"] = _patch(a, 0, "<I", 0x12345678)
    cases["block count"] = _patch(a, 24, "<I", h["n_blocks"] + 1)
    cases["depth"] = _patch(a, 28, "<I", h["depth"] + 1)
    cases["fnv"] = _patch(a, 56, "<Q", h["fnv"] ^ 1)
    cases["prob bits"] = _patch(a, 14, "<B", 11)
    b, k, L, M, O = _first_match(a, orc)
    e = block_entry(a, b)
    cases["level"] = _patch(a, 64 + 32 * b + 16, "<I", e["level"] + 1)
    if e["dep_cnt"]:
        cases["missing dep"] = _patch(a, 64 + 32 * b + 24, "<I", e["dep_cnt"] - 1)
    cases["reserved"] = _patch(a, 64 + 32 * b + 28, "<I", 1)
    lens = stream_desc(a, b, 1)
    offs = stream_desc(a, b, 2)
    assert lens["mode"] == 0 and offs["mode"] == 0
    dst = b * 4096 + int(sum(L[:k + 1]) + sum(M[:k]))
    cases["offset not before destination"] = _patch(a, offs["data_at"] + 4 * k, "<I", dst)
    cases["lengths miss the block length"] = _patch(a, lens["data_at"] + 4 * k + 2, "<H", int(M[k]) - 1)
    cases["stream mode"] = _patch(a, e["payload_off"], "<B", 7)
    cases["payload alignment"] = _patch(a, 64 + 32 * b, "<Q", e["payload_off"] + 4)
    for name, bad in cases.items():
        assert orc.decode_rc(bad) == E, name
    for cut in (0, 10, 63, 64, 64 + 32 * 3, len(a) // 2, len(a) - 1):
        assert orc.decode_rc(a[:cut]) == E, "truncated at %d" % cut


def test_rans_table_corruption(orc):
    x = gen.genome(1 << 16, 6)
    a = orc.encode(x, block_size=4096, interleave=32, flags=1)
    sd = stream_desc(a, 3, 0)
    assert sd["mode"] == 1
    bad = _patch(a, sd["data_at"] + 32, "<H", struct.unpack_from("<H", a, sd["data_at"] + 32)[0] + 1)
    assert orc.decode_rc(bad) == orc.E_CORRUPT
    # a damaged state word fails the final-state check
    nsym = sum(1 for s in range(256) if (a[sd["data_at"] + s // 8] >> (s % 8)) & 1)
    st = sd["data_at"] + ((32 + 2 * nsym + 3) & ~3)
    bad = _patch(a, st, "<I", struct.unpack_from("<I", a, st)[0] ^ 0x40)
    assert orc.decode_rc(bad) == orc.E_CORRUPT


def test_random_bit_flips_never_crash(orc, raw_archive):
    _, a = raw_archive
    rng = np.random.default_rng(1)
    codes = []
    for _ in range(400):
        b = bytearray(a)
        i = int(rng.integers(0, len(b)))
        b[i] ^= 1 << int(rng.integers(0, 8))
        codes.append(orc.decode_rc(bytes(b)))
    assert set(codes) <= {0, orc.E_CORRUPT}
    # only padding bytes may hide a flip
    assert codes.count(orc.E_CORRUPT) >= 0.9 * len(codes)


@pytest.mark.parametrize("name,mm,B,cap", [("mixed", 16, 16384, 8), ("genome", 20, 4096, 0),
                                           ("text", 16, 1000, 0)])
def test_level_parallel_decode_equals_sequential(orc, name, mm, B, cap):
    """The all-cores baseline decodes each dependency level's blocks in
    parallel; its output is the sequential decode's, at any thread count."""
    x = gen.by_name(name, 700_001, 23)
    a = orc.encode(x, block_size=B, interleave=32, min_match=mm, hash_len=mm, max_level=cap)
    for t in (1, 3, 0):
        y, used = orc.decode_levels(a, t)
        assert y == x
        assert used >= 1 and (t == 0 or used == t)


def test_level_parallel_decode_reports_corruption(orc):
    x = gen.fastq(200_000, 5)
    a = bytearray(orc.encode(x, block_size=4096, interleave=8, max_level=4))
    e = block_entry(bytes(a), 7)
    d = stream_desc(bytes(a), 7, 1)
    a[d["data_at"] + d["comp_len"] // 2] ^= 0x40  # damage one block's LEN stream
    with pytest.raises(orc.OracleError) as ex:
        orc.decode_levels(bytes(a), 4)
    assert ex.value.code == orc.E_CORRUPT
    assert ex.value.code == orc.decode_rc(bytes(a))
    assert e["n_seq"] > 0
