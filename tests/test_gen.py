"""The seeded generators: determinism and the shapes of the four profiles."""
import hashlib
import re

import numpy as np
import pytest

import gen


@pytest.mark.parametrize("name", list(gen.PROFILES))
def test_deterministic_and_seed_sensitive(name):
    a = gen.by_name(name, 200_000, 1)
    assert len(a) == 200_000
    assert hashlib.sha256(a).digest() == hashlib.sha256(gen.by_name(name, 200_000, 1)).digest()
    assert a != gen.by_name(name, 200_000, 2)
    assert gen.by_name(name, 0, 1) == b""


def test_genome_alphabet_and_repeats():
    x = gen.genome(1 << 20, 1)
    assert set(x) == set(b"ACGT")
    counts = np.bincount(np.frombuffer(x, dtype=np.uint8))[list(b"ACGT")]
    assert np.all(np.abs(counts / len(x) - 0.25) < 0.01)
    # about 30% of bytes lie in copies of earlier segments (1% substitutions)
    # and 5% in tandem repeats: a sampled 24-mer often occurs earlier
    rng = np.random.default_rng(0)
    pos = rng.integers(1 << 19, (1 << 20) - 24, size=300)
    hits = sum(x.find(x[i:i + 24], 0, i + 23) >= 0 for i in pos)
    assert 0.15 < hits / len(pos) < 0.55


def test_fastq_records():
    x = gen.fastq(1 << 20, 2)
    lines = x.split(b"\n")[:-1]
    recs = len(lines) // 4
    assert recs > 3000
    hdr = re.compile(rb"^@SIM:(\d+):([1-8]):(\d+):(\d+):(\d+)$")
    runs = set()
    for r in range(recs - 1):
        h, s, p, q = lines[4 * r:4 * r + 4]
        m = hdr.match(h)
        assert m, h
        runs.add(m.group(1))
        assert 1101 <= int(m.group(3)) <= 2100 and int(m.group(4)) < 30000 and int(m.group(5)) < 30000
        assert len(s) == 150 and set(s) <= set(b"ACGTN")
        assert p == b"+"
        assert len(q) == 150 and min(q) >= 33 + 2 and max(q) <= 33 + 41
    assert len(runs) == 1
    # quality means fall from about 38 to about 25 along the read
    qs = np.array([np.frombuffer(lines[4 * r + 3], dtype=np.uint8) for r in range(recs - 1)]) - 33
    assert abs(qs[:, 0].mean() - 38) < 1.0 and abs(qs[:, -1].mean() - 25) < 1.0


def test_text_shape():
    x = gen.text(1 << 20, 3)
    assert set(x) <= set(b"abcdefghijklmnopqrstuvwxyz .,;:!?\n")
    lines = x.split(b"\n")[1:-1]
    lens = np.array([len(s) for s in lines])
    assert lens.min() >= 60 and lens.max() <= 100 + 13
    words = re.findall(rb"[a-z]+", x)
    assert 1 <= min(map(len, words)) and max(map(len, words)) <= 12


def test_mixed_has_all_four():
    x = gen.mixed(1 << 20, 4)
    chunks = [x[i:i + 65536] for i in range(0, len(x), 65536)]
    kinds = set()
    for c in chunks:
        s = set(c)
        if s <= set(b"ACGT"):
            kinds.add("genome")
        elif c[:5] == b"@SIM:" or b"\n+\n" in c:
            kinds.add("fastq")
        elif s <= set(b"abcdefghijklmnopqrstuvwxyz .,;:!?\n"):
            kinds.add("text")
        else:
            kinds.add("random")
    assert kinds == {"genome", "fastq", "text", "random"}


def test_seek_requests_bounds():
    lo, hi = gen.seek_requests(1 << 30, 100_000, 4, max_len=4 << 20)
    ln = hi - lo
    assert np.all(hi <= (1 << 30)) and np.all(ln >= 1) and np.all(ln <= (4 << 20))
    # log-uniform lengths: median near sqrt(4 MiB) = 2 KiB, mean near 275 KB
    assert 1500 < np.median(ln) < 2600
    assert 240_000 < ln.mean() < 320_000
