"""Seeded synthetic inputs shaped like the paper's four data profiles.

The paper evaluates on a real FASTQ file, a repetitive genome, English text
and a mixed corpus (Section 6, Table 1).  None of those files is available, so
these generators stand in for them.  They hold none of the codec's arithmetic:
they only produce bytes (and seek request lists) that both the CPU oracle and
the GPU library consume.

Every generator takes (n, seed) and is a pure function of them:
``numpy.random.Generator(PCG64(SeedSequence(seed)))``, with independent child
streams obtained by ``SeedSequence.spawn``.
"""
from __future__ import annotations

import bisect

import numpy as np

__all__ = [
    "genome", "fastq", "text", "random_bytes", "mixed", "by_name",
    "seek_requests", "PROFILES",
]

_ACGT = np.frombuffer(b"ACGT", dtype=np.uint8)


def _rng(seed_seq: np.random.SeedSequence) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(seed_seq))


def _children(seed: int, k: int):
    return [_rng(s) for s in np.random.SeedSequence(seed).spawn(k)]


# ---------------------------------------------------------------------------
# GENOME: uniform ACGT with copied segments (1% substitutions) and tandem repeats
# ---------------------------------------------------------------------------
def genome(n: int, seed: int) -> bytes:
    """Repetitive-genome stand-in.

    Built event by event.  A deficit schedule keeps about 30% of bytes in
    segments of 20..2000 bases copied from uniformly chosen earlier absolute
    positions (each copied base replaced by a different base with p = 0.01),
    about 5% in tandem repeats (period 2..50, 3..40 copies, at most 2000
    bytes), and the rest fresh uniform bases in runs of 20..2000.
    """
    n = int(n)
    if n <= 0:
        return b""
    rng = _rng(np.random.SeedSequence(seed))
    buf = np.empty(n + 2048, dtype=np.uint8)  # base indices 0..3
    pos = copied = tandem = 0
    while pos < n:
        if pos >= 2000 and copied < 0.30 * pos:
            ln = int(rng.integers(20, 2001))
            src = int(rng.integers(0, pos - ln + 1))
            seg = buf[src:src + ln].copy()
            hit = rng.random(ln) < 0.01
            k = int(hit.sum())
            if k:
                seg[hit] = (seg[hit] + rng.integers(1, 4, size=k, dtype=np.uint8)) & 3
            buf[pos:pos + ln] = seg
            copied += ln
        elif tandem < 0.05 * pos:
            period = int(rng.integers(2, 51))
            unit = rng.integers(0, 4, size=period, dtype=np.uint8)
            ln = min(period * int(rng.integers(3, 41)), 2000)
            buf[pos:pos + ln] = np.resize(unit, ln)
            tandem += ln
        else:
            ln = int(rng.integers(20, 2001))
            buf[pos:pos + ln] = rng.integers(0, 4, size=ln, dtype=np.uint8)
        pos += ln
    return _ACGT[buf[:n]].tobytes()


# ---------------------------------------------------------------------------
# FASTQ: 4-line records, 150-bp reads from a 4 Mbp reference
# ---------------------------------------------------------------------------
_READ = 150
_REF = 4_000_000


def fastq(n: int, seed: int) -> bytes:
    """FASTQ-like stand-in (real sequencing reads, the paper's 'clean' profile).

    Record i: ``@SIM:<run>:<lane>:<tile>:<x>:<y>`` with run fixed per file,
    lane = 1 + (i >> 20) mod 8, tile = 1101 + (i // 4096) mod 1000,
    x, y uniform in 0..29999; a 150-bp forward read from a seeded 4 Mbp
    uniform-ACGT reference, each base 'N' with p = 0.001 else substituted with
    p = 0.005; a '+' line; Phred+33 qualities clip(round(mu_j + 3 z), 2, 41)
    with mu_j falling linearly from 38 to 25 along the read.
    """
    n = int(n)
    if n <= 0:
        return b""
    r_ref, r_hdr, r_read, r_qual = _children(seed, 4)
    ref = r_ref.integers(0, 4, size=_REF, dtype=np.uint8)
    run = int(r_hdr.integers(1, 1000))
    mu = 38.0 - 13.0 * np.arange(_READ) / (_READ - 1)
    out = []
    total = 0
    i0 = 0
    chunk = 16384
    while total < n:
        idx = np.arange(i0, i0 + chunk)
        lane = 1 + ((idx >> 20) % 8)
        tile = 1101 + (idx // 4096) % 1000
        xy = r_hdr.integers(0, 30000, size=(chunk, 2))
        starts = r_read.integers(0, _REF - _READ + 1, size=chunk)
        reads = ref[starts[:, None] + np.arange(_READ)[None, :]]
        u = r_read.random((chunk, _READ))
        is_n = u < 0.001
        sub = (~is_n) & (u < 0.006)
        k = int(sub.sum())
        if k:
            reads[sub] = (reads[sub] + r_read.integers(1, 4, size=k, dtype=np.uint8)) & 3
        seq = _ACGT[reads]
        seq[is_n] = ord("N")
        z = r_qual.standard_normal((chunk, _READ))
        q = np.clip(np.rint(mu[None, :] + 3.0 * z), 2, 41).astype(np.uint8) + 33
        body = np.empty((chunk, 2 * _READ + 4), dtype=np.uint8)
        body[:, :_READ] = seq
        body[:, _READ] = 10
        body[:, _READ + 1] = ord("+")
        body[:, _READ + 2] = 10
        body[:, _READ + 3:2 * _READ + 3] = q
        body[:, 2 * _READ + 3] = 10
        rows = body.tobytes()
        w = body.shape[1]
        parts = []
        for j in range(chunk):
            parts.append(b"@SIM:%d:%d:%d:%d:%d\n" % (run, lane[j], tile[j], xy[j, 0], xy[j, 1]))
            parts.append(rows[j * w:(j + 1) * w])
        blob = b"".join(parts)
        out.append(blob)
        total += len(blob)
        i0 += chunk
    return b"".join(out)[:n]


# ---------------------------------------------------------------------------
# TEXT: Zipf(1.1) over 50k pseudo-words, punctuation, line breaks every 60..100
# ---------------------------------------------------------------------------
_NWORDS = 50_000
_PUNCT = np.frombuffer(b".,;:!?", dtype=np.uint8)


def text(n: int, seed: int) -> bytes:
    """English-like text stand-in (the paper's enwik9 profile).

    A vocabulary of 50,000 pseudo-words (length 1..12, letters a..z); word
    rank r drawn with probability proportional to r**-1.1; after each word one
    of '.,;:!?' with p = 0.08; words separated by ' ', except that once a line
    has reached its target length T (drawn uniformly in 60..100 per line) the
    separator is a newline.
    """
    n = int(n)
    if n <= 0:
        return b""
    r_voc, r_tok, r_line = _children(seed, 3)
    wlen = r_voc.integers(1, 13, size=_NWORDS)
    wstart = np.concatenate([[0], np.cumsum(wlen)[:-1]])
    chars = r_voc.integers(ord("a"), ord("z") + 1, size=int(wlen.sum()), dtype=np.uint8)
    p = np.arange(1, _NWORDS + 1, dtype=np.float64) ** -1.1
    cdf = np.cumsum(p / p.sum())
    out = []
    total = 0
    while total < n:
        m = max(1024, min(1 << 22, (n - total) // 5 + 1024))
        ids = np.minimum(np.searchsorted(cdf, r_tok.random(m), side="right"), _NWORDS - 1)
        has_p = r_tok.random(m) < 0.08
        pch = _PUNCT[r_tok.integers(0, 6, size=m)]
        tl = wlen[ids] + has_p  # token length without separator
        # line breaking: the separator after token k is '\n' when the line
        # length after token k reaches T, else ' '.
        c = np.concatenate([[0], np.cumsum(tl)])
        d = c[1:] + np.arange(m)  # D[k] = C[k+1] + k
        sep = np.full(m, ord(" "), dtype=np.uint8)
        # One target length per line, drawn in order; a batch draw yields the
        # same values as one draw at a time, and the generator is then moved
        # on by exactly the number of draws used.
        state = r_line.bit_generator.state
        targets = r_line.integers(60, 101, size=m + 1).tolist()
        dl, cl = d.tolist(), c.tolist()
        a = used = 0
        while a < m:
            t = targets[used]
            used += 1
            k = bisect.bisect_left(dl, cl[a] + a + t)
            if k >= m:
                break
            sep[k] = 10
            a = k + 1
        r_line.bit_generator.state = state
        r_line.integers(60, 101, size=used)
        tot_len = tl + 1
        starts = np.concatenate([[0], np.cumsum(tot_len)[:-1]])
        buf = np.empty(int(tot_len.sum()), dtype=np.uint8)
        wl = wlen[ids]
        # letter j of the chunk: source index into `chars` and destination
        # index into `buf`, both consecutive within a word and jumping to the
        # next word's start between words (built as running sums of steps)
        first = np.cumsum(wl) - wl
        src = np.ones(int(wl.sum()), dtype=np.int64)
        dst = np.ones(src.size, dtype=np.int64)
        ws = wstart[ids]
        src[0], dst[0] = ws[0], starts[0]
        src[first[1:]] = ws[1:] - (ws[:-1] + wl[:-1] - 1)
        dst[first[1:]] = starts[1:] - (starts[:-1] + wl[:-1] - 1)
        np.cumsum(src, out=src)
        np.cumsum(dst, out=dst)
        buf[dst] = chars[src]
        pend = starts + wl
        buf[pend[has_p]] = pch[has_p]
        buf[starts + tl] = sep
        out.append(buf.tobytes())
        total += buf.size
    return b"".join(out)[:n]


def random_bytes(n: int, seed: int) -> bytes:
    """Uniform random bytes (incompressible; exercises raw stream modes)."""
    n = int(n)
    if n <= 0:
        return b""
    return _rng(np.random.SeedSequence(seed)).integers(0, 256, size=n, dtype=np.uint8).tobytes()


_CHUNK = 65536


def mixed(n: int, seed: int) -> bytes:
    """Mixed-corpus stand-in (the paper's silesia profile).

    GENOME, FASTQ, TEXT and RANDOM each produce n/4 bytes, cut into 64 KiB
    chunks; the chunks are interleaved in a seeded shuffled order of their
    labels, each generator's chunks kept in their own order.
    """
    n = int(n)
    if n <= 0:
        return b""
    ss = np.random.SeedSequence(seed).spawn(5)
    seeds = [int(s.generate_state(1)[0]) for s in ss[:4]]
    quarter = -(-n // 4)
    parts = [genome(quarter, seeds[0]), fastq(quarter, seeds[1]),
             text(quarter, seeds[2]), random_bytes(quarter, seeds[3])]
    nch = [-(-len(p) // _CHUNK) for p in parts]
    labels = np.repeat(np.arange(4), nch)
    _rng(ss[4]).shuffle(labels)
    nxt = [0, 0, 0, 0]
    out = []
    for lab in labels:
        lab = int(lab)
        i = nxt[lab]
        out.append(parts[lab][i * _CHUNK:(i + 1) * _CHUNK])
        nxt[lab] = i + 1
    return b"".join(out)[:n]


def tandem(n: int, seed: int) -> bytes:
    """Tandem repeats: a copy of an earlier chunk (20..47 bytes) followed at
    once by its last d bytes (1 <= d <= 15) repeated for 40..899 bytes, with
    short random runs in between.  The second copy's period lies in the
    bytes of the first, so in-block chains of short-period matches are
    common (an edge case of the expansion, not a corpus of the paper)."""
    rng = _rng(np.random.SeedSequence([seed, 5]))
    out = bytearray(rng.integers(0, 256, 4096, dtype=np.uint8).tobytes())
    while len(out) < n:
        if rng.random() < 0.3:
            out += rng.integers(0, 256, int(rng.integers(8, 64)), dtype=np.uint8).tobytes()
        m = int(rng.integers(20, 48))
        o = int(rng.integers(0, len(out) - m))
        chunk = bytes(out[o:o + m])
        d = int(rng.integers(1, 16))
        rep = int(rng.integers(40, 900))
        out += chunk + (chunk[-d:] * (rep // d + 1))[:rep]
    return bytes(out[:n])


PROFILES = {
    "genome": genome,
    "tandem": tandem,
    "fastq": fastq,
    "text": text,
    "random": random_bytes,
    "mixed": mixed,
}


def by_name(name: str, n: int, seed: int) -> bytes:
    return PROFILES[name](n, seed)


def seek_requests(n_total: int, count: int, seed: int, max_len: int = 4 << 20,
                  min_len: int = 1):
    """Seek ranges: length log-uniform in [min_len, max_len], offset uniform.

    Returns two uint64 arrays (lo, hi) with 0 <= lo < hi <= n_total.
    """
    rng = _rng(np.random.SeedSequence(seed))
    max_len = min(max_len, n_total)
    min_len = max(1, min(min_len, max_len))
    ln = np.floor(np.exp(rng.uniform(np.log(min_len), np.log(max_len), size=count))).astype(np.int64)
    ln = np.clip(ln, min_len, max_len)
    lo = (rng.random(count) * (n_total - ln + 1)).astype(np.int64)
    lo = np.minimum(lo, n_total - ln)
    return lo.astype(np.uint64), (lo + ln).astype(np.uint64)
