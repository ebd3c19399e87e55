"""Pins of the oracle's match layer and archive index.

A parse is legal when its sequences reproduce the input under the format's
semantics (L literals, then M bytes copied one at a time from absolute
offset O < destination, overlap allowed, no sequence crossing its block's
end).  Every legal parse of every short string over {a, b} is serialised by
the oracle's assembler and decoded by the oracle's decoder; the output must
be the string.  The enumeration below is written from that definition alone.
"""
import itertools

import numpy as np
import pytest


def block_parses(x, s, e):
    """All sequence lists that rebuild x[s:e] (absolute offsets, overlap ok)."""
    out = []

    def rec(p, lit, seqs):
        if p == e:
            out.append(seqs + [(lit, 0, 0)] if lit else seqs)
            return
        rec(p + 1, lit + 1, seqs)
        for O in range(p):
            M = 0
            while p + M < e and x[O + M] == x[p + M]:
                M += 1
                rec(p + M, 0, seqs + [(lit, M, O)])

    rec(s, 0, [])
    return out


def all_parses(x, B):
    per_block = [block_parses(x, s, min(s + B, len(x))) for s in range(0, len(x), B)]
    return itertools.product(*per_block)


def check_batch(orc, items, B, W, flags):
    """Concatenate (x, parse) pairs, each padded with literals to a whole
    number of blocks, into one archive; decode and compare."""
    xs, counts, L, M, O = [], [], [], [], []
    base = 0
    for x, parse in items:
        nb = -(-len(x) // B)
        pad = nb * B - len(x)
        for bi, seqs in enumerate(parse):
            seqs = [(l, m, (o + base) if m else 0) for (l, m, o) in seqs]
            if bi == nb - 1 and pad:
                if seqs[-1][1] == 0:
                    seqs[-1] = (seqs[-1][0] + pad, 0, 0)
                else:
                    seqs.append((pad, 0, 0))
            counts.append(len(seqs))
            for l, m, o in seqs:
                L.append(l)
                M.append(m)
                O.append(o)
        xs.append(x + b"c" * pad)
        base += nb * B
    blob = b"".join(xs)
    a = orc.assemble(blob, B, W, counts, L, M, O, flags=flags)
    assert orc.decode(a) == blob


@pytest.mark.parametrize("B", [1, 2, 3, 4, 8])
def test_every_parse_of_short_strings(orc, B):
    """All legal parses of all {a,b} strings of length 1..7."""
    batch, k = [], 0
    total = 0
    for n in range(1, 8):
        for t in itertools.product(b"ab", repeat=n):
            x = bytes(t)
            for parse in all_parses(x, B):
                batch.append((x, parse))
                if len(batch) == 4096:
                    check_batch(orc, batch, B, W=[1, 3, 32][k % 3], flags=k % 3)
                    total += len(batch)
                    batch, k = [], k + 1
    if batch:
        check_batch(orc, batch, B, W=2, flags=0)
        total += len(batch)
    # the count of legal parses is itself fixed by the definition; these
    # figures were counted by a separate memoised recursion
    expected = {1: 46232, 2: 55604, 3: 60458, 4: 65554, 8: 72822}
    assert total == expected[B]


def test_sampled_parses_of_length_eight(orc):
    rng = np.random.default_rng(8)
    for B in (1, 2, 3, 4, 8):
        batch = []
        for t in itertools.product(b"ab", repeat=8):
            x = bytes(t)
            parses = list(all_parses(x, B)) if B <= 2 else None
            if parses is None:
                # random legal parse: walk the string choosing uniformly
                per_block = [block_parses(x, s, min(s + B, 8)) for s in range(0, 8, B)]
                for _ in range(6):
                    batch.append((x, tuple(pb[rng.integers(len(pb))] for pb in per_block)))
            else:
                for i in rng.choice(len(parses), size=min(6, len(parses)), replace=False):
                    batch.append((x, parses[i]))
        check_batch(orc, batch, B, W=5, flags=1)


@pytest.mark.parametrize("B", [2, 3, 4])
def test_short_last_block_standalone(orc, B):
    """N not a multiple of B: the last block is short; each parse is its own
    archive so the short block is the archive's real end."""
    for n in range(1, 6):
        if n % B == 0:
            continue
        for t in itertools.product(b"ab", repeat=n):
            x = bytes(t)
            for parse in all_parses(x, B):
                counts = [len(s) for s in parse]
                flat = [q for s in parse for q in s]
                a = orc.assemble(x, B, 2, counts, [q[0] for q in flat], [q[1] for q in flat],
                                 [q[2] for q in flat], flags=1)
                assert orc.decode(a) == x
                assert orc.info(a)["n_blocks"] == -(-n // B)


def test_empty_input(orc):
    a = orc.encode(b"", block_size=16, interleave=4, min_match=4, hash_len=4)
    assert orc.info(a) == dict(n_total=0, block_size=16, n_blocks=0, depth=0, interleave=4)
    assert orc.decode(a) == b""
    assert orc.seek(a, 0, 0) == b""


def test_period_two_overlap_example(orc):
    # "abababab", B = 8: two literals then one match of 6 from offset 0
    a = orc.encode(b"abababab", block_size=8, interleave=1, min_match=2, hash_len=2,
                   max_chain=8, flags=2)
    lit, L, M, O = orc.block_tokens(a, 0)
    assert lit == b"ab" and list(L) == [2] and list(M) == [6] and list(O) == [0]
    assert orc.decode(a) == b"abababab"


def test_all_zero_input_is_a_chain(orc):
    # one period-1 match per block, from the last byte of the previous block
    B, nb = 64, 20
    x = bytes(B * nb)
    a = orc.encode(x, block_size=B, interleave=4, min_match=4, hash_len=4, max_chain=4)
    level, nseq, _ = orc.block_facts(a)
    assert list(level) == list(range(nb))
    assert orc.info(a)["depth"] == nb
    for b in range(1, nb):
        lit, L, M, O = orc.block_tokens(a, b)
        assert (lit, list(L), list(M), list(O)) == (b"", [0], [B], [b * B - 1])
    assert orc.decode(a) == x
    # closure of the last block is every block
    assert list(orc.closure(a, (nb - 1) * B, nb * B)) == list(range(nb))


def test_random_bytes_have_no_dependencies(orc):
    rng = np.random.default_rng(3)
    x = rng.integers(0, 256, size=1 << 16, dtype=np.uint8).tobytes()
    a = orc.encode(x, block_size=4096, interleave=32, min_match=16, hash_len=16)
    level, _, modes = orc.block_facts(a)
    assert np.all(level == 0) and orc.info(a)["depth"] == 1
    assert np.all(modes[:, 0] == 0)  # incompressible literals stay raw
    assert orc.decode(a) == x


@pytest.mark.parametrize("cap", [1, 2, 3, 8])
def test_level_cap_bounds_depth(orc, cap):
    import gen
    x = gen.text(1 << 18, 7)
    a = orc.encode(x, block_size=4096, interleave=32, min_match=8, hash_len=8, max_level=cap)
    level, _, _ = orc.block_facts(a)
    assert level.max() < cap
    assert orc.decode(a) == x
    if cap == 1:
        # no block may reference another block
        for b in range(0, len(level), 9):
            _, _, M, O = orc.block_tokens(a, b)
            assert np.all((M == 0) | (O >= b * 4096))


@pytest.mark.parametrize("cap,B,size", [(2, 1024, 1 << 20), (4, 1024, 1 << 20), (16, 1024, 1 << 20),
                                        (16, 128, 1 << 20)])
def test_level_budget_respected(orc, cap, B, size):
    # the capped parse policy, checked from the tokens: a block of epoch e
    # (64 blocks each, E in all, counted in units of c = max(1, E // 64))
    # references only blocks of earlier epochs whose level is below
    # min(cap - 1, floor(log2(e // c + 1)), max(1, floor(log2(E // c + 1)) - 1));
    # levels then come out geometric
    import gen
    x = gen.fastq(size, 9)
    a = orc.encode(x, block_size=B, interleave=8, min_match=16, hash_len=16, max_level=cap)
    level, _, _ = orc.block_facts(a)
    nb = len(level)
    E = (nb + 63) // 64
    lg = lambda v: v.bit_length() - 1
    n_refs = 0
    for b in range(nb):
        e = b // 64
        cu = max(1, E // 64)
        lam = min(cap - 1, lg(e // cu + 1), max(1, lg(E // cu + 1) - 1))
        _, L, M, O = orc.block_tokens(a, b)
        for m, o in zip(M.tolist(), O.tolist()):
            if m == 0 or o >= b * B:
                continue
            for d in range(o // B, (min(o + m, b * B) - 1) // B + 1):
                assert d < 64 * e and level[d] < lam, (b, d)
                n_refs += 1
    assert n_refs > 1000  # the rule was exercised
    assert level.max() < cap
    if E >= 128:  # epochs counted in units of two or more: the first level is wider
        assert max(1, E // 64) >= 2 and int(np.sum(level == 0)) >= 128
    assert orc.decode(a) == x


def test_dependencies_recomputed_from_tokens(orc):
    import gen
    x = gen.genome(1 << 18, 11)
    B = 4096
    a = orc.encode(x, block_size=B, interleave=32, min_match=20, hash_len=20)
    level, _, _ = orc.block_facts(a)
    lv = []
    for b in range(len(level)):
        _, L, M, O = orc.block_tokens(a, b)
        deps = set()
        for m, o in zip(M, O):
            for q in range(int(o), min(int(o) + int(m), b * B)):
                deps.add(q // B)
        assert all(d < b for d in deps)
        lv.append(0 if not deps else 1 + max(lv[d] for d in deps))
    assert lv == list(level)
