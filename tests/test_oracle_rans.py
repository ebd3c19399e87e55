"""Pins of the oracle's entropy layer (interleaved rANS).

Checked against facts fixed outside the oracle: hand-derived streams
(tests/golden/rans_hand.txt), closed forms of the stream length, the
invariants of the state machine, and the normalisation rule worked by hand.
"""
import os
import struct

import numpy as np
import pytest

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "rans_hand.txt")


def _golden_cases():
    cases = []
    for line in open(GOLDEN):
        line = line.strip()
        if not line.startswith("case "):
            continue
        name, W, freq, syms, states, words = [f.strip() for f in line[5:].split("|")]
        f = np.zeros(256, dtype=np.uint16)
        for tok in freq.split():
            s, v = tok.split(":")
            f[int(s)] = int(v)
        cases.append((name, int(W), f, syms.encode(), [int(v) for v in states.split()],
                      [int(v) for v in words.split()]))
    return cases


@pytest.mark.parametrize("case", _golden_cases(), ids=lambda c: c[0])
def test_hand_derived_streams(orc, case):
    name, W, freq, syms, states, words = case
    assert freq.sum() == 4096
    expect = struct.pack("<%dI" % W, *states) + struct.pack("<%dH" % len(words), *words)
    got = orc.rans_encode(syms, W, freq)
    assert got == expect
    assert orc.rans_decode(got, len(syms), W, freq) == syms


@pytest.mark.parametrize("W", [1, 2, 3, 32, 64])
@pytest.mark.parametrize("n", [1, 5, 63, 64, 65, 1000])
def test_single_symbol_stream_is_states_only(orc, W, n):
    # f = 4096: the state function maps x to x, nothing is ever emitted.
    f = np.zeros(256, dtype=np.uint16)
    f[7] = 4096
    got = orc.rans_encode(bytes([7]) * n, W, f)
    assert got == struct.pack("<I", 65536) * W
    assert orc.rans_decode(got, n, W, f) == bytes([7]) * n


@pytest.mark.parametrize("W", [1, 2, 3, 32, 64])
@pytest.mark.parametrize("n", [0, 1, 31, 32, 33, 64, 65, 129, 4097])
def test_uniform_sixteen_length_closed_form(orc, W, n):
    # f = 16 for all 256 symbols: a lane state alternates between
    # [2^16, 2^16+4096) and [2^24, 2^24+4096), emitting one word every second
    # symbol, so the body is 4W + 2 * sum_j floor(k_j / 2) bytes.
    f = np.full(256, 16, dtype=np.uint16)
    rng = np.random.default_rng(n * 131 + W)
    syms = rng.integers(0, 256, size=n, dtype=np.uint8).tobytes()
    got = orc.rans_encode(syms, W, f)
    k = [len(range(j, n, W)) for j in range(W)]
    assert len(got) == 4 * W + 2 * sum(kj // 2 for kj in k)
    assert orc.rans_decode(got, n, W, f) == syms


def test_lanes_are_independent_scalar_coders(orc):
    # Interleaving only splits the symbols: lane j's final state is the
    # final state of a one-lane coder run on symbols j, j+W, j+2W, ...
    rng = np.random.default_rng(5)
    counts = np.zeros(256, dtype=np.uint64)
    counts[:40] = rng.integers(1, 1000, size=40)
    f = orc.normalize(counts)
    W = 7
    syms = rng.choice(40, size=3001, p=counts[:40] / counts[:40].sum()).astype(np.uint8).tobytes()
    inter = orc.rans_encode(syms, W, f)
    words_total = 0
    for j in range(W):
        solo = orc.rans_encode(syms[j::W], 1, f)
        assert inter[4 * j:4 * j + 4] == solo[:4]
        words_total += (len(solo) - 4) // 2
    assert len(inter) == 4 * W + 2 * words_total


@pytest.mark.parametrize("W", [1, 2, 3, 32, 64])
def test_round_trip_skewed_tables(orc, W):
    rng = np.random.default_rng(W)
    for trial in range(30):
        k = int(rng.integers(1, 257))
        alphabet = rng.choice(256, size=k, replace=False)
        weights = rng.pareto(0.7, size=k) + 1e-3
        n = int(rng.integers(0, 5000))
        syms = rng.choice(alphabet, size=n, p=weights / weights.sum()).astype(np.uint8)
        counts = np.bincount(syms, minlength=256).astype(np.uint64)
        if n == 0:
            counts[alphabet[0]] = 1
        f = orc.normalize(counts)
        assert f.sum() == 4096 and np.all((f > 0) == (counts > 0))
        data = orc.rans_encode(syms.tobytes(), W, f)
        assert orc.rans_decode(data, n, W, f) == syms.tobytes()
        # size is within 1% + the fixed state cost of the ideal code length
        if n:
            ideal = -np.sum(np.log2(f[syms].astype(np.float64) / 4096.0)) / 8.0
            assert len(data) <= ideal * 1.01 + 4 * W + 2 * W + 8


def test_decoder_rejects_damaged_streams(orc):
    f = np.zeros(256, dtype=np.uint16)
    f[97], f[98] = 5, 4091
    good = orc.rans_encode(b"aaaaab", 2, f)
    # a flipped state bit breaks the final-state check
    bad = bytearray(good)
    bad[0] ^= 0x10
    with pytest.raises(orc.OracleError) as e:
        orc.rans_decode(bytes(bad), 6, 2, f)
    assert e.value.code == orc.E_CORRUPT
    # a missing word is an over-run, an extra word is left unused
    for damaged in (good[:-2], good + b"\0\0"):
        with pytest.raises(orc.OracleError) as e:
            orc.rans_decode(damaged, 6, 2, f)
        assert e.value.code == orc.E_CORRUPT
    # a state below 2^16 is rejected up front
    low = struct.pack("<I", 5) + good[4:]
    with pytest.raises(orc.OracleError):
        orc.rans_decode(low, 6, 2, f)


def test_normalisation_worked_examples(orc):
    c = np.zeros(256, dtype=np.uint64)
    c[ord("a")], c[ord("b")] = 1, 3
    f = orc.normalize(c)
    assert f[ord("a")] == 1024 and f[ord("b")] == 3072
    # three equal counts: 1365 each leaves 1; the tie goes to the smallest symbol
    c = np.zeros(256, dtype=np.uint64)
    c[[10, 20, 30]] = 1
    f = orc.normalize(c)
    assert (f[10], f[20], f[30]) == (1366, 1365, 1365)
    # one dominant symbol and 255 singletons: floor gives 4094 + 255 ones,
    # 253 too many, all taken from the dominant symbol
    c = np.ones(256, dtype=np.uint64)
    c[0] = 1_000_000
    f = orc.normalize(c)
    assert f[0] == 3841 and np.all(f[1:] == 1)
