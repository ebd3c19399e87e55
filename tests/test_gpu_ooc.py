"""Out-of-core range decode (paper Section 7): the archive stays in host
memory and each seek stages only its dependency closure's payloads on the
device.  Every output is compared byte for byte with the original and with
the oracle's seek."""
import numpy as np
import pytest

import gen

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

CASES = [
    # profile, n, B, W, cap, flags, min_match
    ("genome", 1 << 20, 16384, 32, 0, 0, 20),
    ("mixed", 2_500_000, 16384, 32, 8, 0, 16),
    ("fastq", 1_500_000, 4096, 64, 0, 0, 20),
    ("genome", 500_000, 1000, 7, 0, 2, 20),           # non-power-of-two blocks, raw streams
    ("mixed", 1_500_007, 16384, 32, 8, 4, 16),        # 8-byte offsets
    ("tandem", 1_000_000, 16384, 32, 8, 0, 16),
]


@pytest.fixture(scope="module")
def dev():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch.device("cuda:0")


@pytest.mark.parametrize("case", CASES, ids=lambda c: "%s-n%d-B%d-W%d-cap%d-f%d" % c[:6])
def test_out_of_core_seeks_match_oracle(dev, orc, case):
    from paper_2606_24531_amd import OutOfCoreArchive
    name, n, B, W, cap, flags, mm = case
    x = gen.by_name(name, n, 37)
    a = orc.encode(x, block_size=B, interleave=W, min_match=mm, hash_len=min(mm, 16), max_level=cap,
                   flags=flags)
    arc = OutOfCoreArchive(a, device=dev)
    rng = np.random.default_rng(8)
    ranges = [(0, n), (n - 1, n), (B - 1, B + 1), (0, 1)]
    for _ in range(12):
        lo = int(rng.integers(0, n))
        ranges.append((lo, min(n, lo + int(np.exp(rng.uniform(0, np.log(4 * B + 1)))))))
    for i, (lo, hi) in enumerate(ranges):
        tuning = dict(mode=(1, 2, 3)[i % 3])
        print("ooc seek", name, n, B, lo, hi, tuning, flush=True)
        got = arc.seek(lo, hi, tuning=tuning)
        arc.check()
        assert got.cpu().numpy().tobytes() == x[lo:hi] == orc.seek(a, lo, hi), (lo, hi, tuning)
    arc.close()


def test_out_of_core_stages_only_the_closure(dev, orc):
    """A one-block seek stages that block's closure, not the archive; the
    handle is refused by the calls that need the archive resident."""
    import ctypes as C
    from paper_2606_24531_amd import OutOfCoreArchive, aceseek
    x = gen.by_name("mixed", 8 << 20, 5)
    a = orc.encode(x, block_size=16384, interleave=32, min_match=16, hash_len=16, max_level=8)
    arc = OutOfCoreArchive(a, device=dev)
    lo = 7 * 16384 + 100
    closure = orc.closure(a, lo, lo + 10)
    need = arc.workspace_bytes(lo, lo + 10)
    if len(closure) < arc.n_blocks // 2:
        assert need < len(a)
    assert arc.seek(lo, lo + 10).cpu().numpy().tobytes() == x[lo:lo + 10]
    arc.check()
    out = torch.empty(len(x), dtype=torch.uint8, device=dev)
    ws = torch.empty(1 << 20, dtype=torch.uint8, device=dev)
    L = aceseek.lib()
    rc = L.ace_decode_all(arc._h, C.c_void_p(out.data_ptr()), len(x), C.c_void_p(ws.data_ptr()), ws.numel(),
                          None, None)
    assert rc == aceseek.E_ARG and b"out of core" in L.ace_last_error()
    arc.close()


def test_out_of_core_seek_writes_only_its_range(dev, orc):
    """The paper's three-phase check on out-of-core seeks: the output buffer
    is filled with a sentinel, the seek writes its range into the middle of
    it, and the bytes around the range keep the sentinel."""
    from paper_2606_24531_amd import OutOfCoreArchive
    x = gen.by_name("genome", 1 << 20, 3)
    a = orc.encode(x, block_size=16384, interleave=32, min_match=20, hash_len=16, max_level=0)
    arc = OutOfCoreArchive(a, device=dev)
    pad = 4096
    for lo, hi in [(0, 16384), (16384 * 5 + 7, 16384 * 9 + 3), (len(x) - 100, len(x)), (12345, 12346)]:
        buf = torch.full((hi - lo + 2 * pad,), 0xA5, dtype=torch.uint8, device=dev)
        arc.seek(lo, hi, out=buf[pad:pad + hi - lo])
        arc.check()
        host = buf.cpu().numpy()
        assert host[pad:pad + hi - lo].tobytes() == x[lo:hi]
        assert (host[:pad] == 0xA5).all() and (host[pad + hi - lo:] == 0xA5).all(), (lo, hi)
    arc.close()
