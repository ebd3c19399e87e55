"""The encoder's rANS step on the GPU (ACE_ENC_DEVICE_ENTROPY): the archive
bytes equal the host encoder's and the oracle encoder's, for every
stream-mode policy and interleave width, and decode back to the input."""
import pytest

import gen

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

CASES = [
    # profile, n, B, W, cap, flags (policy and offset width)
    ("genome", 1 << 20, 16384, 32, 0, 0),
    ("fastq", 2_000_001, 16384, 64, 16, 0),
    ("text", 1_234_567, 4096, 64, 8, 1),       # every stream rANS
    ("mixed", 2_500_000, 16384, 7, 0, 4),      # 8-byte offsets
    ("random", 300_001, 16384, 32, 0, 0),
    ("tandem", 1_000_000, 16384, 1, 8, 0),
    ("mixed", 600_000, 65536, 64, 0, 2),       # every stream raw
    ("text", 100_000, 37, 3, 0, 0),            # tiny blocks
    ("mixed", 32 << 20, 16384, 64, 16, 0),
]


@pytest.fixture(scope="module")
def dev():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch.device("cuda:0")


@pytest.mark.parametrize("case", CASES, ids=lambda c: "%s-n%d-B%d-W%d-cap%d-f%d" % c)
def test_device_entropy_archive_equals_host_and_oracle(dev, orc, case):
    from paper_2606_24531_amd import Archive, aceseek
    name, n, B, W, cap, flags = case
    x = gen.by_name(name, n, 19)
    mm = 20 if name in ("genome", "fastq") else 16
    kw = dict(block_size=B, interleave=W, min_match=mm, hash_len=16, max_chain=32, max_level=cap)
    print("encode", name, n, B, W, cap, flags, flush=True)
    got = aceseek.encode(x, flags=flags | aceseek.ENC_DEVICE_ENTROPY, **kw)
    assert got == aceseek.encode(x, flags=flags, **kw)
    if n <= (4 << 20):
        assert got == orc.encode(x, flags=flags, **kw)
    arc = Archive(got, device=dev)
    out = arc.decode_all()
    arc.check()
    assert bool(torch.equal(out.cpu(), torch.frombuffer(bytearray(x), dtype=torch.uint8)))
    arc.close()
