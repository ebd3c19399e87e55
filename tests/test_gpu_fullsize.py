"""Full-size GPU parity at the benchmark's workload and launch shape.

256 MiB of FASTQ-like records in 16 KiB blocks (the headline decode
workload): the whole-archive decode must equal the original bytes (the
plain definition of decode), and sampled seeks must equal the oracle's seek
of the same archive."""
import numpy as np
import pytest

import gen

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def big():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2606_24531_amd import Archive, encode
    x = gen.fastq(256 << 20, 2)
    a = encode(x, block_size=16384, interleave=32, min_match=20, hash_len=20, max_chain=32,
               max_level=16)
    return x, a, Archive(a, device="cuda:0")


@pytest.mark.parametrize("mode", [2, 1, 3],
                         ids=["persistent", "levels", "overlap"])
def test_full_decode_equals_original(big, mode):
    x, a, arc = big
    out = arc.decode_all(tuning=dict(mode=mode))
    arc.check()
    got = out.cpu().numpy()
    want = np.frombuffer(x, dtype=np.uint8)
    if not np.array_equal(got, want):
        bad = np.nonzero(got != want)[0]
        pytest.fail("%d bytes differ, first at %d (block %d)" % (bad.size, bad[0], bad[0] // 16384))


def test_sampled_seeks_equal_oracle(big, orc):
    x, a, arc = big
    lo, hi = gen.seek_requests(len(x), 24, 77, max_len=1 << 20)
    for l, h in zip(lo.tolist(), hi.tolist()):
        got = arc.seek(l, h).cpu().numpy().tobytes()
        arc.check()
        assert got == orc.seek(a, l, h), (l, h)
