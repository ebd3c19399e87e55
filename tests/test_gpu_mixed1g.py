"""GPU parity at the mixed corpus's full size: 1 GiB of 64 KiB chunks of the
genome, FASTQ-like, text and random profiles in seeded order, 16 KiB and
64 KiB blocks with the level cap, decoded whole in every decode mode and
compared byte for byte with the original (the plain definition of decode);
100,000 seeks (length log-uniform 1 B..4 MiB) replayed as one batch graph,
every output compared; and an uncapped archive with thousands of dependency
levels decoded whole.  Expected bytes are the generator's input: no value
here comes from the GPU path."""
import numpy as np
import pytest

import gen

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def _first_difference(got, want):
    bad = torch.nonzero(got != want)
    return int(bad[0]) if bad.numel() else -1


@pytest.fixture(scope="module")
def corpus():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    x = gen.mixed(1 << 30, 3)
    x_dev = torch.from_numpy(np.frombuffer(x, dtype=np.uint8).copy()).to("cuda:0")
    return x, x_dev


@pytest.fixture(scope="module")
def arc16(corpus):
    from paper_2606_24531_amd import Archive, encode
    x, _ = corpus
    a = encode(x, block_size=16384, interleave=64, min_match=16, hash_len=16, max_chain=32, max_level=16)
    return Archive(a, device="cuda:0")


@pytest.mark.parametrize("B", [16384, 65536], ids=["16KiB", "64KiB"])
@pytest.mark.parametrize("mode", [1, 2], ids=["levels", "persistent"])
def test_mixed1g_full_decode_equals_original(corpus, arc16, B, mode):
    from paper_2606_24531_amd import Archive, encode
    x, x_dev = corpus
    if B == 16384:
        arc = arc16
    else:
        a = encode(x, block_size=B, interleave=64, min_match=16, hash_len=16, max_chain=32, max_level=16)
        arc = Archive(a, device="cuda:0")
    assert arc.depth <= 16
    out = torch.full((arc.n_total,), 0x5A, dtype=torch.uint8, device="cuda:0")
    arc.decode_all(out=out, tuning=dict(mode=mode))
    arc.check()
    at = _first_difference(out, x_dev)
    assert at < 0, "first difference at byte %d (block %d)" % (at, at // B)


def test_mixed1g_100k_batch_every_output(corpus, arc16):
    x, x_dev = corpus
    n_req = 100_000
    lo, hi = gen.seek_requests(len(x), n_req, 4, max_len=4 << 20)
    ln = (hi - lo).astype(np.int64)
    offs = np.concatenate([[0], np.cumsum(ln)[:-1]]).astype(np.uint64)
    out = torch.empty(int(ln.sum()), dtype=torch.uint8, device="cuda:0")
    bt = arc16.batch(n_req, tuning=dict(mode=1))
    bt.run((lo, hi), out, offs)
    torch.cuda.synchronize()
    bt.check()
    bad = [i for i in range(n_req)
           if not torch.equal(out[int(offs[i]):int(offs[i]) + int(ln[i])], x_dev[int(lo[i]):int(hi[i])])]
    bt.close()
    assert not bad, "%d requests differ, first %d [%d, %d)" % (len(bad), bad[0], lo[bad[0]], hi[bad[0]])


@pytest.mark.parametrize("mode", [1, 2], ids=["levels", "persistent"])
def test_uncapped_thousands_of_levels(mode):
    from paper_2606_24531_amd import Archive, encode
    x = gen.fastq(64 << 20, 2)
    a = encode(x, block_size=16384, interleave=64, min_match=20, hash_len=20, max_chain=32, max_level=0)
    arc = Archive(a, device="cuda:0")
    assert arc.depth > 1000
    out = arc.decode_all(tuning=dict(mode=mode))
    arc.check()
    x_dev = torch.from_numpy(np.frombuffer(x, dtype=np.uint8).copy()).to("cuda:0")
    at = _first_difference(out, x_dev)
    assert at < 0, "first difference at byte %d" % at
