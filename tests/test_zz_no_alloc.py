"""The allocation-free seek (ace_seek_static, the library's fixed device
scratch as workspace) against the plain seek (ace_seek with a caller
workspace), through the C ABI, byte for byte: two calls in a row, the second
smaller, so the second runs on the scratch the first left behind."""
import pytest

import gen

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def dev():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch.device("cuda:0")


def _host(t):
    torch.cuda.synchronize()
    return t.cpu().numpy().tobytes()


@pytest.mark.parametrize("profile,n,B,W,cap", [("mixed", 3_000_001, 16384, 32, 0),
                                               ("fastq", 2_000_003, 4096, 64, 16)])
def test_static_scratch_seek_matches_plain_seek(dev, profile, n, B, W, cap):
    from paper_2606_24531_amd import Archive, encode
    x = gen.by_name(profile, n, 17)
    a = encode(x, block_size=B, interleave=W, min_match=16, hash_len=16, max_level=cap)
    arc = Archive(a, device=dev)
    status = torch.full((1,), 77, dtype=torch.int32, device=dev)
    for lo, hi in [(n // 3, n // 3 + 5 * B + 123), (n // 2 + 7, n // 2 + B // 3)]:  # the second smaller
        ref = arc.seek(lo, hi)
        arc.check()
        out = torch.full((hi - lo,), 0xA5, dtype=torch.uint8, device=dev)
        arc.seek_static(lo, hi, out, status)
        assert int(status.item()) == 0
        assert _host(out) == _host(ref) == x[lo:hi]


def test_static_scratch_seek_refuses_beyond_its_scratch(dev):
    from paper_2606_24531_amd import Archive, aceseek, encode
    n = 40 << 20
    x = gen.random_bytes(n, 5)
    a = encode(x, block_size=16 << 20, interleave=64, min_match=16, hash_len=16)
    arc = Archive(a, device=dev)
    status = torch.zeros((1,), dtype=torch.int32, device=dev)
    out = torch.empty(n, dtype=torch.uint8, device=dev)
    with pytest.raises(aceseek.AceError) as e:
        arc.seek_static(1, n - 1, out, status)
    assert e.value.code == aceseek.E_NOSPACE and "fixed scratch" in str(e.value)
    # a seek that fits still works after the refusal
    arc.seek_static(5, 1000, out, status)
    assert int(status.item()) == 0 and _host(out[:995]) == x[5:1000]
