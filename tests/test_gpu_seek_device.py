"""Single seeks planned on the device (the batch planner's kernels for one
request, the archive's plan resident) against the original bytes and against
host-planned seeks of the same ranges, in every decode mode; and the choice
between the two by workspace size."""
import numpy as np
import pytest

import gen

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def dev():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch.device("cuda:0")


@pytest.mark.parametrize("name,n,B,W,cap", [("mixed", 8 << 20, 16384, 64, 16), ("genome", 1 << 20, 16384, 32, 0),
                                            ("text", 3_000_001, 4096, 32, 8)])
@pytest.mark.parametrize("mode", [1, 2, 3])
def test_device_planned_seek_matches_host_planned(dev, name, n, B, W, cap, mode):
    from paper_2606_24531_amd import Archive, encode
    x = gen.by_name(name, n, 21)
    a = encode(x, block_size=B, interleave=W, min_match=16, hash_len=16, max_level=cap)
    arc = Archive(a, device=dev)
    lo, hi = gen.seek_requests(n, 40, 22, max_len=4 * B)
    ranges = [(int(l), int(h)) for l, h in zip(lo, hi)] + [(0, n), (n - 1, n), (B - 1, B + 1)]
    ws = torch.zeros(max(arc.seek_device_bytes(), arc.workspace_bytes([0, n])), dtype=torch.uint8, device=dev)
    for l, h in ranges:
        d = arc.seek(l, h, ws=ws, tuning=dict(mode=mode), plan="device")
        hp = arc.seek(l, h, ws=ws, tuning=dict(mode=mode), plan="host")
        arc.check(ws)
        want = x[l:h]
        assert d.cpu().numpy().tobytes() == want, (l, h, "device-planned")
        assert hp.cpu().numpy().tobytes() == want, (l, h, "host-planned")


def test_workspace_size_selects_the_planner(dev):
    """With the resident plan, a workspace of seek_device_bytes plans on the
    device (no host closure walk: the host time stays small even for a range
    whose closure spans the archive); a smaller one plans on the host."""
    from paper_2606_24531_amd import Archive, aceseek, encode
    x = gen.mixed(16 << 20, 23)
    a = encode(x, block_size=16384, interleave=64, min_match=16, hash_len=16, max_level=16)
    arc = Archive(a, device=dev)
    n = len(x)
    lo, hi = n - 5000, n - 10
    ws = torch.zeros(arc.seek_device_bytes(), dtype=torch.uint8, device=dev)
    aceseek.set_timing(True)
    try:
        out = arc.seek(lo, hi, ws=ws)
        torch.cuda.synchronize()
        plan_dev, _ = aceseek.last_host_times()
        out_h = arc.seek(lo, hi, ws=ws, plan="host")
        torch.cuda.synchronize()
        plan_host, _ = aceseek.last_host_times()
    finally:
        aceseek.set_timing(False)
    arc.check(ws)
    assert out.cpu().numpy().tobytes() == x[lo:hi] == out_h.cpu().numpy().tobytes()
    assert plan_dev < plan_host
