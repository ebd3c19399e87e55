"""The graph-replayed batched seek: device-side planning plus one decode of
the union of closures plus one gather, replayed for batches of different
sizes; every request must equal the original bytes and its solo seek."""
import numpy as np
import pytest

import gen

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.mark.parametrize("tuning", [dict(mode=1), dict(mode=3),
                                    dict(mode=3, waves_per_block=8, blocks_per_wg=1),
                                    dict(mode=2)],
                         ids=["levels", "overlap", "overlap-8waves-1stream", "persistent"])
def test_graph_batch_replays(orc, tuning):
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2606_24531_amd import Archive, encode
    x = gen.mixed(3 << 20, 12)
    a = encode(x, block_size=16384, interleave=32, min_match=16, hash_len=16, max_level=8)
    arc = Archive(a, device="cuda:0")
    bt = arc.batch(500, tuning=tuning)
    for it, (count, max_len, seed) in enumerate([(500, 200_000, 1), (37, 1 << 20, 2),
                                                 (1, 5, 3), (0, 10, 4), (400, 30_000, 5)]):
        lo, hi = gen.seek_requests(len(x), max(count, 1), seed, max_len=max_len)
        lo, hi = lo[:count], hi[:count]
        lens = (hi - lo).astype(np.int64)
        out = torch.full((max(int(lens.sum()), 1),), 0x5A, dtype=torch.uint8, device="cuda:0")
        bt.run((lo, hi), out)
        bt.check()
        got = out.cpu().numpy().tobytes()
        pos = 0
        for i in range(count):
            l, h = int(lo[i]), int(hi[i])
            assert got[pos:pos + h - l] == x[l:h], (it, i)
            pos += h - l
    bt.close()


@pytest.mark.parametrize("levels,W,tuning", [(1, 32, None), (2, 32, None), ("all", 32, None),
                                             (2, 64, dict(mode=3)), (1, 64, dict(mode=1, waves_per_block=4))],
                         ids=["keep1", "keep2", "keep-all", "keep2-W64-overlap", "keep1-W64-4waves"])
def test_graph_batch_with_kept_levels(orc, levels, W, tuning):
    """Keeping the lowest dependency levels decoded (ace_batch_pin): later
    batches neither plan nor decode those blocks, and every request still
    equals the original bytes, including requests that lie entirely in kept
    blocks, across several replays."""
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2606_24531_amd import Archive, encode
    from paper_2606_24531_amd.aceseek import AceError, E_ARG
    x = gen.mixed(3 << 20, 13)
    # uncapped: 54 dependency levels on this input
    a = encode(x, block_size=16384, interleave=W, min_match=16, hash_len=16, max_level=0)
    arc = Archive(a, device="cuda:0")
    assert arc.depth >= 3
    keep = arc.depth if levels == "all" else levels
    bt = arc.batch(300, tuning=tuning)
    with pytest.raises(AceError) as ei:
        bt.pin(arc.depth + 1)
    assert ei.value.code == E_ARG
    bt.pin(keep)
    with pytest.raises(AceError) as ei:
        bt.pin(1)
    assert ei.value.code == E_ARG
    B = 16384
    for it, (count, max_len, seed) in enumerate([(300, 200_000, 21), (50, 40, 22), (1, 5, 23), (0, 10, 24),
                                                 (200, 1 << 20, 25)]):
        lo, hi = gen.seek_requests(len(x), max(count, 1), seed, max_len=max_len)
        lo, hi = lo[:count].copy(), hi[:count].copy()
        if count >= 2:  # one request inside block 0 (level 0, always kept)
            lo[0], hi[0] = 100, 100 + min(500, B - 100)
        lens = (hi - lo).astype(np.int64)
        out = torch.full((max(int(lens.sum()), 1),), 0x5A, dtype=torch.uint8, device="cuda:0")
        bt.run((lo, hi), out)
        bt.check()
        got = out.cpu().numpy().tobytes()
        pos = 0
        for i in range(count):
            l, h = int(lo[i]), int(hi[i])
            assert got[pos:pos + h - l] == x[l:h], (it, i)
            pos += h - l
    bt.close()
