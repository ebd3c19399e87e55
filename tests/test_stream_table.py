"""Per-stream entropy effect (the paper's Table 2 view, Section 6.1) on the
synthetic profiles: rANS compresses literals but inflates the structural
offset stream of genomic data, and the encoder's per-stream choice (rANS only
where it is smaller) never loses to coding every stream."""
import pytest

import gen


@pytest.fixture(scope="module")
def lib():
    from paper_2606_24531_amd import aceseek
    return aceseek


@pytest.mark.parametrize("name,mm", [("genome", 20), ("fastq", 20), ("text", 16), ("mixed", 16)])
def test_per_stream_ratios(lib, name, mm):
    x = gen.by_name(name, 4 << 20, 7)
    kw = dict(block_size=16384, interleave=32, min_match=mm, hash_len=mm, max_level=16)
    forced = lib.encode(x, flags=1, **kw)
    adaptive = lib.encode(x, flags=0, **kw)
    tf, ta = lib.stream_table(forced), lib.stream_table(adaptive)
    assert tf["LIT"]["ratio"] > 1.2
    assert tf["OFF"]["ratio"] < 1.0           # absolute offsets: rANS inflates them
    assert ta["OFF"]["ratio"] >= 1.0 - 1e-9   # ... so the encoder stores them raw
    assert len(adaptive) <= len(forced)
    for s in ("LIT", "LEN", "OFF"):
        assert ta[s]["raw"] == tf[s]["raw"]
        assert ta[s]["stored"] <= tf[s]["stored"]
    if name in ("genome", "fastq"):
        assert tf["LEN"]["ratio"] < 1.0
