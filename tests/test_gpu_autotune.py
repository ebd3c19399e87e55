"""The autotuner: every candidate it times is checked bit-exact by the tuner
itself, and the shape it picks decodes a larger archive of the same profile
bit-exact (whole-archive decode and a replayed batch of seeks)."""
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


def test_tuned_choice_decodes_bit_exact(dev, tmp_path):
    from paper_2606_24531_amd import Archive, encode
    from paper_2606_24531_amd.autotune import candidates, tune, tune_batch
    x = gen.mixed(6 << 20, 11)
    best = tune(x[:2 << 20], "mixed", block_size=16384, min_match=16, max_level=16, reps=1,
                cache_path=str(tmp_path / "tune.json"))
    assert best["interleave"] in (32, 64) and best["mode"] in (1, 2, 3)
    assert any(all(best[k] == c[k] for k in c) for c in candidates(best["interleave"], 2560))
    a = encode(x, block_size=16384, interleave=best["interleave"], min_match=16, hash_len=16,
               max_level=16)
    arc = Archive(a, device=dev)
    shape = {k: best[k] for k in ("mode", "waves_per_block", "blocks_per_wg", "grid_wgs")}
    out = arc.decode_all(tuning=shape)
    arc.check()
    torch.cuda.synchronize()
    assert out.cpu().numpy().tobytes() == x
    x_dev = torch.from_numpy(np.frombuffer(x, dtype=np.uint8).copy()).to(dev)
    lo, hi = gen.seek_requests(len(x), 40, 5, max_len=1 << 20)
    bb = tune_batch(arc, x_dev, lo, hi, reps=1)
    assert bb["mode"] in (1, 2, 3) and len(bb["all"]) >= 4
