"""Autotuner host logic (no GPU): every compiled (tile shape, backward
batch) pair is timed, the fastest is returned and cached with its batch, and
a cached entry from before the batch dimension is tuned again.  The library
is the real one (which pairs are compiled); the step timing and the GPU
buffers are stand-ins."""
import torch

from paper_2501_08174_amd import autotune as at


class _FakeRast:
    def __init__(self, n, views, *a, **k):
        self.views, self.batch = views, 0

    def plan_capacity(self, p, slack=1.0):
        return 0

    def set_bwd_batch(self, b):
        self.batch = b


class _FakeViews:
    def __init__(self, cams, tile=(16, 16), device="cuda"):
        self.tile = tile


def _params(n=10):
    z = lambda *s: torch.zeros(*s)
    return at.Params(z(n, 3), z(n, 2), z(n, 4), z(n), z(n, 16, 3))


def test_times_every_compiled_pair_and_keeps_the_fastest(monkeypatch, tmp_path):
    timed = []
    cost = {((16, 16), 64): 1.0}

    def fake_time(rast, p, g, mask, target, used, steps):
        key = (rast.views.tile, rast.batch)
        timed.append(key)
        return cost.get(key, 5.0)

    monkeypatch.setattr(at, "ViewBatch", _FakeViews)
    monkeypatch.setattr(at, "Rasterizer", _FakeRast)
    monkeypatch.setattr(at, "time_step", fake_time)
    monkeypatch.setattr(at, "CACHE", str(tmp_path / "autotune.json"))
    monkeypatch.setattr(at, "cache_key", lambda cams, n, deg: "k")
    report = {}
    tile, batch = at.autotune([], _params(), 3, 16, None, None, report=report)
    assert (tile, batch) == ((16, 16), 64)
    want = {((16, 16), b) for b in (32, 64, 128, 256)} | {((32, 8), b) for b in (32, 64, 128, 256)} | \
        {((16, 8), b) for b in (32, 64, 128)} | {((8, 8), b) for b in (32, 64)}
    assert set(timed) == want and len(timed) == len(want)
    assert report["batch"] == 64 and report["tile"] == [16, 16] and len(report["ms"]) == len(want)
    # the cache answers the next call without timing
    timed.clear()
    assert at.autotune([], _params(), 3, 16, None, None) == ((16, 16), 64)
    assert timed == []


def test_entry_without_batch_is_tuned_again(monkeypatch, tmp_path):
    monkeypatch.setattr(at, "ViewBatch", _FakeViews)
    monkeypatch.setattr(at, "Rasterizer", _FakeRast)
    monkeypatch.setattr(at, "time_step", lambda rast, *a: 1.0 if rast.views.tile == (32, 8) and rast.batch == 128
                        else 2.0)
    monkeypatch.setattr(at, "CACHE", str(tmp_path / "autotune.json"))
    monkeypatch.setattr(at, "cache_key", lambda cams, n, deg: "k")
    at._store({"k": {"tile": [16, 16], "ms": {"16x16": 1.0}}})
    assert at.autotune([], _params(), 3, 16, None, None) == ((32, 8), 128)
    assert at._load()["k"]["batch"] == 128
