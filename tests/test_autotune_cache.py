"""Host logic of the spreading-shape autotuner cache (no GPU)."""
import json

from paper_2305_06482_amd import autotune


class FakeCtx:
    """Stands in for a Context: records the shape it is given and counts the
    timing runs."""

    ndim = 2
    N = 1000

    def __init__(self, best=3):
        self.best = best
        self.timed = 0
        self.cfg = None

    def grid_shape(self):
        return (80, 80, 1)

    def autotune_spread(self, maps, reps):
        self.timed += 1
        self.cfg = self.best
        return self.best, [1.0 + i for i in range(6)]

    def set_spread_cfg(self, cfg):
        self.cfg = cfg


class Maps:
    shape = (64, 64, 12)


def test_key_distinguishes_geometry_and_chunk():
    k = autotune.geometry_key(3, (160, 240, 240), 9216000, 12)
    assert k == "3d/160x240x240/N9216000/c12"
    assert autotune.geometry_key(3, (160, 240, 240), 9216000, 32).endswith("/c16")
    assert k != autotune.geometry_key(3, (160, 240, 240), 9216001, 12)


def test_tune_times_once_then_reuses(tmp_path):
    path = str(tmp_path / "sub" / "cache.json")
    a = FakeCtx(best=4)
    shape, ms, hit = autotune.tune(a, Maps(), path=path)
    assert (shape, hit, a.timed) == (4, False, 1) and len(ms) == 6
    stored = json.load(open(path))
    assert list(stored.values())[0]["shape"] == 4
    b = FakeCtx(best=0)
    shape, _, hit = autotune.tune(b, Maps(), path=path)
    assert (shape, hit, b.timed, b.cfg) == (4, True, 0, 4)


def test_corrupt_cache_is_retuned(tmp_path):
    path = tmp_path / "cache.json"
    path.write_text("{not json")
    c = FakeCtx(best=2)
    shape, _, hit = autotune.tune(c, Maps(), path=str(path))
    assert (shape, hit, c.timed) == (2, False, 1)
    assert json.load(open(path))
