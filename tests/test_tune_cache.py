"""Host logic of the launch-shape cache (no GPU): keys, round trip, refresh,
the shipped table."""
import json

from paper_2210_00947_amd import tune


class FakeParams:
    dim, nelx, nely, nelz, levels, precision = 3, 128, 128, 128, 6, 0


class FakeHandle:
    def __init__(self):
        self.shapes = {}
        self.timed = 0

    def mgar_autotune(self, reps):
        self.timed += 1
        self.shapes[(0, 0, 1)] = [1, 8, 2, 3]
        return [[[0.0] * 7 for _ in range(6)] for _ in range(2)]

    def mgar_tune_get(self, c, l, m):
        return list(self.shapes.get((c, l, m), [1, 12, 1, 3]))

    def mgar_tune_set(self, c, l, m, v):
        self.shapes[(c, l, m)] = list(v)


def test_cache_key_separates_arch_grid_and_precision():
    p = FakeParams()
    k = tune.cache_key(p, "gfx950")
    assert k == "gfx950|d3|128x128x128|L6|prec0"
    q = FakeParams()
    q.precision = 1
    assert tune.cache_key(q, "gfx950") != k
    assert tune.cache_key(p, "gfx942") != k


def test_timed_then_cached(tmp_path):
    path = str(tmp_path / "tune.json")
    h = FakeHandle()
    shapes, src = tune.autotune(h, FakeParams(), "gfx950", path=path, shipped=None)
    assert src == "timed" and h.timed == 1
    assert shapes["0/0/1"] == [1, 8, 2, 3]
    assert len(shapes) == 2 * 6 * 7
    data = json.load(open(path))
    assert "gfx950|d3|128x128x128|L6|prec0" in data
    h2 = FakeHandle()
    shapes2, src2 = tune.autotune(h2, FakeParams(), "gfx950", path=path, shipped=None)
    assert src2 == "cache" and h2.timed == 0
    assert h2.shapes[(0, 0, 1)] == [1, 8, 2, 3]
    assert shapes2 == shapes
    h3 = FakeHandle()
    _, src3 = tune.autotune(h3, FakeParams(), "gfx950", path=path, refresh=True, shipped=None)
    assert src3 == "timed" and h3.timed == 1


def test_corrupt_cache_is_retimed(tmp_path):
    path = tmp_path / "tune.json"
    path.write_text("{not json")
    h = FakeHandle()
    _, src = tune.autotune(h, FakeParams(), "gfx950", path=str(path), shipped=None)
    assert src == "timed"
    assert json.load(open(path))


def test_shipped_table_used_when_cache_misses(tmp_path):
    shipped = tmp_path / "shipped.json"
    key = tune.cache_key(FakeParams(), "gfx950")
    shapes = {"0/0/1": [2, 10, 1, 3], "1/0/1": [2, 8, 1, 2]}
    shipped.write_text(json.dumps({key: {"shapes": shapes}}))
    path = str(tmp_path / "tune.json")
    h = FakeHandle()
    got, src = tune.autotune(h, FakeParams(), "gfx950", path=path, shipped=str(shipped))
    assert src == "shipped" and h.timed == 0
    assert got == shapes and h.shapes[(0, 0, 1)] == [2, 10, 1, 3]
    # another architecture misses both tables and is timed
    h2 = FakeHandle()
    _, src2 = tune.autotune(h2, FakeParams(), "gfx942", path=path, shipped=str(shipped))
    assert src2 == "timed" and h2.timed == 1
    # the user's cache wins over the shipped table; refresh times again
    h3 = FakeHandle()
    _, src3 = tune.autotune(h3, FakeParams(), "gfx942", path=path, shipped=str(shipped))
    assert src3 == "cache"
    h4 = FakeHandle()
    _, src4 = tune.autotune(h4, FakeParams(), "gfx950", path=path, shipped=str(shipped), refresh=True)
    assert src4 == "timed" and h4.timed == 1


def test_shipped_table_entries_are_valid_shapes():
    """Every shipped shape is a 4-int shape of a known kind for a known mode."""
    table = tune._load(tune.SHIPPED)
    for key, entry in table.items():
        assert key.count("|") == 4
        for k, v in entry["shapes"].items():
            c, l, m = (int(s) for s in k.split("/"))
            assert c in (0, 1) and 0 <= m < tune.NMODES and l >= 0
            assert len(v) == 4 and v[0] in (0, 1, 2)
