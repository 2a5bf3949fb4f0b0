"""The autotuner's winner cache (host logic only): graph-shape buckets and
the JSON store, with stand-in graph objects."""
import json

from paper_2407_19562_amd import autotune


class _P:
    def __init__(self, precision):
        self.precision = precision


class _G:
    def __init__(self, n, m, precision=64):
        self.n = n
        self._m = m
        self.params = _P(precision)

    def size(self):
        return self.n, self._m


def test_bucket_separates_shapes():
    a = autotune.shape_bucket([_G(1 << 16, 1 << 20)] * 4, "async")
    b = autotune.shape_bucket([_G(1 << 16, 1 << 20)] * 4, "async")
    assert a == b == "async/fp64/g2/n18/m22"
    assert autotune.shape_bucket([_G(1 << 16, 1 << 20, 32)] * 4, "async") != a
    assert autotune.shape_bucket([_G(1 << 16, 1 << 20)] * 64, "async") != a
    assert autotune.shape_bucket([_G(1 << 20, 1 << 24)], "sync") == "sync/fp64/g0/n20/m24"


def test_cache_round_trip(tmp_path, monkeypatch):
    path = tmp_path / "sub" / "tune.json"
    monkeypatch.setenv("DFPR_TUNE_CACHE", str(path))
    assert autotune._load_cache() == {}
    autotune._store_cache("k1", {"chunk": 1024, "block_size": 256})
    autotune._store_cache("k2", {"chunk": 0, "block_size": 64})
    assert json.loads(path.read_text()) == {
        "k1": {"block_size": 256, "chunk": 1024},
        "k2": {"block_size": 64, "chunk": 0}}
    path.write_text("not json")
    assert autotune._load_cache() == {}
