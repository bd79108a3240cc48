"""The autotuner's JSON cache (host logic, no GPU): keys separate size
classes, tolerances, precision modes and devices; entries survive rewrites."""
import json

from paper_2210_07021_amd import tune


def test_cache_key_classes():
    k = tune.cache_key("MI355X", 10_000_000, 3_145_728, 1e-10, 0, {})
    assert k == tune.cache_key("MI355X", 10_400_000, 3_145_728, 1e-10, 0, {})  # same quarter decade
    assert k != tune.cache_key("MI355X", 20_000_000, 3_145_728, 1e-10, 0, {})
    assert k != tune.cache_key("MI355X", 10_000_000, 3_145_728, 1e-6, 0, {})
    assert k != tune.cache_key("MI355X", 10_000_000, 3_145_728, 1e-10, 1, {})
    assert k != tune.cache_key("other", 10_000_000, 3_145_728, 1e-10, 0, {})
    assert k != tune.cache_key("MI355X", 10_000_000, 3_145_728, 1e-10, 0, {"c_s": 3.0})
    assert tune.cache_key("g", 0, 0, 1e-10, 0, {}).count("1e0|") == 2


def test_cache_store_and_load(tmp_path):
    path = str(tmp_path / "t.json")
    assert tune.cache_load(path, "a") is None
    tune.cache_store(path, "a", {"options": {"leaf_size": 56}, "seconds": 0.01})
    tune.cache_store(path, "b", {"options": {"leaf_size": 32}, "seconds": 0.02})
    assert tune.cache_load(path, "a")["options"] == {"leaf_size": 56}
    assert tune.cache_load(path, "b")["seconds"] == 0.02
    assert set(json.load(open(path))) == {"a", "b"}
    open(path, "w").write("{not json")
    assert tune.cache_load(path, "a") is None
    tune.cache_store(path, "c", {"options": {}, "seconds": 1.0})  # a broken file is replaced
    assert tune.cache_load(path, "c")["seconds"] == 1.0
