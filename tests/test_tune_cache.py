"""The pair-shape tuning cache (paper_1209_3362_amd/tune_cache.py) and the
validation of cached shapes by nfs_set_pair_shapes, without a GPU."""
import json

import paper_1209_3362_amd.tune_cache as tc


def test_key_separates_what_changes_the_shapes():
    k = tc.cache_key("gfx950", 1024, [1, 2, 3], "f32", "plain")
    assert k != tc.cache_key("gfx942", 1024, [1, 2, 3], "f32", "plain")
    assert k != tc.cache_key("gfx950", 512, [1, 2, 3], "f32", "plain")
    assert k != tc.cache_key("gfx950", 1024, [1, 2, 4], "f32", "plain")
    assert k != tc.cache_key("gfx950", 1024, [1, 2, 3], "bf16", "plain")
    assert k != tc.cache_key("gfx950", 1024, [1, 2, 3], "f32", "kahan")
    assert k == tc.cache_key("gfx950", 1024, (1, 2, 3), "f32", "plain")


def test_store_lookup_and_environment(tmp_path, monkeypatch):
    path = str(tmp_path / "sub" / "shapes.json")
    monkeypatch.setenv("NFS_TUNE_CACHE", path)
    assert tc.cache_path() == path
    assert tc.lookup(path, "a") is None
    tc.store(path, "a", [(16, 8), (8, 6)])
    tc.store(path, "b", [(0, 0)])
    assert tc.lookup(path, "a") == [(16, 8), (8, 6)]
    assert tc.lookup(path, "b") == [(0, 0)]
    assert json.load(open(path))["a"] == [[16, 8], [8, 6]]
    # A damaged file reads as empty and is replaced on the next store.
    open(path, "w").write("{not json")
    assert tc.lookup(path, "a") is None
    tc.store(path, "c", [(16, 4)])
    assert tc.lookup(path, "c") == [(16, 4)]
    monkeypatch.setenv("NFS_TUNE_CACHE", "off")
    assert tc.cache_path() is None and tc.lookup(None, "c") is None
    monkeypatch.setenv("NFS_TUNE_REFRESH", "1")
    assert tc.refresh()
    monkeypatch.setenv("NFS_TUNE_REFRESH", "0")
    assert not tc.refresh()
