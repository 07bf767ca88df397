"""Autotuner host logic (CPU): size buckets, cache keys, the JSON cache, choice of the fastest."""
import json

import pytest

from paper_2410_21207_amd import tune


def test_buckets_and_keys():
    assert [tune._bucket(x) for x in (1, 2, 3, 240, 256, 257, 2160)] == [1, 2, 4, 256, 256, 512, 4096]
    assert tune.key_single("gfx950", 1080, 1920) == "gfx950/single/2048x2048"
    assert tune.key_batch("gfx950", [(240, 300), (2000, 1000), (500, 2160)]) == "gfx950/batch/2048x4096/n4"


def test_cache_roundtrip(tmp_path, monkeypatch):
    path = str(tmp_path / "cache.json")
    monkeypatch.setenv("SC_TUNE_CACHE", path)
    monkeypatch.setattr(tune, "_cache", None)
    assert tune.lookup("gfx950/single/64x64") is None
    tune.save({"gfx950/single/64x64": {"variant": 5, "team": 4, "ms": 1.0}})
    tune.save({"gfx950/batch/256x256/n8": {"variant": 7, "team": 16, "ms": 2.0}})
    assert tune.lookup("gfx950/single/64x64") == (5, 4)
    assert tune.lookup("gfx950/batch/256x256/n8") == (7, 16)
    monkeypatch.setattr(tune, "_cache", None)  # a fresh process reads the file
    assert tune.lookup("gfx950/single/64x64") == (5, 4)
    with open(path) as f:
        assert set(json.load(f)) == {"gfx950/single/64x64", "gfx950/batch/256x256/n8"}


def test_cache_rejects_garbage(tmp_path, monkeypatch):
    path = tmp_path / "bad.json"
    path.write_text("[1, 2, 3]")
    monkeypatch.setattr(tune, "_cache", None)
    with pytest.raises(ValueError):
        tune.load(str(path))


def test_pick_fastest_first_on_ties():
    t = {(1, 8): 0.30, (5, 16): 0.25, (7, 16): 0.25, (7, 32): 0.40}
    assert tune.pick(t) == (5, 16)


def test_candidates_are_known_variants():
    # variant ids the tuner tries must exist in the library's variant table (10 compiled variants)
    for v, g in tune.BATCH_CANDIDATES + tune.SINGLE_CANDIDATES:
        assert 0 <= v < 10 and 1 <= g <= 32


def test_packaged_cache_is_consistent():
    """The cache shipped in the package: every entry names a compiled variant and a team the
    library accepts, records its fastest candidate, and the keys cover the benchmarked shapes
    (the 256-image batch, 1920x1080 and 3840x2160 single images)."""
    import json
    import re

    with open(tune.DEFAULT_CACHE) as f:
        data = json.load(f)
    assert data, "empty cache"
    for key, e in data.items():
        assert re.fullmatch(r"gfx\w+/(single/\d+x\d+|batch/\d+x\d+/n\d+)", key), key
        assert 0 <= e["variant"] < 10 and 1 <= e["team"] <= 32, (key, e)
        cands = {k: v for k, v in e.get("candidates", {}).items()}
        if cands:
            best = min(cands.values())
            assert cands[f"v{e['variant']}/g{e['team']}"] == best == e["ms"], key
    assert tune.key_single("gfx950", 1080, 1920) in data
    assert tune.key_single("gfx950", 2160, 3840) in data
    assert tune.key_batch("gfx950", [(2160, 2160)] * 256) in data
