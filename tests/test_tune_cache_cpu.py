"""The tuning cache (host logic only): keys, round trips through the JSON file,
atomic replacement and the refusals of malformed files and entries."""
import json
import os

import pytest

from paper_2606_09058_amd import tune_cache as TC

ENTRY = {"tiles_per_workgroup": 4, "nseg": 2, "seg_first": [0, 100], "seg_tiles": [4, 2],
         "backtr_block": 256, "gemm_big_min_k": 256, "dc_leaf": 32}


def test_key_format():
    k = TC.cache_key("gfx950-256cu", "gevd", "real64", 6656, 1, "collinear", "fp64", "onestage")
    assert k == "gfx950-256cu/gevd/real64/6656/1/collinear/fp64/onestage"
    with pytest.raises(ValueError):
        TC.cache_key("gfx950/x", "gevd", "real64", 10, 1, "collinear", "fp64", "onestage")
    with pytest.raises(ValueError):
        TC.cache_key("gfx950", "gevd", "real64", 0, 1, "collinear", "fp64", "onestage")
    with pytest.raises(ValueError):
        TC.cache_key("", "gevd", "real64", 10, 1, "collinear", "fp64", "onestage")


def test_round_trip_and_replace(tmp_path):
    path = str(tmp_path / "sub" / "tune.json")
    assert TC.load(path) == {}
    assert TC.lookup(path, "a/b") is None
    TC.store(path, "k1", ENTRY)
    TC.store(path, "k2", dict(ENTRY, dc_leaf=16))
    assert TC.lookup(path, "k1") == ENTRY
    assert TC.lookup(path, "k2")["dc_leaf"] == 16
    TC.store(path, "k1", dict(ENTRY, backtr_block=128))
    assert TC.lookup(path, "k1")["backtr_block"] == 128
    assert TC.lookup(path, "k2")["dc_leaf"] == 16
    doc = json.load(open(path))
    assert doc["version"] == TC.VERSION and sorted(doc["entries"]) == ["k1", "k2"]
    # no temporary files left behind
    assert sorted(os.listdir(tmp_path / "sub")) == ["tune.json"]


def test_refusals(tmp_path):
    path = str(tmp_path / "tune.json")
    bad = dict(ENTRY)
    del bad["dc_leaf"]
    with pytest.raises(ValueError):
        TC.store(path, "k", bad)
    assert not os.path.exists(path)
    with open(path, "w") as f:
        json.dump({"version": TC.VERSION + 1, "entries": {}}, f)
    with pytest.raises(ValueError):
        TC.load(path)
    with open(path, "w") as f:
        json.dump({"version": TC.VERSION, "entries": {"k": bad}}, f)
    with pytest.raises(ValueError):
        TC.lookup(path, "k")
