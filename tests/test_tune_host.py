"""Host logic of the autotuner without a GPU: the cache path follows
HEGRID_TUNE_CACHE, choices round-trip through the JSON file, a damaged file
reads as empty, and the candidate lists stay inside what hg_opts accepts."""
import json

from paper_2207_04584_amd import api, tune


def test_cache_round_trip(tmp_path, monkeypatch):
    path = tmp_path / "sub" / "tune.json"
    monkeypatch.setenv("HEGRID_TUNE_CACHE", str(path))
    assert tune.cache_path() == str(path)
    assert tune._load() == {}
    tune._store("k1", {"chunk": 48, "waves": 16, "chan_block": 256, "ms": 3.4})
    tune._store("k2", {"waves": 8, "chan_block": 128, "ms": 90.0})
    data = json.loads(path.read_text())
    assert data["k1"]["chunk"] == 48 and data["k2"]["waves"] == 8
    assert tune._load()["k1"]["ms"] == 3.4


def test_damaged_cache_reads_as_empty(tmp_path, monkeypatch):
    path = tmp_path / "tune.json"
    path.write_text("{not json")
    monkeypatch.setenv("HEGRID_TUNE_CACHE", str(path))
    assert tune._load() == {}


def test_candidates_are_valid_options():
    for waves, cb in tune.SHAPES:
        assert waves in (8, 16) and cb in (64, 128, 256)
    for prec, chunks in tune.CHUNKS.items():
        assert prec in (api.HG_PREC_FP32, api.HG_PREC_MFMA_BF16, api.HG_PREC_MFMA_F16)
        top = 64 if prec == api.HG_PREC_FP32 else 112
        assert all(8 <= c <= top and c % 8 == 0 for c in chunks)
