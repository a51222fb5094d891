"""The autotuner's file cache (host only): round trip through GS_TUNE_CACHE, and
GS_TUNE_CACHE=off."""
import json

from paper_1901_07643_amd import tune


def test_file_cache_round_trip(tmp_path, monkeypatch):
    path = tmp_path / "sub" / "tune.json"
    monkeypatch.setenv("GS_TUNE_CACHE", str(path))
    monkeypatch.setattr(tune, "_file_key", lambda key, device: repr(key))
    key = ("batch", ((12, 300), (14, 900)), "bic", None)
    assert tune._file_get(key, None) is None
    tune._file_put(key, None, [10, {"9": 0.71, "10": 0.70}])
    tune._file_put(("plan", 26, 5000, "bic", None), None, 13)
    assert tune._file_get(key, None) == [10, {"9": 0.71, "10": 0.70}]
    assert tune._file_get(("plan", 26, 5000, "bic", None), None) == 13
    assert len(json.loads(path.read_text())) == 2


def test_file_cache_off_and_unreadable(tmp_path, monkeypatch):
    monkeypatch.setattr(tune, "_file_key", lambda key, device: repr(key))
    monkeypatch.setenv("GS_TUNE_CACHE", "off")
    tune._file_put(("plan", 8, 100, "bic", None), None, 7)
    assert tune._file_get(("plan", 8, 100, "bic", None), None) is None
    bad = tmp_path / "tune.json"
    bad.write_text("not json")
    monkeypatch.setenv("GS_TUNE_CACHE", str(bad))
    assert tune._file_get(("plan", 8, 100, "bic", None), None) is None
    tune._file_put(("plan", 8, 100, "bic", None), None, 7)  # replaces the broken file
    assert tune._file_get(("plan", 8, 100, "bic", None), None) == 7
