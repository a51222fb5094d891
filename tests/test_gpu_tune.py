"""The autotuner on the device, and its file cache: a second process-level lookup
(in-process cache cleared) returns the stored choice without timing anything."""
import pytest
import torch

pytestmark = pytest.mark.gpu


def test_tune_plan_is_kept_in_the_file_cache(tmp_path, monkeypatch):
    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    from paper_1901_07643_amd import tune
    monkeypatch.setenv("GS_TUNE_CACHE", str(tmp_path / "tune.json"))
    tune.clear_cache()
    k = tune.tune_plan(9, 120, reps=2)
    assert k in tune.k_candidates(9)
    tune.clear_cache()

    def no_timing(*a, **kw):
        raise AssertionError("the cached choice should not be timed again")
    monkeypatch.setattr(tune, "_timed", no_timing)
    assert tune.tune_plan(9, 120, reps=2) == k
    shapes = [(8, 100), (9, 150)]
    monkeypatch.undo()
    monkeypatch.setenv("GS_TUNE_CACHE", str(tmp_path / "tune.json"))
    tune.clear_cache()
    cap, times = tune.tune_batch(shapes, reps=2)
    tune.clear_cache()
    monkeypatch.setattr(tune, "_timed", no_timing)
    assert tune.tune_batch(shapes, reps=2) == (cap, times)
    tune.clear_cache()
