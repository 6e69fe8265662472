"""Host logic of the layout autotuner: shape classes and the result cache."""
import json

import torch

from paper_2306_11612_amd import tune


def test_shape_key_rounds_to_powers_of_two():
    a = tune.shape_key(501_195_808, 4, torch.float32, 1920)
    b = tune.shape_key(480_000_000, 4, torch.float32, 2048)
    assert a == b == "n2^29_m4_float32_w2^11"
    assert tune.shape_key(10_000_000, 8, torch.bfloat16, 1024) == "n2^23_m8_bfloat16_w2^10"


def test_cache_round_trip(tmp_path, monkeypatch):
    monkeypatch.setenv("DVL_TUNE_CACHE", str(tmp_path / "sub" / "tune.json"))
    assert tune._load() == {}
    tune._store({"k": {"tile_steps": 8, "run_waves": 0, "ms": 1.0}})
    assert json.loads((tmp_path / "sub" / "tune.json").read_text())["k"]["tile_steps"] == 8
    assert tune._load()["k"]["ms"] == 1.0


def test_best_layout_uses_cache_without_measuring(tmp_path, monkeypatch):
    monkeypatch.setenv("DVL_TUNE_CACHE", str(tmp_path / "tune.json"))
    x = torch.zeros(1000, dtype=torch.int32)
    fields = [torch.zeros(1000)] * 4
    key = tune.shape_key(1000, 4, torch.float32, 64)
    tune._store({key: {"tile_steps": 32, "run_waves": 4096, "ms": 0.5}})

    def boom(*a, **k):
        raise AssertionError("must not measure when cached")
    monkeypatch.setattr(tune, "tune", boom)
    assert tune.best_layout(x, x, x, x, fields, 64)["tile_steps"] == 32


def test_candidates_are_valid_build_options():
    for ts, wpc in tune.CANDIDATES:
        assert ts in (8, 16, 32)
        assert wpc == 0 or 64 <= wpc * 256 <= 65536
