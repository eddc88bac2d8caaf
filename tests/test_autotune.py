"""The autotuner's table (CPU): every entry is a configuration the batched launcher can run in one
mixed launch, choose() returns the nearest grid point, and a missing table falls back to the defaults."""
import importlib.util
import json
import os

import pytest

# loaded from its file: the package itself loads the HIP library, which these CPU tests do not need
_PATH = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "paper_2009_07914_amd",
                     "autotune.py")
_spec = importlib.util.spec_from_file_location("hc_autotune", _PATH)
autotune = importlib.util.module_from_spec(_spec)
_spec.loader.exec_module(autotune)

# (group size, window) pairs of the batched launcher's mixed launch
MIXED = {(1, 8), (2, 8), (4, 8), (8, 8), (2, 16), (4, 16), (8, 16), (16, 16), (4, 32), (8, 32), (16, 32)}


def test_tuning_table_entries_are_runnable():
    pts = json.load(open(autotune.TUNING_PATH))["points"]
    assert len(pts) >= 18
    for p in pts:
        assert p["scheme"] in ("linear", "quadratic", "double")
        assert (p["group_insert"], p["window"]) in MIXED and (p["group_query"], p["window"]) in MIXED
        assert p["insert_gops"] > 0 and p["retrieve_gops"] > 0


@pytest.mark.parametrize("log2_cap,load", [(10, 0.6), (16, 0.8), (24, 0.95), (22, 0.6)])
def test_choose_returns_the_grid_point(log2_cap, load):
    pts = json.load(open(autotune.TUNING_PATH))["points"]
    exp = [p for p in pts if p["log2_capacity"] == log2_cap and p["load"] == load][0]
    got = autotune.choose(1 << log2_cap, load)
    assert got == {k: exp[k] for k in ("scheme", "window", "group_insert", "group_query")}
    # a nearby capacity and load map to the same point
    assert autotune.choose(int((1 << log2_cap) * 1.2), load + 0.02) == got


def test_missing_table_falls_back_to_defaults(monkeypatch, tmp_path):
    monkeypatch.setattr(autotune, "TUNING_PATH", str(tmp_path / "absent.json"))
    monkeypatch.setattr(autotune, "_cache", None)
    assert autotune.choose(1 << 20, 0.9) == autotune.DEFAULT
