"""Launch-shape choice (host logic only): the tuned table, its workload keys
and explicit overrides."""
import json

from paper_1709_00821_amd import tune as TU


def _table(tmp_path, monkeypatch):
    t = {"gfx950": {"f32": {"large": {"tile_cells": 768, "steps_per_pass": 64, "tile_waves": 1,
                                      "vacuum_tile_cells": 1024},
                            "batched": {"tile_cells": 256, "steps_per_pass": 32, "tile_waves": 2}}}}
    p = tmp_path / "tuning.json"
    p.write_text(json.dumps(t))
    monkeypatch.setattr(TU, "CACHE", str(p))


def test_pick_reads_workload_keys(tmp_path, monkeypatch):
    _table(tmp_path, monkeypatch)
    assert TU.pick("f32", 1 << 24) == {"tile_cells": 768, "steps_per_pass": 64, "tile_waves": 1,
                                       "vacuum_tile_cells": 1024}
    assert TU.pick("f32", 1 << 24, batched=True) == {"tile_cells": 256, "steps_per_pass": 32, "tile_waves": 2,
                                                     "vacuum_tile_cells": 0}
    # no "small" entry and no f64 entries: the defaults
    assert TU.pick("f32", 1000) == TU.DEFAULT
    assert TU.pick("f64", 1 << 24) == TU.DEFAULT


def test_pick_overrides_win(tmp_path, monkeypatch):
    _table(tmp_path, monkeypatch)
    got = TU.pick("f32", 1 << 24, tile_cells=512, steps_per_pass=16, tile_waves=4)
    assert got == {"tile_cells": 512, "steps_per_pass": 16, "tile_waves": 4, "vacuum_tile_cells": 0}
    # the wide vacuum tiles are kept only where the library takes them: wider
    # than the other tiles, one-wave tiles, not the FP32 delta ablation
    assert TU.pick("f32", 1 << 24, tile_cells=512)["vacuum_tile_cells"] == 1024
    assert TU.pick("f32", 1 << 24, tile_cells=1024)["vacuum_tile_cells"] == 0
    assert TU.pick("f32d", 1 << 24)["vacuum_tile_cells"] == 0


def test_pick_survives_a_broken_table(tmp_path, monkeypatch):
    p = tmp_path / "tuning.json"
    p.write_text("{not json")
    monkeypatch.setattr(TU, "CACHE", str(p))
    assert TU.pick("f32", 1 << 24) == TU.DEFAULT


def test_shipped_table_is_valid():
    """Every shipped entry is a launch shape the library accepts."""
    table = json.load(open(TU.CACHE))["gfx950"]
    for prec, ents in table.items():
        for wl, e in ents.items():
            assert wl in ("large", "small", "batched"), wl
            assert e["tile_cells"] % 64 == 0 and e["tile_cells"] // 64 in (4, 8, 12, 16)
            assert e["steps_per_pass"] % 4 == 0 and 4 <= e["steps_per_pass"] <= 64
            assert e["tile_waves"] in (1, 2, 4, 8)
            v = e.get("vacuum_tile_cells", 0)
            assert v == 0 or (v in TU.VACUUM_WIDTHS and v > e["tile_cells"] and e["tile_waves"] == 1
                              and prec != "f32d")
