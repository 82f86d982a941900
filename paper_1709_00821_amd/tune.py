"""Launch-shape choice for the temporally blocked executor.

pick() returns the (tile_cells, steps_per_pass) to use for a precision and
grid size: an explicit override, else the best entry measured by
`python -m paper_1709_00821_amd.tune` on this GPU (tuning.json next to this
file), else a default.
"""
from __future__ import annotations

import json
import os

HERE = os.path.dirname(os.path.abspath(__file__))
CACHE = os.path.join(HERE, "tuning.json")
DEFAULT = {"tile_cells": 512, "steps_per_pass": 16}


def _bucket(n: int) -> str:
    return "large" if n >= (1 << 20) else "small"


def pick(precision: str, n: int, tile_cells: int = 0, steps_per_pass: int = 0) -> dict:
    out = dict(DEFAULT)
    if os.path.exists(CACHE):
        try:
            table = json.load(open(CACHE))
            ent = table.get("gfx950", {}).get(precision, {}).get(_bucket(n))
            if ent:
                out.update({k: int(ent[k]) for k in ("tile_cells", "steps_per_pass")})
        except (OSError, ValueError, KeyError):
            pass
    if tile_cells:
        out["tile_cells"] = tile_cells
    if steps_per_pass:
        out["steps_per_pass"] = steps_per_pass
    return out
