"""Launch-shape choice for the temporally blocked executor.

pick() returns the (tile_cells, steps_per_pass, tile_waves, vacuum_tile_cells) to use
for a precision and workload: an explicit override, else the best entry measured by
`python -m paper_1709_00821_amd.tune` on this GPU (tuning.json next to this
file), else a default.  Three workloads are tuned: one long grid ("large":
half plasma, CPML ends), a batch of short independent slabs ("batched": Mur
ends, a source and two probes per slab, so that tiles holding a grid end are
a sizeable share) and one short grid ("small": 8000 nodes, where a launch is
a few waves and latency rather than throughput decides).  After the shape
sweep, the width of the all-vacuum tiles (vacuum_tile_cells) is swept at the
best shape.
"""
from __future__ import annotations

import json
import os

HERE = os.path.dirname(os.path.abspath(__file__))
CACHE = os.path.join(HERE, "tuning.json")
DEFAULT = {"tile_cells": 512, "steps_per_pass": 48, "tile_waves": 1, "vacuum_tile_cells": 0}
VACUUM_WIDTHS = (768, 1024, 1536, 2048)


def _bucket(n: int, batched: bool = False) -> str:
    if batched:
        return "batched"
    return "large" if n >= (1 << 20) else "small"


def pick(precision: str, n: int, tile_cells: int = 0, steps_per_pass: int = 0, tile_waves: int = 0,
         batched: bool = False) -> dict:
    out = dict(DEFAULT)
    if os.path.exists(CACHE):
        try:
            table = json.load(open(CACHE)).get("gfx950", {})
            ent = table.get(precision, {}).get(_bucket(n, batched))
            if ent is None and precision == "f32d":   # the FP32 ablation, untuned: the FP32 shapes
                ent = table.get("f32", {}).get(_bucket(n, batched))
            if ent:
                out.update({k: int(ent[k]) for k in ("tile_cells", "steps_per_pass", "tile_waves",
                                                     "vacuum_tile_cells") if k in ent})
        except (OSError, ValueError, KeyError):
            pass
    if tile_cells:
        out["tile_cells"] = tile_cells
        if out["vacuum_tile_cells"] <= tile_cells:
            out["vacuum_tile_cells"] = 0
    if steps_per_pass:
        out["steps_per_pass"] = steps_per_pass
    if tile_waves:
        out["tile_waves"] = tile_waves
    if out["tile_waves"] > 1 or precision == "f32d":
        out["vacuum_tile_cells"] = 0
    return out


def _workload(workload: str, n: int, steps: int):
    from . import workloads as W
    if workload == "batched":
        p = W.batch_c4(n_slabs=max(1, n // 4096), steps=steps)
        return p, sum(q.n for q in p)
    if workload == "small":
        p = W.adjoint_c5(steps=steps)
        return p, p.n
    return W.large_c2(n=n, steps=steps), n


def _time_run(p, steps: int, reps: int, precision: str, **shape) -> float:
    """Median ms of reps runs of run(steps) (graph replay, after one
    capturing run)."""
    import torch
    from .plasma import FdtdPlasma
    h = FdtdPlasma(p, precision=precision, exec="tiled", **shape)
    h.run(steps)
    h.synchronize()
    ts = []
    for _ in range(reps):
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record(h.stream)
        h.run(steps)
        e1.record(h.stream)
        e1.synchronize()
        ts.append(e0.elapsed_time(e1))
    h.close()
    ts.sort()
    return 0.5 * (ts[(reps - 1) // 2] + ts[reps // 2])


VACUUM_MARGIN = 1.01    # a wider vacuum tile is kept only if it beats width 0 by 1%


def sweep_vacuum(precision: str, shape: dict, n: int = 1 << 22, steps: int = 2000, reps: int = 5,
                 log=print, workload: str = "large"):
    """At a launch shape (one-wave tiles), time run(steps) with every tile as
    wide as the others (0) and with the all-vacuum tiles of each wider width
    (median of reps runs each); returns [(vacuum_tile_cells, Mcell-updates/s)]."""
    p, n = _workload(workload, n, steps)
    out = []
    for v in (0,) + tuple(w for w in VACUUM_WIDTHS if w > shape["tile_cells"]):
        ms = _time_run(p, steps, reps, precision, vacuum_tile_cells=v, **shape)
        rate = n * steps / (ms / 1e3) / 1e6
        out.append((v, rate))
        log(f"tune {workload} {precision} {shape} vacuum_tile_cells={v:5d}: {ms:8.3f} ms {rate:10.0f} Mcell/s")
    return out


def sweep(precision: str, n: int = 1 << 22, steps: int = 2000, reps: int = 2,
          tiles=(256, 512, 768, 1024), depths=(8, 12, 16, 24, 32, 48, 64), waves=(1,), log=print,
          workload: str = "large"):
    """Time run(steps) for every launch shape on a plasma/vacuum grid of n
    cells (workload "large"), on a batch of n // 4096 slabs of 200-8000
    cells (workload "batched") or on one 8000-node grid (workload "small");
    returns ([(tile_cells, steps_per_pass, tile_waves, Mcell-updates/s)],
    nodes of the workload)."""
    p, n = _workload(workload, n, steps)
    out = []
    for wv in waves:
        for tc in tiles:
            if wv > 1 and tc > 512:
                continue
            for k in depths:
                if wv * tc <= 2 * k + 64:
                    continue
                ms = _time_run(p, steps, reps, precision, tile_cells=tc, steps_per_pass=k, tile_waves=wv)
                rate = n * steps / (ms / 1e3) / 1e6
                out.append((tc, k, wv, rate))
                log(f"tune {workload} {precision} tile_cells={tc:5d} steps_per_pass={k:3d} tile_waves={wv}: "
                    f"{ms:8.3f} ms {rate:10.0f} Mcell/s")
    return out, n


def main(argv=None):
    import argparse
    ap = argparse.ArgumentParser(description="sweep launch shapes and record the best")
    ap.add_argument("--precision", nargs="+", default=["f32", "f64", "f32d"])
    ap.add_argument("--workload", nargs="+", default=["large", "batched", "small"],
                    choices=["large", "batched", "small"])
    ap.add_argument("--cells", type=int, default=1 << 22)
    ap.add_argument("--steps", type=int, default=2000)
    ap.add_argument("--out", default=CACHE)
    ap.add_argument("--tiles", type=int, nargs="+", default=[256, 512, 768, 1024])
    ap.add_argument("--depths", type=int, nargs="+", default=[8, 12, 16, 24, 32, 48, 64])
    ap.add_argument("--waves", type=int, nargs="+", default=[1, 2, 4, 8])
    ap.add_argument("--vacuum-only", action="store_true",
                    help="keep the recorded shapes; sweep only the vacuum tile width at each")
    args = ap.parse_args(argv)
    table = {}
    if os.path.exists(args.out):
        try:
            table = json.load(open(args.out))
        except ValueError:
            table = {}
    g = table.setdefault("gfx950", {})
    log = lambda m: print(m, flush=True)
    for wl in args.workload:
        for prec in args.precision:
            ent = g.setdefault(prec, {})
            if not args.vacuum_only:
                res, cells = sweep(prec, n=args.cells, steps=args.steps, tiles=tuple(args.tiles),
                                   depths=tuple(args.depths), waves=tuple(args.waves), log=log, workload=wl)
                tc, k, wv, rate = max(res, key=lambda r: r[3])
                ent[wl] = {"tile_cells": tc, "steps_per_pass": k, "tile_waves": wv, "mcells": round(rate, 1),
                           "cells": cells, "steps": args.steps,
                           "sweep": [[a, b, c, round(r, 1)] for a, b, c, r in res]}
                ent.pop("sweep", None)
                print(f"best {wl} {prec}: tile_cells={tc} steps_per_pass={k} tile_waves={wv} {rate:.0f} Mcell/s",
                      flush=True)
            e = ent.get(wl)
            if e is None or e["tile_waves"] != 1 or prec == "f32d":
                continue
            shape = {k: e[k] for k in ("tile_cells", "steps_per_pass", "tile_waves")}
            vres = sweep_vacuum(prec, shape, n=args.cells, steps=args.steps, log=log, workload=wl)
            v, vrate = max(vres, key=lambda r: r[1])
            if vrate < VACUUM_MARGIN * vres[0][1]:      # within the noise of width 0
                v, vrate = vres[0]
            e["vacuum_tile_cells"] = v
            e["vacuum_sweep"] = [[a, round(r, 1)] for a, r in vres]
            print(f"best {wl} {prec}: vacuum_tile_cells={v} {vrate:.0f} Mcell/s", flush=True)
    json.dump(table, open(args.out, "w"), indent=1)


if __name__ == "__main__":
    main()
