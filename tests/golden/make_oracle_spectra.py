"""Stored oracle spectra for the accuracy figures of the bench.

Writes c2_oracle_spectra.json, c1_oracle_spectra.json and
c4_oracle_spectra.json next to this file (or the ones named: c2 c1 c4).
The first holds the FP64 serial oracle's
probe spectra X[probe][frequency] of the default bench workload (the
2^24-cell half-plasma grid with CPML ends, 20000 steps, eqs.(11)-(15)) and of
its plasma-free reference run, from which the two-run reflection and
transmission follow.  Outside the source's light cone the fields of a
zero-initial-state run stay exactly zero for the whole run, so the oracle
runs on the trimmed grid (PEC ends beyond the cone), which yields the full
grid's spectra exactly.  The second holds the same two spectra of the
1000-cell slab with Mur ends (4096 steps), on which the bench states the
error of the FP32 modes.  Calls only the oracle and the seeded generators.

    python tests/golden/make_oracle_spectra.py [c2] [c1] [c4]

The third holds, for six slabs of the 4096-slab batch (8000 steps, 64
frequencies), the oracle spectra of the slab and of its plasma-free run.
"""
from __future__ import annotations

import json
import os
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
OUT = os.path.join(HERE, "c2_oracle_spectra.json")
OUT_C1 = os.path.join(HERE, "c1_oracle_spectra.json")
CELLS, STEPS = 1 << 24, 20000


def lightcone_spectra(p, steps):
    import oracle
    from paper_1709_00821_amd import workloads as W
    lo, hi = W.light_cone(p, steps)
    wp2 = p.wp2[lo:hi].copy()
    wp2[0] = wp2[-1] = 0.0
    q = p.copy(n=hi - lo, wp2=wp2, nu=p.nu[lo:hi].copy(), src_cell=p.src_cell - lo,
               probes=p.probes - lo, bc="pec", cpml_cells=0)
    return oracle.run(q, steps)["X"]


def compute(cells=CELLS, steps=STEPS):
    from paper_1709_00821_amd import workloads as W
    p = W.large_c2(n=cells, steps=steps)
    out = {"workload": "large_c2", "cells": cells, "steps": steps,
           "freqs_hz": [float(f) for f in p.freqs]}
    for name, q in (("plasma", p), ("vacuum", p.vacuum())):
        X = lightcone_spectra(q, steps)
        out[name] = {"re": [[float(v) for v in row.real] for row in X],
                     "im": [[float(v) for v in row.imag] for row in X]}
    return out


def compute_c1():
    import oracle
    from paper_1709_00821_amd import workloads as W
    p = W.slab_c1()
    out = {"workload": "slab_c1", "cells": p.n, "steps": p.steps, "freqs_hz": [float(f) for f in p.freqs]}
    for name, q in (("plasma", p), ("vacuum", p.vacuum())):
        X = oracle.run(q, p.steps)["X"]
        out[name] = {"re": [[float(v) for v in row.real] for row in X],
                     "im": [[float(v) for v in row.imag] for row in X]}
    return out


OUT_C4 = os.path.join(HERE, "c4_oracle_spectra.json")
# the batch's sampled slabs: first, last, shortest, longest, two more
C4_SLABS = "first, last, shortest, longest, 1000, 3000"


def c4_sample(slabs):
    import numpy as np
    lens = np.array([q.n for q in slabs])
    return sorted({0, len(slabs) - 1, int(np.argmin(lens)), int(np.argmax(lens)), 1000, 3000})


def compute_c4():
    """Oracle spectra of the sampled slabs of the 4096-slab batch (8000 steps,
    64 frequencies) and of their plasma-free runs, slab by slab."""
    import oracle
    from paper_1709_00821_amd import workloads as W
    slabs = W.batch_c4()
    pick = c4_sample(slabs)
    steps = slabs[0].steps
    out = {"workload": "batch_c4", "slabs": pick, "steps": steps,
           "freqs_hz": [float(f) for f in slabs[0].freqs], "plasma": [], "vacuum": []}
    for b in pick:
        for name, q in (("plasma", slabs[b]), ("vacuum", slabs[b].vacuum())):
            X = oracle.run(q, steps)["X"]
            out[name].append({"re": [[float(v) for v in row.real] for row in X],
                              "im": [[float(v) for v in row.imag] for row in X]})
    return out


def load_c4(path=OUT_C4):
    """(config dict, X plasma [slab][probe][f], X vacuum) as complex arrays."""
    import numpy as np
    d = json.load(open(path))
    X = {k: np.array([np.array(e["re"]) + 1j * np.array(e["im"]) for e in d[k]]) for k in ("plasma", "vacuum")}
    return d, X["plasma"], X["vacuum"]


def load(path=OUT):
    """(config dict, X plasma, X vacuum) as complex arrays [probe][frequency]."""
    import numpy as np
    d = json.load(open(path))
    X = {k: np.array(d[k]["re"]) + 1j * np.array(d[k]["im"]) for k in ("plasma", "vacuum")}
    return d, X["plasma"], X["vacuum"]


if __name__ == "__main__":
    sys.path.insert(0, ROOT)
    which = sys.argv[1:] or ["c2", "c1", "c4"]
    for key, fn, out in (("c2", compute, OUT), ("c1", compute_c1, OUT_C1), ("c4", compute_c4, OUT_C4)):
        if key in which:
            json.dump(fn(), open(out, "w"))
            print("wrote", out)
