"""Stored oracle spectra for the accuracy figures of the bench.

Writes c2_oracle_spectra.json and c1_oracle_spectra.json next to this file.
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

    python tests/golden/make_oracle_spectra.py
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


def load(path=OUT):
    """(config dict, X plasma, X vacuum) as complex arrays [probe][frequency]."""
    import numpy as np
    d = json.load(open(path))
    X = {k: np.array(d[k]["re"]) + 1j * np.array(d[k]["im"]) for k in ("plasma", "vacuum")}
    return d, X["plasma"], X["vacuum"]


if __name__ == "__main__":
    sys.path.insert(0, ROOT)
    json.dump(compute(), open(OUT, "w"))
    json.dump(compute_c1(), open(OUT_C1, "w"))
    print("wrote", OUT, OUT_C1)
