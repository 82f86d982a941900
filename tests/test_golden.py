"""The stored oracle spectra that bench.py reads for its accuracy figures are
the oracle's own output: regenerating them reproduces the file exactly."""
import os
import sys

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.join(HERE, "golden"))
import make_oracle_spectra as G  # noqa: E402


def test_stored_c2_spectra_are_the_oracles():
    d, Xo, Xvo = G.load()
    assert (d["cells"], d["steps"]) == (G.CELLS, G.STEPS)
    new = G.compute()
    assert new["freqs_hz"] == d["freqs_hz"]
    for name, X in (("plasma", Xo), ("vacuum", Xvo)):
        Y = np.array(new[name]["re"]) + 1j * np.array(new[name]["im"])
        assert np.array_equal(X, Y), name
    # the plasma-free run transmits the pulse: a nonzero spectrum at both probes
    assert np.all(np.abs(Xvo) > 0)


def test_stored_c1_spectra_are_the_oracles():
    d, Xo, Xvo = G.load(G.OUT_C1)
    new = G.compute_c1()
    assert (d["cells"], d["steps"], d["freqs_hz"]) == (new["cells"], new["steps"], new["freqs_hz"])
    for name, X in (("plasma", Xo), ("vacuum", Xvo)):
        Y = np.array(new[name]["re"]) + 1j * np.array(new[name]["im"])
        assert np.array_equal(X, Y), name


def test_stored_c4_spectra_are_the_oracles():
    d, Xo, Xvo = G.load_c4()
    new = G.compute_c4()
    assert (d["slabs"], d["steps"], d["freqs_hz"]) == (new["slabs"], new["steps"], new["freqs_hz"])
    for name, X in (("plasma", Xo), ("vacuum", Xvo)):
        Y = np.array([np.array(e["re"]) + 1j * np.array(e["im"]) for e in new[name]])
        assert np.array_equal(X, Y), name
    # the reflection probe sits next to the source; the transmission probe of
    # a slab longer than the pulse travels in 8000 steps sees nothing
    assert np.all(np.abs(Xvo[:, 0]) > 0)
