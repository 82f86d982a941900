"""fdtd_plasma_create_static (the workspace is the library's static device
array) against fdtd_plasma_create with an allocated workspace: the same
descriptor advanced the same way gives the same spectra and fields bit for
bit, on two handles in a row, the second on a smaller grid; a second static
handle while one is live is refused."""
import ctypes
import sys

import numpy as np
import pytest

from paper_1709_00821_amd import workloads as W

pytestmark = pytest.mark.gpu


def say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def _static_run(L, p, T, precision, stream):
    from paper_1709_00821_amd.plasma import make_desc
    d, keep = make_desc(p, precision=precision, exec="tiled", stream_handle=stream.cuda_stream)
    h = ctypes.c_void_p()
    L.check(L.lib().fdtd_plasma_create_static(ctypes.byref(d), ctypes.byref(h)))
    try:
        # while it is live, the device's array is taken
        h2 = ctypes.c_void_p()
        assert L.lib().fdtd_plasma_create_static(ctypes.byref(d), ctypes.byref(h2)) == L.E_STATE
        assert not h2.value
        L.check(L.lib().fdtd_plasma_step(h, T))
        P, F = d.n_probes, d.n_freqs
        re, im = np.zeros(P * F), np.zeros(P * F)
        L.check(L.lib().fdtd_plasma_probe_spectra(h, re.ctypes.data, im.ctypes.data))
        n = p.n
        E, H, J = np.zeros(n), np.zeros(n - 1), np.zeros(n)
        L.check(L.lib().fdtd_plasma_get_fields(h, 0, E.ctypes.data, H.ctypes.data, J.ctypes.data))
    finally:
        L.lib().fdtd_plasma_destroy(h)
    return (re + 1j * im).reshape(P, F), {"E": E, "H": H, "J": J}


@pytest.mark.parametrize("precision", ["f64", "f32"])
def test_static_workspace_matches_allocated(precision):
    import torch
    assert torch.cuda.is_available()
    from paper_1709_00821_amd import _lib as L
    from paper_1709_00821_amd.plasma import FdtdPlasma
    stream = torch.cuda.Stream()
    cases = [(W.slab_c1(), 1500),
             (W.slab_c1(n=300, slab=(120, 160), src=40, probes=(20, 260), n_freqs=16), 600)]
    for p, T in cases:
        say(f"case no-alloc {precision} n={p.n} steps={T}")
        Xs, Fs = _static_run(L, p, T, precision, stream)
        with FdtdPlasma(p, precision=precision, exec="tiled") as h:
            h.step(T)
            X = h.spectra()[0]
            F = h.fields()
        assert np.array_equal(Xs, X)
        for k in ("E", "H", "J"):
            assert np.array_equal(Fs[k], F[k]), k
        assert np.max(np.abs(X)) > 0
