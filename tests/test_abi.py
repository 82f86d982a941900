"""C-ABI contract on the CPU: the library loads, exports every function the
public header declares, and validates descriptors (no GPU work is issued:
fdtd_plasma_workspace_bytes only plans)."""
import ctypes
import os
import subprocess

import numpy as np
import pytest

from paper_1709_00821_amd import workloads as W

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SO = os.path.join(ROOT, "paper_1709_00821_amd", "libfdtd_plasma.so")


@pytest.fixture(scope="module")
def L():
    if not os.path.exists(SO):
        from paper_1709_00821_amd import build
        build.build()
    from paper_1709_00821_amd import _lib
    _lib.lib()
    return _lib


def test_exports_every_header_function(L):
    syms = L.header_symbols()
    assert len(syms) >= 10
    out = subprocess.run(["nm", "-D", "--defined-only", SO], capture_output=True, text=True,
                         check=True).stdout
    exported = {line.split()[-1] for line in out.splitlines() if line.strip()}
    missing = [s for s in syms if s not in exported]
    assert not missing, missing
    lib = L.lib()
    for s in syms:
        assert hasattr(lib, s)


def _desc(problems, **kw):
    from paper_1709_00821_amd.plasma import make_desc
    return make_desc(problems, **kw)


def _code(d):
    L_ = __import__("paper_1709_00821_amd._lib", fromlist=["lib"])
    n = ctypes.c_size_t()
    return L_.lib().fdtd_plasma_workspace_bytes(ctypes.byref(d), ctypes.byref(n)), n.value


def test_valid_descriptor_plans(L):
    d, keep = _desc(W.slab_c1())
    rc, n = _code(d)
    assert rc == 0 and n > 0
    # the state of 1000 nodes in FP64 plus spectra fits in a few MB
    assert n < 64 << 20


@pytest.mark.parametrize("mutate,code", [
    (lambda p: p.copy(dt=p.dz / 299792458.0 * 1.01), -2),        # Courant > 1
    (lambda p: p.copy(wp2=np.where(np.arange(p.n) == 5, -1.0, p.wp2)), -1),
    (lambda p: p.copy(nu=np.where(np.arange(p.n) == 7, np.nan, p.nu)), -1),
    (lambda p: p.copy(src_cell=0), -1),
    (lambda p: p.copy(src_cell=p.n - 1), -1),
    (lambda p: p.copy(probes=np.array([0, p.n])), -1),
    (lambda p: p.copy(wp2=np.where(np.arange(p.n) == 0, 1e20, p.wp2)), -1),
    (lambda p: p.copy(bc="cpml", cpml_cells=500), -1),
    (lambda p: p.copy(bc="cpml", cpml_cells=0), -1),
    (lambda p: p.copy(bc="cpml", cpml_cells=450), -7),             # plasma inside the CPML
    (lambda p: p.copy(freqs=np.array([])), -1),
])
def test_invalid_descriptors_rejected(L, mutate, code):
    p = mutate(W.slab_c1())
    d, keep = _desc(p)
    rc, _ = _code(d)
    assert rc == code
    assert len(L.lib().fdtd_plasma_last_error()) > 0


def test_struct_size_mismatch_rejected(L):
    d, keep = _desc(W.slab_c1())
    d.struct_size = 8
    rc, _ = _code(d)
    assert rc == -1 and b"struct_size" in L.lib().fdtd_plasma_last_error()


def test_bad_tuning_rejected(L):
    for kw, code in [({"tile_cells": 300}, -1), ({"steps_per_pass": 6}, -1),
                     ({"steps_per_pass": 128}, -1)]:
        d, keep = _desc(W.slab_c1(), **kw)
        assert _code(d)[0] == code


def test_resident_rejects_cpml_and_long_grids(L):
    p = W.slab_c1().copy(bc="cpml", cpml_cells=20, wp2=np.zeros(1000))
    d, keep = _desc(p, exec="resident")
    assert _code(d)[0] == -7
    big = W.slab_c1(n=200000, slab=(1000, 2000), probes=(10, 150000))
    d, keep = _desc(big, exec="resident")
    assert _code(d)[0] == -1
    d, keep = _desc(big, exec="auto")
    assert _code(d)[0] == 0


def test_null_handle_calls_fail_cleanly(L):
    lib = L.lib()
    assert lib.fdtd_plasma_step(None, 1) == -1
    assert lib.fdtd_plasma_destroy(None) == 0
    v = ctypes.c_int64()
    assert lib.fdtd_plasma_steps_done(None, ctypes.byref(v)) == -1


@pytest.mark.parametrize("exec_", ["step", "tiled", "resident", "auto"])
def test_create_runs_host_setup_without_gpu(L, exec_):
    """create() plans and builds its tables on the host before it touches the
    device; without a GPU it must fail with FDTD_E_DEVICE, not crash."""
    import torch
    if torch.cuda.is_available():
        pytest.skip("a GPU is present")
    rng = np.random.default_rng(5)
    probs = [W.random_slab(rng, n, n_freqs=3) for n in (100, 513, 3000)]
    probs = [q.copy(freqs=probs[0].freqs) for q in probs]
    d, keep = _desc(probs, exec=exec_)
    h = ctypes.c_void_p()
    rc = L.lib().fdtd_plasma_create(ctypes.byref(d), None, 0, ctypes.byref(h))
    assert rc == -4 and h.value is None
