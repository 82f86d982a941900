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


def test_vacuum_tile_cells_validated(L):
    """Wide vacuum tiles: 768, 1024, 1536 or 2048 nodes, wider than the other
    tiles, one-wave tiles, not in the FP32 delta ablation."""
    p = W.slab_c1()
    for kw in ({"vacuum_tile_cells": 1024}, {"vacuum_tile_cells": 2048, "tile_cells": 256},
               {"vacuum_tile_cells": 768, "precision": "f32"}):
        d, keep = _desc(p, exec="tiled", **kw)
        assert _code(d)[0] == 0, kw
    for kw in ({"vacuum_tile_cells": 1000}, {"vacuum_tile_cells": 512},
               {"vacuum_tile_cells": 768, "tile_cells": 1024}, {"vacuum_tile_cells": 1024, "tile_waves": 2},
               {"vacuum_tile_cells": 1024, "precision": "f32d"}):
        d, keep = _desc(p, exec="tiled", **kw)
        assert _code(d)[0] == -1, kw
        assert b"vacuum_tile_cells" in L.lib().fdtd_plasma_last_error() or \
            b"FDTD_F32_DELTA" in L.lib().fdtd_plasma_last_error()


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


# ---- 3D library (include/fdtd_plasma3d.h) ----------------------------------

def _p3(**kw):
    from tests.test_oracle3d_pins import mk
    base = dict(cpml=2, source="tfsf", b0=4, b1=9,
                points=np.array([(0, 5, 5, 5), (4, 6, 5, 7)], np.int32))
    base.update(kw)
    return mk(12, 12, 16, **base)


def _code3(p, **kw):
    from paper_1709_00821_amd.plasma3d import make_desc3
    d, keep = make_desc3(p, **kw)
    n = ctypes.c_size_t()
    from paper_1709_00821_amd import _lib
    rc = _lib.lib().fdtd3d_workspace_bytes(ctypes.byref(d), ctypes.byref(n))
    return rc, n.value, d


def test_3d_exports_every_header_function(L):
    syms = L.header_symbols(L.HEADER3)
    assert len(syms) >= 10 and all(s.startswith("fdtd3d_") for s in syms)
    out = subprocess.run(["nm", "-D", "--defined-only", SO], capture_output=True, text=True,
                         check=True).stdout
    exported = {line.split()[-1] for line in out.splitlines() if line.strip()}
    assert not [s for s in syms if s not in exported]


def test_3d_valid_descriptor_plans(L):
    rc, n, _ = _code3(_p3())
    assert rc == 0 and n > 0
    rc64, n64, _ = _code3(_p3(), precision="f64")
    assert rc64 == 0 and n64 > n          # FP64 fields take more room


def test_3d_plasma_support_is_compact(L):
    """Only rows holding plasma carry J and coefficients: a one-row plasma
    costs far less than a full one."""
    p = _p3()
    w_one = np.zeros_like(p.wp2)
    w_one[0, 6, 6, 3:9] = 1e21
    w_all = np.full_like(p.wp2, 1e21)
    _, n_vac, _ = _code3(p)
    _, n_one, _ = _code3(p.copy(wp2=w_one))
    _, n_all, _ = _code3(p.copy(wp2=w_all))
    assert n_one - n_vac < 4096
    assert n_all - n_vac >= 0.95 * 12 * 12 * 16 * (3 * 4 + 6 * 8)   # J (f32) + wp2, nu (f64)


@pytest.mark.parametrize("mutate,code", [
    (lambda p: p.copy(dt=p.dt * 1.2), -2),                       # c dt/d above 1/sqrt(3)
    (lambda p: p.copy(b0=0), -1),
    (lambda p: p.copy(b1=12), -1),                                # past the walled x face
    (lambda p: p.copy(cpml=8), -1),
    (lambda p: p.copy(points=np.array([(6, 0, 0, 0)], np.int32)), -1),
    (lambda p: p.copy(points=np.array([(0, 12, 0, 0)], np.int32)), -1),
    (lambda p: p.copy(source="planar", src_comp=2), -1),
    (lambda p: p.copy(source="planar", src_k=16), -1),
    (lambda p: p.copy(wp2=np.where(np.arange(16) == 3, -1.0, p.wp2)), -1),
    (lambda p: p.copy(nu=np.where(np.arange(16) == 3, np.nan, p.nu)), -1),
])
def test_3d_invalid_descriptors_rejected(L, mutate, code):
    rc, _, _ = _code3(mutate(_p3()))
    assert rc == code
    assert len(L.lib().fdtd3d_last_error()) > 0


def test_3d_struct_size_and_slots(L):
    rc, _, d = _code3(_p3(), sample_slots=33)
    assert rc == -1
    d.sample_slots = 0
    d.struct_size -= 8
    n = ctypes.c_size_t()
    assert L.lib().fdtd3d_workspace_bytes(ctypes.byref(d), ctypes.byref(n)) == -1


def test_3d_null_handle(L):
    lib = L.lib()
    assert lib.fdtd3d_step(None, 1) == -1
    assert lib.fdtd3d_destroy(None) == 0


def test_fp32_delta_ablation_plans(L):
    """FDTD_F32_DELTA (FP32 eq.(11) ablation) plans on the per-step executor
    and on one-wave tiles of 256 or 512 nodes; the resident and mixed
    executors, other tile shapes and checkpoints are refused."""
    p = W.slab_c1()
    for kw in ({"exec": "auto"}, {"exec": "step"}, {"exec": "tiled"}, {"exec": "tiled", "tile_cells": 256}):
        d, keep = _desc(p, precision="f32d", **kw)
        assert _code(d)[0] == 0, kw
    for kw in ({"exec": "resident"}, {"exec": "mixed"}, {"exec": "tiled", "tile_cells": 768},
               {"exec": "tiled", "tile_waves": 2}, {"checkpoint": 64}):
        d, keep = _desc(p, precision="f32d", **kw)
        assert _code(d)[0] == -1, kw
        assert b"FDTD_F32_DELTA" in L.lib().fdtd_plasma_last_error()


def test_grid_length_limit(L):
    """Tiles address nodes with 32-bit indices: a grid of 2^31 nodes is
    rejected (before any node array is read)."""
    p = W.slab_c1(n=64, slab=(20, 30), src=10, probes=(5, 50))
    d, keep = _desc(p)
    big = np.array([1 << 31], np.int64)
    d.cells = big.ctypes.data
    rc, _ = _code(d)
    assert rc == -1
    msg = L.lib().fdtd_plasma_last_error()
    msg = msg.decode() if isinstance(msg, bytes) else str(msg)
    assert "2^31 - 1" in msg


def test_static_workspace_limit(L):
    """fdtd_plasma_create_static refuses a descriptor whose workspace exceeds
    the static array before any device call (so this runs without a GPU)."""
    p = W.slab_c1(n=600000, slab=(1000, 2000), src=500, probes=(100, 599000))
    d, keep = _desc(p)
    rc, need = _code(d)
    assert rc == 0 and need > (16 << 20)
    h = ctypes.c_void_p()
    rc = L.lib().fdtd_plasma_create_static(ctypes.byref(d), ctypes.byref(h))
    assert rc == -3 and not h.value
    msg = L.lib().fdtd_plasma_last_error()
    msg = msg.decode() if isinstance(msg, bytes) else str(msg)
    assert "static" in msg


def test_2d_exports_and_validation(L):
    syms = L.header_symbols(L.HEADER2)
    assert "fdtd2d_create" in syms and "fdtd2d_run" in syms
    lib = L.lib()
    for s in syms:
        assert hasattr(lib, s)
    from paper_1709_00821_amd.plasma2d import make_desc2
    p = W.random_2d(np.random.default_rng(3), "te", 20, 24)
    for q, code in ((p, 0), (p.copy(dt=0.75 * p.d / 299792458.0), -2),
                    (p.copy(probes=np.array([[2, 1, 1]])), -1), (p.copy(src=(20, 3)), -1),
                    (p.copy(wp2=-p.wp2 - 1.0), -1)):
        d, keep = make_desc2(q)
        n = ctypes.c_size_t()
        assert lib.fdtd2d_workspace_bytes(ctypes.byref(d), ctypes.byref(n)) == code
