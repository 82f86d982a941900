"""ctypes binding of libfdtd_plasma.so (argument marshalling only).

torch is imported first so that the library binds to the HIP runtime torch
already loaded (both use the soname libamdhip64.so.7), letting torch tensors
serve as device workspaces and torch streams as launch streams.
"""
from __future__ import annotations

import ctypes
import os
import re

import torch  # noqa: F401  (must precede loading the HIP library)

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libfdtd_plasma.so")
HEADER = os.path.join(os.path.dirname(HERE), "include", "fdtd_plasma.h")
HEADER3 = os.path.join(os.path.dirname(HERE), "include", "fdtd_plasma3d.h")
HEADER2 = os.path.join(os.path.dirname(HERE), "include", "fdtd_plasma2d.h")

# status codes and enums (include/fdtd_plasma.h)
OK, E_INVALID, E_UNSTABLE, E_WORKSPACE, E_DEVICE, E_STATE, E_NONFINITE, E_UNSUPPORTED = \
    0, -1, -2, -3, -4, -5, -6, -7
F64, F32, F32_DELTA = 0, 1, 2
BC = {"mur": 0, "cpml": 1, "pec": 2}
EXEC = {"auto": 0, "step": 1, "tiled": 2, "resident": 3, "mixed": 4}
FLAG_CHECKPOINT = 0x1
FLAG_RECORD = 0x2


class FdtdError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"fdtd_plasma error {code}: {msg}")
        self.code = code


class Desc(ctypes.Structure):
    _fields_ = [
        ("struct_size", ctypes.c_uint32),
        ("precision", ctypes.c_int32),
        ("scheme", ctypes.c_int32),
        ("bc", ctypes.c_int32),
        ("exec", ctypes.c_int32),
        ("flags", ctypes.c_int32),
        ("batch", ctypes.c_int64),
        ("cells", ctypes.c_void_p),
        ("dz", ctypes.c_double),
        ("dt", ctypes.c_double),
        ("wp2", ctypes.c_void_p),
        ("nu", ctypes.c_void_p),
        ("src_cell", ctypes.c_void_p),
        ("src_tau", ctypes.c_double),
        ("src_t0", ctypes.c_double),
        ("src_amp", ctypes.c_double),
        ("n_probes", ctypes.c_int32),
        ("n_freqs", ctypes.c_int32),
        ("probe_cells", ctypes.c_void_p),
        ("freqs_hz", ctypes.c_void_p),
        ("cpml_cells", ctypes.c_int32),
        ("tile_cells", ctypes.c_int32),
        ("cpml_m", ctypes.c_double),
        ("cpml_sigma_max", ctypes.c_double),
        ("steps_per_pass", ctypes.c_int32),
        ("checkpoint_steps", ctypes.c_int32),
        ("tile_waves", ctypes.c_int32),
        ("record_steps", ctypes.c_int32),
        ("vacuum_tile_cells", ctypes.c_int32),
        ("stream", ctypes.c_void_p),
    ]


class Desc3(ctypes.Structure):
    """fdtd3d_desc (include/fdtd_plasma3d.h)."""
    _fields_ = [
        ("struct_size", ctypes.c_int32),
        ("precision", ctypes.c_int32),
        ("nx", ctypes.c_int64), ("ny", ctypes.c_int64), ("nz", ctypes.c_int64),
        ("d", ctypes.c_double), ("dt", ctypes.c_double),
        ("wp2", ctypes.c_void_p * 3),
        ("nu", ctypes.c_void_p * 3),
        ("periodic_x", ctypes.c_int32), ("periodic_y", ctypes.c_int32),
        ("cpml_cells", ctypes.c_int32),
        ("source", ctypes.c_int32),
        ("src_comp", ctypes.c_int32),
        ("src_k", ctypes.c_int64),
        ("src_tau", ctypes.c_double), ("src_t0", ctypes.c_double), ("src_amp", ctypes.c_double),
        ("tf_lo", ctypes.c_int64), ("tf_hi", ctypes.c_int64),
        ("n_points", ctypes.c_int32), ("n_freqs", ctypes.c_int32),
        ("points", ctypes.c_void_p),
        ("freqs_hz", ctypes.c_void_p),
        ("sample_slots", ctypes.c_int32),
        ("exec", ctypes.c_int32),
        ("x_planes", ctypes.c_int32),
        ("reserved", ctypes.c_int32),
        ("stream", ctypes.c_void_p),
    ]


SRC3 = {"none": 0, "planar": 1, "tfsf": 2}
EXEC3 = {"auto": 0, "split": 1, "fused": 2}
FIELDS3 = ("Ex", "Ey", "Ez", "Hx", "Hy", "Hz", "Jx", "Jy", "Jz")

class Desc2(ctypes.Structure):
    """fdtd2d_desc (include/fdtd_plasma2d.h)."""
    _fields_ = [
        ("struct_size", ctypes.c_uint32),
        ("mode", ctypes.c_int32),
        ("precision", ctypes.c_int32),
        ("periodic_x", ctypes.c_int32),
        ("periodic_y", ctypes.c_int32),
        ("nx", ctypes.c_int64),
        ("ny", ctypes.c_int64),
        ("d", ctypes.c_double),
        ("dt", ctypes.c_double),
        ("wp2", ctypes.c_void_p),
        ("nu", ctypes.c_void_p),
        ("has_src", ctypes.c_int32),
        ("n_probes", ctypes.c_int32),
        ("src_i", ctypes.c_int64),
        ("src_j", ctypes.c_int64),
        ("src_tau", ctypes.c_double),
        ("src_t0", ctypes.c_double),
        ("src_amp", ctypes.c_double),
        ("n_freqs", ctypes.c_int32),
        ("reserved", ctypes.c_int32),
        ("probes", ctypes.c_void_p),
        ("freqs_hz", ctypes.c_void_p),
        ("stream", ctypes.c_void_p),
    ]


_lib = None


def lib():
    """Load the HIP library; raises if it has not been built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(
                f"{LIB_PATH} is missing: build it with `python -c 'import __graft_entry__ as g; g.build()'`")
        L = ctypes.CDLL(LIB_PATH)
        p, i32, i64, d = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_double
        sig = {
            "fdtd_plasma_workspace_bytes": [p, p],
            "fdtd_plasma_create": [p, p, ctypes.c_size_t, p],
            "fdtd_plasma_create_static": [p, p],
            "fdtd_plasma_step": [p, i64],
            "fdtd_plasma_run": [p, i64],
            "fdtd_plasma_probe_spectra": [p, p, p],
            "fdtd_plasma_probe_series": [p, p],
            "fdtd_plasma_probe_fft": [p, i64, p, p],
            "fdtd_plasma_get_fields": [p, i64, p, p, p],
            "fdtd_plasma_steps_done": [p, p],
            "fdtd_plasma_grad_r2": [p, i64, i32, p, p, p, p],
            "fdtd_plasma_loss_r2": [p, i32, p, p, p],
            "fdtd_plasma_profile": [p, i64, i32, p, p, p, p, p],
            "fdtd_plasma_destroy": [p],
            "fdtd3d_workspace_bytes": [p, p],
            "fdtd3d_create": [p, p, ctypes.c_size_t, p],
            "fdtd3d_step": [p, i64],
            "fdtd3d_run": [p, i64],
            "fdtd3d_spectra": [p, p, p],
            "fdtd3d_get_fields": [p, i32, p],
            "fdtd3d_set_fields": [p, i32, p],
            "fdtd3d_steps_done": [p, p],
            "fdtd3d_profile": [p, i32],
            "fdtd3d_profile_read": [p, i32, p, p, p, p, p],
            "fdtd3d_destroy": [p],
            "fdtd2d_workspace_bytes": [p, p],
            "fdtd2d_create": [p, p, ctypes.c_size_t, p],
            "fdtd2d_step": [p, i64],
            "fdtd2d_run": [p, i64],
            "fdtd2d_spectra": [p, p, p],
            "fdtd2d_get_fields": [p, i32, p],
            "fdtd2d_steps_done": [p, p],
            "fdtd2d_destroy": [p],
        }
        for name, args in sig.items():
            fn = getattr(L, name)
            fn.argtypes = args
            fn.restype = ctypes.c_int
        L.fdtd_plasma_last_error.argtypes = []
        L.fdtd_plasma_last_error.restype = ctypes.c_char_p
        L.fdtd3d_last_error.argtypes = []
        L.fdtd3d_last_error.restype = ctypes.c_char_p
        L.fdtd2d_last_error.argtypes = []
        L.fdtd2d_last_error.restype = ctypes.c_char_p
        _lib = L
    return _lib


def check(rc: int):
    if rc != OK:
        msg = lib().fdtd_plasma_last_error().decode(errors="replace")
        raise FdtdError(rc, msg)
    return rc


def check3(rc: int):
    if rc != OK:
        msg = lib().fdtd3d_last_error().decode(errors="replace")
        raise FdtdError(rc, msg)
    return rc


def check2(rc: int):
    if rc != OK:
        msg = lib().fdtd2d_last_error().decode(errors="replace")
        raise FdtdError(rc, msg)
    return rc


def header_symbols(path: str = HEADER):
    """Function names a public header declares."""
    txt = open(path).read()
    return sorted(set(re.findall(r"\b(fdtd(?:_plasma|3d|2d)_[a-z0-9_]+)\s*\(", txt)))
