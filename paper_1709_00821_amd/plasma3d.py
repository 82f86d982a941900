"""Python face of the 3D library (include/fdtd_plasma3d.h): argument
marshalling only.  Every step of the time loop runs in the HIP kernels; torch
provides the device workspace (a uint8 tensor) and the stream."""
from __future__ import annotations

import ctypes
from typing import Optional, Union

import numpy as np
import torch

from . import _lib as L
from .workloads import Problem3D


def make_desc3(p: Problem3D, precision: str = "f32", sample_slots: int = 0, stream_handle: int = 0,
               exec: str = "auto", x_planes: int = 0):
    """The C descriptor of a 3D problem; returns (desc, arrays it points into)."""
    wp2 = [np.ascontiguousarray(p.wp2[c], np.float64) for c in range(3)]
    if p.nu.ndim == 3:
        nu0 = np.ascontiguousarray(p.nu, np.float64)
        nu = [nu0, nu0, nu0]
    else:
        nu = [np.ascontiguousarray(p.nu[c], np.float64) for c in range(3)]
    pts = np.ascontiguousarray(np.asarray(p.points, np.int32).reshape(-1, 4))
    freqs = np.ascontiguousarray(p.freqs, np.float64)
    d = L.Desc3()
    d.struct_size = ctypes.sizeof(L.Desc3)
    d.precision = {"f64": L.F64, "f32": L.F32}[precision]
    d.nx, d.ny, d.nz = p.nx, p.ny, p.nz
    d.d, d.dt = p.d, p.dt
    d.wp2 = (ctypes.c_void_p * 3)(*[a.ctypes.data for a in wp2])
    d.nu = (ctypes.c_void_p * 3)(*[a.ctypes.data for a in nu])
    d.periodic_x, d.periodic_y = int(p.periodic_x), int(p.periodic_y)
    d.cpml_cells = p.cpml
    d.source = L.SRC3[p.source]
    d.src_comp, d.src_k = p.src_comp, p.src_k
    d.src_tau, d.src_t0, d.src_amp = p.src_tau, p.src_t0, p.src_amp
    d.tf_lo, d.tf_hi = p.b0, p.b1
    d.n_points, d.n_freqs = len(pts), len(freqs)
    d.points = pts.ctypes.data if len(pts) else None
    d.freqs_hz = freqs.ctypes.data if len(freqs) else None
    d.sample_slots = sample_slots
    d.exec = L.EXEC3[exec]
    d.x_planes = x_planes
    d.stream = stream_handle or None
    return d, [wp2, nu, pts, freqs]


def workspace_bytes3(desc) -> int:
    n = ctypes.c_size_t()
    L.check3(L.lib().fdtd3d_workspace_bytes(ctypes.byref(desc), ctypes.byref(n)))
    return n.value


class FdtdPlasma3D:
    """One 3D Yee-RKETD grid."""

    def __init__(self, problem: Problem3D, precision: str = "f32", sample_slots: int = 0,
                 exec: str = "auto", x_planes: int = 0, stream: Optional[torch.cuda.Stream] = None,
                 device: Union[int, str, torch.device] = "cuda"):
        self.problem = problem
        self.precision = precision
        self.dtype = np.float64 if precision == "f64" else np.float32
        self.device = torch.device(device)
        self.stream = stream if stream is not None else torch.cuda.Stream(device=self.device)
        d, keep = make_desc3(problem, precision, sample_slots, self.stream.cuda_stream, exec, x_planes)
        self.desc = d
        self.workspace_bytes = workspace_bytes3(d)
        with torch.cuda.stream(self.stream):
            self.workspace = torch.empty(max(1, self.workspace_bytes), dtype=torch.uint8, device=self.device)
        h = ctypes.c_void_p()
        L.check3(L.lib().fdtd3d_create(ctypes.byref(d), ctypes.c_void_p(self.workspace.data_ptr()),
                                       self.workspace_bytes, ctypes.byref(h)))
        del keep                       # create copied what it needs
        self.h = h

    # -- time loop ---------------------------------------------------------
    def step(self, nsteps: int) -> "FdtdPlasma3D":
        L.check3(L.lib().fdtd3d_step(self.h, int(nsteps)))
        return self

    def run(self, nsteps: int) -> "FdtdPlasma3D":
        L.check3(L.lib().fdtd3d_run(self.h, int(nsteps)))
        return self

    def steps_done(self) -> int:
        v = ctypes.c_int64()
        L.check3(L.lib().fdtd3d_steps_done(self.h, ctypes.byref(v)))
        return v.value

    # -- results -----------------------------------------------------------
    def spectra(self, allow_nonfinite: bool = False) -> np.ndarray:
        """Running DFT of every sample point, complex [n_points, n_freqs]."""
        P, F = self.desc.n_points, self.desc.n_freqs
        re = np.zeros(max(P * F, 1))
        im = np.zeros(max(P * F, 1))
        rc = L.lib().fdtd3d_spectra(self.h, re.ctypes.data, im.ctypes.data)
        if not (allow_nonfinite and rc == L.E_NONFINITE):
            L.check3(rc)
        return (re[:P * F] + 1j * im[:P * F]).reshape(P, F)

    def field(self, name: str) -> np.ndarray:
        """One field ('Ex' .. 'Hz', 'Jx' .. 'Jz') as [nx, ny, nz] in the storage precision."""
        p = self.problem
        out = np.zeros((p.nx, p.ny, p.nz), self.dtype)
        L.check3(L.lib().fdtd3d_get_fields(self.h, L.FIELDS3.index(name), out.ctypes.data))
        return out

    def set_field(self, name: str, values: np.ndarray):
        p = self.problem
        v = np.ascontiguousarray(np.broadcast_to(values, (p.nx, p.ny, p.nz)), self.dtype)
        L.check3(L.lib().fdtd3d_set_fields(self.h, L.FIELDS3.index(name), v.ctypes.data))

    def profile(self, on: bool = True):
        """Per-launch HIP events on (graph capture off) or off; clears records."""
        L.check3(L.lib().fdtd3d_profile(self.h, int(on)))

    def profile_read(self) -> dict:
        """{kernel: (total ms, launches, cell-updates)} since profile(True)."""
        mx = 8
        names = (ctypes.c_char_p * mx)()
        ms = np.zeros(mx)
        calls = np.zeros(mx, np.int64)
        cells = np.zeros(mx)
        cnt = ctypes.c_int32()
        L.check3(L.lib().fdtd3d_profile_read(self.h, mx, names, ms.ctypes.data, calls.ctypes.data,
                                             cells.ctypes.data, ctypes.byref(cnt)))
        return {names[j].decode(): (float(ms[j]), int(calls[j]), float(cells[j]))
                for j in range(min(cnt.value, mx))}

    def synchronize(self):
        self.stream.synchronize()

    # -- lifetime ----------------------------------------------------------
    def close(self):
        if getattr(self, "h", None):
            L.lib().fdtd3d_destroy(self.h)
            self.h = None
            self.workspace = None

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
