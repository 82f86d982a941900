"""Python binding of the 2D library (include/fdtd_plasma2d.h): argument
marshalling only; torch supplies the device workspace and the stream."""
from __future__ import annotations

import ctypes
from typing import Optional, Union

import numpy as np
import torch

from . import _lib as L
from .workloads import Problem2D


def make_desc2(p: Problem2D, precision: str = "f64", stream_handle: int = 0):
    """The C descriptor of p; returns (desc, arrays it points into)."""
    nc = p.ncomp
    keep = [np.ascontiguousarray(np.asarray(p.wp2, np.float64).reshape(nc, p.nx, p.ny)),
            np.ascontiguousarray(np.asarray(p.nu, np.float64).reshape(nc, p.nx, p.ny)),
            np.ascontiguousarray(np.asarray(p.probes, np.int64).reshape(-1, 3)),
            np.ascontiguousarray(p.freqs, np.float64)]
    wp2, nu, probes, freqs = keep
    d = L.Desc2()
    d.struct_size = ctypes.sizeof(L.Desc2)
    d.mode = 0 if p.mode == "tm" else 1
    d.precision = {"f64": L.F64, "f32": L.F32}[precision]
    d.periodic_x, d.periodic_y = int(p.periodic_x), int(p.periodic_y)
    d.nx, d.ny = p.nx, p.ny
    d.d, d.dt = p.d, p.dt
    d.wp2, d.nu = wp2.ctypes.data, nu.ctypes.data
    d.has_src = int(p.src is not None)
    if p.src is not None:
        d.src_i, d.src_j = int(p.src[0]), int(p.src[1])
    d.src_tau, d.src_t0, d.src_amp = p.src_tau, p.src_t0, p.src_amp
    d.n_probes = len(probes)
    d.probes = probes.ctypes.data if len(probes) else None
    d.n_freqs = len(freqs)
    d.freqs_hz = freqs.ctypes.data
    d.stream = stream_handle or None
    return d, keep


class FdtdPlasma2D:
    """One 2D grid (TM or TE) on the GPU."""

    def __init__(self, p: Problem2D, precision: str = "f64", stream: Optional[torch.cuda.Stream] = None,
                 device: Union[int, str, torch.device] = "cuda"):
        self.problem = p
        self.device = torch.device(device)
        self.stream = stream if stream is not None else torch.cuda.Stream(device=self.device)
        d, self._keep = make_desc2(p, precision, self.stream.cuda_stream)
        self.desc = d
        n = ctypes.c_size_t()
        L.check2(L.lib().fdtd2d_workspace_bytes(ctypes.byref(d), ctypes.byref(n)))
        self.workspace_bytes = n.value
        with torch.cuda.stream(self.stream):
            self.workspace = torch.empty(max(1, n.value), dtype=torch.uint8, device=self.device)
        h = ctypes.c_void_p()
        L.check2(L.lib().fdtd2d_create(ctypes.byref(d), ctypes.c_void_p(self.workspace.data_ptr()), n.value,
                                       ctypes.byref(h)))
        self.h = h

    def step(self, nsteps: int) -> "FdtdPlasma2D":
        L.check2(L.lib().fdtd2d_step(self.h, int(nsteps)))
        return self

    def run(self, nsteps: int) -> "FdtdPlasma2D":
        L.check2(L.lib().fdtd2d_run(self.h, int(nsteps)))
        return self

    def steps_done(self) -> int:
        v = ctypes.c_int64()
        L.check2(L.lib().fdtd2d_steps_done(self.h, ctypes.byref(v)))
        return v.value

    def spectra(self) -> np.ndarray:
        """Probe spectra, complex [n_probes, n_freqs]."""
        P, F = self.desc.n_probes, self.desc.n_freqs
        re, im = np.zeros(P * F), np.zeros(P * F)
        L.check2(L.lib().fdtd2d_spectra(self.h, re.ctypes.data, im.ctypes.data))
        return (re + 1j * im).reshape(P, F)

    def fields(self) -> dict:
        """{"E": [ncomp, nx, ny], "H": [nh, nx, ny], "J": [ncomp, nx, ny]} (float64)."""
        p = self.problem
        nc, nh = p.ncomp, (2 if p.mode == "tm" else 1)
        out = []
        for w in range(2 * nc + nh):
            a = np.zeros(p.nx * p.ny)
            L.check2(L.lib().fdtd2d_get_fields(self.h, w, a.ctypes.data))
            out.append(a.reshape(p.nx, p.ny))
        return {"E": np.stack(out[:nc]), "H": np.stack(out[nc:nc + nh]), "J": np.stack(out[nc + nh:])}

    def synchronize(self):
        self.stream.synchronize()

    def close(self):
        if getattr(self, "h", None):
            L.lib().fdtd2d_destroy(self.h)
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
