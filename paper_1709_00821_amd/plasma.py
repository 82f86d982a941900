"""Python face of the library: one handle over one or many 1D grids.

Only marshalling happens here; every step of the time loop (H, E, J, source,
ends, probe DFT) runs in the HIP kernels behind the C ABI.  torch provides
the device workspace (a uint8 tensor) and the stream.
"""
from __future__ import annotations

import ctypes
from typing import List, Optional, Sequence, Union

import numpy as np
import torch

from . import _lib as L
from .workloads import Problem1D


def _as_list(problems) -> List[Problem1D]:
    return [problems] if isinstance(problems, Problem1D) else list(problems)


def make_desc(problems, precision: str = "f64", exec: str = "auto", tile_cells: int = 0,
              steps_per_pass: int = 0, checkpoint: int = 0, stream_handle: int = 0,
              tile_waves: int = 0, record: int = 0, vacuum_tile_cells: int = 0):
    """Build the C descriptor; returns (desc, arrays it points into)."""
    probs = _as_list(problems)
    p0 = probs[0]
    for q in probs[1:]:
        if (q.dz, q.dt, q.bc, q.scheme, q.cpml_cells, len(q.probes)) != \
           (p0.dz, p0.dt, p0.bc, p0.scheme, p0.cpml_cells, len(p0.probes)) or \
           not np.array_equal(q.freqs, p0.freqs) or \
           (q.src_tau, q.src_t0, q.src_amp) != (p0.src_tau, p0.src_t0, p0.src_amp):
            raise ValueError("all grids of one handle must share dz, dt, ends, source shape, "
                             "probe count and frequencies")
    keep = [
        np.array([q.n for q in probs], np.int64),
        np.ascontiguousarray(np.concatenate([q.wp2 for q in probs]), np.float64),
        np.ascontiguousarray(np.concatenate([q.nu for q in probs]), np.float64),
        np.array([q.src_cell for q in probs], np.int64),
        np.ascontiguousarray(np.concatenate([q.probes for q in probs]), np.int64),
        np.ascontiguousarray(p0.freqs, np.float64),
    ]
    cells, wp2, nu, src, probes, freqs = keep
    d = L.Desc()
    d.struct_size = ctypes.sizeof(L.Desc)
    d.precision = {"f64": L.F64, "f32": L.F32, "f32d": L.F32_DELTA}[precision]
    d.scheme = p0.scheme
    d.bc = L.BC[p0.bc]
    d.exec = L.EXEC[exec]
    d.flags = (L.FLAG_CHECKPOINT if checkpoint else 0) | (L.FLAG_RECORD if record else 0)
    d.checkpoint_steps = int(checkpoint) if checkpoint else 0
    d.record_steps = int(record) if record else 0
    d.batch = len(probs)
    d.cells = cells.ctypes.data
    d.dz, d.dt = p0.dz, p0.dt
    d.wp2, d.nu = wp2.ctypes.data, nu.ctypes.data
    d.src_cell = src.ctypes.data
    d.src_tau, d.src_t0, d.src_amp = p0.src_tau, p0.src_t0, p0.src_amp
    d.n_probes, d.n_freqs = len(p0.probes), len(freqs)
    d.probe_cells, d.freqs_hz = probes.ctypes.data, freqs.ctypes.data
    d.cpml_cells = p0.cpml_cells
    d.tile_cells = tile_cells
    d.tile_waves = tile_waves
    d.vacuum_tile_cells = vacuum_tile_cells
    d.cpml_m, d.cpml_sigma_max = p0.cpml_m, p0.cpml_sigma_max
    d.steps_per_pass = steps_per_pass
    d.stream = stream_handle or None
    return d, keep


def workspace_bytes(desc) -> int:
    nbytes = ctypes.c_size_t()
    L.check(L.lib().fdtd_plasma_workspace_bytes(ctypes.byref(desc), ctypes.byref(nbytes)))
    return nbytes.value


class FdtdPlasma:
    """A set of independent 1D RKETD-FDTD grids sharing dz, dt, ends, source
    shape, probe count and DFT frequencies."""

    def __init__(self, problems: Union[Problem1D, Sequence[Problem1D]], precision: str = "f64",
                 exec: str = "auto", tile_cells: int = 0, steps_per_pass: int = 0, tile_waves: int = 0,
                 checkpoint: int = 0, stream: Optional[torch.cuda.Stream] = None,
                 device: Union[int, str, torch.device] = "cuda", record: int = 0, vacuum_tile_cells: int = 0):
        probs = _as_list(problems)
        self.problems = probs
        self.device = torch.device(device)
        self.stream = stream if stream is not None else torch.cuda.Stream(device=self.device)
        self.cells = np.array([q.n for q in probs], np.int64)
        self.offsets = np.concatenate([[0], np.cumsum(self.cells)])
        d, self._keep = make_desc(probs, precision, exec, tile_cells, steps_per_pass, checkpoint,
                                  self.stream.cuda_stream, tile_waves, record, vacuum_tile_cells)
        self.desc = d
        self.precision = precision
        self.workspace_bytes = workspace_bytes(d)
        with torch.cuda.stream(self.stream):
            self.workspace = torch.empty(max(1, self.workspace_bytes), dtype=torch.uint8,
                                         device=self.device)
        h = ctypes.c_void_p()
        L.check(L.lib().fdtd_plasma_create(ctypes.byref(d), ctypes.c_void_p(self.workspace.data_ptr()),
                                           self.workspace_bytes, ctypes.byref(h)))
        self.h = h

    # -- time loop ---------------------------------------------------------
    def step(self, nsteps: int) -> "FdtdPlasma":
        L.check(L.lib().fdtd_plasma_step(self.h, int(nsteps)))
        return self

    def run(self, nsteps: int) -> "FdtdPlasma":
        L.check(L.lib().fdtd_plasma_run(self.h, int(nsteps)))
        return self

    def steps_done(self) -> int:
        v = ctypes.c_int64()
        L.check(L.lib().fdtd_plasma_steps_done(self.h, ctypes.byref(v)))
        return v.value

    # -- results -----------------------------------------------------------
    def spectra(self, allow_nonfinite: bool = False) -> np.ndarray:
        """Running DFT, complex [batch, n_probes, n_freqs]."""
        B, P, F = len(self.problems), self.desc.n_probes, self.desc.n_freqs
        re = np.zeros(B * P * F)
        im = np.zeros(B * P * F)
        rc = L.lib().fdtd_plasma_probe_spectra(self.h, re.ctypes.data, im.ctypes.data)
        if not (allow_nonfinite and rc == L.E_NONFINITE):
            L.check(rc)
        return (re + 1j * im).reshape(B, P, F)

    def series(self) -> np.ndarray:
        """Recorded probe samples (record=steps at construction), float64
        [batch, n_probes, steps]: entry m-1 is E^m."""
        B, P, T = len(self.problems), self.desc.n_probes, self.steps_done()
        out = np.zeros(B * P * T)
        L.check(L.lib().fdtd_plasma_probe_series(self.h, out.ctypes.data))
        return out.reshape(B, P, T)

    def fft(self, nfft: int) -> np.ndarray:
        """dt-scaled FFT of the recorded series zero-padded to nfft points,
        complex [batch, n_probes, nfft] (bin k at f = k / (nfft dt))."""
        B, P = len(self.problems), self.desc.n_probes
        re = np.zeros(B * P * nfft)
        im = np.zeros(B * P * nfft)
        L.check(L.lib().fdtd_plasma_probe_fft(self.h, int(nfft), re.ctypes.data, im.ctypes.data))
        return (re + 1j * im).reshape(B, P, nfft)

    def fields(self, grid: int = 0) -> dict:
        n = int(self.cells[grid])
        E, H, J = np.zeros(n), np.zeros(max(n - 1, 1)), np.zeros(n)
        L.check(L.lib().fdtd_plasma_get_fields(self.h, grid, E.ctypes.data, H.ctypes.data,
                                               J.ctypes.data))
        return {"E": E, "H": H, "J": J}

    def loss_r2(self, xref: np.ndarray, probe: int = 0) -> np.ndarray:
        """L_b = sum_f |(X_b - xref_b)/xref_b|^2 at `probe`, per grid; xref [batch, F]."""
        B, F = len(self.problems), self.desc.n_freqs
        xr = np.ascontiguousarray(np.real(xref).reshape(B, F), np.float64)
        xi = np.ascontiguousarray(np.imag(xref).reshape(B, F), np.float64)
        loss = np.zeros(B)
        L.check(L.lib().fdtd_plasma_loss_r2(self.h, probe, xr.ctypes.data, xi.ctypes.data,
                                            loss.ctypes.data))
        return loss

    def grad_r2(self, nsteps: int, xref: np.ndarray, probe: int = 0):
        """(loss [batch], dL/d wp2 [sum cells]) by the discrete adjoint with
        sqrt(T) checkpoints (needs checkpoint >= nsteps at construction)."""
        B, F = len(self.problems), self.desc.n_freqs
        xr = np.ascontiguousarray(np.real(xref).reshape(B, F), np.float64)
        xi = np.ascontiguousarray(np.imag(xref).reshape(B, F), np.float64)
        loss = np.zeros(B)
        grad = np.zeros(int(self.cells.sum()))
        L.check(L.lib().fdtd_plasma_grad_r2(self.h, int(nsteps), probe, xr.ctypes.data,
                                            xi.ctypes.data, loss.ctypes.data, grad.ctypes.data))
        return loss, grad

    def profile(self, nsteps: int) -> dict:
        """Advance nsteps eagerly with HIP events around every launch on the
        handle's stream: {kernel group: (total ms, launches, nodes advanced)}."""
        mx = 16
        names = ctypes.create_string_buffer(32 * mx)
        ms = np.zeros(mx)
        calls = np.zeros(mx, np.int64)
        units = np.zeros(mx, np.int64)
        cnt = ctypes.c_int32()
        L.check(L.lib().fdtd_plasma_profile(self.h, int(nsteps), mx, names, ms.ctypes.data,
                                            calls.ctypes.data, units.ctypes.data, ctypes.byref(cnt)))
        out = {}
        for j in range(cnt.value):
            nm = names.raw[32 * j:32 * j + 32].split(b"\0")[0].decode()
            out[nm] = (float(ms[j]), int(calls[j]), int(units[j]))
        return out

    def synchronize(self):
        self.stream.synchronize()

    # -- lifetime ----------------------------------------------------------
    def close(self):
        if getattr(self, "h", None):
            L.lib().fdtd_plasma_destroy(self.h)
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


def reflect_transmit(problem: Problem1D, nsteps: int, refl: int = 0, trans: int = 1, **kw):
    """Two-run R = (X_refl - X_refl^vac)/X_refl^vac and T = X_trans/X_trans^vac,
    both grids advanced in one handle (batch of 2)."""
    with FdtdPlasma([problem, problem.vacuum()], **kw) as h:
        h.run(nsteps)
        X = h.spectra()
    s, v = X[0], X[1]
    return (s[refl] - v[refl]) / v[refl], s[trans] / v[trans], s, v
