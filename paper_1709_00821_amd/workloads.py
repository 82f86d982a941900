"""Seeded synthetic inputs for the 1D RKETD-FDTD plasma problems.

This module only *describes* problems: grid, time step, per-cell plasma
parameters, source, probes and frequencies.  It holds none of the method's
arithmetic, so both the GPU library's tests and the FP64 oracle draw their
inputs from here.

Problem families (paper section IV-B gives the slab geometry the first one is
built on: dz = 75 um, a Drude slab with wp = 2 pi 28.7 GHz and nu = 20 GHz, a
Gaussian-derivative pulse eq.(15) with tau = 15 dt):

* ``slab_c1``      - 1000 cells, 120-cell uniform slab, Mur ends, 4096 steps.
* ``large_c2``     - 2^24 cells, plasma on the middle half with a seeded
                     sinusoidal wp^2 profile and per-cell nu, CPML ends.
* ``batch_c4``     - thousands of independent slabs of uneven length with
                     piecewise-linear wp^2 profiles and per-slab nu.
* ``adjoint_c5``   - 8000 cells, a 2000-cell piecewise-linear plasma region.
* ``paper_preset`` - the paper's own 4096-cell domain with a 1200-cell slab.
"""
from __future__ import annotations

import dataclasses
import math
from typing import List, Optional

import numpy as np

C0 = 299792458.0          # m/s (exact)
GHZ = 1e9


@dataclasses.dataclass
class Problem1D:
    """One 1D grid: E nodes 0..n-1, H nodes at k+1/2 for k = 0..n-2."""

    n: int
    dz: float
    dt: float
    wp2: np.ndarray                   # [n] float64, rad^2/s^2
    nu: np.ndarray                    # [n] float64, 1/s
    src_cell: int
    src_tau: float
    src_t0: float
    src_amp: float
    probes: np.ndarray                # int64 cell indices
    freqs: np.ndarray                 # float64 Hz
    bc: str = "mur"                   # "mur" | "cpml" | "pec" | "periodic"
    cpml_cells: int = 0
    cpml_m: float = 3.0
    cpml_sigma_max: float = 0.0       # 0: the default 0.8 (m+1)/(eta0 dz)
    scheme: int = 0                   # 0 consistent, 1 printed eq.(13), 2 eq.(9)
    steps: int = 0                    # the run length this problem is quoted at

    def vacuum(self) -> "Problem1D":
        """The same grid with the plasma switched off (the reference run)."""
        return dataclasses.replace(self, wp2=np.zeros_like(self.wp2))

    def copy(self, **kw) -> "Problem1D":
        return dataclasses.replace(self, **kw)


def pulse_params(dt: float, tau_steps: float = 15.0):
    """eq.(15): tau = 15 dt, centred at 5 tau, scaled so the peak is 1."""
    tau = tau_steps * dt
    return tau, 5.0 * tau, math.exp(0.5) / tau


def _base(n, dz, dt, wp2, nu, src, probes, freqs, **kw) -> Problem1D:
    tau, t0, amp = pulse_params(dt)
    return Problem1D(n=n, dz=dz, dt=dt, wp2=np.ascontiguousarray(wp2, np.float64),
                     nu=np.ascontiguousarray(nu, np.float64), src_cell=int(src),
                     src_tau=tau, src_t0=t0, src_amp=amp,
                     probes=np.asarray(probes, np.int64),
                     freqs=np.ascontiguousarray(freqs, np.float64), **kw)


def slab_c1(n: int = 1000, dz: float = 75e-6, slab=(400, 520),
            wp: float = 2 * math.pi * 28.7 * GHZ, nu: float = 2e10,
            src: int = 100, probes=(50, 900), n_freqs: int = 256,
            steps: int = 4096, bc: str = "mur") -> Problem1D:
    """Uniform Drude slab on E nodes [slab[0], slab[1]), dt = dz/(2c)."""
    dt = dz / (2.0 * C0)
    wp2 = np.zeros(n)
    wp2[slab[0]:slab[1]] = wp * wp
    nuv = np.full(n, float(nu))
    freqs = np.linspace(1 * GHZ, 100 * GHZ, n_freqs)
    return _base(n, dz, dt, wp2, nuv, src, probes, freqs, bc=bc, steps=steps)


def paper_preset(steps: int = 8192) -> Problem1D:
    """The paper's 4096-cell domain: 1200-cell (9 cm) slab in the middle,
    dt = 125 fs taken literally, a 5-cell absorbing layer at each end."""
    n, dz, dt = 4096, 75e-6, 125e-15
    wp = 2 * math.pi * 28.7 * GHZ
    wp2 = np.zeros(n)
    lo = (n - 1200) // 2
    wp2[lo:lo + 1200] = wp * wp
    nuv = np.full(n, 2e10)
    freqs = np.linspace(1 * GHZ, 100 * GHZ, 256)
    return _base(n, dz, dt, wp2, nuv, 600, (300, n - 300), freqs,
                 bc="cpml", cpml_cells=5, steps=steps)


def large_c2(n: int = 1 << 24, steps: int = 20000, seed: int = 1709,
             cpml: int = 32, n_freqs: int = 256) -> Problem1D:
    """2^24-cell plain run: plasma on [n/4, 3n/4) with
    wp^2 = clip(wpmax^2 (0.5 + sum_i A_i sin(2 pi k/lambda_i + phi_i)), 0, wpmax^2),
    A_i ~ U(0, 0.25), lambda_i log-uniform in [2^6, 2^22] cells, phi_i ~ U[0, 2pi),
    nu ~ U[5, 40] GHz (a rate, no 2 pi) per cell.  Source 2048 cells before the
    plasma, probes 4096 cells either side of the plasma front."""
    rng = np.random.default_rng(seed)
    dz = 75e-6
    dt = dz / (2.0 * C0)
    wpmax2 = (2 * math.pi * 40 * GHZ) ** 2
    p0, p1 = n // 4, 3 * n // 4
    A = rng.uniform(0.0, 0.25, 8)
    lam = np.exp(rng.uniform(math.log(2.0 ** 6), math.log(2.0 ** 22), 8))
    ph = rng.uniform(0.0, 2 * math.pi, 8)
    k = np.arange(p1 - p0, dtype=np.float64)
    prof = np.full(k.shape, 0.5)
    for i in range(8):
        prof += A[i] * np.sin(2 * math.pi * k / lam[i] + ph[i])
    wp2 = np.zeros(n)
    wp2[p0:p1] = np.clip(wpmax2 * prof, 0.0, wpmax2)
    nu = rng.uniform(5 * GHZ, 40 * GHZ, n)
    freqs = np.linspace(1 * GHZ, 100 * GHZ, n_freqs)
    src = p0 - 2048
    return _base(n, dz, dt, wp2, nu, src, (p0 - 4096, p0 + 4096), freqs,
                 bc="cpml", cpml_cells=cpml, steps=steps)


def _piecewise_linear(rng, length: int, n_knots: int, vmax: float) -> np.ndarray:
    """Knots at both ends plus sorted uniform interior positions, values U[0, vmax]."""
    inner = np.sort(rng.uniform(0.0, length - 1, n_knots - 2))
    xs = np.concatenate([[0.0], inner, [length - 1.0]])
    ys = rng.uniform(0.0, vmax, n_knots)
    return np.interp(np.arange(length, dtype=np.float64), xs, ys)


def batch_c4(n_slabs: int = 4096, seed: int = 1710, lmin: int = 200,
             lmax: int = 8000, pad: int = 64, n_freqs: int = 64,
             steps: int = 8000) -> List[Problem1D]:
    """Independent slabs: L_i ~ U{lmin..lmax} plasma cells with `pad` vacuum
    cells on each side, Mur ends, source at node 32, probes at 16 and
    L_i + 2 pad - 16.  wp^2 piecewise linear with 4-16 knots in
    [0, (2 pi 40 GHz)^2]; nu ~ U[1, 50] GHz per slab."""
    rng = np.random.default_rng(seed)
    dz = 75e-6
    dt = dz / (2.0 * C0)
    wpmax2 = (2 * math.pi * 40 * GHZ) ** 2
    freqs = np.linspace(1 * GHZ, 100 * GHZ, n_freqs)
    out = []
    for _ in range(n_slabs):
        L = int(rng.integers(lmin, lmax + 1))
        kn = int(rng.integers(4, 17))
        n = L + 2 * pad
        wp2 = np.zeros(n)
        wp2[pad:pad + L] = _piecewise_linear(rng, L, kn, wpmax2)
        nu = np.full(n, float(rng.uniform(1 * GHZ, 50 * GHZ)))
        out.append(_base(n, dz, dt, wp2, nu, pad // 2, (pad // 4, n - pad // 4),
                         freqs, bc="mur", steps=steps))
    return out


def adjoint_c5(n: int = 8000, plasma=(3000, 5000), seed: int = 1711,
               steps: int = 20000, n_freqs: int = 32) -> Problem1D:
    """8000 cells, piecewise-linear (8 knots) plasma on [3000, 5000),
    nu = 20 GHz, source at 1000, probes at 500 (reflection) and 7000."""
    rng = np.random.default_rng(seed)
    dz = 75e-6
    dt = dz / (2.0 * C0)
    wpmax2 = (2 * math.pi * 40 * GHZ) ** 2
    wp2 = np.zeros(n)
    wp2[plasma[0]:plasma[1]] = _piecewise_linear(rng, plasma[1] - plasma[0], 8, wpmax2)
    nu = np.full(n, 2e10)
    freqs = np.linspace(5 * GHZ, 100 * GHZ, n_freqs)
    return _base(n, dz, dt, wp2, nu, 1000, (500, 7000), freqs, bc="mur", steps=steps)


def random_slab(rng: np.random.Generator, n: int, *, bc: str = "mur",
                n_freqs: int = 8, wpmax_ghz: float = 40.0,
                nu_ghz=(1.0, 50.0), cpml_cells: int = 0,
                dz: float = 75e-6, courant: float = 0.5,
                plasma_frac=(0.2, 0.8)) -> Problem1D:
    """A small random problem for parity tests: random plasma extent, per-cell
    wp^2 and nu, random source and probe positions."""
    dt = courant * dz / C0
    wpmax2 = (2 * math.pi * wpmax_ghz * GHZ) ** 2
    margin = max(2, cpml_cells + 1)
    if n - 2 * margin < 2:
        raise ValueError("grid too short for its absorbing layers")
    a = max(margin, min(int(n * plasma_frac[0]), n - margin - 2))
    lo = int(rng.integers(margin, a + 1))
    b = max(lo + 1, min(int(n * plasma_frac[1]), n - margin))
    hi = int(rng.integers(b, n - margin + 1))
    wp2 = np.zeros(n)
    wp2[lo:hi] = rng.uniform(0.0, wpmax2, hi - lo)
    nu = rng.uniform(nu_ghz[0] * GHZ, nu_ghz[1] * GHZ, n)
    src = int(rng.integers(margin, n - margin))
    probes = rng.integers(margin, n - margin, 2)
    freqs = np.sort(rng.uniform(1 * GHZ, 100 * GHZ, n_freqs))
    return _base(n, dz, dt, wp2, nu, src, probes, freqs, bc=bc,
                 cpml_cells=cpml_cells)


def light_cone(p: Problem1D, steps: int, extra: int = 2) -> Optional[tuple]:
    """Cells [lo, hi) outside which a zero-initial-state run with a single
    source stays exactly zero for `steps` steps (the stencil reaches one cell
    per step), widened to cover the probes.  None if it reaches an end."""
    pts = [p.src_cell] + [int(q) for q in p.probes]
    lo = min(p.src_cell - steps - extra, min(pts) - extra)
    hi = max(p.src_cell + steps + extra + 1, max(pts) + extra + 1)
    if lo <= 0 or hi >= p.n:
        return None
    return lo, hi
