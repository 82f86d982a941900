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


def paper_preset(steps: int = 8192, n: int = 4096) -> Problem1D:
    """The paper's domain (4096 cells by default): 1200-cell (9 cm) slab in the
    middle, dt = 125 fs taken literally, a 5-cell absorbing layer at each end,
    source 600 cells in and probes 300 cells from the ends.  Other n (the cell
    counts of the paper's timing table) scale source and probe positions by
    n / 4096 and shorten the slab to n / 3 where 1200 cells do not fit."""
    dz, dt = 75e-6, 125e-15
    wp = 2 * math.pi * 28.7 * GHZ
    wp2 = np.zeros(n)
    slab = min(1200, n // 3)
    lo = (n - slab) // 2
    wp2[lo:lo + slab] = wp * wp
    nuv = np.full(n, 2e10)
    freqs = np.linspace(1 * GHZ, 100 * GHZ, 256)
    src = int(round(600 * n / 4096))
    return _base(n, dz, dt, wp2, nuv, src, (src // 2, n - src // 2), freqs,
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


# ---------------------------------------------------------------------------
# 3D problems (Yee lattice, cubic cells; components at their staggered
# positions, arrays [i][j][k] with k fastest)
# ---------------------------------------------------------------------------

# component codes of sample points: E then H
COMPONENTS = ("Ex", "Ey", "Ez", "Hx", "Hy", "Hz")

# half-cell offsets of each component's position, (x, y, z)
STAGGER = {
    "Ex": (0.5, 0.0, 0.0), "Ey": (0.0, 0.5, 0.0), "Ez": (0.0, 0.0, 0.5),
    "Hx": (0.0, 0.5, 0.5), "Hy": (0.5, 0.0, 0.5), "Hz": (0.5, 0.5, 0.0),
}

# incident-grid margin of the TF/SF source: the 1D grid spans z in
# [b0 - AUX_MARGIN, b1 + AUX_MARGIN] with its soft source AUX_SRC nodes in
AUX_MARGIN = 8
AUX_SRC = 3


@dataclasses.dataclass
class Problem3D:
    nx: int
    ny: int
    nz: int
    d: float
    dt: float
    wp2: np.ndarray                   # [3, nx, ny, nz] float64 per E component
    nu: np.ndarray                    # [3, nx, ny, nz] or [nx, ny, nz] (shared)
    src_tau: float
    src_t0: float
    src_amp: float
    freqs: np.ndarray
    points: np.ndarray                # int32 [n, 4]: component code, i, j, k
    periodic_x: bool = False
    periodic_y: bool = False
    cpml: int = 0
    source: str = "none"              # "none" | "planar" | "tfsf"
    src_comp: int = 0                 # planar source: 0 Ex, 1 Ey
    src_k: int = 0
    b0: int = 0                       # TF box [b0, b1]
    b1: int = 0
    steps: int = 0

    @property
    def ncells(self) -> int:
        return self.nx * self.ny * self.nz

    def nu_comp(self, c: int) -> np.ndarray:
        return self.nu[c] if self.nu.ndim == 4 else self.nu

    def aux_layout(self):
        """(naux, aux_off, aux_src) of the incident 1D grid: aux node q is at
        z = q - aux_off."""
        naux = self.b1 - self.b0 + 2 * AUX_MARGIN + 1
        return naux, AUX_MARGIN - self.b0, AUX_SRC

    def vacuum(self) -> "Problem3D":
        return dataclasses.replace(self, wp2=np.zeros_like(self.wp2))

    def copy(self, **kw) -> "Problem3D":
        return dataclasses.replace(self, **kw)


def box_points(lo: int, hi: int, nx: int, ny: int, nz: int) -> np.ndarray:
    """Sample points on the six faces of the box [lo, hi]^3: on each face the
    four field components tangential to it at the face's index (face x = lo:
    Ey, Ez, Hy, Hz with i = lo), over the nodes whose other two coordinates
    lie in [lo, hi].  E nodes lie in the face plane, H nodes half a cell
    towards +axis.  Faces
    in the order x-lo, x-hi, y-lo, y-hi, z-lo, z-hi; within a face component by
    component, nodes in [i][j][k] order."""
    if not (0 <= lo < hi < min(nx, ny, nz)):
        raise ValueError("box outside the grid")
    tang = {0: ("Ey", "Ez", "Hy", "Hz"), 1: ("Ex", "Ez", "Hx", "Hz"), 2: ("Ex", "Ey", "Hx", "Hy")}
    out = []
    for axis in range(3):
        for face in (lo, hi):
            for name in tang[axis]:
                off = STAGGER[name]
                rng_ = []
                for a in range(3):
                    if a == axis:
                        rng_.append(np.array([face]))
                    else:
                        # nodes whose position lies within [lo, hi]
                        top = hi - 1 if off[a] == 0.5 else hi
                        rng_.append(np.arange(lo, top + 1))
                I, J, K = np.meshgrid(*rng_, indexing="ij")
                c = np.full(I.size, COMPONENTS.index(name))
                out.append(np.stack([c, I.ravel(), J.ravel(), K.ravel()], axis=1))
    return np.ascontiguousarray(np.concatenate(out), np.int32)


def sphere_wp2(nx: int, ny: int, nz: int, centre, radius: float, cutoff: float,
               wp2_peak: float) -> np.ndarray:
    """wp^2(r) = peak exp(-(r/radius)^2) for r <= cutoff (cells), else 0,
    sampled at each E component's own position; [3, nx, ny, nz]."""
    out = np.zeros((3, nx, ny, nz))
    c = np.asarray(centre, np.float64)
    lo = [max(0, int(math.floor(c[a] - cutoff - 1))) for a in range(3)]
    hi = [min(n, int(math.ceil(c[a] + cutoff + 1)) + 1) for a, n in enumerate((nx, ny, nz))]
    for comp, name in enumerate(("Ex", "Ey", "Ez")):
        off = STAGGER[name]
        x = np.arange(lo[0], hi[0]) + off[0] - c[0]
        y = np.arange(lo[1], hi[1]) + off[1] - c[1]
        z = np.arange(lo[2], hi[2]) + off[2] - c[2]
        r2 = x[:, None, None] ** 2 + y[None, :, None] ** 2 + z[None, None, :] ** 2
        v = wp2_peak * np.exp(-r2 / radius ** 2)
        v[r2 > cutoff ** 2] = 0.0
        out[comp, lo[0]:hi[0], lo[1]:hi[1], lo[2]:hi[2]] = v
    return out


def sphere_c3(n: int = 384, steps: int = 2000, d: float = 0.5e-3, courant: float = 0.5,
              n_freqs: int = 16, cpml: int = 10, tf: Optional[tuple] = None,
              box: Optional[tuple] = None, box_dft: bool = True) -> Problem3D:
    """Plasma sphere in a TF/SF plane wave: n^3 cells of d = 0.5 mm at Courant
    number c dt / d = 0.5; wp^2 = (2 pi 20 GHz)^2 exp(-(r/R)^2) for r <= 1.5 R,
    R = n/4, centred; nu = 10 GHz; x-polarised +z plane wave with the eq.(15)
    pulse; CPML of `cpml` cells on every face; TF box faces at 18 and n - 19
    (scaled for other n); FP64 DFT at 16 frequencies over 2-40 GHz of the
    tangential E and H on a box in the scattered-field region, midway between
    the CPML and the TF box (faces at 14 and 369 for n = 384)."""
    dt = courant * d / C0
    tau, t0, amp = pulse_params(dt)
    R = n / 4.0
    wp2 = sphere_wp2(n, n, n, (n / 2.0,) * 3, R, 1.5 * R, (2 * math.pi * 20 * GHZ) ** 2)
    nu = np.full((n, n, n), 1e10)
    if tf is None:
        tf = (max(cpml + 2, round(18 * n / 384)), n - max(cpml + 3, round(19 * n / 384)))
    if box is None:       # midway between the CPML and the TF box
        box = ((cpml + tf[0]) // 2, (tf[1] + n - cpml) // 2)
    pts = box_points(box[0], box[1], n, n, n) if box_dft else np.zeros((0, 4), np.int32)
    freqs = np.linspace(2 * GHZ, 40 * GHZ, n_freqs)
    return Problem3D(nx=n, ny=n, nz=n, d=d, dt=dt, wp2=wp2, nu=nu, src_tau=tau,
                     src_t0=t0, src_amp=amp, freqs=freqs, points=pts, cpml=cpml,
                     source="tfsf", b0=int(tf[0]), b1=int(tf[1]), steps=steps)


# ---------------------------------------------------------------------------
# 2D problems (square cells in the x-y plane, fields uniform along z; arrays
# [i][j] with j fastest)
# ---------------------------------------------------------------------------

# E-like components of each 2D mode (each carries its own plasma current)
MODES_2D = {"tm": ("Ez",), "te": ("Ex", "Ey")}
# half-cell offsets (x, y) of each 2D component's position
STAGGER_2D = {"Ez": (0.0, 0.0), "Hx": (0.0, 0.5), "Hy": (0.5, 0.0),
              "Ex": (0.5, 0.0), "Ey": (0.0, 0.5), "Hz": (0.5, 0.5)}


@dataclasses.dataclass
class Problem2D:
    """One 2D grid of nx x ny square cells of side d.  TM: Ez at (i, j), Hx at
    (i, j+1/2), Hy at (i+1/2, j).  TE: Ex at (i+1/2, j), Ey at (i, j+1/2), Hz at
    (i+1/2, j+1/2).  wp2, nu: [ncomp, nx, ny] at each E component's position."""

    mode: str                         # "tm" | "te"
    nx: int
    ny: int
    d: float
    dt: float
    wp2: np.ndarray
    nu: np.ndarray
    src: tuple                        # (i, j) of the soft point source (Ez / Ey), or None
    src_tau: float
    src_t0: float
    src_amp: float
    probes: np.ndarray                # int64 [n, 3]: E component index, i, j
    freqs: np.ndarray
    periodic_x: bool = False
    periodic_y: bool = False
    steps: int = 0

    @property
    def ncells(self) -> int:
        return self.nx * self.ny

    @property
    def ncomp(self) -> int:
        return len(MODES_2D[self.mode])

    def vacuum(self) -> "Problem2D":
        return dataclasses.replace(self, wp2=np.zeros_like(self.wp2))

    def copy(self, **kw) -> "Problem2D":
        return dataclasses.replace(self, **kw)


def cylinder_wp2(mode: str, nx: int, ny: int, centre, radius: float, wp2_peak: float,
                 edge: float = 0.0) -> np.ndarray:
    """Plasma cylinder along z: wp^2 = peak inside radius (cells), a Gaussian
    falloff exp(-((r - radius)/edge)^2) outside it out to radius + 3 edge,
    sampled at each E component's own position; [ncomp, nx, ny]."""
    comps = MODES_2D[mode]
    out = np.zeros((len(comps), nx, ny))
    for c, name in enumerate(comps):
        ox, oy = STAGGER_2D[name]
        x = np.arange(nx) + ox - centre[0]
        y = np.arange(ny) + oy - centre[1]
        r = np.sqrt(x[:, None] ** 2 + y[None, :] ** 2)
        v = np.where(r <= radius, wp2_peak, 0.0)
        if edge > 0:
            fall = wp2_peak * np.exp(-((r - radius) / edge) ** 2)
            v = np.where((r > radius) & (r <= radius + 3 * edge), fall, v)
        out[c] = v
    return out


def cylinder_2d(mode: str = "tm", n: int = 4096, steps: int = 2000, d: float = 75e-6,
                courant: float = 0.5, n_freqs: int = 64, seed: int = 1714) -> Problem2D:
    """n x n cells of d = 75 um (Courant c dt/d = 0.5), PEC walls; a plasma
    cylinder of radius n/8 at the centre (wp = 2 pi 40 GHz, Gaussian edge of
    n/64 cells, nu = 20 GHz); the eq.(15) pulse as a soft point source a
    quarter of the way in; 8 probes at seeded angles on a circle of radius
    n/5 about the source (within the pulse's reach after 2000 steps at
    n = 4096); 64 frequencies over 1-100 GHz."""
    rng = np.random.default_rng(seed)
    dt = courant * d / C0
    tau, t0, amp = pulse_params(dt)
    wp2 = cylinder_wp2(mode, n, n, (n / 2.0, n / 2.0), n / 8.0, (2 * math.pi * 40 * GHZ) ** 2, n / 64.0)
    nu = np.full((len(MODES_2D[mode]), n, n), 2e10)
    comp = 0 if mode == "tm" else 1
    ang = rng.uniform(0.0, 2 * math.pi, 8)
    pi = np.clip(np.round(n // 4 + n / 5.0 * np.cos(ang)), 1, n - 2).astype(np.int64)
    pj = np.clip(np.round(n // 2 + n / 5.0 * np.sin(ang)), 1, n - 2).astype(np.int64)
    probes = np.stack([np.full(8, comp), pi, pj], axis=1).astype(np.int64)
    return Problem2D(mode=mode, nx=n, ny=n, d=d, dt=dt, wp2=wp2, nu=nu, src=(n // 4, n // 2),
                     src_tau=tau, src_t0=t0, src_amp=amp, probes=probes,
                     freqs=np.linspace(1 * GHZ, 100 * GHZ, n_freqs), steps=steps)


def random_2d(rng: np.random.Generator, mode: str, nx: int, ny: int, *, periodic_x: bool = False,
              periodic_y: bool = False, n_freqs: int = 6, courant: float = 0.5, d: float = 75e-6,
              plasma: bool = True) -> Problem2D:
    """A small random 2D problem for parity tests: a random rectangle of
    per-cell random wp^2 and nu, random source and E probes."""
    dt = courant * d / C0
    tau, t0, amp = pulse_params(dt)
    nc = len(MODES_2D[mode])
    wp2 = np.zeros((nc, nx, ny))
    if plasma:
        i0, i1 = sorted(rng.integers(1, nx, 2))
        j0, j1 = sorted(rng.integers(1, ny, 2))
        wp2[:, i0:i1 + 1, j0:j1 + 1] = rng.uniform(0, (2 * math.pi * 40 * GHZ) ** 2, (nc, i1 - i0 + 1, j1 - j0 + 1))
    nu = rng.uniform(1 * GHZ, 50 * GHZ, (nc, nx, ny))
    src = (int(rng.integers(1, nx - 1)), int(rng.integers(1, ny - 1)))
    probes = np.stack([rng.integers(0, nc, 4), rng.integers(1, nx - 1, 4), rng.integers(1, ny - 1, 4)],
                      axis=1).astype(np.int64)
    return Problem2D(mode=mode, nx=nx, ny=ny, d=d, dt=dt, wp2=wp2, nu=nu, src=src, src_tau=tau,
                     src_t0=t0, src_amp=amp, probes=probes,
                     freqs=np.sort(rng.uniform(1 * GHZ, 100 * GHZ, n_freqs)),
                     periodic_x=periodic_x, periodic_y=periodic_y)
