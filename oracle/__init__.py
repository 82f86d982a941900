"""FP64 serial oracle for the 1D RKETD-FDTD plasma step (test infrastructure).

Only the test suite, the smoke check and the benchmark's CPU-baseline leg may
import this package.  It wraps ``liboracle.so`` (plain C in this directory,
written from the paper's section II equations) with ctypes and numpy; it shares
no code with the GPU library.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from typing import Optional

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SO = os.path.join(_HERE, "liboracle.so")
_SRCS = ["rketd1d.c", "adjoint1d.c", "rketd3d.c", "rketd2d.c"]
_lib = None
# faster builds of the same sources: "native" is the serial oracle with -O3
# -march=native, "omp" adds -fopenmp (the 1D node loops and the 2D cell loops
# carry OpenMP pragmas, ignored by the other builds; their iterations are
# independent, so the order of the arithmetic is unchanged).  Every build
# keeps -ffp-contract=off, so all give the same results bit for bit.  Used by
# the benchmark's CPU-baseline leg and by the largest parity cases.
_TIMING = {"native": ["-O3", "-march=native"], "omp": ["-O3", "-march=native", "-fopenmp"]}
_timing_libs = {}

BC = {"mur": 0, "cpml": 1, "pec": 2, "periodic": 3}

# plain serial build: -ffp-contract=off keeps every multiply and add separately
# rounded, as written
CFLAGS = ["-O2", "-fPIC", "-shared", "-ffp-contract=off", "-std=c99"]


def build(out: str = _SO, extra: Optional[list] = None) -> str:
    srcs = [os.path.join(_HERE, s) for s in _SRCS if os.path.exists(os.path.join(_HERE, s))]
    cmd = ["gcc", *CFLAGS, *(extra or []), "-o", out, *srcs, "-lm"]
    subprocess.run(cmd, check=True)
    return out


def timing_lib(kind: str):
    """The "native" or "omp" timing build (built on first use, under /tmp)."""
    if kind not in _timing_libs:
        import tempfile
        out = os.path.join(tempfile.gettempdir(), f"liboracle_{kind}_{os.getpid()}.so")
        build(out, _TIMING[kind])
        L = ctypes.CDLL(out)
        _declare(L)
        _timing_libs[kind] = L
    return _timing_libs[kind]


def lib(kind: Optional[str] = None):
    if kind is not None:
        return timing_lib(kind)
    global _lib
    if _lib is None:
        srcs = [os.path.join(_HERE, s) for s in _SRCS if os.path.exists(os.path.join(_HERE, s))]
        if not os.path.exists(_SO) or any(os.path.getmtime(s) > os.path.getmtime(_SO) for s in srcs):
            build()
        _lib = ctypes.CDLL(_SO)
        _declare(_lib)
    return _lib


class _Problem(ctypes.Structure):
    _fields_ = [
        ("n", ctypes.c_int64), ("dz", ctypes.c_double), ("dt", ctypes.c_double),
        ("wp2", ctypes.c_void_p), ("nu", ctypes.c_void_p),
        ("bc", ctypes.c_int32), ("scheme", ctypes.c_int32),
        ("cpml_cells", ctypes.c_int64), ("cpml_m", ctypes.c_double),
        ("cpml_sigma_max", ctypes.c_double),
        ("src_cell", ctypes.c_int64), ("src_tau", ctypes.c_double),
        ("src_t0", ctypes.c_double), ("src_amp", ctypes.c_double),
        ("n_probes", ctypes.c_int32), ("n_freqs", ctypes.c_int32),
        ("probe_cells", ctypes.c_void_p), ("freqs", ctypes.c_void_p),
    ]


class _State(ctypes.Structure):
    _fields_ = [
        ("E", ctypes.c_void_p), ("H", ctypes.c_void_p), ("J", ctypes.c_void_p),
        ("psiE", ctypes.c_void_p), ("psiH", ctypes.c_void_p),
        ("Xre", ctypes.c_void_p), ("Xim", ctypes.c_void_p),
        ("step", ctypes.c_int64),
    ]


def _declare(L):
    d, i64, p = ctypes.c_double, ctypes.c_int64, ctypes.c_void_p
    L.or_c0.restype = d
    L.or_eps0.restype = d
    L.or_mu0.restype = d
    L.or_phi.argtypes = [d, p, p, p]
    L.or_coeffs.argtypes = [i64, p, p, d, d, ctypes.c_int, p]
    L.or_source.argtypes = [d, d, d, d]
    L.or_source.restype = d
    L.or_twiddle.argtypes = [d, d, i64, p, p]
    L.or_dft_accumulate.argtypes = [i64, p, i64, ctypes.c_int, p, d, p, p]
    L.or1d_check.argtypes = [p]
    L.or1d_step.argtypes = [p, p, i64]
    L.or3d_check.argtypes = [p]
    L.or3d_step.argtypes = [p, p, i64]
    L.or2d_check.argtypes = [p]
    L.or2d_step.argtypes = [p, p, i64]
    if hasattr(L, "or1d_adjoint_r2"):
        L.or1d_adjoint_r2.argtypes = [p, i64, ctypes.c_int32, p, p, p, p, p]
        L.or1d_adjoint_step.argtypes = [p, p, p, p]


def _ptr(a: np.ndarray) -> int:
    return a.ctypes.data


def constants():
    L = lib()
    return {"c0": L.or_c0(), "eps0": L.or_eps0(), "mu0": L.or_mu0()}


def phi(x: float):
    a, p1, p2 = (ctypes.c_double() for _ in range(3))
    lib().or_phi(x, ctypes.byref(a), ctypes.byref(p1), ctypes.byref(p2))
    return a.value, p1.value, p2.value


COEFF_NAMES = ("a", "phi1", "phi2", "D", "CA", "CJ", "CH", "b1", "b2")


def coeffs(wp2, nu, dt, dz, scheme=0) -> dict:
    wp2 = np.ascontiguousarray(wp2, np.float64)
    nu = np.ascontiguousarray(nu, np.float64)
    out = np.zeros((wp2.size, 9))
    lib().or_coeffs(wp2.size, _ptr(wp2), _ptr(nu), dt, dz, scheme, _ptr(out))
    return {k: out[:, i].copy() for i, k in enumerate(COEFF_NAMES)}


def source(t, tau, t0, amp) -> float:
    return lib().or_source(t, tau, t0, amp)


def dft(samples, m0, freqs, dt) -> np.ndarray:
    """sum_i samples[i] dt exp(-j 2 pi f (m0+i) dt), accumulated term by term."""
    s = np.ascontiguousarray(samples, np.float64)
    f = np.ascontiguousarray(freqs, np.float64)
    xr = np.zeros(f.size)
    xi = np.zeros(f.size)
    lib().or_dft_accumulate(s.size, _ptr(s), m0, f.size, _ptr(f), dt, _ptr(xr), _ptr(xi))
    return xr + 1j * xi


class _Keep:
    """Holds the numpy buffers a ctypes struct points into."""

    def __init__(self):
        self.bufs = []

    def arr(self, a, dtype):
        a = np.ascontiguousarray(a, dtype)
        self.bufs.append(a)
        return a


def _problem(p, keep: _Keep) -> _Problem:
    wp2 = keep.arr(p.wp2, np.float64)
    nu = keep.arr(p.nu, np.float64)
    probes = keep.arr(p.probes, np.int64)
    freqs = keep.arr(p.freqs, np.float64)
    return _Problem(
        n=p.n, dz=p.dz, dt=p.dt, wp2=_ptr(wp2), nu=_ptr(nu), bc=BC[p.bc],
        scheme=p.scheme, cpml_cells=p.cpml_cells, cpml_m=p.cpml_m,
        cpml_sigma_max=p.cpml_sigma_max, src_cell=p.src_cell, src_tau=p.src_tau,
        src_t0=p.src_t0, src_amp=p.src_amp, n_probes=len(probes),
        n_freqs=len(freqs), probe_cells=_ptr(probes), freqs=_ptr(freqs))


def new_state(p) -> dict:
    n = p.n
    return {"E": np.zeros(n), "H": np.zeros(n), "J": np.zeros(n),
            "psiE": np.zeros(n), "psiH": np.zeros(n),
            "X": np.zeros((len(p.probes), len(p.freqs)), np.complex128), "step": 0}


def check(p) -> int:
    keep = _Keep()
    pb = _problem(p, keep)
    return lib().or1d_check(ctypes.byref(pb))


def run(p, nsteps: int, state: Optional[dict] = None, kind: Optional[str] = None) -> dict:
    """Advance `state` (default: zero fields at step 0) by nsteps; returns a new
    dict.  kind: a timing build ("native", "omp") instead of the plain one."""
    st = new_state(p) if state is None else {k: (v.copy() if isinstance(v, np.ndarray) else v)
                                            for k, v in state.items()}
    keep = _Keep()
    pb = _problem(p, keep)
    Xre = np.ascontiguousarray(st["X"].real)
    Xim = np.ascontiguousarray(st["X"].imag)
    for k in ("E", "H", "J", "psiE", "psiH"):
        st[k] = np.ascontiguousarray(st[k], np.float64)
    cs = _State(E=_ptr(st["E"]), H=_ptr(st["H"]), J=_ptr(st["J"]),
                psiE=_ptr(st["psiE"]), psiH=_ptr(st["psiH"]),
                Xre=_ptr(Xre), Xim=_ptr(Xim), step=st["step"])
    rc = lib(kind).or1d_step(ctypes.byref(pb), ctypes.byref(cs), nsteps)
    if rc != 0:
        raise ValueError(f"oracle rejected the problem (code {rc})")
    st["X"] = Xre + 1j * Xim
    st["step"] = cs.step
    return st


def probe_series(p, nsteps: int) -> np.ndarray:
    """E^m at every probe for m = 1 .. nsteps, [n_probes, nsteps]: the oracle
    advanced one step at a time (section IV-B records the probe field over
    the run)."""
    st = new_state(p)
    out = np.zeros((len(p.probes), nsteps))
    for m in range(nsteps):
        st = run(p, 1, st)
        out[:, m] = st["E"][np.asarray(p.probes)]
    return out


def series_fft(series: np.ndarray, nfft: int, dt: float) -> np.ndarray:
    """X[k] = dt sum_{m=1}^{T} E^m exp(-j 2 pi k m / nfft) of series [..., T]
    (entry m-1 is E^m), zero-padded to nfft points: numpy's FFT of the
    sequence 0, E^1, .., E^T, 0, .. (the running DFT at f = k / (nfft dt))."""
    T = series.shape[-1]
    x = np.zeros(series.shape[:-1] + (nfft,))
    x[..., 1:T + 1] = series
    return dt * np.fft.fft(x, axis=-1)


def reflect_transmit(p, nsteps: int, refl: int = 0, trans: int = 1):
    """Two-run R and T: R = (X_refl - X_refl^vac)/X_refl^vac, T = X_trans/X_trans^vac."""
    s = run(p, nsteps)["X"]
    v = run(p.vacuum(), nsteps)["X"]
    return (s[refl] - v[refl]) / v[refl], s[trans] / v[trans], s, v


def adjoint_step(p, lE, lH, lJ):
    """lambda^{n+1} -> lambda^n through the transposed linear step (no source)."""
    keep = _Keep()
    pb = _problem(p, keep)
    lE = np.ascontiguousarray(lE, np.float64).copy()
    lH = np.ascontiguousarray(lH, np.float64).copy()
    lJ = np.ascontiguousarray(lJ, np.float64).copy()
    rc = lib().or1d_adjoint_step(ctypes.byref(pb), _ptr(lE), _ptr(lH), _ptr(lJ))
    if rc != 0:
        raise ValueError(f"oracle adjoint rejected the problem (code {rc})")
    return lE, lH, lJ


def adjoint_r2(p, nsteps: int, xv: np.ndarray, probe: int = 0, kind: Optional[str] = None):
    """L = sum_f |(X_f - xv_f)/xv_f|^2 at probe `probe`, and dL/d wp2 (full trajectory)."""
    keep = _Keep()
    pb = _problem(p, keep)
    xr = np.ascontiguousarray(np.real(xv), np.float64)
    xi = np.ascontiguousarray(np.imag(xv), np.float64)
    loss = ctypes.c_double()
    grad = np.zeros(p.n)
    F = len(p.freqs)
    X = np.zeros(2 * F)
    rc = lib(kind).or1d_adjoint_r2(ctypes.byref(pb), nsteps, probe, _ptr(xr), _ptr(xi),
                               ctypes.addressof(loss), _ptr(grad), _ptr(X))
    if rc != 0:
        raise ValueError(f"oracle adjoint rejected the problem (code {rc})")
    return loss.value, grad, X[:F] + 1j * X[F:]


# ---------------------------------------------------------------------------
# 3D (rketd3d.c)
# ---------------------------------------------------------------------------

class _Problem3(ctypes.Structure):
    _fields_ = [
        ("nx", ctypes.c_int64), ("ny", ctypes.c_int64), ("nz", ctypes.c_int64),
        ("d", ctypes.c_double), ("dt", ctypes.c_double),
        ("wp2", ctypes.c_void_p * 3), ("nu", ctypes.c_void_p * 3),
        ("periodic_x", ctypes.c_int32), ("periodic_y", ctypes.c_int32),
        ("cpml", ctypes.c_int64), ("source", ctypes.c_int32), ("src_comp", ctypes.c_int32),
        ("src_k", ctypes.c_int64), ("src_tau", ctypes.c_double), ("src_t0", ctypes.c_double),
        ("src_amp", ctypes.c_double), ("b0", ctypes.c_int64), ("b1", ctypes.c_int64),
        ("naux", ctypes.c_int64), ("aux_off", ctypes.c_int64), ("aux_src", ctypes.c_int64),
        ("n_points", ctypes.c_int32), ("n_freqs", ctypes.c_int32),
        ("points", ctypes.c_void_p), ("freqs", ctypes.c_void_p),
    ]


class _State3(ctypes.Structure):
    _fields_ = [
        ("E", ctypes.c_void_p * 3), ("H", ctypes.c_void_p * 3), ("J", ctypes.c_void_p * 3),
        ("psi", ctypes.c_void_p), ("Einc", ctypes.c_void_p), ("Hinc", ctypes.c_void_p),
        ("Xre", ctypes.c_void_p), ("Xim", ctypes.c_void_p), ("step", ctypes.c_int64),
    ]


SOURCE3 = {"none": 0, "planar": 1, "tfsf": 2}


def _problem3(p, keep: _Keep) -> _Problem3:
    wp2 = [keep.arr(p.wp2[c], np.float64) for c in range(3)]
    nu = [keep.arr(p.nu_comp(c), np.float64) for c in range(3)]
    pts = keep.arr(np.asarray(p.points, np.int32).reshape(-1, 4), np.int32)
    freqs = keep.arr(p.freqs, np.float64)
    naux, aoff, asrc = p.aux_layout() if p.source == "tfsf" else (0, 0, 0)
    return _Problem3(
        nx=p.nx, ny=p.ny, nz=p.nz, d=p.d, dt=p.dt,
        wp2=(ctypes.c_void_p * 3)(*[_ptr(a) for a in wp2]),
        nu=(ctypes.c_void_p * 3)(*[_ptr(a) for a in nu]),
        periodic_x=int(p.periodic_x), periodic_y=int(p.periodic_y), cpml=p.cpml,
        source=SOURCE3[p.source], src_comp=p.src_comp, src_k=p.src_k,
        src_tau=p.src_tau, src_t0=p.src_t0, src_amp=p.src_amp, b0=p.b0, b1=p.b1,
        naux=naux, aux_off=aoff, aux_src=asrc, n_points=len(pts), n_freqs=len(freqs),
        points=_ptr(pts), freqs=_ptr(freqs))


def new_state3(p) -> dict:
    shp = (3, p.nx, p.ny, p.nz)
    naux = p.aux_layout()[0] if p.source == "tfsf" else 1
    return {"E": np.zeros(shp), "H": np.zeros(shp), "J": np.zeros(shp),
            "psi": np.zeros((12, p.nx, p.ny, p.nz)) if p.cpml > 0 else np.zeros(1),
            "Einc": np.zeros(naux), "Hinc": np.zeros(naux),
            "X": np.zeros((len(p.points), len(p.freqs)), np.complex128), "step": 0}


def check3(p) -> int:
    keep = _Keep()
    return lib().or3d_check(ctypes.byref(_problem3(p, keep)))


def run3d(p, nsteps: int, state: Optional[dict] = None, kind: Optional[str] = None) -> dict:
    """Advance a 3D state (default: zero fields at step 0) by nsteps; returns a
    new dict with E, H, J [3, nx, ny, nz], psi, Einc, Hinc, X [points, freqs]."""
    st = new_state3(p) if state is None else {k: (v.copy() if isinstance(v, np.ndarray) else v)
                                             for k, v in state.items()}
    keep = _Keep()
    pb = _problem3(p, keep)
    for k in ("E", "H", "J", "psi", "Einc", "Hinc"):
        st[k] = np.ascontiguousarray(st[k], np.float64)
    Xre = np.ascontiguousarray(st["X"].real)
    Xim = np.ascontiguousarray(st["X"].imag)
    arr3 = lambda a: (ctypes.c_void_p * 3)(*[a[c].ctypes.data for c in range(3)])
    cs = _State3(E=arr3(st["E"]), H=arr3(st["H"]), J=arr3(st["J"]),
                 psi=_ptr(st["psi"]) if p.cpml > 0 else None,
                 Einc=_ptr(st["Einc"]), Hinc=_ptr(st["Hinc"]),
                 Xre=_ptr(Xre), Xim=_ptr(Xim), step=st["step"])
    rc = lib(kind).or3d_step(ctypes.byref(pb), ctypes.byref(cs), nsteps)
    if rc != 0:
        raise ValueError(f"3D oracle rejected the problem (code {rc})")
    st["X"] = Xre + 1j * Xim
    st["step"] = cs.step
    return st


# ---------------------------------------------------------------------------
# 2D (rketd2d.c)
# ---------------------------------------------------------------------------

class _Problem2(ctypes.Structure):
    _fields_ = [
        ("mode", ctypes.c_int32), ("nx", ctypes.c_int64), ("ny", ctypes.c_int64),
        ("d", ctypes.c_double), ("dt", ctypes.c_double),
        ("wp2", ctypes.c_void_p * 2), ("nu", ctypes.c_void_p * 2),
        ("periodic_x", ctypes.c_int32), ("periodic_y", ctypes.c_int32),
        ("has_src", ctypes.c_int32), ("src_i", ctypes.c_int64), ("src_j", ctypes.c_int64),
        ("src_tau", ctypes.c_double), ("src_t0", ctypes.c_double), ("src_amp", ctypes.c_double),
        ("n_probes", ctypes.c_int32), ("n_freqs", ctypes.c_int32),
        ("probes", ctypes.c_void_p), ("freqs", ctypes.c_void_p),
    ]


class _State2(ctypes.Structure):
    _fields_ = [
        ("E", ctypes.c_void_p * 2), ("H", ctypes.c_void_p * 2), ("J", ctypes.c_void_p * 2),
        ("Xre", ctypes.c_void_p), ("Xim", ctypes.c_void_p), ("step", ctypes.c_int64),
    ]


def _problem2(p, keep: _Keep) -> _Problem2:
    nc = 1 if p.mode == "tm" else 2
    wp2 = [keep.arr(p.wp2[c], np.float64) for c in range(nc)]
    nu = [keep.arr(p.nu[c], np.float64) for c in range(nc)]
    while len(wp2) < 2:
        wp2.append(wp2[0])
        nu.append(nu[0])
    pr = keep.arr(np.asarray(p.probes, np.int64).reshape(-1, 3), np.int64)
    fr = keep.arr(p.freqs, np.float64)
    src = p.src if p.src is not None else (0, 0)
    return _Problem2(
        mode=0 if p.mode == "tm" else 1, nx=p.nx, ny=p.ny, d=p.d, dt=p.dt,
        wp2=(ctypes.c_void_p * 2)(*[_ptr(a) for a in wp2]), nu=(ctypes.c_void_p * 2)(*[_ptr(a) for a in nu]),
        periodic_x=int(p.periodic_x), periodic_y=int(p.periodic_y), has_src=int(p.src is not None),
        src_i=int(src[0]), src_j=int(src[1]), src_tau=p.src_tau, src_t0=p.src_t0, src_amp=p.src_amp,
        n_probes=len(pr), n_freqs=len(fr), probes=_ptr(pr), freqs=_ptr(fr))


def new_state2(p) -> dict:
    nc = 1 if p.mode == "tm" else 2
    nh = 2 if p.mode == "tm" else 1
    return {"E": np.zeros((nc, p.nx, p.ny)), "H": np.zeros((nh, p.nx, p.ny)), "J": np.zeros((nc, p.nx, p.ny)),
            "X": np.zeros((len(p.probes), len(p.freqs)), np.complex128), "step": 0}


def check2(p) -> int:
    keep = _Keep()
    return lib().or2d_check(ctypes.byref(_problem2(p, keep)))


def run2d(p, nsteps: int, state: Optional[dict] = None, kind: Optional[str] = None) -> dict:
    """Advance a 2D state (default: zero at step 0) by nsteps; returns a new dict
    with E [ncomp, nx, ny], H [2 (TM: Hx, Hy) or 1 (TE: Hz), nx, ny], J, X."""
    st = new_state2(p) if state is None else {k: (v.copy() if isinstance(v, np.ndarray) else v)
                                             for k, v in state.items()}
    keep = _Keep()
    pb = _problem2(p, keep)
    for k in ("E", "H", "J"):
        st[k] = np.ascontiguousarray(st[k], np.float64)
    Xre = np.ascontiguousarray(st["X"].real)
    Xim = np.ascontiguousarray(st["X"].imag)
    two = lambda a: (ctypes.c_void_p * 2)(*[a[min(c, a.shape[0] - 1)].ctypes.data for c in range(2)])
    cs = _State2(E=two(st["E"]), H=two(st["H"]), J=two(st["J"]), Xre=_ptr(Xre), Xim=_ptr(Xim), step=st["step"])
    rc = lib(kind).or2d_step(ctypes.byref(pb), ctypes.byref(cs), nsteps)
    if rc != 0:
        raise ValueError(f"2D oracle rejected the problem (code {rc})")
    st["X"] = Xre + 1j * Xim
    st["step"] = cs.step
    return st
