"""Pins of the FP64 3D oracle against what the mathematics fixes:

* a PEC (and a periodic-x/y) cavity eigenmode of the Yee lattice oscillates at
  the lattice's own dispersion frequency, sin(w dt/2) = (c dt/2)|s| with
  s_a = (2/d) sin(k_a d/2) -- every curl term, sign and neighbour index and
  both wall rules enter it;
* the discrete electromagnetic energy of a vacuum PEC box is conserved;
* a field uniform across two axes is the 1D problem along the third: the 3D
  oracle reproduces the 1D oracle (itself pinned in test_oracle_pins.py) along
  z (Ex/Hy, Ey/Hx, planar source), along x (Ez/Hy) and along y (Ez/Hx), with
  plasma, PEC or CPML walls;
* a total-field/scattered-field plane wave in vacuum leaves the scattered
  region at rounding level and the total region equal to the incident wave;
* the incident grid is the 1D oracle's Mur grid, and the running DFT uses
  t = m dt for E and (m - 1/2) dt for H.
"""
import math

import numpy as np
import pytest

import oracle
from paper_1709_00821_amd import workloads as W

C0 = 299792458.0


def mk(nx, ny, nz, *, d=75e-6, courant=0.5, wp2=None, nu=None, points=None, n_freqs=6, **kw):
    dt = courant * d / C0
    tau, t0, amp = W.pulse_params(dt)
    if wp2 is None:
        wp2 = np.zeros((3, nx, ny, nz))
    if nu is None:
        nu = np.full((3, nx, ny, nz), 2e10)
    if points is None:
        points = np.zeros((0, 4), np.int32)
    return W.Problem3D(nx=nx, ny=ny, nz=nz, d=d, dt=dt, wp2=wp2, nu=nu, src_tau=tau,
                       src_t0=t0, src_amp=amp, freqs=np.linspace(2e9, 60e9, n_freqs),
                       points=np.asarray(points, np.int32), **kw)


# --------------------------------------------------------------------------
# cavity eigenmode
# --------------------------------------------------------------------------

def _mode(p, mnp, periodic, rng):
    """E pattern with amplitude A (s . A = 0) and H pattern with amplitude s x A."""
    n = (p.nx, p.ny, p.nz)
    k = [(2 if periodic[a] else 1) * math.pi * mnp[a] / (n[a] * p.d) for a in range(3)]
    s = np.array([2.0 / p.d * math.sin(k[a] * p.d / 2) for a in range(3)])
    A = np.cross(s, rng.normal(size=3))
    A /= np.max(np.abs(A))
    Cv = np.cross(s, A)
    idx = [np.arange(m, dtype=np.float64) for m in n]

    def pat(offs):
        # along axis a: cos at half-integer positions, sin at integer ones
        f = []
        for a in range(3):
            x = (idx[a] + offs[a]) * p.d
            f.append(np.cos(k[a] * x) if offs[a] == 0.5 else np.sin(k[a] * x))
        return f[0][:, None, None] * f[1][None, :, None] * f[2][None, None, :]

    E = np.stack([A[c] * pat(W.STAGGER[nm]) for c, nm in enumerate(("Ex", "Ey", "Ez"))])
    Hp = np.stack([Cv[c] * pat(W.STAGGER[nm]) for c, nm in enumerate(("Hx", "Hy", "Hz"))])
    return E, Hp, s


@pytest.mark.parametrize("periodic", [False, True])
def test_cavity_eigenmode_frequency(periodic):
    p = mk(6, 7, 9, periodic_x=periodic, periodic_y=periodic)
    rng = np.random.default_rng(41)
    mu0 = oracle.constants()["mu0"]
    E0, Hp, s = _mode(p, (1, 2, 1) if not periodic else (1, 1, 2), (periodic, periodic, False), rng)
    sw = C0 * p.dt / 2 * np.linalg.norm(s)
    w = 2 * math.asin(sw) / p.dt
    gam = -(p.dt / mu0) / (2 * sw)
    st = oracle.new_state3(p)
    st["E"] = E0.copy()
    st["H"] = gam * math.sin(-w * p.dt / 2) * Hp        # H^{-1/2}
    for n in (1, 37, 300):
        out = oracle.run3d(p, n, st)
        e_ref = math.cos(w * n * p.dt) * E0
        h_ref = gam * math.sin(w * (n - 0.5) * p.dt) * Hp
        assert np.max(np.abs(out["E"] - e_ref)) <= 1e-12 * np.max(np.abs(E0)), n
        assert np.max(np.abs(out["H"] - h_ref)) <= 1e-12 * np.max(np.abs(Hp * gam)), n


def test_cavity_mode_detects_wrong_frequency():
    """The pin is sensitive: the continuous-space frequency differs from the
    lattice one by far more than the tolerance after 300 steps."""
    p = mk(6, 7, 9)
    E0, Hp, s = _mode(p, (1, 2, 1), (False, False, False), np.random.default_rng(41))
    kc = np.linalg.norm([math.pi / (6 * p.d), 2 * math.pi / (7 * p.d), math.pi / (9 * p.d)])
    w_lat = 2 * math.asin(C0 * p.dt / 2 * np.linalg.norm(s)) / p.dt
    assert abs(math.cos(w_lat * 300 * p.dt) - math.cos(C0 * kc * 300 * p.dt)) > 1e-3


def test_vacuum_pec_energy_conserved():
    p = mk(8, 9, 10)
    rng = np.random.default_rng(42)
    mu0, eps0 = oracle.constants()["mu0"], oracle.constants()["eps0"]
    st = oracle.new_state3(p)
    st["E"] = rng.normal(size=st["E"].shape)
    st["H"] = rng.normal(size=st["H"].shape) / 377.0
    # tangential E on the index-0 walls is held at zero
    st["E"][1, 0] = st["E"][2, 0] = 0
    st["E"][0, :, 0] = st["E"][2, :, 0] = 0
    st["E"][0, :, :, 0] = st["E"][1, :, :, 0] = 0
    Wn = []
    for _ in range(400):
        # W^n = eps0/2 |E^n|^2 + mu0/2 H^{n-1/2} . H^{n+1/2}
        e_n, h_prev = st["E"], st["H"]
        st = oracle.run3d(p, 1, st)
        Wn.append(0.5 * eps0 * np.sum(e_n ** 2) + 0.5 * mu0 * np.sum(st["H"] * h_prev))
    Wn = np.array(Wn)
    assert np.max(np.abs(Wn - Wn[0])) <= 1e-12 * abs(Wn[0])


# --------------------------------------------------------------------------
# equivalence with the 1D oracle
# --------------------------------------------------------------------------

def _profile(rng, n, lo, hi):
    w = np.zeros(n)
    w[lo:hi] = rng.uniform(0, (2 * math.pi * 40e9) ** 2, hi - lo)
    nu = rng.uniform(1e9, 5e10, n)
    return w, nu


def _p1d(p3, n, w, nu, bc, P, src=-1, probes=(), freqs=None):
    return W.Problem1D(n=n, dz=p3.d, dt=p3.dt, wp2=w, nu=nu, src_cell=src, src_tau=p3.src_tau,
                       src_t0=p3.src_t0, src_amp=p3.src_amp, probes=np.asarray(probes, np.int64),
                       freqs=p3.freqs if freqs is None else freqs, bc=bc, cpml_cells=P)


def _close(a, b, exact, scale=None):
    if exact:
        return np.array_equal(a, b)
    s = np.max(np.abs(b)) if scale is None else scale
    return np.max(np.abs(a - b)) <= 1e-13 * s


@pytest.mark.parametrize("comp", [0, 1])
@pytest.mark.parametrize("bc", ["pec", "cpml"])
def test_z_uniform_layer_equals_1d(comp, bc):
    rng = np.random.default_rng(43 + comp)
    nz, P = 120, (10 if bc == "cpml" else 0)
    w, nu = _profile(rng, nz + 1, 40, 80)
    wp2 = np.broadcast_to(w[:nz], (3, 3, 4, nz)).copy()
    nuv = np.broadcast_to(nu[:nz], (3, 3, 4, nz)).copy()
    pts = [(comp, 1, 2, 30), (comp, 0, 3, 100), (3 + (1 - comp), 2, 0, 30)]
    p3 = mk(3, 4, nz, wp2=wp2, nu=nuv, periodic_x=True, periodic_y=True, cpml=P,
            source="planar", src_comp=comp, src_k=20, points=pts)
    p1 = _p1d(p3, nz + 1, w, nu, bc, P, src=20, probes=(30, 100))
    T = 400
    o3 = oracle.run3d(p3, T)
    o1 = oracle.run(p1, T)
    exact = bc == "pec"
    sgn = 1.0 if comp == 0 else -1.0          # Hy = H1d for Ex, Hx = -H1d for Ey
    hcomp = 1 if comp == 0 else 0
    for i in range(3):
        for j in range(4):
            assert _close(o3["E"][comp, i, j], o1["E"][:nz], exact)
            assert _close(o3["J"][comp, i, j], o1["J"][:nz], exact)
            assert _close(sgn * o3["H"][hcomp, i, j], o1["H"][:nz], exact)
    others = [c for c in range(3) if c != comp]
    assert not np.any(o3["E"][others]) and not np.any(o3["J"][others])
    assert not np.any(o3["H"][[c for c in range(3) if c != hcomp]])
    assert _close(o3["X"][:2], o1["X"], exact, np.max(np.abs(o1["X"])))
    # the H sample runs half a step behind E: it is not the E spectrum
    assert np.max(np.abs(o3["X"][2])) > 0


@pytest.mark.parametrize("axis", ["x", "y"])
@pytest.mark.parametrize("bc", ["pec", "cpml"])
def test_transverse_axis_equals_1d(axis, bc):
    """Ez polarised wave along x (H1d = -Hy) or along y (H1d = Hx), plasma and
    an initial field profile varying along that axis."""
    rng = np.random.default_rng(47 if axis == "x" else 48)
    n, P = 90, (8 if bc == "cpml" else 0)
    w, nu = _profile(rng, n + 1, 30, 60)
    e1 = rng.normal(size=n + 1)
    e1[0] = e1[n] = 0.0
    h1 = rng.normal(size=n + 1) / 377.0
    h1[n] = 0.0
    j1 = rng.normal(size=n + 1) * 1e-3
    j1[0] = j1[n] = 0.0
    nz = 2 * P + 2 if P else 4            # z is walled (and lined) too
    if axis == "x":
        shape, expand = (n, 2, nz), (lambda v: np.broadcast_to(v[:n, None, None], (n, 2, nz)))
        kw = dict(periodic_x=False, periodic_y=True)
        hcomp, sgn = 1, -1.0
    else:
        shape, expand = (2, n, nz), (lambda v: np.broadcast_to(v[None, :n, None], (2, n, nz)))
        kw = dict(periodic_x=True, periodic_y=False)
        hcomp, sgn = 0, 1.0
    wp2 = np.zeros((3,) + shape)
    wp2[2] = expand(w)
    nuv = np.broadcast_to(expand(nu), (3,) + shape).copy()
    p3 = mk(*shape, wp2=wp2, nu=nuv, cpml=P, **kw)
    st = oracle.new_state3(p3)
    st["E"][2] = expand(e1)
    st["H"][hcomp] = sgn * expand(h1)
    st["J"][2] = expand(j1)
    p1 = _p1d(p3, n + 1, w, nu, bc, P)
    s1 = oracle.new_state(p1)
    s1["E"], s1["H"], s1["J"] = e1.copy(), h1.copy(), j1.copy()
    T = 300
    o3 = oracle.run3d(p3, T, st)
    o1 = oracle.run(p1, T, s1)
    exact = bc == "pec"
    mv = (lambda a: np.moveaxis(a, 0, 0)) if axis == "x" else (lambda a: np.moveaxis(a, 1, 0))
    Ez, Hh, Jz = mv(o3["E"][2]), mv(o3["H"][hcomp]), mv(o3["J"][2])
    for a in range(Ez.shape[1]):
        for b in range(Ez.shape[2]):
            assert _close(Ez[:, a, b], o1["E"][:n], exact)
            assert _close(sgn * Hh[:, a, b], o1["H"][:n], exact)
            assert _close(Jz[:, a, b], o1["J"][:n], exact)
    assert not np.any(o3["E"][:2]) and not np.any(o3["J"][:2])
    assert not np.any(o3["H"][[c for c in range(3) if c != hcomp]])


# --------------------------------------------------------------------------
# total-field / scattered-field source
# --------------------------------------------------------------------------

def _tfsf_problem(periodic, cpml=4, points=None):
    if periodic:
        return mk(3, 4, 40, periodic_x=True, periodic_y=True, cpml=cpml, source="tfsf",
                  b0=8, b1=30, points=points)
    return mk(16, 18, 40, cpml=cpml, source="tfsf", b0=6, b1=12, points=points)


def _tf_mask(p, comp):
    """Which nodes of a component lie in the total-field box."""
    off = W.STAGGER[W.COMPONENTS[comp]]
    masks = []
    for a, (m, per) in enumerate(((p.nx, p.periodic_x), (p.ny, p.periodic_y), (p.nz, False))):
        x = np.arange(m) + off[a]
        masks.append(np.ones(m, bool) if per else (x >= p.b0) & (x <= p.b1))
    return masks[0][:, None, None] & masks[1][None, :, None] & masks[2][None, None, :]


@pytest.mark.parametrize("periodic", [False, True])
def test_tfsf_vacuum_no_leak(periodic):
    p = _tfsf_problem(periodic)
    naux, ao, _ = p.aux_layout()
    st = None
    peak = 0.0
    for _ in range(12):
        st = oracle.run3d(p, 25, st)
        Ei, Hi = st["Einc"], st["Hinc"]
        peak = max(peak, np.max(np.abs(Ei)))
        for c in range(6):
            F = st["E"][c] if c < 3 else st["H"][c - 3]
            tf = _tf_mask(p, c)
            ref = np.zeros(F.shape)
            q = np.clip(np.arange(p.nz) + ao, 0, naux - 1)   # aux node of each z (box only)
            if c == 0:
                ref[:] = Ei[q][None, None, :]
            elif c == 4:
                ref[:] = Hi[q][None, None, :]
            ref[~tf] = 0.0
            scale = peak if c < 3 else peak / 376.7
            assert np.max(np.abs(F - ref)) <= 1e-12 * scale, (st["step"], c)
    assert peak > 0.5          # the pulse went through the box


def test_scattered_region_quiet_only_with_the_split():
    """Sensitivity of the leak pin: a plain planar source on the box face (no
    total/scattered split) radiates into the region below it."""
    p = _tfsf_problem(False)
    q = p.copy(source="planar", src_k=p.b0)
    st = oracle.run3d(q, 150)
    assert np.max(np.abs(st["E"][0][:, :, :p.b0 - 1])) > 1e-3


def test_incident_grid_is_the_1d_mur_grid():
    p = _tfsf_problem(False)
    naux, ao, asrc = p.aux_layout()
    T = 260
    o3 = oracle.run3d(p, T)
    p1 = _p1d(p, naux, np.zeros(naux), np.zeros(naux), "mur", 0, src=asrc)
    o1 = oracle.run(p1, T)
    assert np.array_equal(o3["Einc"], o1["E"])
    assert np.array_equal(o3["Hinc"][:naux - 1], o1["H"][:naux - 1])


def test_sample_times_e_and_h():
    """X(f) = sum_m v_m dt exp(-j 2 pi f t_m), t_m = m dt (E), (m - 1/2) dt (H)."""
    pts = np.array([(0, 8, 9, 9), (4, 8, 9, 9), (2, 7, 9, 10), (5, 9, 11, 3)], np.int32)
    p = _tfsf_problem(False, points=pts)
    st = None
    series = []
    for _ in range(120):
        st = oracle.run3d(p, 1, st)
        series.append([st["E"][c][i, j, k] if c < 3 else st["H"][c - 3][i, j, k] for c, i, j, k in pts])
    v = np.array(series)                          # [m-1, point]
    m = np.arange(1, 121)
    for q, (c, *_ ) in enumerate(pts):
        t = (m if c < 3 else m - 0.5) * p.dt
        ref = np.array([np.sum(v[:, q] * p.dt * np.exp(-2j * np.pi * f * t)) for f in p.freqs])
        assert np.max(np.abs(st["X"][q] - ref)) <= 1e-12 * max(np.max(np.abs(ref)), 1e-300), q
    assert np.max(np.abs(v[:, 0])) > 0.1 and np.max(np.abs(v[:, 1])) > 1e-4


def test_box_points_are_tangential_and_on_the_box():
    """Each face carries its four tangential components: E in the face plane,
    H half a cell towards +axis (the H node of the same index)."""
    lo, hi = 3, 9
    pts = W.box_points(lo, hi, 12, 13, 14)
    m = hi - lo
    assert len(pts) == 6 * 4 * m * (m + 1)
    per_face = np.split(pts, 6)
    for f, face in enumerate(per_face):
        axis, plane = f // 2, (lo, hi)[f % 2]
        assert len({tuple(r) for r in face.tolist()}) == len(face)
        for c, i, j, k in face:
            off = W.STAGGER[W.COMPONENTS[c]]
            idx = (i, j, k)
            assert off[axis] == (0.0 if c < 3 else 0.5)      # tangential to the face
            assert idx[axis] == plane
            for a in range(3):
                if a != axis:
                    assert lo <= idx[a] + off[a] <= hi


def test_check_rejects():
    p = _tfsf_problem(False)
    assert oracle.check3(p) == 0
    assert oracle.check3(p.copy(b0=0)) == -1
    assert oracle.check3(p.copy(dt=p.dt * 1.2)) == -2      # c dt / d = 0.6 > 1/sqrt(3)
    bad = p.wp2.copy()
    bad[0, 1, 1, 1] = -1.0
    assert oracle.check3(p.copy(wp2=bad)) == -1
