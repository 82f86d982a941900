"""GPU 3D Yee-RKETD against the FP64 3D oracle (itself pinned in
test_oracle3d_pins.py): every field and every sample spectrum, FP64 within
1e-12 and FP32 within the stated FP32 bound, on grids whose k extent leaves a
ragged 64-node tail and whose j extent a ragged 4-row tail; plus step
composition, graph replay, field I/O, and full-size (384^3) properties."""
import math
import sys

import numpy as np
import pytest

import oracle
from paper_1709_00821_amd import workloads as W
from tests.test_oracle3d_pins import mk, _mode

pytestmark = pytest.mark.gpu
C0 = 299792458.0
NAMES = ("Ex", "Ey", "Ez", "Hx", "Hy", "Hz", "Jx", "Jy", "Jz")


def say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def G():
    import torch
    assert torch.cuda.is_available()
    from paper_1709_00821_amd import plasma3d
    return plasma3d


def sphere_small(**kw):
    """28 x 27 x 70 cells (ragged 64-node k tail, ragged 4-row j tail), CPML 4,
    TF box [6, 21] around a Gaussian plasma sphere, DFT box faces at 4 and 23."""
    nx, ny, nz = 28, 27, 70
    d = 0.5e-3
    p = mk(nx, ny, nz, d=d, cpml=4, source="tfsf", b0=6, b1=21, n_freqs=16, **kw)
    wp2 = W.sphere_wp2(nx, ny, nz, (13.5, 13.0, 14.0), 4.0, 6.0, (2 * math.pi * 20e9) ** 2)
    pts = W.box_points(4, 23, nx, ny, nz)
    return p.copy(wp2=wp2, nu=np.full((nx, ny, nz), 1e10), points=pts,
                  freqs=np.linspace(2e9, 40e9, 16))


def layer_planar(rng):
    nx, ny, nz = 3, 5, 150
    w = np.zeros(nz)
    w[60:110] = rng.uniform(0, (2 * math.pi * 40e9) ** 2, 50)
    wp2 = np.broadcast_to(w, (3, nx, ny, nz)).copy()
    nu = np.broadcast_to(rng.uniform(1e9, 5e10, nz), (3, nx, ny, nz)).copy()
    pts = np.array([(1, 0, 0, 30), (1, 2, 4, 130), (3, 1, 1, 30)], np.int32)
    return mk(nx, ny, nz, wp2=wp2, nu=nu, periodic_x=True, periodic_y=True, cpml=8,
              source="planar", src_comp=1, src_k=20, points=pts)


def tfsf_periodic(rng):
    nx, ny, nz = 4, 3, 130
    w = np.zeros(nz)
    w[50:90] = rng.uniform(0, (2 * math.pi * 40e9) ** 2, 40)
    wp2 = np.broadcast_to(w, (3, nx, ny, nz)).copy()
    pts = np.array([(0, 0, 0, 12), (4, 3, 2, 12), (0, 1, 1, 120), (4, 2, 0, 100)], np.int32)
    return mk(nx, ny, nz, wp2=wp2, periodic_x=True, periodic_y=True, cpml=6, source="tfsf",
              b0=16, b1=110, points=pts)


def blob_pec(rng):
    nx, ny, nz = 13, 10, 67
    wp2 = np.zeros((3, nx, ny, nz))
    wp2[:, 3:10, 2:8, 20:40] = rng.uniform(0, (2 * math.pi * 40e9) ** 2, (3, 7, 6, 20))
    nu = rng.uniform(1e9, 5e10, (3, nx, ny, nz))
    pts = np.array([(0, 6, 5, 10), (2, 6, 5, 50), (5, 4, 4, 45)], np.int32)
    return mk(nx, ny, nz, wp2=wp2, nu=nu, source="planar", src_comp=0, src_k=8, points=pts)


CASES = {
    "sphere_tfsf_cpml": lambda rng: sphere_small(),
    "layer_planar_periodic": layer_planar,
    "tfsf_periodic_layer": tfsf_periodic,
    "blob_planar_pec": blob_pec,
}


def gpu_fields(h):
    return {nm: h.field(nm).astype(np.float64) for nm in NAMES}


def oracle_fields(o):
    out = {}
    for c in range(3):
        out[NAMES[c]] = o["E"][c]
        out[NAMES[3 + c]] = o["H"][c]
        out[NAMES[6 + c]] = o["J"][c]
    return out


ETA0 = 376.730313668


def scales(of, Xo, pts, dt):
    """Per-group field scales (E, H, J) and per-kind spectrum scales (E, H).
    E and H scales are tied through eta0, and a spectrum's scale is at least
    one sample of its field's scale (v dt): a point the wave has not reached
    holds rounding noise, which is no scale."""
    s = {grp: max(np.max(np.abs(of[nm])) for nm in NAMES if nm[0] == grp) for grp in "EHJ"}
    s["E"], s["H"] = max(s["E"], ETA0 * s["H"]), max(s["H"], s["E"] / ETA0)
    isH = np.asarray(pts)[:, 0] >= 3 if len(pts) else np.zeros(0, bool)
    xe = np.max(np.abs(Xo[~isH])) if np.any(~isH) else 0.0
    xh = np.max(np.abs(Xo[isH])) if np.any(isH) else 0.0
    s["XE"] = max(xe, ETA0 * xh, s["E"] * dt)
    s["XH"] = max(xh, xe / ETA0, s["H"] * dt)
    return s


def compare(gf, of, Xg, Xo, pts, rtol, what, sc):
    """Max errors against rtol times the scales sc (those of the livelier of
    the states compared, once the pulse has left the grid)."""
    for nm in NAMES:
        s = sc[nm[0]]
        if s == 0:
            assert not np.any(gf[nm]), (what, nm)
            continue
        err = np.max(np.abs(gf[nm] - of[nm]))
        assert err <= rtol * s, f"{what} {nm}: {err:.3e} vs scale {s:.3e}"
    if len(pts):
        isH = np.asarray(pts)[:, 0] >= 3
        for sel, key in ((~isH, "XE"), (isH, "XH")):
            if not np.any(sel):
                continue
            err = np.max(np.abs(Xg[sel] - Xo[sel]))
            assert err <= rtol * sc[key], f"{what} spectra: {err:.3e} vs scale {sc[key]:.3e}"


def max_scales(a, b):
    return {k: max(a[k], b[k]) for k in a}


@pytest.mark.parametrize("case", list(CASES))
def test_3d_matches_oracle(G, case):
    """Both executors against the oracle at step 110 (pulse on the grid) and
    240; split and fused agree bit for bit."""
    rng = np.random.default_rng(1900 + list(CASES).index(case))
    p = CASES[case](rng)
    T1, T2 = 110, 240
    say(f"case 3d {case} grid {p.nx}x{p.ny}x{p.nz} steps {T1}+{T2 - T1}: oracle")
    o1 = oracle.run3d(p, T1)
    o2 = oracle.run3d(p, T2 - T1, o1)
    of1, of2 = oracle_fields(o1), oracle_fields(o2)
    sc1 = scales(of1, o1["X"], p.points, p.dt)
    sc2 = max_scales(sc1, scales(of2, o2["X"], p.points, p.dt))
    for prec, rtol in (("f64", 1e-12), ("f32", 2e-5)):
        got = {}
        for ex in ("split", "fused"):
            say(f"case 3d {case} {prec} {ex}")
            with G.FdtdPlasma3D(p, precision=prec, sample_slots=7, exec=ex) as h:
                h.step(T1)
                compare(gpu_fields(h), of1, h.spectra(), o1["X"], p.points, rtol, f"{case} {prec} {ex} @{T1}", sc1)
                h.step(T2 - T1)
                gf = gpu_fields(h)
                X = h.spectra()
            compare(gf, of2, X, o2["X"], p.points, rtol, f"{case} {prec} {ex} @{T2}", sc2)
            got[ex] = (gf, X)
        assert all(np.array_equal(got["split"][0][nm], got["fused"][0][nm]) for nm in NAMES)
        assert np.array_equal(got["split"][1], got["fused"][1])


def test_3d_cavity_mode_via_set_fields(G):
    """Initial-value run from a lattice eigenmode (vacuum PEC box)."""
    p = mk(6, 7, 9)
    E0, Hp, s = _mode(p, (1, 2, 1), (False, False, False), np.random.default_rng(41))
    mu0 = oracle.constants()["mu0"]
    sw = C0 * p.dt / 2 * np.linalg.norm(s)
    w = 2 * math.asin(sw) / p.dt
    H0 = -(p.dt / mu0) / (2 * sw) * math.sin(-w * p.dt / 2) * Hp
    st = oracle.new_state3(p)
    st["E"], st["H"] = E0.copy(), H0.copy()
    o = oracle.run3d(p, 150, st)
    for ex in ("fused", "split"):
        say(f"case 3d cavity f64 {ex}")
        with G.FdtdPlasma3D(p, precision="f64", exec=ex) as h:
            for c in range(3):
                h.set_field(NAMES[c], E0[c])
                h.set_field(NAMES[3 + c], H0[c])
            h.step(75)
            h.step(75)
            for c in range(3):
                assert np.max(np.abs(h.field(NAMES[c]) - o["E"][c])) <= 1e-12 * np.max(np.abs(E0))
                assert np.max(np.abs(h.field(NAMES[3 + c]) - o["H"][c])) <= 1e-12 * np.max(np.abs(H0))


@pytest.mark.parametrize("prec,ex", [("f32", "fused"), ("f64", "fused"), ("f32", "split")])
def test_3d_step_composition_and_replay(G, prec, ex):
    p = sphere_small()
    say(f"case 3d composition {prec} {ex}")
    with G.FdtdPlasma3D(p, precision=prec, sample_slots=5, exec=ex) as h:
        h.run(120)
        ref = gpu_fields(h)
        Xr = h.spectra()
        h.run(120)                      # graph replay
        assert all(np.array_equal(ref[nm], h.field(nm)) for nm in NAMES)
        assert np.array_equal(Xr, h.spectra())
        h.run(119)                      # odd length: the other ping-pong copy
        h.run(120)
        assert all(np.array_equal(ref[nm], h.field(nm)) for nm in NAMES)
    with G.FdtdPlasma3D(p, precision=prec, sample_slots=5, exec=ex) as h:
        h.step(37)
        h.spectra()                     # folding the window must not disturb later steps
        h.step(83)
        assert h.steps_done() == 120
        assert all(np.array_equal(ref[nm], h.field(nm)) for nm in NAMES)
        assert np.array_equal(Xr, h.spectra())


def test_3d_field_io_roundtrip_and_support(G):
    p = blob_pec(np.random.default_rng(5))
    with G.FdtdPlasma3D(p, precision="f64") as h:
        h.step(40)
        J = h.field("Jx")
        assert np.any(J)
        assert not np.any(J[p.wp2[0] == 0])        # no current where the x component has no plasma
        rng = np.random.default_rng(6)
        v = rng.normal(size=J.shape) * (p.wp2[0] > 0)
        h.set_field("Jx", v)
        assert np.array_equal(h.field("Jx"), v)
        bad = np.zeros(J.shape)
        bad[0, 0, 0] = 1.0
        with pytest.raises(Exception):
            h.set_field("Jx", bad)


def test_3d_c3_scaled_96_matches_oracle(G):
    """The 384^3 sphere problem scaled to 96^3 (same shape: sphere radius n/4,
    Gaussian falloff, TF box and CPML scaled, box DFT), 200 steps."""
    p = W.sphere_c3(96, cpml=4, n_freqs=16)
    T = 200
    say(f"case 3d c3@96: oracle ({p.ncells} cells, {len(p.points)} sample points)")
    o = oracle.run3d(p, T)
    of = oracle_fields(o)
    for prec, rtol in (("f64", 1e-12), ("f32", 2e-5)):
        say(f"case 3d c3@96 {prec}")
        with G.FdtdPlasma3D(p, precision=prec) as h:
            h.run(T)
            compare(gpu_fields(h), of, h.spectra(), o["X"], p.points, rtol, f"c3@96 {prec}",
                    scales(of, o["X"], p.points, p.dt))


def test_3d_c3_full_size_vacuum_properties(G):
    """384^3 in the benchmark's configuration with the plasma off: the
    scattered-field region stays quiet, the total-field region carries exactly
    the incident wave of the 1D Mur grid (computed by the 1D oracle), and the
    scattered-field DFT box sees nothing."""
    p = W.sphere_c3(384, box_dft=True).vacuum()
    T = 700
    naux, ao, asrc = p.aux_layout()
    inc = W.Problem1D(n=naux, dz=p.d, dt=p.dt, wp2=np.zeros(naux), nu=np.zeros(naux), src_cell=asrc,
                      src_tau=p.src_tau, src_t0=p.src_t0, src_amp=p.src_amp,
                      probes=np.array([p.b0 + ao], np.int64), freqs=p.freqs, bc="mur")
    oi = oracle.run(inc, T)
    Ei, Xinc = oi["E"], oi["X"][0]
    say("case 3d c3 full size vacuum f32")
    with G.FdtdPlasma3D(p, precision="f32") as h:
        h.run(T)
        Ex = h.field("Ex")
        X = h.spectra()
        Ey = h.field("Ey")
    peak = np.max(np.abs(Ei))
    assert peak > 0.5
    b0, b1 = p.b0, p.b1
    tf = Ex[b0:b1, b0:b1 + 1, b0:b1 + 1].astype(np.float64)
    err_tf = np.max(np.abs(tf - Ei[np.arange(b0, b1 + 1) + ao][None, None, :]))
    sf = np.abs(Ex.astype(np.float64))
    sf[b0:b1, b0:b1 + 1, b0:b1 + 1] = 0.0
    say(f"full size: TF error {err_tf:.2e}, SF max {sf.max():.2e}, Ey max {np.abs(Ey).max():.2e}, peak {peak:.3f}")
    assert err_tf <= 1e-4 * peak
    assert sf.max() <= 1e-4 * peak
    assert np.abs(Ey).max() <= 1e-4 * peak
    assert np.all(np.isfinite(X))
    # the box spectra against the incident spectrum at the TF face
    isE = p.points[:, 0] < 3
    say(f"full size: box E spectra {np.abs(X[isE]).max():.2e} vs incident {np.abs(Xinc).max():.2e}")
    assert np.abs(X[isE]).max() <= 1e-3 * np.abs(Xinc).max()
