"""Pins of the 2D oracle (oracle/rketd2d.c) against what the lattice and the
already-pinned 1D oracle fix, on the CPU:

* a lattice eigenmode of a PEC box (TM: Ez = sin sin; TE: Hz = cos cos),
  started from its spatial shape, keeps that shape and follows the leapfrog
  recurrence u^{n+1} + u^{n-1} = (2 - lam) u^n with
  lam = 4 S^2 (sin^2(pi p / 2nx) + sin^2(pi q / 2ny)), S = c dt / d: every curl
  term, sign, neighbour index and wall rule enters;
* vacuum energy eps0/2 |E^n|^2 + mu0/2 <H^{n-1/2}, H^{n+1/2}> is conserved
  from random fields (walled and periodic), and decays with a collisional
  plasma;
* a field uniform along one axis (that axis periodic) equals the 1D oracle
  along the other, bit for bit, with plasma, in both modes and along both
  axes (the 1D oracle is pinned by test_oracle_pins.py);
* the probes take the running DFT of the E samples at t = m dt.
"""
import numpy as np
import pytest

import oracle
from paper_1709_00821_amd import workloads as W

EPS0 = 8.8541878128e-12
C0 = 299792458.0
MU0 = 1.0 / (EPS0 * C0 * C0)


def _vac(mode, nx, ny, **kw):
    dt = 0.5 * 75e-6 / C0
    tau, t0, amp = W.pulse_params(dt)
    nc = 1 if mode == "tm" else 2
    return W.Problem2D(mode=mode, nx=nx, ny=ny, d=75e-6, dt=dt, wp2=np.zeros((nc, nx, ny)),
                       nu=np.full((nc, nx, ny), 2e10), src=None, src_tau=tau, src_t0=t0, src_amp=amp,
                       probes=np.zeros((0, 3), np.int64), freqs=np.array([1e10]), **kw)


@pytest.mark.parametrize("mode", ["tm", "te"])
def test_pec_box_eigenmode_recurrence(mode):
    nx, ny, pq = 20, 24, (2, 3)
    p = _vac(mode, nx, ny)
    S = C0 * p.dt / p.d
    lam = 4 * S * S * (np.sin(np.pi * pq[0] / (2 * nx)) ** 2 + np.sin(np.pi * pq[1] / (2 * ny)) ** 2)
    i = np.arange(nx)[:, None]
    j = np.arange(ny)[None, :]
    st = oracle.new_state2(p)
    if mode == "tm":
        shape = np.sin(np.pi * pq[0] * i / nx) * np.sin(np.pi * pq[1] * j / ny)
        st["E"][0] = shape
        get = lambda s: s["E"][0]
    else:
        shape = np.cos(np.pi * pq[0] * (i + 0.5) / nx) * np.cos(np.pi * pq[1] * (j + 0.5) / ny)
        st["H"][0] = shape
        get = lambda s: s["H"][0]
    amps = []
    for n in range(200):
        st = oracle.run2d(p, 1, st)
        u = get(st)
        k = np.argmax(np.abs(shape))
        a = u.ravel()[k] / shape.ravel()[k]
        # the field keeps the mode's shape
        assert np.max(np.abs(u - a * shape)) <= 1e-12 * max(1.0, abs(a)), n
        amps.append(a)
    amps = np.array(amps)
    r = amps[2:] + amps[:-2] - (2 - lam) * amps[1:-1]
    assert np.max(np.abs(r)) <= 1e-12 * np.max(np.abs(amps))
    # and it oscillates (a sensitivity check: lam is far from 0 and 4)
    assert 0.05 < lam < 3.9 and np.min(amps) < -0.5 * np.max(amps)


def _step_energy(p, st):
    """One step; returns (new state, W^n = eps0/2 |E^n|^2 + mu0/2 <H^{n-1/2},
    H^{n+1/2}>) with E^n, H^{n-1/2} the state before the step."""
    E0, H0 = st["E"].copy(), st["H"].copy()
    st = oracle.run2d(p, 1, st)
    return st, 0.5 * EPS0 * np.sum(E0 ** 2) + 0.5 * MU0 * np.sum(H0 * st["H"])


@pytest.mark.parametrize("mode,per", [("tm", False), ("te", False), ("tm", True), ("te", True)])
def test_vacuum_energy_conserved(mode, per):
    rng = np.random.default_rng(7)
    p = _vac(mode, 18, 22, periodic_x=per, periodic_y=per)
    st = oracle.new_state2(p)
    st["E"] = rng.normal(size=st["E"].shape)
    st["H"] = rng.normal(size=st["H"].shape) / 376.73
    if not per:   # the held (tangential) wall values start at zero
        if mode == "tm":
            st["E"][0, 0, :] = 0.0
            st["E"][0, :, 0] = 0.0
        else:
            st["E"][1, 0, :] = 0.0
            st["E"][0, :, 0] = 0.0
    st, w0 = _step_energy(p, st)
    for n in range(300):
        st, w = _step_energy(p, st)
        assert abs(w - w0) <= 1e-12 * abs(w0), n


def test_plasma_energy_decays():
    rng = np.random.default_rng(8)
    p = _vac("tm", 16, 16)
    # a dense, strongly collisional plasma: the random field's lattice modes
    # (up to ~1 THz here) feel it
    p = p.copy(wp2=np.full((1, 16, 16), (2 * np.pi * 300e9) ** 2), nu=np.full((1, 16, 16), 5e11))
    st = oracle.new_state2(p)
    st["E"][0, 1:, 1:] = rng.normal(size=(15, 15))
    st, w0 = _step_energy(p, st)
    for n in range(400):
        st, w = _step_energy(p, st)
    assert 0 < w < 0.5 * w0


def _oracle1d(n, dt, d, wp2, nu, bc):
    tau, t0, amp = W.pulse_params(dt)
    return W.Problem1D(n=n, dz=d, dt=dt, wp2=wp2, nu=nu, src_cell=-1, src_tau=tau, src_t0=t0, src_amp=amp,
                       probes=np.array([0], np.int64), freqs=np.array([1e10]), bc=bc)


@pytest.mark.parametrize("mode,axis,walled", [("tm", "x", True), ("tm", "x", False), ("te", "x", True),
                                              ("te", "x", False), ("tm", "y", True), ("te", "y", True)])
def test_uniform_field_equals_1d_oracle(mode, axis, walled):
    """Fields and plasma uniform across `axis`' partner (periodic there) are the
    1D problem along `axis`: TM along x is (E, H) = (Ez, -Hy), TE along x
    (Ey, Hz), TM along y (Ez, Hx), TE along y (Ex, -Hz)."""
    rng = np.random.default_rng(11)
    n = 40
    m = 3                                       # cells across the uniform axis
    nx, ny = (n, m) if axis == "x" else (m, n)
    p = _vac(mode, nx, ny, periodic_x=(axis == "y") or not walled, periodic_y=(axis == "x") or not walled)
    comp = {("tm", "x"): 0, ("te", "x"): 1, ("tm", "y"): 0, ("te", "y"): 0}[(mode, axis)]
    hidx = {("tm", "x"): 1, ("te", "x"): 0, ("tm", "y"): 0, ("te", "y"): 0}[(mode, axis)]
    hsign = {("tm", "x"): -1.0, ("te", "x"): 1.0, ("tm", "y"): 1.0, ("te", "y"): -1.0}[(mode, axis)]
    prof = np.zeros(n)
    prof[10:30] = rng.uniform(0, (2 * np.pi * 40e9) ** 2, 20)
    nuv = rng.uniform(1e9, 5e10, n)
    e = rng.normal(size=n)
    h = rng.normal(size=n) / 376.73
    jv = rng.normal(size=n) * 1e-3
    if walled:
        e[0] = 0.0
        jv[0] = 0.0
    st = oracle.new_state2(p)
    wp2, nu = p.wp2.copy(), p.nu.copy()
    if axis == "x":
        wp2[comp] = prof[:, None]
        nu[comp] = nuv[:, None]
        st["E"][comp] = e[:, None]
        st["H"][hidx] = hsign * h[:, None]
        st["J"][comp] = jv[:, None]
    else:
        wp2[comp] = prof[None, :]
        nu[comp] = nuv[None, :]
        st["E"][comp] = e[None, :]
        st["H"][hidx] = hsign * h[None, :]
        st["J"][comp] = jv[None, :]
    p = p.copy(wp2=wp2, nu=nu)
    T = 150
    o2 = oracle.run2d(p, T, st)
    # the 1D problem: PEC adds the far wall node (held zero); periodic wraps
    n1 = n + 1 if walled else n
    pad = lambda a: np.concatenate([a, [0.0]]) if walled else a
    q = _oracle1d(n1, p.dt, p.d, pad(prof), pad(nuv), "pec" if walled else "periodic")
    s1 = oracle.new_state(q)
    s1["E"], s1["H"], s1["J"] = pad(e), pad(h), pad(jv)
    o1 = oracle.run(q, T, s1)
    take = (lambda a: a[:, 0]) if axis == "x" else (lambda a: a[0, :])
    for r in range(m):
        takr = (lambda a: a[:, r]) if axis == "x" else (lambda a: a[r, :])
        assert np.array_equal(takr(o2["E"][comp]), o1["E"][:n])
        assert np.array_equal(hsign * takr(o2["H"][hidx]), o1["H"][:n])
        assert np.array_equal(takr(o2["J"][comp]), o1["J"][:n])
    assert np.max(np.abs(take(o2["J"][comp]))) > 0


def test_probe_dft_convention():
    rng = np.random.default_rng(12)
    p = W.random_2d(rng, "te", 24, 20, n_freqs=5)
    T = 120
    st = oracle.new_state2(p)
    samp = np.zeros((len(p.probes), T))
    for m in range(T):
        st = oracle.run2d(p, 1, st)
        for k, (c, i, j) in enumerate(p.probes):
            samp[k, m] = st["E"][c, i, j]
    X = oracle.run2d(p, T)["X"]
    mm = np.arange(1, T + 1)
    for k in range(len(p.probes)):
        ref = np.array([np.sum(samp[k] * p.dt * np.exp(-2j * np.pi * f * p.dt * mm)) for f in p.freqs])
        assert np.max(np.abs(X[k] - ref)) <= 1e-12 * max(np.max(np.abs(ref)), 1e-300)
    assert np.max(np.abs(X)) > 0


def test_courant_limit_2d():
    p = _vac("tm", 8, 8)
    assert oracle.check2(p) == 0
    q = p.copy(dt=0.75 * p.d / C0)
    assert oracle.check2(q) == -2


def test_openmp_build_gives_the_same_bits():
    """The OpenMP build (cell loops in parallel, used for the largest parity
    case) and the -O3 -march=native build equal the plain build bit for bit."""
    rng = np.random.default_rng(31)
    for mode, px in (("tm", False), ("te", True)):
        p = W.random_2d(rng, mode, 40, 52, periodic_x=px)
        a = oracle.run2d(p, 120)
        for kind in ("omp", "native"):
            b = oracle.run2d(p, 120, kind=kind)
            for k in ("E", "H", "J", "X"):
                assert np.array_equal(a[k], b[k]), (mode, kind, k)
