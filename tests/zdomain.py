"""Frequency-domain (z-transform) solution of the discrete 1D scheme, written
from the paper's unsolved equations (11), (12), (14), the Mur / CPML
recursions and the soft-source order, for pinning the oracle's time stepping.

At z = exp(j w dt) the per-node E amplitudes satisfy one tridiagonal system;
the infinite-time running DFT at a node is dt * E(z) there.  Per-node a, phi1,
phi2 come from scipy's matrix exponential, not from the oracle.
"""
import numpy as np
import scipy.linalg

C0 = 299792458.0
EPS0 = 8.8541878128e-12
MU0 = 1.0 / (EPS0 * C0 * C0)


def phi_expm(x):
    """First row of expm([[-x,1,0],[0,0,1],[0,0,0]]) = [e^-x, phi1(x), phi2(x)]."""
    A = np.array([[-x, 1.0, 0.0], [0.0, 0.0, 1.0], [0.0, 0.0, 0.0]])
    r = scipy.linalg.expm(A)[0]
    return r[0], r[1], r[2]


def phi_table(nu, dt):
    u, inv = np.unique(np.asarray(nu), return_inverse=True)
    vals = np.array([phi_expm(v * dt) for v in u])
    return vals[inv, 0], vals[inv, 1], vals[inv, 2]


def cpml_ab(n, P, dz, dt, m=3.0, smax=0.0):
    """b = exp(-sigma dt/eps0), a = b - 1 on E nodes and H nodes (at k+1/2),
    sigma = smax (depth/P)^m, depth counted in cells from the inner interface."""
    eta0 = np.sqrt(MU0 / EPS0)
    if smax <= 0:
        smax = 0.8 * (m + 1.0) / (eta0 * dz)

    def prof(pos):
        d = np.maximum(np.maximum(P - pos, pos - (n - 1 - P)), 0.0)
        b = np.exp(-smax * (d / P) ** m * dt / EPS0)
        return b, b - 1.0
    bE, aE = prof(np.arange(n, dtype=float))
    bH, aH = prof(np.arange(n, dtype=float) + 0.5)
    return bE, aE, bH, aH


def source_ztransform(p, w, nmax=None):
    """S(w) = sum_{n>=1} s(n dt) exp(-j w n dt), summed until the pulse is gone."""
    if nmax is None:
        nmax = int((p.src_t0 + 14 * p.src_tau) / p.dt) + 2
    t = np.arange(1, nmax + 1) * p.dt
    u = t - p.src_t0
    s = p.src_amp * u * np.exp(-(u * u) / (2 * p.src_tau ** 2))
    return np.exp(-1j * np.outer(w, t)) @ s


def solve(p, freqs=None):
    """Infinite-time DFT at every node, [F, n] complex."""
    freqs = p.freqs if freqs is None else np.asarray(freqs)
    n, dz, dt = p.n, p.dz, p.dt
    ce, ch = dt / (EPS0 * dz), dt / (MU0 * dz)
    S = C0 * dt / dz
    cm = (S - 1) / (S + 1)
    a, p1, p2 = phi_table(p.nu, dt)
    if p.bc == "cpml":
        bE, aE, bH, aH = cpml_ab(n, p.cpml_cells, dz, dt, p.cpml_m, p.cpml_sigma_max)
    w = 2 * np.pi * freqs
    Sw = source_ztransform(p, w)
    out = np.zeros((len(freqs), n), complex)
    for i, (wi, si) in enumerate(zip(w, Sw)):
        z = np.exp(1j * wi * dt)
        sE = np.ones(n, complex)
        sH = np.ones(n, complex)
        if p.bc == "cpml":
            sE = 1 + aE * z / (z - bE)
            sH = 1 + aH * z / (z - bH)
        # eq.(11) in z: J = eps0 wp2 dt (phi1 + phi2 (z-1)) / (z-a) * E
        jfac = EPS0 * p.wp2 * dt * (p1 + p2 * (z - 1)) / (z - a)
        diag = (z - 1) + (dt / (2 * EPS0)) * (z + 1) * jfac
        # eq.(14) in z: H[k] = -ch sH[k] (E[k+1]-E[k])/(z-1); eq.(12): + ce z sE curl H
        g = ce * ch * z / (z - 1)
        lo = np.zeros(n, complex)
        up = np.zeros(n, complex)
        dg = np.zeros(n, complex)
        for k in range(1, n - 1):
            dg[k] = diag[k] + g * sE[k] * (sH[k] + sH[k - 1])
            up[k] = -g * sE[k] * sH[k]
            lo[k] = -g * sE[k] * sH[k - 1]
        rhs = np.zeros(n, complex)
        Dsrc = 1 + (dt / (2 * EPS0)) * EPS0 * p.wp2[p.src_cell] * dt * p2[p.src_cell]
        rhs[p.src_cell] = z * si * Dsrc
        if p.bc == "mur":
            # E0^{n+1} = E1^n + cm (E1^{n+1} - E0^n)
            dg[0], up[0] = z + cm, -(1 + cm * z)
            dg[n - 1], lo[n - 1] = z + cm, -(1 + cm * z)
        else:
            dg[0], dg[n - 1] = 1.0, 1.0
        ab = np.zeros((3, n), complex)
        ab[0, 1:] = up[:-1]
        ab[1, :] = dg
        ab[2, :-1] = lo[1:]
        out[i] = dt * scipy.linalg.solve_banded((1, 1), ab, rhs)
    return out


def drude_slab(freqs, wp2, nu, d):
    """Closed-form R, T of a uniform Drude slab of thickness d in vacuum
    (e^{+j w t} convention): eps = 1 - wp^2/(w (w - j nu))."""
    w = 2 * np.pi * np.asarray(freqs)
    eps = 1 - wp2 / (w * (w - 1j * nu))
    nn = np.sqrt(eps)
    r = (1 - nn) / (1 + nn)
    e2 = np.exp(-2j * w * nn * d / C0)
    R = r * (1 - e2) / (1 - r * r * e2)
    T = (1 - r * r) * np.exp(-1j * w * nn * d / C0) / (1 - r * r * e2)
    return R, T
