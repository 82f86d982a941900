"""CPU model of where FP32 storage rounds the 1D plasma step (test infrastructure).

A plain numpy re-statement of one time step (eq.(14) for H, eqs.(11)+(12)
solved for E with J carried as P = J - b2 E, the eq.(15) soft source, first-
order Mur ends, the probe samples) with the precision of every stage
selectable, so that the reflection/transmission error of an FP32 storage
scheme can be predicted on the CPU and compared with what the GPU measures:

* ``arith32``   every field operation in FP32 (the fields rounded after every
                  operation), J and its update in FP64;
* ``round_every=K``  FP64 arithmetic, E and H rounded to FP32 every K steps
                  (K = 1: after every step; K = the run length: never inside
                  the run).

The coefficients come from the oracle's own build (``oracle.coeffs``), so the
model adds only the rounding schedule.  Used by ``test_fp32_model.py``; run
as a script it prints the error table for the 1000-cell slab (the 2^24-cell
grid takes its light cone, ~40k cells x 20000 steps, a few minutes):

    python tests/fp32_rounding_model.py [c2]
"""
from __future__ import annotations

import os
import sys

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

import oracle  # noqa: E402
from paper_1709_00821_amd import workloads as W  # noqa: E402

F32 = np.float32


def _fma32(a, b, c):
    """a*b + c rounded once to FP32 (the FP64 product of two FP32 numbers is exact)."""
    return (np.asarray(a, np.float64) * np.asarray(b, np.float64) + np.asarray(c, np.float64)).astype(F32)


def spectra(p, steps, arith32=False, round_every=0, lo=0, hi=None, mur=True):
    """Probe spectra of p over nodes [lo, hi) (outside: zero for the whole run,
    as on a light-cone-trimmed grid, then mur=False)."""
    hi = p.n if hi is None else hi
    n = hi - lo
    cf = oracle.coeffs(p.wp2[lo:hi], p.nu[lo:hi], p.dt, p.dz, p.scheme)
    const = oracle.constants()
    ch = p.dt / (const["mu0"] * p.dz)
    CJ, CH, a, b1, b2 = cf["CJ"], cf["CH"], cf["a"], cf["b1"], cf["b2"]
    eP = cf["CA"] - CJ * b2          # E^{n+1} = eP E^n - CJ P^{n-1} - CH curl
    eP1 = (cf["CA"] - 1.0) - CJ * b2  # the same, less one (FP32 delta form)
    pc = a * b2 + b1                  # P^n = a P^{n-1} + pc E^n
    S = const["c0"] * p.dt / p.dz
    cm = (S - 1.0) / (S + 1.0)
    src, probes = p.src_cell - lo, np.asarray(p.probes) - lo
    E = np.zeros(n, F32 if arith32 else np.float64)
    H = np.zeros(n - 1, E.dtype)
    P = np.zeros(n)
    samp = np.zeros((len(probes), steps))
    for m in range(1, steps + 1):
        e0, e1, eR, eR1 = E[0], E[1], E[-1], E[-2]
        Pn = pc * E.astype(np.float64) + a * P
        if arith32:
            H = _fma32(F32(-ch), (E[1:] - E[:-1]).astype(F32), H)
            curl = (H[1:] - H[:-1]).astype(F32)
            t = _fma32(eP1[1:-1].astype(F32), E[1:-1], E[1:-1])
            t = _fma32((-CJ[1:-1]).astype(F32), P[1:-1].astype(F32), t)
            E[1:-1] = _fma32((-CH[1:-1]).astype(F32), curl, t)
        else:
            H = H - ch * (E[1:] - E[:-1])
            E[1:-1] = eP[1:-1] * E[1:-1] - CJ[1:-1] * P[1:-1] - CH[1:-1] * (H[1:] - H[:-1])
        P = Pn
        s = oracle.source(m * p.dt, p.src_tau, p.src_t0, p.src_amp)
        E[src] = E.dtype.type(float(E[src]) + s)
        if mur:
            if arith32:
                E[0] = F32(e1 + F32(cm) * F32(E[1] - e0))
                E[-1] = F32(eR1 + F32(cm) * F32(E[-2] - eR))
            else:
                E[0] = e1 + cm * (E[1] - e0)
                E[-1] = eR1 + cm * (E[-2] - eR)
        samp[:, m - 1] = E[probes]    # sampled from the registers, before a store rounds them
        if round_every and m % round_every == 0:
            E = E.astype(F32).astype(np.float64)
            H = H.astype(F32).astype(np.float64)
    mm = np.arange(1, steps + 1)
    X = np.zeros((len(probes), len(p.freqs)), complex)
    for i, f in enumerate(p.freqs):
        cyc = f * p.dt * mm
        cyc = cyc - np.rint(cyc)
        X[:, i] = samp @ (p.dt * np.exp(-2j * np.pi * cyc))
    return X


def rt_error(p, steps, ref, **kw):
    """max_f | |R| - |R_ref| |, max_f | |T| - |T_ref| | of the two-run R, T."""
    s = spectra(p, steps, **kw)
    v = spectra(p.vacuum(), steps, **kw)
    R, T = (s[0] - v[0]) / v[0], s[1] / v[1]
    Rr, Tr = ref
    return float(np.max(np.abs(np.abs(R) - np.abs(Rr)))), float(np.max(np.abs(np.abs(T) - np.abs(Tr))))


def c1_table(round_every=(1, 16, 32, 60, 64, 128, 4096)):
    p = W.slab_c1()
    Ro, To, _, _ = oracle.reflect_transmit(p, p.steps)
    rows = [("FP32 arithmetic", rt_error(p, p.steps, (Ro, To), arith32=True))]
    for K in round_every:
        rows.append((f"FP64 arithmetic, rounded every {K} steps",
                     rt_error(p, p.steps, (Ro, To), round_every=K)))
    return rows


def c2_table(round_every=(1, 60)):
    import json
    p = W.large_c2()
    lo, hi = W.light_cone(p, p.steps)
    g = json.load(open(os.path.join(ROOT, "tests", "golden", "c2_oracle_spectra.json")))
    s = np.array(g["plasma"]["re"]) + 1j * np.array(g["plasma"]["im"])
    v = np.array(g["vacuum"]["re"]) + 1j * np.array(g["vacuum"]["im"])
    ref = ((s[0] - v[0]) / v[0], s[1] / v[1])
    rows = [("FP32 arithmetic", rt_error(p, p.steps, ref, arith32=True, lo=lo, hi=hi, mur=False))]
    for K in round_every:
        rows.append((f"FP64 arithmetic, rounded every {K} steps",
                     rt_error(p, p.steps, ref, round_every=K, lo=lo, hi=hi, mur=False)))
    return rows


if __name__ == "__main__":
    table = c2_table() if sys.argv[1:] == ["c2"] else c1_table()
    for name, (dR, dT) in table:
        print(f"{name:45s} max|dR| {dR:.2e}  max|dT| {dT:.2e}", flush=True)
