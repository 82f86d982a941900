#!/usr/bin/env python3
"""Benchmark of the 1D RKETD-FDTD plasma hot path on one MI355X.

One bench "step" is one full run of the plain workload: 2^24 cells x 20000
time steps (H-curl, E-curl minus J, ETD2 J advance, source, CPML ends, probe
DFT), seeded synthetic plasma (sinusoidal wp^2 profile over the middle half,
per-cell nu).  Inputs are resident in HBM before timing; each run() replays a
captured HIP graph.  Prints one JSON line.

  python bench.py [--steps K] [--warmup W] [--precision f32|f64] [--no-cpu]
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = ("Mcell-updates/s & %HBM roofline (plain vs batched vs adjoint) at stated "
          "|R|,|T| error")
HBM_PEAK_GBS = 8000.0


def log(msg):
    print(msg, file=sys.stderr, flush=True)


def algorithmic_bytes_per_node(precision: str, plasma: bool) -> int:
    """What one pass must move per node: read and write E, H once (and J, held
    in FP64 at either precision, on plasma nodes), plus the two FP64 material
    words (wp2, nu) on plasma nodes."""
    es = 8 if precision == "f64" else 4
    return (2 * 2 * es + 2 * 8 + 16) if plasma else 2 * 2 * es


def run_precision(p, precision, T, K, W, tune):
    import torch
    from paper_1709_00821_amd.plasma import FdtdPlasma
    h = FdtdPlasma(p, precision=precision, exec="tiled", **tune)
    log(f"bench: {precision} tile_cells={h.desc.tile_cells} steps_per_pass={h.desc.steps_per_pass}"
        f" workspace {h.workspace_bytes / 2**30:.2f} GiB")
    for i in range(W):
        h.run(T)
        h.synchronize()
        log(f"bench: warmup {i + 1}/{W} done")
    ev0 = torch.cuda.Event(enable_timing=True)
    ev1 = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    ev0.record(h.stream)
    for i in range(K):
        h.run(T)
    ev1.record(h.stream)
    torch.cuda.synchronize()
    ms = ev0.elapsed_time(ev1)
    X = h.spectra()[0]
    log(f"bench: {precision} timed {K} runs: {ms / K:.2f} ms/run")
    # per-launch durations on the handle's stream (HIP events inside the library)
    prof_steps = min(T, 4000)
    h.run(0)
    prof = h.profile(prof_steps)
    h.close()
    return ms / K, X, prof


def roofline(prof, precision):
    """Dominant kernel: achieved = algorithmic bytes per launch (bytes per node
    x nodes the launch advances, as the library reports) / mean launch time."""
    name, (ms_tot, calls, units) = max(prof.items(), key=lambda kv: kv[1][0])
    per = algorithmic_bytes_per_node(precision, name in ("tiled_plasma", "tiled_cpml", "tiled_role", "resident",
                                                         "step_h_e"))
    bytes_per_launch = per * units / calls
    avg_s = ms_tot / calls / 1e3
    achieved = bytes_per_launch / avg_s / 1e9
    return {"kernel": name, "bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS,
            "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": None,
            "bytes_per_launch": int(bytes_per_launch), "avg_launch_us": round(avg_s * 1e6, 2),
            "launches": calls}


# Algorithmic floating-point operations per node-update (eqs.(14), (12)+(11)
# solved, (11)): H: subtract + FMA = 3; vacuum E: 3; plasma E: subtract,
# multiply, two FMAs = 6; J: multiply + two FMAs = 5.  FP64 and FP32 storage
# both compute them in FP64 registers; the all-FP32 ablation in FP32.
FLOPS_VAC = 6
FLOPS_PLASMA = 14
# MI355X vector peaks from the unit counts: 256 CUs x 2.4 GHz x 2 flops (FMA)
# x 128 FP32 lanes a CU-cycle = 157.3 TFLOP/s (reached by the two-operand FP32
# forms without packed math: a wave64 v_fmac_f32 / v_sub_f32 issues every
# ~2.4 cycles on the box), x 64 FP64 lanes = 78.6 TFLOP/s.
FP32_PEAK_TFLOPS = 157.3
FP64_PEAK_TFLOPS = 78.6


def alu_peak(kernel, precision):
    """Peak of the arithmetic the kernel runs: FP64 (FP64 storage, and FP32
    storage, whose updates run in FP64 registers), or FP32 (the all-FP32
    ablation)."""
    return FP32_PEAK_TFLOPS if precision == "f32d" else FP64_PEAK_TFLOPS


def alu_roofline(prof, kernel, steps_per_launch, precision):
    """The tiled kernels do K steps per launch on data held in VGPRs; their
    ceiling is VALU issue: achieved = algorithmic flops of the node-updates a
    launch delivers / mean launch time, against the vector peak of the
    precision they compute in."""
    ms_tot, calls, units = prof[kernel]
    per = FLOPS_PLASMA if kernel in ("tiled_plasma", "tiled_cpml", "tiled_role") else FLOPS_VAC
    flops = per * units / calls * steps_per_launch
    avg_s = ms_tot / calls / 1e3
    ach = flops / avg_s / 1e12
    peak = round(alu_peak(kernel, precision), 1)
    return {"kernel": kernel, "bound": "alu", "achieved": round(ach, 2), "peak": peak,
            "unit": "TFLOP/s", "frac": round(ach / peak, 4), "traffic": None,
            "peak_basis": ("FP32 vector 157.3 TFLOP/s (the all-FP32 ablation)" if precision == "f32d" else
                           "FP64 vector 78.6 TFLOP/s (the updates run in FP64 registers)"),
            "flops_per_launch": int(flops), "avg_launch_us": round(avg_s * 1e6, 2), "launches": calls}


def batched_leg(precision="f32", n_slabs=4096, T=8000, reps=2):
    """4096 independent slabs of uneven length in one handle."""
    import torch
    from paper_1709_00821_amd import workloads as W
    from paper_1709_00821_amd import tune as TU
    from paper_1709_00821_amd.plasma import FdtdPlasma
    slabs = W.batch_c4(n_slabs=n_slabs, steps=T)
    cells = sum(q.n for q in slabs)
    tune = TU.pick(precision, cells, batched=True)
    h = FdtdPlasma(slabs, precision=precision, exec="auto", **tune)
    h.run(T)
    h.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(h.stream)
    for _ in range(reps):
        h.run(T)
    e1.record(h.stream)
    e1.synchronize()
    ms = e0.elapsed_time(e1) / reps
    X = h.spectra()
    h.close()
    log(f"bench: batched {n_slabs} slabs ({cells} nodes) x {T} steps: {ms:.2f} ms")
    acc = batched_accuracy(slabs, X, precision, T, tune) if n_slabs == 4096 and T == 8000 else None
    value = cells * T / (ms / 1e3) / 1e6
    plasma = sum(int(np.count_nonzero(q.wp2)) for q in slabs)
    ss = (plasma * algorithmic_bytes_per_node(precision, True)
          + (cells - plasma) * algorithmic_bytes_per_node(precision, False)) / cells
    return {"value": round(value, 1), "unit": "Mcell-updates/s",
            "ms": round(ms, 3), "slabs": n_slabs, "nodes": cells, "time_steps": T,
            "precision": precision, "exec": "auto (tiled over the concatenated slabs)",
            "tile_cells": tune["tile_cells"], "steps_per_pass": tune["steps_per_pass"],
            "vacuum_tile_cells": tune.get("vacuum_tile_cells", 0),
            "single_step_equivalent": {"gbs": round(value * 1e6 * ss / 1e9, 1),
                                       "frac_of_hbm_peak": round(value * 1e6 * ss / 1e9 / HBM_PEAK_GBS, 2),
                                       "bytes_per_cell_update": round(ss, 2)},
            "accuracy": acc}


def batched_accuracy(slabs, X, precision, T, tune):
    """Two-run |R|, |T| and spectra errors of the sampled slabs against the
    stored FP64 oracle spectra (tests/golden/c4_oracle_spectra.json): the
    plasma runs are the timed batch's, the plasma-free runs a batch of the
    sampled slabs at the same precision and launch shape."""
    from paper_1709_00821_amd.plasma import FdtdPlasma
    sys.path.insert(0, os.path.join(ROOT, "tests", "golden"))
    import make_oracle_spectra as G
    try:
        d, Xo, Xvo = G.load_c4()
    except (OSError, ValueError, KeyError):
        return None
    pick = d["slabs"]
    if d["steps"] != T or pick != G.c4_sample(slabs):
        return None
    with FdtdPlasma([slabs[b].vacuum() for b in pick], precision=precision, exec="auto", **tune) as hv:
        hv.run(T)
        Xv = hv.spectra()
    spec, dR, dT = [], [], []
    for i, b in enumerate(pick):
        spec.append(float(np.max(np.abs(X[b] - Xo[i])) / np.max(np.abs(Xo[i]))))
        R, Ro = (X[b][0] - Xv[i][0]) / Xv[i][0], (Xo[i][0] - Xvo[i][0]) / Xvo[i][0]
        dR.append(float(np.max(np.abs(np.abs(R) - np.abs(Ro)))))
        # transmission where the pulse reaches the far probe within the run
        if np.all(np.abs(Xvo[i][1]) > 0):
            Tt, To = X[b][1] / Xv[i][1], Xo[i][1] / Xvo[i][1]
            dT.append(float(np.max(np.abs(np.abs(Tt) - np.abs(To)))))
    return {"slabs": pick, "spectra_rel_err_max": max(spec), "max_abs_R_err": max(dR),
            "max_abs_T_err": max(dT) if dT else None, "transmission_slabs": len(dT),
            "oracle": "stored FP64 oracle spectra (tests/golden/c4_oracle_spectra.json)"}


def adjoint_leg(precision="f32"):
    """Gradient of sum_f |R|^2 w.r.t. wp2 per node: 8000 nodes, 20000 steps,
    forward with sqrt(T) checkpoints + reverse sweep with recompute."""
    import torch
    from paper_1709_00821_amd import workloads as W
    from paper_1709_00821_amd import tune as TU
    from paper_1709_00821_amd.plasma import FdtdPlasma
    p = W.adjoint_c5()
    T = p.steps
    tune = TU.pick(precision, p.n)
    with FdtdPlasma(p.vacuum(), precision="f64", exec="tiled") as hv:
        hv.run(T)
        xv = hv.spectra()[0, 0].reshape(1, -1)
    h = FdtdPlasma(p, precision=precision, exec="tiled", checkpoint=T, **tune)
    h.run(T)
    h.grad_r2(T, xv)                 # first call captures the reverse sweep's graph
    h.synchronize()
    e0, e1, e2 = (torch.cuda.Event(enable_timing=True) for _ in range(3))
    e0.record(h.stream)
    h.run(T)
    e1.record(h.stream)
    L, g = h.grad_r2(T, xv)          # reuses the checkpointed forward run
    e2.record(h.stream)
    e2.synchronize()
    fwd_ms, adj_ms = e0.elapsed_time(e1), e1.elapsed_time(e2)
    h.close()
    tot = fwd_ms + adj_ms
    log(f"bench: adjoint {p.n} nodes x {T} steps: forward {fwd_ms:.2f} ms, reverse {adj_ms:.2f} ms")
    return {"value": round(p.n * T / (tot / 1e3) / 1e6, 1), "unit": "forward-equivalent Mcell/s",
            "forward_ms": round(fwd_ms, 3), "reverse_ms": round(adj_ms, 3),
            "gradient_over_forward": round(tot / fwd_ms, 3),
            "vs_same_grid_forward": round(fwd_ms / tot, 4),
            "nodes": p.n, "time_steps": T, "precision": precision,
            "checkpoint_interval": int(math.ceil(math.sqrt(T))), "forward_tile_cells": tune["tile_cells"],
            "forward_steps_per_pass": tune["steps_per_pass"]}


# GPU times (ms) of the paper's timing table (Table 2): 1000 steps of the
# plasma-slab setup at each cell count, on the GeForce GTX 1080 it names, and
# the serial CPU program's times on its Core i7-6700.  Context only.
PAPER_TABLE2_MS = {1024: (33, 279), 5120: (33, 379), 10240: (33, 504), 20480: (34, 753), 30720: (46, 982),
                   40960: (53, 1231), 51200: (61, 1467), 61440: (64, 1701)}


def table2_leg(precision="f64", reps=5):
    """The paper's timing experiment on this GPU: 1000 steps of its slab setup
    at each cell count of its Table 2 (FP64: the paper states no precision),
    launch shape from the tuner; beside it the paper's GTX 1080 times."""
    import torch
    from paper_1709_00821_amd import workloads as W
    from paper_1709_00821_amd import tune as TU
    from paper_1709_00821_amd.plasma import FdtdPlasma
    T = 1000
    rows = []
    for n, (gpu_ms, ser_ms) in PAPER_TABLE2_MS.items():
        p = W.paper_preset(steps=T, n=n)
        tune = TU.pick(precision, n)
        with FdtdPlasma(p, precision=precision, exec="auto", **tune) as h:
            h.run(T)
            h.synchronize()
            times = []
            for _ in range(reps):
                e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
                e0.record(h.stream)
                h.run(T)
                e1.record(h.stream)
                e1.synchronize()
                times.append(e0.elapsed_time(e1))
        ms = sorted(times)[len(times) // 2]
        rows.append({"cells": n, "ms": round(ms, 4), "mcells": round(n * T / ms / 1e3, 1),
                     "paper_gtx1080_ms": gpu_ms, "paper_gtx1080_mcells": round(n * T / gpu_ms / 1e3, 1),
                     "vs_paper_gpu": round(gpu_ms / ms, 1)})
        log(f"bench: table-2 size {n}: {ms:.3f} ms (paper GPU {gpu_ms} ms)")
    return {"context": "paper Table 2 setup, 1000 steps; paper numbers are its own hardware's, not targets",
            "precision": precision, "rows": rows}


def table2_serial(cpu, leg):
    """The serial oracle's time for one Table 2 size (measured in the CPU
    baseline leg) beside this GPU's, as the paper sets its serial column beside
    its GPU's."""
    s = cpu.get("paper_table2_serial")
    if not s:
        return None
    gpu = next((r["ms"] for r in leg["rows"] if r["cells"] == s["cells"]), None)
    if gpu is None:
        return None
    return {"cells": s["cells"], "ms": s["ms"], "cores": 1, "speedup_gpu_vs_serial": round(s["ms"] / gpu, 1),
            "paper_speedup_gpu_vs_serial": round(PAPER_TABLE2_MS[s["cells"]][1] / PAPER_TABLE2_MS[s["cells"]][0], 2)}


def c1_leg(reps=5):
    """The 1000-cell slab (latency bound: the state would fit one CU; the
    register tiles beat the one-workgroup resident executor here)."""
    import torch
    from paper_1709_00821_amd import workloads as W
    from paper_1709_00821_amd import tune as TU
    from paper_1709_00821_amd.plasma import FdtdPlasma
    p = W.slab_c1()
    T = p.steps
    tune = TU.pick("f64", p.n)
    h = FdtdPlasma(p, precision="f64", exec="auto", **tune)
    h.run(T)
    h.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(h.stream)
    for _ in range(reps):
        h.run(T)
    e1.record(h.stream)
    e1.synchronize()
    ms = e0.elapsed_time(e1) / reps
    h.close()
    return {"value": round(p.n * T / (ms / 1e3) / 1e6, 1), "unit": "Mcell-updates/s",
            "ms": round(ms, 3), "nodes": p.n, "time_steps": T, "precision": "f64",
            "exec": "auto (register tiles)", "tile_cells": tune["tile_cells"],
            "steps_per_pass": tune["steps_per_pass"]}


def c3_leg(precision="f32", n=384, T=2000, prof_steps=64, compare_f64=True, exec="auto"):
    """3D Yee-RKETD: n^3 cells, plasma sphere in a TF/SF plane wave, CPML,
    FP64 DFT of the tangential E and H on a box in the scattered-field region.
    Whole-job throughput of run(T) (graph replay), plus per-kernel event
    timings and the algorithmic HBM rate of the two field kernels."""
    import torch
    from paper_1709_00821_amd import workloads as W
    from paper_1709_00821_amd.plasma3d import FdtdPlasma3D
    log(f"bench: 3D leg, {n}^3 cells x {T} steps ({precision})")
    p = W.sphere_c3(n, steps=T)
    N = p.ncells
    es = 8 if precision == "f64" else 4
    # plasma support as the library keeps it: per row, first..last node with wp2 > 0
    m = (p.wp2 > 0).any(axis=0)
    has = m.any(axis=2)
    k0 = np.argmax(m, axis=2)
    k1 = p.nz - np.argmax(m[:, :, ::-1], axis=2)
    S = int(np.sum(np.where(has, k1 - k0, 0)))
    del m
    P = p.cpml
    slab = 2 * P * (p.ny * p.nz + p.nx * p.nz + p.nx * p.ny)
    npts, F = len(p.points), len(p.freqs)
    # algorithmic bytes per launch: E, H read and the updated component group
    # written; J read+written and wp2, nu read on the support; two CPML
    # auxiliaries read+written per slab cell and axis
    bytes_h = 9 * es * N + 4 * es * slab
    bytes_e = 9 * es * N + S * (6 * es + 3 * 16) + 4 * es * slab
    # the one-pass kernel: E and H read once and written once, both groups of
    # CPML auxiliaries, the plasma terms of the E pass
    bytes_f = 12 * es * N + S * (6 * es + 3 * 16) + 8 * es * slab
    with FdtdPlasma3D(p, precision=precision, exec=exec) as h:
        h.profile(True)
        h.step(prof_steps)
        prof = h.profile_read()
        h.profile(False)
        h.run(T)                                   # capture + first replay
        h.synchronize()
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        with torch.cuda.stream(h.stream):
            e0.record(h.stream)
            h.run(T)
            e1.record(h.stream)
        e1.synchronize()
        ms = e0.elapsed_time(e1)
        X = h.spectra()
    kern = {}
    for k, (kms, calls, cells) in prof.items():
        kern[k] = {"us_per_launch": round(kms / calls * 1e3, 2), "launches": calls}
    out = {"value": round(N * T / (ms / 1e3) / 1e6, 1), "unit": "Mcell-updates/s",
           "ms": round(ms, 2), "cells": N, "time_steps": T, "precision": precision, "exec": exec,
           "plasma_support_cells": S, "cpml_slab_cells": slab, "sample_points": npts,
           "freqs": F, "spectra_finite": bool(np.all(np.isfinite(X))), "kernels": kern}
    if precision != "f64" and compare_f64:
        # the same run in FP64 on the GPU: the FP64 path is held to the oracle
        # within 1e-12 on the same problem scaled to 96^3 (tests/test_gpu3d.py)
        with FdtdPlasma3D(p, precision="f64", exec=exec) as h64:
            h64.run(T)
            X64 = h64.spectra()
        err = np.abs(X - X64)
        out["accuracy"] = {"spectra_rel_err_vs_fp64": float(np.max(err) / np.max(np.abs(X64))),
                           "reference": "the FP64 GPU run of the same problem (within 1e-12 of the "
                                        "oracle at 96^3)"}
        log(f"bench: 3D fp32 vs fp64 spectra {out['accuracy']['spectra_rel_err_vs_fp64']:.2e}")
    for k, b in (("k_e3d", bytes_e), ("k_h3d", bytes_h), ("k_fused3d", bytes_f)):
        if k in prof:
            kms, calls, _ = prof[k]
            gbs = b / (kms / calls / 1e3) / 1e9
            out["kernels"][k].update({"algorithmic_bytes": int(b), "achieved_gbs": round(gbs, 1),
                                      "frac_hbm": round(gbs / HBM_PEAK_GBS, 3)})
    return out


def c2d_leg(n=4096, T=2000, reps=3):
    """2D Yee-RKETD, TM and TE: n^2 cells, plasma cylinder (radius n/8 with a
    Gaussian edge), PEC walls, soft point source, 8 probes at 64 frequencies;
    FP32 storage (FP64 registers), an H pass and an E/J pass per step.
    Whole-job throughput of run(T) (graph replay), the split passes' effective
    HBM rate at their algorithmic bytes, and the FP32 spectra against the FP64
    GPU run of the same problem (the FP64 path is held to the 2D oracle within
    1e-12 in tests/test_gpu2d.py)."""
    import torch
    from paper_1709_00821_amd import workloads as W
    from paper_1709_00821_amd.plasma2d import FdtdPlasma2D
    out = {}
    for mode in ("tm", "te"):
        p = W.cylinder_2d(mode, n=n, steps=T)
        N = p.ncells
        S = int(np.count_nonzero(p.wp2.any(axis=0)))     # cells of the plasma support (at least)
        res = {}
        for prec in ("f32", "f64"):
            with FdtdPlasma2D(p, precision=prec) as h:
                h.run(T)
                h.synchronize()
                ts = []
                for _ in range(reps):
                    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
                    e0.record(h.stream)
                    h.run(T)
                    e1.record(h.stream)
                    e1.synchronize()
                    ts.append(e0.elapsed_time(e1))
                res[prec] = (sorted(ts)[len(ts) // 2], h.spectra())
        ms, X = res["f32"]
        es = 4
        nf = 3                                 # field arrays: TM Ez, Hx, Hy; TE Ex, Ey, Hz
        ncomp = 1 if mode == "tm" else 2
        # algorithmic bytes per step: every field read and written once; on the
        # plasma support the currents (FP64) read and written and wp2, nu read
        alg = N * nf * 2 * es + S * ncomp * (16 + 16)
        gbs = alg * T / (ms / 1e3) / 1e9
        err = float(np.max(np.abs(X - res["f64"][1])) / np.max(np.abs(res["f64"][1])))
        out[mode] = {"value": round(N * T / (ms / 1e3) / 1e6, 1), "unit": "Mcell-updates/s", "ms": round(ms, 2),
                     "cells": N, "time_steps": T, "precision": "f32", "fp64_ms": round(res["f64"][0], 2),
                     "plasma_support_cells": S,
                     "algorithmic_bytes_per_step": int(alg), "effective_gbs": round(gbs, 1),
                     "frac_hbm": round(gbs / HBM_PEAK_GBS, 3),
                     "spectra_rel_err_vs_fp64": err}
        log(f"bench: 2D {mode} {n}^2 x {T}: {ms:.2f} ms ({out[mode]['value']} Mcell/s), fp32 vs fp64 {err:.2e}")
    return out


# the sources the 1D tiled kernels are compiled from (what the counter
# summary describes); other files of the library do not change them
TILED_SOURCES = ("physics.h", "internal.h", "tile1d.h", "blocked1d.hip")


def kernel_source_hash() -> str:
    import hashlib
    d = os.path.join(ROOT, "paper_1709_00821_amd", "csrc")
    h = hashlib.sha256()
    for f in TILED_SOURCES:
        with open(os.path.join(d, f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def counter_traffic(kernel, precision, tune, cells):
    """HBM bytes per launch from the committed rocprofv3 FETCH_SIZE/WRITE_SIZE
    summary, if it was taken on these kernel sources and this launch shape."""
    path = os.path.join(ROOT, "profiles", "tiled_c2_f32_hbm_traffic.md")
    try:
        txt = open(path).read()
        blk = json.loads(txt.split("```json", 1)[1].split("```", 1)[0])
    except (OSError, IndexError, ValueError):
        return None
    if (blk.get("source_sha256") != kernel_source_hash() or blk.get("precision") != precision
            or blk.get("tile_cells") != tune["tile_cells"]
            or blk.get("steps_per_pass") != tune["steps_per_pass"] or blk.get("cells") != cells
            or blk.get("vacuum_tile_cells", 0) != tune.get("vacuum_tile_cells", 0)):
        return None
    k = blk.get("kernels", {}).get(kernel)
    return None if k is None else int(k["traffic_bytes_per_launch"])


def cpu_info():
    """The host CPU as the box reports it."""
    model = None
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    return {"model": model, "nproc": os.cpu_count(), "cpus_available": len(os.sched_getaffinity(0)),
            "omp_num_threads": os.environ.get("OMP_NUM_THREADS")}


class pinned:
    """Run the calling thread on one CPU (the serial oracle's timing rule),
    restoring its affinity afterwards."""

    def __init__(self, cpu):
        self.cpu = cpu

    def __enter__(self):
        self.old = os.sched_getaffinity(0)
        os.sched_setaffinity(0, {self.cpu})

    def __exit__(self, *exc):
        os.sched_setaffinity(0, self.old)


def median_time(fn, reps=3, warmup=1):
    for _ in range(warmup):
        fn()
    ts = []
    for _ in range(reps):
        t = time.perf_counter()
        fn()
        ts.append(time.perf_counter() - t)
    return sorted(ts)[len(ts) // 2]


def cpu_baseline(p, steps, table2_cells=10240, contexts=True):
    """The FP64 oracle on this host, built -O3 -march=native -ffp-contract=off,
    serial on one pinned CPU, median of 3 runs after one warm-up: a bounded
    sample of the headline workload (the full grid for `steps` steps, the
    coefficient build timed separately and excluded).  Context beside it: the
    same sample on the OpenMP build over every available CPU, and samples of
    the other configurations (the 1000-cell slab in full, the 3D sphere
    problem scaled to 160^3 for 4 steps, 64 slabs of the batch for 1000 steps,
    the 8000-cell adjoint once, one size of the paper's Table 2 setup)."""
    import oracle
    from paper_1709_00821_amd import workloads as W
    info = cpu_info()
    cpu0 = min(os.sched_getaffinity(0))
    log(f"bench: cpu baseline on {info['model']} ({info['cpus_available']} CPUs): oracle, full {p.n}-cell grid, "
        f"{steps} steps, serial on CPU {cpu0}")
    oracle.timing_lib("native")
    oracle.timing_lib("omp")
    # a run of 1 step holds the setup (coefficient build, first touch of the
    # state): the sample is the difference to a run of steps + 1
    with pinned(cpu0):
        setup = median_time(lambda: oracle.run(p, 1, kind="native"), reps=1, warmup=0)
        tot = median_time(lambda: oracle.run(p, steps + 1, kind="native"))
    run_s = max(tot - setup, 1e-9)
    out = {"value": round(p.n * steps / run_s / 1e6, 2), "unit": "Mcell-updates/s", "cores": 1,
           "kind": "oracle",
           "sample": f"full {p.n}-cell grid, {steps} of {p.steps} steps, serial FP64 oracle "
                     f"(-O3 -march=native -ffp-contract=off) pinned to CPU {cpu0}, median of 3 after "
                     f"1 warm-up, {run_s:.2f} s a run (a run of steps + 1 less a run of 1 step: "
                     f"setup and first touch, {setup:.2f} s, excluded)",
           "host": info}
    nthr = len(os.sched_getaffinity(0))
    tot_omp = median_time(lambda: oracle.run(p, steps + 1, kind="omp"))
    setup_omp = median_time(lambda: oracle.run(p, 1, kind="omp"), reps=1, warmup=0)
    omp_s = max(tot_omp - setup_omp, 1e-9)
    out["openmp"] = {"value": round(p.n * steps / omp_s / 1e6, 2), "unit": "Mcell-updates/s",
                     "threads": int(info["omp_num_threads"] or nthr),
                     "speedup_vs_serial": round(run_s / omp_s, 2),
                     "sample": "the same sample on the OpenMP build (node loops in parallel)"}
    log(f"bench: cpu baseline serial {out['value']} Mcell/s, OpenMP {out['openmp']['value']} Mcell/s")
    if not contexts:
        return out
    ctx = {}
    with pinned(cpu0):
        q = W.slab_c1()
        t = median_time(lambda: oracle.run(q, q.steps, kind="native"))
        ctx["c1"] = {"ms": round(t * 1e3, 2), "mcells": round(q.n * q.steps / t / 1e6, 2),
                     "sample": f"the whole 1000-cell slab run, {q.steps} steps"}
        q3 = W.sphere_c3(160, steps=4)
        s3 = median_time(lambda: oracle.run3d(q3, 1, kind="native"), reps=1, warmup=0)
        t3 = median_time(lambda: oracle.run3d(q3, 5, kind="native"), reps=1, warmup=0)
        ctx["c3"] = {"mcells": round(q3.ncells * 4 / max(t3 - s3, 1e-9) / 1e6, 2),
                     "sample": "the 3D sphere problem scaled to 160^3, 4 steps, setup excluded, one run"}
        del q3
        slabs = W.batch_c4(n_slabs=4096)
        rng = np.random.default_rng(1713)
        sub = [slabs[i] for i in sorted(rng.choice(len(slabs), 64, replace=False))]
        del slabs
        nodes = sum(x.n for x in sub)
        t4 = median_time(lambda: [oracle.run(x, 1000, kind="native") for x in sub], reps=1, warmup=0)
        ctx["c4"] = {"mcells": round(nodes * 1000 / t4 / 1e6, 2),
                     "sample": f"64 seeded slabs of the batch ({nodes} nodes), 1000 steps each, one run"}
        q5 = W.adjoint_c5()
        xv = oracle.run(q5.vacuum(), q5.steps, kind="native")["X"][0]
        t5 = median_time(lambda: oracle.adjoint_r2(q5, q5.steps, xv, kind="native"), reps=1, warmup=0)
        ctx["c5"] = {"s": round(t5, 2), "forward_equivalent_mcells": round(q5.n * q5.steps / t5 / 1e6, 2),
                     "sample": "the 8000-cell, 20000-step loss and gradient (full-trajectory adjoint), once"}
        q2 = W.paper_preset(steps=1000, n=table2_cells)
        t2 = median_time(lambda: oracle.run(q2, 1000, kind="native"))
        ctx["paper_table2"] = {"cells": table2_cells, "steps": 1000, "ms": round(t2 * 1e3, 1)}
    out["contexts"] = ctx
    out["paper_table2_serial"] = ctx["paper_table2"]
    return out


def vacuum_spectra(p, precision, T, tune):
    """Probe spectra of the plasma-free run of p on the GPU (the reference run
    of the two-run reflection and transmission)."""
    from paper_1709_00821_amd.plasma import FdtdPlasma
    with FdtdPlasma(p.vacuum(), precision=precision, exec="tiled", **tune) as h:
        h.run(T)
        return h.spectra()[0]


def stored_oracle_spectra(p, T):
    """The FP64 oracle's spectra of this workload (plasma run, plasma-free
    run), as written by tests/golden/make_oracle_spectra.py; None when the
    stored run is another size."""
    sys.path.insert(0, os.path.join(ROOT, "tests", "golden"))
    import make_oracle_spectra as G
    try:
        d, Xo, Xvo = G.load()
    except (OSError, ValueError, KeyError):
        return None
    if d["cells"] != p.n or d["steps"] != T or not np.array_equal(np.array(d["freqs_hz"]), p.freqs):
        return None
    return Xo, Xvo


def c1_precision_errors():
    """|R|, |T| errors of each precision mode on the 1000-cell slab against the
    stored oracle spectra: FP64, FP32 storage (the executor AUTO picks, and the
    register tiles), and the all-FP32 ablation."""
    sys.path.insert(0, os.path.join(ROOT, "tests", "golden"))
    import make_oracle_spectra as G
    from paper_1709_00821_amd import workloads as W
    from paper_1709_00821_amd.plasma import reflect_transmit
    p = W.slab_c1()
    try:
        d, Xo, Xvo = G.load(G.OUT_C1)
    except (OSError, ValueError, KeyError):
        return None
    if d["cells"] != p.n or d["steps"] != p.steps or not np.array_equal(np.array(d["freqs_hz"]), p.freqs):
        return None
    Ro, To = (Xo[0] - Xvo[0]) / Xvo[0], Xo[1] / Xvo[1]
    hi = p.freqs >= 12e9
    out = {"workload": "slab_c1 (1000 cells, 4096 steps, Mur ends)"}
    for prec, ex in (("f64", "auto"), ("f32", "auto"), ("f32_tiled", "tiled"), ("f32d", "auto")):
        R, Tt, s, _ = reflect_transmit(p, p.steps, precision=prec.split("_")[0], exec=ex)
        dR, dT = np.abs(np.abs(R) - np.abs(Ro)), np.abs(np.abs(Tt) - np.abs(To))
        out[prec] = {"spectra_rel_err": float(np.max(np.abs(s - Xo)) / np.max(np.abs(Xo))),
                     "max_abs_R_err": float(dR.max()), "max_abs_T_err": float(dT.max()),
                     "max_abs_R_err_f_ge_12ghz": float(dR[hi].max()),
                     "max_abs_T_err_f_ge_12ghz": float(dT[hi].max())}
    out["f32"]["exec"] = "auto (resident: fields rounded to FP32 once per sample window)"
    out["f32_tiled"]["exec"] = "register tiles (fields rounded to FP32 once per launch)"
    out["f32d"]["mode"] = ("ablation: every field update in FP32 arithmetic, eq.(11) in FP32 with FP32 "
                           "delta-form coefficients")
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--precision", default="f32", choices=["f32", "f64"])
    ap.add_argument("--cells", type=int, default=1 << 24)
    ap.add_argument("--time-steps", type=int, default=20000)
    ap.add_argument("--tile-cells", type=int, default=0)
    ap.add_argument("--steps-per-pass", type=int, default=0)
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-check", action="store_true")
    ap.add_argument("--no-fp64", action="store_true")
    ap.add_argument("--no-ablation", action="store_true",
                    help="skip the FP32 delta-form ablation run (eq.(11) in FP32)")
    ap.add_argument("--no-legs", action="store_true", help="skip the batched, adjoint and C1 legs")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="first run one plain 1 GiB device copy (counter calibration)")
    ap.add_argument("--cpu-steps", type=int, default=16)
    ap.add_argument("--only", choices=["c3", "batched", "adjoint", "c1", "table2", "c2d"],
                    help="run just this leg and print its JSON (profiling runs)")
    ap.add_argument("--c3-steps", type=int, default=2000)
    ap.add_argument("--c3-exec", default="auto", choices=["auto", "split", "fused"])
    ap.add_argument("--c2d-steps", type=int, default=2000)
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only; --gpus {args.gpus} is not supported "
              f"(the method's independent grids would shard by cell ranges with a halo exchange, "
              f"not built here)", file=sys.stderr)
        sys.exit(2)

    import torch
    assert torch.cuda.is_available(), "bench.py needs a GPU"
    if args.copy_calibration:
        # one plain device-to-device blit of known size (the HIP runtime's copy
        # kernel), for scaling the hardware byte counters
        import ctypes
        hip = ctypes.CDLL("libamdhip64.so.7")
        nbytes = 1 << 30
        x = torch.full((nbytes // 4,), 1.0, dtype=torch.float32, device="cuda")
        y = torch.empty_like(x)
        torch.cuda.synchronize()
        rc = hip.hipMemcpy(ctypes.c_void_p(y.data_ptr()), ctypes.c_void_p(x.data_ptr()),
                           ctypes.c_size_t(nbytes), 3)          # hipMemcpyDeviceToDevice
        torch.cuda.synchronize()
        log(f"bench: copy calibration: hipMemcpy of {nbytes} bytes (rc {rc})")
        del x, y
    if args.only:
        leg = {"c3": lambda: c3_leg(T=args.c3_steps, exec=args.c3_exec), "batched": batched_leg, "adjoint": adjoint_leg,
               "c1": c1_leg, "table2": table2_leg, "c2d": lambda: c2d_leg(T=args.c2d_steps)}[args.only]
        print(json.dumps({args.only: leg()}), flush=True)
        return
    from paper_1709_00821_amd import workloads as W
    from paper_1709_00821_amd import tune as TU

    T = args.time_steps
    log(f"bench: building the {args.cells}-cell workload")
    p = W.large_c2(n=args.cells, steps=T)
    results = {}
    for prec in ([args.precision] + ([] if args.no_fp64 else [x for x in ("f64",) if x != args.precision])
                 + ([] if args.no_ablation else ["f32d"])):
        tune = TU.pick(prec, p.n, tile_cells=args.tile_cells, steps_per_pass=args.steps_per_pass)
        ms, X, prof = run_precision(p, prec, T, args.steps, args.warmup, tune)
        results[prec] = (ms, X, prof, tune)

    ms, X, prof, tune = results[args.precision]
    cells = p.n
    value = cells * T / (ms / 1e3) / 1e6
    dom = max(prof.items(), key=lambda kv: kv[1][0])[0]
    rl = alu_roofline(prof, dom, tune["steps_per_pass"], args.precision)
    hv = roofline(prof, args.precision)
    rl["traffic"] = hv["traffic"] = counter_traffic(dom, args.precision, tune, cells)
    # single-step algorithmic bytes per cell-update of this workload (half plasma)
    ss_bytes = 0.5 * algorithmic_bytes_per_node(args.precision, True) + \
        0.5 * algorithmic_bytes_per_node(args.precision, False)
    out = {
        "metric": METRIC, "value": round(value, 1), "unit": "Mcell-updates/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(ms, 3),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": args.precision, "data": "synthetic",
        "config": {"workload": f"1D plain RKETD-FDTD, {cells} cells x {T} steps, CPML 32, "
                               f"seeded sinusoidal wp2 on the middle half, per-cell nu",
                   "cells": cells, "time_steps": T, "exec": "tiled",
                   "tile_cells": tune["tile_cells"], "steps_per_pass": tune["steps_per_pass"],
                   "vacuum_tile_cells": tune.get("vacuum_tile_cells", 0),
                   "fields": args.precision, "coefficients_dft": "f64"},
        "roofline": rl,
        "hbm_view": hv,
        "single_step_bound_mcells": round(HBM_PEAK_GBS * 1e9 / ss_bytes / 1e6, 1),
        # what a one-step-per-pass kernel would have to move to match this rate
        "single_step_equivalent": {"gbs": round(value * 1e6 * ss_bytes / 1e9, 1),
                                   "frac_of_hbm_peak": round(value * 1e6 * ss_bytes / 1e9 / HBM_PEAK_GBS, 2),
                                   "bytes_per_cell_update": ss_bytes},
        "kernels": {k: {"ms": round(v[0], 3), "launches": v[1], "nodes": v[2]}
                    for k, v in prof.items()},
    }
    for prec, (ms2, X2, prof2, tune2) in results.items():
        if prec == args.precision:
            continue
        dom2 = max(prof2.items(), key=lambda kv: kv[1][0])[0]
        out[prec] = {"value": round(cells * T / (ms2 / 1e3) / 1e6, 1), "ms_per_step": round(ms2, 3),
                     "roofline": alu_roofline(prof2, dom2, tune2["steps_per_pass"], prec),
                     "hbm_view": roofline(prof2, prec),
                     "tile_cells": tune2["tile_cells"], "steps_per_pass": tune2["steps_per_pass"],
                     "vacuum_tile_cells": tune2.get("vacuum_tile_cells", 0)}
        if prec == "f32d":
            out[prec]["mode"] = ("ablation: FP32 fields with eq.(11) and every coefficient in FP32 "
                                 "(delta form), not the specified FP32 mode")
    if not args.no_legs:
        out["batched"] = batched_leg()
        out["batched"]["vs_plain"] = round(out["batched"]["value"] / out["value"], 3)
        # the same node class: the plain workload is half vacuum (whose tiles
        # run about twice as fast), the batch 97% plasma; its whole-job rate
        # against the plain run's plasma-tile rate (kernel time only)
        if "tiled_plasma" in prof:
            ms_t, calls, units = prof["tiled_plasma"]
            rate = units / calls * tune["steps_per_pass"] / (ms_t / calls / 1e3) / 1e6
            out["batched"]["plain_plasma_tile_rate"] = round(rate, 1)
            out["batched"]["vs_plain_plasma_tiles"] = round(out["batched"]["value"] / rate, 3)
        out["adjoint"] = adjoint_leg()
        out["c1_latency"] = c1_leg()
        out["c3_3d"] = c3_leg()
        out["c2d_2d"] = c2d_leg()
        out["paper_table2"] = table2_leg()
    stored = None if args.no_check else stored_oracle_spectra(p, T)
    if stored is not None:
        Xo, Xvo = stored
        Ro, To = (Xo[0] - Xvo[0]) / Xvo[0], Xo[1] / Xvo[1]
        acc, rerr, terr = {}, {}, {}
        for prec, r in results.items():
            acc[prec] = float(np.max(np.abs(r[1] - Xo)) / np.max(np.abs(Xo)))
            # two-run reflection and transmission, the vacuum run at the same precision
            Xv = vacuum_spectra(p, prec, T, r[3])
            R, Tt = (r[1][0] - Xv[0]) / Xv[0], r[1][1] / Xv[1]
            rerr[prec] = float(np.max(np.abs(np.abs(R) - np.abs(Ro))))
            terr[prec] = float(np.max(np.abs(np.abs(Tt) - np.abs(To))))
            hi = p.freqs >= 12e9
            rerr[prec + "_f_ge_12ghz"] = float(np.max(np.abs(np.abs(R[hi]) - np.abs(Ro[hi]))))
            terr[prec + "_f_ge_12ghz"] = float(np.max(np.abs(np.abs(Tt[hi]) - np.abs(To[hi]))))
        out["accuracy"] = {"spectra_rel_err_vs_fp64_oracle": acc, "max_abs_R_err": rerr, "max_abs_T_err": terr,
                           "frequencies_ghz": [round(float(p.freqs[0]) / 1e9, 3), round(float(p.freqs[-1]) / 1e9, 3)],
                           "oracle": "stored FP64 oracle spectra (tests/golden/c2_oracle_spectra.json)"}
    elif not args.no_check:
        out["accuracy"] = {"skipped": "stored oracle spectra cover 2^24 cells x 20000 steps only"}
    if not args.no_check:
        out["accuracy_c1_precisions"] = c1_precision_errors()
    if not args.no_cpu:
        out["cpu_baseline"] = cpu_baseline(p, args.cpu_steps)
        if "paper_table2" in out:
            out["paper_table2"]["serial_oracle_ms_at"] = table2_serial(out["cpu_baseline"], out["paper_table2"])
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
