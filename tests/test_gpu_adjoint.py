"""GPU adjoint: dL/d(wp2) of L = sum_f |R(f)|^2 by the library's discrete
adjoint (sqrt(T) checkpoints) against the FP64 oracle's full-trajectory
adjoint and against FP64 central finite differences."""
import sys

import numpy as np
import pytest

import oracle
from paper_1709_00821_amd import workloads as W

pytestmark = pytest.mark.gpu


def say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def G():
    import torch
    assert torch.cuda.is_available()
    from paper_1709_00821_amd import plasma
    return plasma


def small_problem(seed=3, n=300, bc="mur"):
    rng = np.random.default_rng(seed)
    p = W.random_slab(rng, n, n_freqs=8, bc=bc)
    return p.copy(probes=np.array([10, n - 20]), src_cell=30)


@pytest.mark.parametrize("bc,T", [("mur", 800), ("pec", 700), ("mur", 150)])
def test_fp64_adjoint_matches_oracle(G, bc, T):
    p = small_problem(bc=bc)
    say(f"case adjoint fp64 bc={bc} n={p.n} steps={T}")
    xv = oracle.run(p.vacuum(), T)["X"][0]
    Lo, go, Xo = oracle.adjoint_r2(p, T, xv)
    with G.FdtdPlasma(p, precision="f64", exec="tiled", checkpoint=T) as h:
        L, g = h.grad_r2(T, xv.reshape(1, -1))
        X = h.spectra()[0]
    Xr = Xo[0] if np.ndim(Xo) > 1 else Xo
    # the forward run's spectra themselves: the FP64 bar
    ex = float(np.max(np.abs(X[0] - Xr)) / np.max(np.abs(Xr)))
    # L = sum |R|^2 with R = (X - Xv)/Xv (two-run reflection): the spectra's
    # relative bound 1e-12, amplified by the condition number of that
    # difference, 2 max |X| / |X - Xv| (about 3e4 for the 150-step run, whose
    # reflected part is still small; 80 for the longer runs)
    cond = 2.0 * float(np.max(np.abs(Xr) / np.abs(Xr - xv)))
    eL = abs(L[0] - Lo) / abs(Lo)
    # the gradient is linear in the adjoint source 2 conj(R)/Xv, so R's error
    # (the same cond times the spectra's) enters it with the same factor; the
    # transposed steps add their own rounding at the forward run's 1e-12 level
    eg = float(np.max(np.abs(g - go)) / np.max(np.abs(go)))
    say(f"spectra {ex:.2e}, loss {eL:.2e}, gradient {eg:.2e}, condition {cond:.1e}")
    assert ex <= 1e-12
    assert eL <= 1e-12 * max(1.0, cond)
    assert eg <= 1e-12 * (1.0 + cond)


@pytest.mark.parametrize("precision,bc", [("f64", "mur"), ("f32", "mur"), ("f64", "pec")])
def test_tiled_reverse_matches_per_step_bitwise(G, precision, bc):
    """The register-tile reverse sweep (up to 48 transposed steps per launch
    on 256-node tiles) gives the per-step reverse sweep's loss and gradient
    bit for bit: grids spanning several tiles with ragged tails, probes at
    both ends, T = 3000 so each 55-step checkpoint segment takes two launches.
    FP32 storage: each executor's forward run rounds the FP64 register fields
    at its own launch ends, so the losses and gradients agree to that
    rounding (1e-6 of the largest gradient) rather than bit for bit."""
    rng = np.random.default_rng(31)
    probs = [W.random_slab(rng, n, n_freqs=6, bc=bc) for n in (150, 701, 2100)]
    probs = [q.copy(freqs=probs[0].freqs, probes=np.array([5, q.n - 6]), src_cell=30) for q in probs]
    T = 3000
    say(f"case tiled reverse bitwise {precision} {bc} lens={[q.n for q in probs]} steps={T}")
    xrefs = np.stack([oracle.run(q.vacuum(), T)["X"][0] for q in probs])
    out = {}
    for ex in ("step", "tiled", "resident"):
        with G.FdtdPlasma(probs, precision=precision, exec=ex, checkpoint=T) as h:
            out[ex] = h.grad_r2(T, xrefs, probe=1 if bc == "pec" else 0)
    for ex in ("tiled", "resident"):
        if precision == "f64":
            assert np.array_equal(out[ex][0], out["step"][0]), ex
            assert np.array_equal(out[ex][1], out["step"][1]), ex
        else:
            gl = np.max(np.abs(out["step"][1]))
            eL = np.max(np.abs(out[ex][0] - out["step"][0]) / np.abs(out["step"][0]))
            eg = np.max(np.abs(out[ex][1] - out["step"][1])) / gl
            say(f"fp32 {ex} vs step: loss {eL:.2e} gradient {eg:.2e}")
            assert eL <= 1e-5 and eg <= 1e-5, ex
    assert np.all(np.isfinite(out["step"][1])) and np.max(np.abs(out["step"][1])) > 0


def test_batched_adjoint_and_loss(G):
    rng = np.random.default_rng(9)
    probs = [W.random_slab(rng, n, n_freqs=6) for n in (150, 420, 900)]
    # probes 25 nodes from the source so that every reference spectrum is nonzero
    probs = [q.copy(freqs=probs[0].freqs, probes=np.array([5, q.n - 6]), src_cell=30) for q in probs]
    T = 600
    say(f"case batched adjoint lens={[q.n for q in probs]} steps={T}")
    xrefs = np.stack([oracle.run(q.vacuum(), T)["X"][0] for q in probs])
    with G.FdtdPlasma(probs, precision="f64", exec="resident", checkpoint=T) as h:
        h.run(T)
        L1 = h.loss_r2(xrefs)
        L, g = h.grad_r2(T, xrefs)
        L2, g2 = h.grad_r2(T, xrefs)         # reuses the checkpoints
    assert np.array_equal(L, L1) and np.array_equal(g, g2)
    o = 0
    for b, q in enumerate(probs):
        Lo, go, Xo = oracle.adjoint_r2(q, T, xrefs[b])
        # R = (X - Xref)/Xref cancels when |R| is small: the spectra's 1e-14
        # relative error enters L through 2 |R| |X/Xref|, not through L itself
        R = (Xo - xrefs[b]) / xrefs[b]
        cond = np.sum(2 * np.abs(R) * np.abs(Xo / xrefs[b]))
        assert abs(L[b] - Lo) <= 1e-12 * (abs(Lo) + cond), b
        gb = g[o:o + q.n]
        assert np.max(np.abs(gb - go)) <= 1e-10 * np.max(np.abs(go)), b
        o += q.n


def test_autograd_matches_grad(G):
    import torch
    from paper_1709_00821_amd.autograd import reflection_loss
    p = small_problem(seed=5, n=200)
    T = 400
    say("case autograd RLoss")
    xv = oracle.run(p.vacuum(), T)["X"][0]
    w = torch.tensor(p.wp2, dtype=torch.float64, requires_grad=True)
    L = reflection_loss(w, p, xv, T, precision="f64")
    L.backward(torch.tensor(2.0, dtype=torch.float64))
    Lo, go, _ = oracle.adjoint_r2(p, T, xv)
    assert abs(L.item() - Lo) <= 1e-12 * Lo
    assert np.max(np.abs(w.grad.numpy() - 2 * go)) <= 1e-10 * np.max(np.abs(2 * go))


def fd_gradients(G, p, T, xv, cells, dirs, hrel=1e-3):
    """FP64 central differences, all perturbed grids in one batched launch."""
    h_abs = hrel * np.max(p.wp2)
    probs = []
    for k in cells:
        for s in (+1, -1):
            w = p.wp2.copy()
            hk = hrel * w[k] if w[k] > 0 else h_abs
            w[k] += s * hk
            probs.append(p.copy(wp2=w))
    for v in dirs:                      # relative perturbation hrel * v_k * wp2_k
        for s in (+1, -1):
            probs.append(p.copy(wp2=p.wp2 * (1 + s * hrel * v)))
    with G.FdtdPlasma(probs, precision="f64", exec="tiled") as hh:
        hh.run(T)
        Lb = hh.loss_r2(np.tile(xv, (len(probs), 1)))
    out = []
    for i, k in enumerate(cells):
        hk = hrel * p.wp2[k] if p.wp2[k] > 0 else h_abs
        out.append((Lb[2 * i] - Lb[2 * i + 1]) / (2 * hk))
    base = 2 * len(cells)
    dd = [(Lb[base + 2 * j] - Lb[base + 2 * j + 1]) / (2 * hrel) for j in range(len(dirs))]
    return np.array(out), np.array(dd)


def test_c5_fp32_adjoint_vs_fd_and_oracle(G):
    """The 8000-cell, 20000-step gradient: FP32 forward + adjoint against FP64
    central differences (h = 1e-3 relative) on 64 seeded cells and 4 random
    directions, and against the FP64 oracle adjoint (full trajectory)."""
    p = W.adjoint_c5()
    T = p.steps
    rng = np.random.default_rng(1712)
    cells = np.sort(rng.choice(np.arange(3000, 5000), 64, replace=False))
    dirs = [np.clip(rng.normal(size=p.n), -3, 3) for _ in range(4)]
    say(f"case c5 adjoint fp32 n={p.n} steps={T}: vacuum reference")
    with G.FdtdPlasma(p.vacuum(), precision="f64", exec="tiled") as hv:
        hv.run(T)
        xv = hv.spectra()[0, 0]
    say("case c5: fp32 forward + adjoint")
    with G.FdtdPlasma(p, precision="f32", exec="tiled", checkpoint=T) as h:
        L32, g32 = h.grad_r2(T, xv.reshape(1, -1))
    say("case c5: fp64 finite differences (batched)")
    fd, fdd = fd_gradients(G, p, T, xv, cells, dirs)
    rel = np.linalg.norm(g32[cells] - fd) / np.linalg.norm(fd)
    say(f"c5 fp32 adjoint vs fp64 FD: rel {rel:.2e}")
    assert rel <= 1e-4
    big = np.abs(fd) >= 1e-2 * np.max(np.abs(fd))
    assert np.all(np.abs(g32[cells][big] - fd[big]) <= 1e-4 * np.abs(fd[big]) + 1e-4 * np.max(np.abs(fd)))
    proj = np.array([g32 @ (v * p.wp2) for v in dirs])   # d/d(eps) L(wp2 (1 + eps v))
    say(f"c5 directional derivatives: adjoint {proj}, FD {fdd}")
    assert np.linalg.norm(proj - fdd) <= 1e-4 * np.linalg.norm(fdd)
    say("case c5: fp64 oracle adjoint (full trajectory)")
    Lo, go, _ = oracle.adjoint_r2(p, T, xv)
    relo = np.linalg.norm(g32 - go) / np.linalg.norm(go)
    say(f"c5 fp32 adjoint vs fp64 oracle adjoint: rel {relo:.2e}; loss {L32[0]:.6e} vs {Lo:.6e}")
    assert relo <= 1e-4
