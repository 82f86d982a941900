// Discrete adjoint of the 1D RKETD-FDTD step for the reflection loss
//   L_b = sum_f |R_b(f)|^2,  R_b(f) = (X_b(f) - Xref_b(f)) / Xref_b(f),
// X_b the running DFT at one probe.  The forward step applies, in order,
//   H update (eq.(14)), E update (eqs.(11)+(12) solved), source (eq.(15)),
//   J update (eq.(11)), Mur/PEC ends, probe sample;
// the adjoint applies the transposes of ends, J, E and H in reverse order (the
// source does not depend on the plasma).  dL/d(wp2) collects, per step,
//   lambda_E* (dCA E^n - dCJ J^n - dCH curl H^{n+1/2}) + lambda_J (db1 E^n + db2 E^{n+1}).
#include <hip/hip_runtime.h>

#include "tile1d.h"

namespace fdtdp {

__device__ __forceinline__ int grid_of_adj(const Grids &g, int64_t i)
{
    int64_t lo = 0, hi = g.batch - 1;
    while (lo < hi) {
        const int64_t mid = (lo + hi + 1) >> 1;
        if (g.off[mid] <= i) lo = mid; else hi = mid - 1;
    }
    return (int)lo;
}

// Per-node coefficients and their wp2-derivatives, SoA [12][nodes]:
// CA, CJ, CH, a, b1, b2, dCA, dCJ, dCH, db1, db2, 1/CJ (the last turns the
// forward state's carried Q = CJ (J - b2 E) back into J).
__global__ void k_adj_coef(Grids g, int64_t total, double *tab)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= total) return;
    const double w = g.wp2[i], v = g.nu[i];
    const Coef c = node_coef(w, v, g.dt, g.dz, 0);
    const DCoef d = node_dcoef(w, v, g.dt, g.dz);
    const double vals[12] = {c.CA, c.CJ, c.CH, c.a, c.b1, c.b2, d.dCA, d.dCJ, d.dCH, d.db1, d.db2, 1.0 / c.CJ};
#pragma unroll
    for (int q = 0; q < 12; ++q) tab[(int64_t)q * total + i] = vals[q];
}

// Per grid: R_f, loss_b = sum_f |R_f|^2 and G_f = conj(R_f) / Xref_f.  One wave
// per grid, frequencies strided over lanes, fixed shuffle-tree sum.
__global__ __launch_bounds__(64) void k_adj_prepare(const double2 *X, int P, int F, int probe,
                                                    const double2 *xref, double2 *G, double *loss)
{
    const int b = blockIdx.x;
    const int lane = threadIdx.x;
    double acc = 0.0;
    for (int f = lane; f < F; f += 64) {
        const double2 x = X[((int64_t)b * P + probe) * F + f];
        const double2 r0 = xref[(int64_t)b * F + f];
        const double den = r0.x * r0.x + r0.y * r0.y;
        const double nr = x.x - r0.x, ni = x.y - r0.y;
        const double Rr = (nr * r0.x + ni * r0.y) / den;
        const double Ri = (ni * r0.x - nr * r0.y) / den;
        acc += Rr * Rr + Ri * Ri;
        // conj(R) / xref = conj(R) conj(xref) / |xref|^2
        G[(int64_t)b * F + f] = make_double2((Rr * r0.x - Ri * r0.y) / den,
                                             (-Rr * r0.y - Ri * r0.x) / den);
    }
#pragma unroll
    for (int d = 32; d >= 1; d >>= 1) acc += __shfl_xor(acc, d, 64);
    if (lane == 0) loss[b] = acc;
}

// dL/dE^m at the probe, m = 1..T: 2 sum_f Re(G_f dt e^{-j 2 pi f m dt}).
__global__ void k_adj_source(const double *freqs, int F, double dt, const double2 *G,
                             int64_t batch, int64_t T, double *gsrc)
{
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= batch * T) return;
    const int64_t b = t / T, m = t % T + 1;
    double acc = 0.0;
    for (int f = 0; f < F; ++f) {
        double re, im;
        twiddle(freqs[f] * dt, dt, m, re, im);
        const double2 Gf = G[b * F + f];
        acc += Gf.x * re - Gf.y * im;
    }
    gsrc[t] = 2.0 * acc;
}

template <typename T>
struct AdjView {
    const T *lE, *lH, *lJ;      // lambda^{m+1}
    T *nE, *nH, *nJ;            // lambda^m
    const T *En;                // forward E^m
    const double *Jn;           // forward Q^{m-1} = CJ (J^m - b2 E^m) (FP64)
    const T *Hh, *En1;          // forward H^{m+1/2}, E^{m+1}
};

// One transposed step m+1 -> m for every node of every grid.
template <typename T>
__global__ void k_adj_step(Grids g, AdjView<T> v, const double *tab, int64_t total,
                           const double *gsrc, int64_t T_, int64_t m, int probe, double *grad)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= total) return;
    const int b = grid_of_adj(g, i);
    const int64_t off = g.off[b], n = g.n[b], k = i - off;
    if (k >= n) return;
    const double *CA = tab, *CJ = tab + total, *CH = tab + 2 * total, *A = tab + 3 * total,
                 *B1 = tab + 4 * total, *B2 = tab + 5 * total;
    const bool mur = g.bc == 0;
    const double cm = g.cm, ch = g.ch;
    const int64_t pc = g.probe[(int64_t)b * g.P + probe];
    const double src = gsrc[(int64_t)b * T_ + m];      // dL/dE^{m+1}[pc]
    // lambda_E^{m+1} after the probe's adjoint source, at grid node j
    auto lEp = [&](int64_t j) -> double {
        const double l = (double)v.lE[off + j];
        return j == pc ? l + src : l;
    };
    // adjoint of E* at interior node j (1..n-2): ends (Mur) and the J update's b2
    auto lEs = [&](int64_t j) -> double {
        double s = lEp(j);
        if (mur && j == 1) s += cm * lEp(0);
        if (mur && j == n - 2) s += cm * lEp(n - 1);
        return s + B2[off + j] * (double)v.lJ[off + j];
    };
    // adjoint of H^{m+1/2} at H node j (0..n-2) after the E* transpose
    auto lHn = [&](int64_t j) -> double {
        double s = (double)v.lH[off + j];
        if (j + 1 <= n - 2) s += CH[off + j + 1] * lEs(j + 1);
        if (j >= 1) s -= CH[off + j] * lEs(j);
        return s;
    };
    double nE, nJ = 0.0;
    if (k == 0 || k == n - 1) {
        if (mur) {
            nE = -cm * lEp(k) + (k == 0 ? ch * lHn(0) : -ch * lHn(n - 2));
        } else {
            nE = 0.0;
        }
    } else {
        const double es = lEs(k);
        const double lj = (double)v.lJ[off + k];
        nJ = A[off + k] * lj - CJ[off + k] * es;
        nE = CA[off + k] * es + B1[off + k] * lj + ch * (lHn(k) - lHn(k - 1));
        if (mur && k == 1) nE += lEp(0);
        if (mur && k == n - 2) nE += lEp(n - 1);
        // gradient with respect to wp2 at node k
        const double dCA = tab[6 * total + off + k], dCJ = tab[7 * total + off + k];
        const double dCH = tab[8 * total + off + k], dB1 = tab[9 * total + off + k];
        const double dB2 = tab[10 * total + off + k];
        // the stored forward state carries Q^{m-1} = CJ (J^m - b2 E^m)
        const double e0 = (double)v.En[off + k];
        const double j0 = __builtin_fma(B2[off + k], e0, v.Jn[off + k] * tab[11 * total + off + k]);
        const double curl = (double)v.Hh[off + k] - (double)v.Hh[off + k - 1];
        const double e1 = (double)v.En1[off + k];
        grad[off + k] += es * (dCA * e0 - dCJ * j0 - dCH * curl) + lj * (dB1 * e0 + dB2 * e1);
    }
    v.nE[off + k] = (T)nE;
    v.nJ[off + k] = (T)nJ;
    if (k <= n - 2) v.nH[off + k] = (T)lHn(k);
}

void launch_adj_coef(const Grids &g, int64_t total, double *tab, hipStream_t st)
{
    hipLaunchKernelGGL(k_adj_coef, dim3((unsigned)((total + 255) / 256)), dim3(256), 0, st, g, total,
                       tab);
}

void launch_adj_prepare(const double2 *X, int64_t batch, int P, int F, int probe, const double2 *xref,
                        double2 *G, double *loss, hipStream_t st)
{
    hipLaunchKernelGGL(k_adj_prepare, dim3((unsigned)batch), dim3(64), 0, st, X, P, F, probe, xref, G,
                       loss);
}

void launch_adj_source(const double *freqs, int F, double dt, const double2 *G, int64_t batch,
                       int64_t T, double *gsrc, hipStream_t st)
{
    const int64_t tot = batch * T;
    hipLaunchKernelGGL(k_adj_source, dim3((unsigned)((tot + 255) / 256)), dim3(256), 0, st, freqs, F,
                       dt, G, batch, T, gsrc);
}

template <typename T>
void launch_adj_step(const Grids &g, const T *const lam[3], T *const out[3], const T *En,
                     const double *Jn, const T *Hh, const T *En1, const double *tab, int64_t total,
                     const double *gsrc, int64_t T_, int64_t m, int probe, double *grad,
                     hipStream_t st)
{
    AdjView<T> v{lam[0], lam[1], lam[2], out[0], out[1], out[2], En, Jn, Hh, En1};
    hipLaunchKernelGGL(k_adj_step<T>, dim3((unsigned)((total + 255) / 256)), dim3(256), 0, st, g, v,
                       tab, total, gsrc, T_, m, probe, grad);
}

template void launch_adj_step<float>(const Grids &, const float *const[3], float *const[3],
                                     const float *, const double *, const float *, const float *,
                                     const double *, int64_t, const double *, int64_t, int64_t, int,
                                     double *, hipStream_t);
template void launch_adj_step<double>(const Grids &, const double *const[3], double *const[3],
                                      const double *, const double *, const double *, const double *,
                                      const double *, int64_t, const double *, int64_t, int64_t, int,
                                      double *, hipStream_t);

__global__ void k_copy(uint4 *dst, const uint4 *src, int64_t n16)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t j = i; j < n16; j += stride) dst[j] = src[j];
}

// Device-to-device copy as a kernel (capturable like any launch).
void launch_copy(void *dst, const void *src, int64_t bytes, hipStream_t st)
{
    const int64_t n16 = bytes / 16;
    if (n16 <= 0) return;
    int64_t nb = (n16 + 255) / 256;
    if (nb > 65536) nb = 65536;
    hipLaunchKernelGGL(k_copy, dim3((unsigned)nb), dim3(256), 0, st, (uint4 *)dst, (const uint4 *)src,
                       n16);
}

// ------------------------------------------------------------ trace

// Forward recompute for the adjoint: the tiles of every grid advance nsteps
// steps from segment slot slot0 and store the state of their output nodes
// after every step into slots slot0 + 1 .. slot0 + nsteps (slot i at
// seg + i * slot_bytes: E [nodes], H at + arr_bytes, J (FP64) at + 2 arr_bytes).
// Same per-node functions as k_tiled, hence the forward run's bits.  Tiles
// read only slot slot0, which no tile of the launch writes.  Mur or PEC ends;
// no probes (g.P = 0); the source values come from g.srcv indexed by slot.
template <typename T, int C>
__global__ __launch_bounds__(256) void k_trace(Grids g, char *seg, int64_t slot_bytes, int64_t arr_bytes,
                                               const Tile *tiles, int64_t ntiles, int nsteps, int slot0)
{
    const int lane = threadIdx.x & 63;
    const int64_t blk = xcd_block(blockIdx.x, gridDim.x);
    const int64_t t = blk * (blockDim.x >> 6) + uniform(threadIdx.x >> 6);
    if (t >= ntiles) return;
    const Tile tl = tiles[t];
    const int b = tl.grid;
    const int64_t off = g.off[b], n = g.n[b];
    const int64_t k0 = (int64_t)tl.lo + (int64_t)lane * C;
    auto slotE = [&](int i) { return (T *)(seg + (int64_t)i * slot_bytes); };
    auto slotH = [&](int i) { return (T *)(seg + (int64_t)i * slot_bytes + arr_bytes); };
    auto slotJ = [&](int i) { return (double *)(seg + (int64_t)i * slot_bytes + 2 * arr_bytes); };
    State<T> s0;
    s0.E[0] = slotE(slot0);
    s0.H[0] = slotH(slot0);
    s0.J[0] = slotJ(slot0);
    Chunk<T, C, true, false> ck;
    typedef typename Chunk<T, C, true, false>::R R;
    chunk_load<T, C, true, false>(ck, g, s0, 0, b, off, n, k0, tl.hi);
    auto er = [](R e0) { return shfl_down1(e0); };
    auto hl = [](R h) { return shfl_up1(h); };
    auto post = [&](int st) {
        const int i = slot0 + st + 1;
        store_chunk_as<T, C>(slotE(i) + off, k0, tl.out_lo, tl.out_hi, ck.E);
        store_chunk_as<T, C>(slotH(i) + off, k0, tl.out_lo, tl.out_hi < n ? tl.out_hi : n - 1, ck.H);
        store_chunk<double, C>(slotJ(i) + off, k0, tl.out_lo, tl.out_hi, ck.J);
    };
    const WaveRole role = wave_role<C>(g, b, n, tl.lo, tl.hi);
    if (!has_role(role)) {
        for (int st = 0; st < nsteps; ++st) {
            chunk_step_plain<T, C, true, false>(ck, g, er, hl);
            post(st);
        }
    } else {
        WaveProbes wp;
        wp.n = 0;
        run_role<T, C, true, false>(ck, g, role, wp, lane, b, tl.lo, tl.out_lo, tl.out_hi, nsteps, slot0, er, hl,
                                    post);
    }
}

template <typename T>
void launch_trace(const Grids &g, char *seg, int64_t slot_bytes, int64_t arr_bytes, const Tile *tiles,
                  int64_t ntiles, int nsteps, int slot0, hipStream_t st)
{
    hipLaunchKernelGGL((k_trace<T, kTraceCells / 64>), dim3((unsigned)((ntiles + 3) / 4)), dim3(256), 0, st, g, seg,
                       slot_bytes, arr_bytes, tiles, ntiles, nsteps, slot0);
}

template void launch_trace<float>(const Grids &, char *, int64_t, int64_t, const Tile *, int64_t, int, int,
                                  hipStream_t);
template void launch_trace<double>(const Grids &, char *, int64_t, int64_t, const Tile *, int64_t, int, int,
                                   hipStream_t);

// ------------------------------------------------------------ reverse

// Transposed steps of the adjoint on register tiles: lane holds C nodes of
// lambda_E, lambda_H, lambda_J (storage precision, as between the steps of
// the per-step kernel), the twelve coefficient and derivative values and the
// gradient of its nodes (FP64).  Reverse step m (lambda^{m+1} -> lambda^m),
// for interior nodes k, with es the adjoint of the E update's input, lHn the
// adjoint of H^{m+1/2}:
//   lEp = lambda_E (+ dL/dE^{m+1} at the probe node)
//   es  = lEp (+ cm lEp(0) at node 1, + cm lEp(n-1) at node n-2, Mur) + b2 lambda_J
//   lHn = lambda_H + CH(k+1) es(k+1) [k+1 <= n-2] - CH(k) es(k) [k >= 1]
//   lambda_J' = a lambda_J - CJ es
//   lambda_E' = CA es + b1 lambda_J + ch (lHn(k) - lHn(k-1)) (+ lEp(0) at 1, + lEp(n-1) at n-2)
//   grad += es (dCA E^m - dCJ J^m - dCH curl H^{m+1/2}) + lambda_J (db1 E^m + db2 E^{m+1})
// and at the end nodes lambda_E' = -cm lEp(k) +- ch lHn (Mur) or 0 (PEC).
// The expressions and their order are those of the per-step kernel, so the
// two give the same bits.  The stencil radius is one node per step, as in
// the forward step, so a tile with a kAdjHalo halo runs up to kAdjHalo steps.
// ROLE: the tile holds a grid end or the probe node (conditions evaluated per
// node); otherwise every held node is interior.
template <typename T, int C, bool ROLE>
__device__ __forceinline__ void adj_tile_steps(const Grids &g, const AdjTileArgs<T> &a, const Tile &tl, int b,
                                               int64_t off, int64_t n, int64_t k0, int lane, int64_t mtop,
                                               int nsteps, T (&lE)[C], T (&lH)[C], T (&lJ)[C],
                                               double (&gr)[C])
{
    const int64_t tot = a.total;
    double CA[C], CJ[C], CH[C], CHn[C], A[C], B1[C], B2[C], dCA[C], dCJ[C], dCH[C], dB1[C], dB2[C], ICJ[C];
    load_chunk<double, C>(a.tab + 0 * tot + off, k0, tl.hi, CA);
    load_chunk<double, C>(a.tab + 1 * tot + off, k0, tl.hi, CJ);
    load_chunk<double, C>(a.tab + 2 * tot + off, k0, tl.hi, CH);
    load_chunk<double, C>(a.tab + 3 * tot + off, k0, tl.hi, A);
    load_chunk<double, C>(a.tab + 4 * tot + off, k0, tl.hi, B1);
    load_chunk<double, C>(a.tab + 5 * tot + off, k0, tl.hi, B2);
    load_chunk<double, C>(a.tab + 6 * tot + off, k0, tl.hi, dCA);
    load_chunk<double, C>(a.tab + 7 * tot + off, k0, tl.hi, dCJ);
    load_chunk<double, C>(a.tab + 8 * tot + off, k0, tl.hi, dCH);
    load_chunk<double, C>(a.tab + 9 * tot + off, k0, tl.hi, dB1);
    load_chunk<double, C>(a.tab + 10 * tot + off, k0, tl.hi, dB2);
    load_chunk<double, C>(a.tab + 11 * tot + off, k0, tl.hi, ICJ);
    {
        const double nx = shfl_down1(CH[0]);
#pragma unroll
        for (int i = 0; i < C; ++i) CHn[i] = (i + 1 < C) ? CH[i + 1] : nx;
    }
    const bool mur = g.bc == 0;
    const double cm = g.cm, ch = g.ch;
    // the probe node, if this tile holds it (wave-uniform)
    const int64_t pc = g.probe[(int64_t)b * g.P + a.probe];
    const bool has_p = ROLE && pc >= tl.lo && pc < tl.hi;
    const int p_lane = uniform(has_p ? (pc - tl.lo) / C : -1), p_reg = uniform(has_p ? (pc - tl.lo) % C : 0);
    const int nn = (int)n;
    auto slotp = [&](int64_t m, int q) { return a.seg + (m - a.m0) * a.slot_bytes + q * a.arr_bytes; };
    // forward states of step st (m = mtop - st): E^m and Q^{m-1} (slot m),
    // H^{m+1/2} (slot m+1), and E^{m+1}, which is step st-1's E^m.  The first
    // three (and the probe's adjoint source) are loaded kAdjPrefetch steps
    // ahead into a ring of registers: they do not depend on the adjoint
    // arithmetic, and a step waits only on the loads issued for it.
    constexpr int D = kAdjPrefetch;
    T qe[D][C], qh[D][C];
    double qj[D][C], qs[D];
    auto fetch = [&](int st, T (&e)[C], double (&j)[C], T (&h)[C], double &sv) {
        const int64_t m = mtop - st;
        load_chunk<T, C>((const T *)slotp(m, 0) + off, k0, tl.hi, e);
        load_chunk<double, C>((const double *)slotp(m, 2) + off, k0, tl.hi, j);
        load_chunk<T, C>((const T *)slotp(m + 1, 1) + off, k0, tl.hi, h);
        sv = has_p ? a.gsrc[(int64_t)b * a.T_ + m] : 0.0;
    };
#pragma unroll
    for (int d = 0; d < D; ++d)
        if (d < nsteps) fetch(d, qe[d], qj[d], qh[d], qs[d]);
    T e1[C];
    load_chunk<T, C>((const T *)slotp(mtop + 1, 0) + off, k0, tl.hi, e1);
    for (int base = 0; base < nsteps; base += D) {
#pragma unroll
        for (int d = 0; d < D; ++d) {
            const int st = base + d;
            if (st >= nsteps) break;
            T e0[C], hh[C];
            double j0[C];
#pragma unroll
            for (int i = 0; i < C; ++i) {
                e0[i] = qe[d][i];
                j0[i] = qj[d][i];
                hh[i] = qh[d][i];
            }
            const double src = qs[d];
            if (st + D < nsteps) fetch(st + D, qe[d], qj[d], qh[d], qs[d]);
            double lEp[C], es[C], lHn[C];
#pragma unroll
            for (int i = 0; i < C; ++i) {
                const double l = (double)lE[i];
                lEp[i] = (ROLE && lane == p_lane && i == p_reg) ? l + src : l;
            }
            double lEp0 = 0.0, lEpN = 0.0;
            if constexpr (ROLE) {
                // lEp at node 0 for node 1 (same lane: node 0 sits in register 0
                // or 1 of lane 0), at node n-1 for node n-2 (same lane, or the
                // next lane's register 0)
                const int r0 = uniform(tl.lo <= 0 ? -tl.lo : 0);
                lEp0 = upick<double, C>(lEp, r0);
                const int64_t pr = n - 1 - tl.lo;
                const int rr = uniform(pr >= 0 && pr < 64LL * C ? pr % C : 1);
                const double nx = shfl_down1(lEp[0]);
                const double own = upick<double, C>(lEp, rr);
                lEpN = (rr > 0) ? own : nx;
            }
#pragma unroll
            for (int i = 0; i < C; ++i) {
                double s = lEp[i];
                if constexpr (ROLE) {
                    const int k = (int)(k0 + i);
                    s = (mur && k == 1) ? s + cm * lEp0 : s;
                    s = (mur && k == nn - 2) ? s + cm * lEpN : s;
                }
                es[i] = s + B2[i] * (double)lJ[i];
            }
            const double esn = shfl_down1(es[0]);
#pragma unroll
            for (int i = 0; i < C; ++i) {
                const double en = (i + 1 < C) ? es[i + 1] : esn;
                double s = (double)lH[i];
                if constexpr (ROLE) {
                    const int k = (int)(k0 + i);
                    s = (k + 1 <= nn - 2) ? s + CHn[i] * en : s;
                    s = (k >= 1) ? s - CH[i] * es[i] : s;
                } else {
                    s += CHn[i] * en;
                    s -= CH[i] * es[i];
                }
                lHn[i] = s;
            }
            const double lHp = shfl_up1(lHn[C - 1]);
            const T hhp = shfl_up1(hh[C - 1]);
#pragma unroll
            for (int i = 0; i < C; ++i) {
                const double lhm = (i > 0) ? lHn[i - 1] : lHp;
                const double lj = (double)lJ[i];
                double nJ = A[i] * lj - CJ[i] * es[i];
                double nE = CA[i] * es[i] + B1[i] * lj + ch * (lHn[i] - lhm);
                const double curl = (double)hh[i] - (double)((i > 0) ? hh[i - 1] : hhp);
                const double e0d = (double)e0[i], e1d = (double)e1[i];
                const double jm = __builtin_fma(B2[i], e0d, j0[i] * ICJ[i]);   // J^m from the stored Q^{m-1}
                const double gnew =
                    gr[i] + (es[i] * (dCA[i] * e0d - dCJ[i] * jm - dCH[i] * curl) + lj * (dB1[i] * e0d + dB2[i] * e1d));
                if constexpr (ROLE) {
                    const int k = (int)(k0 + i);
                    nE = (mur && k == 1) ? nE + lEp0 : nE;
                    nE = (mur && k == nn - 2) ? nE + lEpN : nE;
                    const bool end = k == 0 || k == nn - 1;
                    const double nEe = mur ? -cm * lEp[i] + (k == 0 ? ch * lHn[i] : -ch * lhm) : 0.0;
                    nE = end ? nEe : nE;
                    nJ = end ? 0.0 : nJ;
                    gr[i] = (k >= 1 && k <= nn - 2) ? gnew : gr[i];
                } else {
                    gr[i] = gnew;
                }
                lE[i] = (T)nE;
                lJ[i] = (T)nJ;
                lH[i] = (T)lHn[i];
            }
#pragma unroll
            for (int i = 0; i < C; ++i) e1[i] = e0[i];
        }
    }
}

template <typename T, int C>
__global__ __launch_bounds__(256) void k_adj_tiled(Grids g, AdjTileArgs<T> a, const Tile *tiles, int64_t ntiles,
                                                   int64_t mtop, int nsteps)
{
    const int lane = threadIdx.x & 63;
    const int64_t blk = xcd_block(blockIdx.x, gridDim.x);
    const int64_t t = blk * (blockDim.x >> 6) + uniform(threadIdx.x >> 6);
    if (t >= ntiles) return;
    const Tile tl = tiles[t];
    const int b = tl.grid;
    const int64_t off = g.off[b], n = g.n[b];
    const int64_t k0 = (int64_t)tl.lo + (int64_t)lane * C;
    T lE[C], lH[C], lJ[C];
    double gr[C];
    load_chunk<T, C>(a.lE + off, k0, tl.hi, lE);
    load_chunk<T, C>(a.lH + off, k0, tl.hi, lH);
    load_chunk<T, C>(a.lJ + off, k0, tl.hi, lJ);
    load_chunk<double, C>(a.grad + off, k0, tl.hi, gr);
    const int64_t pc = g.probe[(int64_t)b * g.P + a.probe];
    const bool role = tl.lo <= 0 || tl.hi >= n || (pc >= tl.lo && pc < tl.hi);
    if (role)
        adj_tile_steps<T, C, true>(g, a, tl, b, off, n, k0, lane, mtop, nsteps, lE, lH, lJ, gr);
    else
        adj_tile_steps<T, C, false>(g, a, tl, b, off, n, k0, lane, mtop, nsteps, lE, lH, lJ, gr);
    store_chunk<T, C>(a.nE + off, k0, tl.out_lo, tl.out_hi, lE);
    store_chunk<T, C>(a.nH + off, k0, tl.out_lo, tl.out_hi < n ? tl.out_hi : n - 1, lH);
    store_chunk<T, C>(a.nJ + off, k0, tl.out_lo, tl.out_hi, lJ);
    store_chunk<double, C>(a.grad + off, k0, tl.out_lo, tl.out_hi, gr);
}

template <typename T>
void launch_adj_tiled(const Grids &g, const AdjTileArgs<T> &a, const Tile *tiles, int64_t ntiles, int64_t mtop,
                      int nsteps, hipStream_t st)
{
    hipLaunchKernelGGL((k_adj_tiled<T, kAdjCells / 64>), dim3((unsigned)((ntiles + 3) / 4)), dim3(256), 0, st, g,
                       a, tiles, ntiles, mtop, nsteps);
}

template void launch_adj_tiled<float>(const Grids &, const AdjTileArgs<float> &, const Tile *, int64_t, int64_t,
                                      int, hipStream_t);
template void launch_adj_tiled<double>(const Grids &, const AdjTileArgs<double> &, const Tile *, int64_t, int64_t,
                                       int, hipStream_t);

}  // namespace fdtdp
