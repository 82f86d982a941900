// Discrete adjoint of the 1D RKETD-FDTD step for the reflection loss
//   L_b = sum_f |R_b(f)|^2,  R_b(f) = (X_b(f) - Xref_b(f)) / Xref_b(f),
// X_b the running DFT at one probe.  The forward step applies, in order,
//   H update (eq.(14)), E update (eqs.(11)+(12) solved), source (eq.(15)),
//   J update (eq.(11)), Mur/PEC ends, probe sample;
// the adjoint applies the transposes of ends, J, E and H in reverse order (the
// source does not depend on the plasma).  dL/d(wp2) collects, per step,
//   lambda_E* (dCA E^n - dCJ J^n - dCH curl H^{n+1/2}) + lambda_J (db1 E^n + db2 E^{n+1}).
#include <hip/hip_runtime.h>

#include "internal.h"

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

// Per-node coefficients and their wp2-derivatives, SoA [11][nodes]:
// CA, CJ, CH, a, b1, b2, dCA, dCJ, dCH, db1, db2.
__global__ void k_adj_coef(Grids g, int64_t total, double *tab)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= total) return;
    const double w = g.wp2[i], v = g.nu[i];
    const Coef c = node_coef(w, v, g.dt, g.dz, 0);
    const DCoef d = node_dcoef(w, v, g.dt, g.dz);
    const double vals[11] = {c.CA, c.CJ, c.CH, c.a, c.b1, c.b2, d.dCA, d.dCJ, d.dCH, d.db1, d.db2};
#pragma unroll
    for (int q = 0; q < 11; ++q) tab[(int64_t)q * total + i] = vals[q];
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
    const double *Jn;           // forward J^m (FP64)
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
        const double e0 = (double)v.En[off + k], j0 = (double)v.Jn[off + k];
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

}  // namespace fdtdp
