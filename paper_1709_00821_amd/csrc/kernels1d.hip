// 1D RKETD-FDTD kernels for gfx950: per-step reference kernels, the
// temporally blocked register-tile kernel, probe DFT, setup helpers.
// Every kernel advances nodes through the same per-node functions of
// physics.h, so all execution modes agree bit for bit.
#include <hip/hip_runtime.h>

#include "internal.h"

namespace fdtdp {

// ---------------------------------------------------------------- helpers

__device__ __forceinline__ int grid_of(const Grids &g, int64_t i)
{
    // largest b with off[b] <= i (off is increasing)
    int64_t lo = 0, hi = g.batch - 1;
    while (lo < hi) {
        const int64_t mid = (lo + hi + 1) >> 1;
        if (g.off[mid] <= i) lo = mid; else hi = mid - 1;
    }
    return (int)lo;
}

// Index into the compact CPML arrays [batch][2][P] and table slot for E node k
// (returns -1 outside the layers; the PEC end nodes carry no psi).
__device__ __forceinline__ int cpml_e_slot(int P, int64_t n, int64_t k, int &tab)
{
    if (k >= 1 && k < P) { tab = P - 1 - (int)k; return (int)k; }
    if (k > n - 1 - P && k <= n - 2) {
        const int d = (int)(k - (n - 1 - P));   // depth 1..P-1
        tab = d - 1;
        return P + (int)(k - (n - P));
    }
    return -1;
}

// Same for H node k (position k+1/2), k = 0..n-2.
__device__ __forceinline__ int cpml_h_slot(int P, int64_t n, int64_t k, int &tab)
{
    if (k < P) { tab = P - 1 - (int)k; return (int)k; }      // depth P-k-1/2
    if (k >= n - 1 - P && k <= n - 2) {
        tab = (int)(k - (n - 1 - P));                         // depth j+1/2
        return P + tab;
    }
    return -1;
}

// ------------------------------------------------------ per-step reference

// Arithmetic of the per-step kernels: R is the register type (FP64, or FP32 in
// the FP32 ablation); values are read from and rounded to the storage type T
// every step.

// H^{n+1/2} of node k of grid b (and its psi, written to buffer nxt).
template <typename T, typename R>
__device__ __forceinline__ R step_h_val(const Grids &g, const State<T> &s, int cur, int b, int64_t off,
                                        int64_t n, int64_t k)
{
    const int nxt = cur ^ 1;
    const T *E = s.E[cur] + off;
    const R El = (R)E[k], Er = (R)E[k + 1];
    const R Ho = (R)s.H[cur][off + k];
    if (g.bc == 1) {
        int tab;
        const int slot = cpml_h_slot(g.cpmlP, n, k, tab);
        if (slot >= 0) {
            const int64_t ps = (int64_t)b * 2 * g.cpmlP + slot;
            const R dE = Er - El;
            const R bH = (R)g.cpml[2 * g.cpmlP + tab], aH = (R)g.cpml[3 * g.cpmlP + tab];
            const R psi = fmat(aH, dE, bH * (R)s.psiH[cur][ps]);
            s.psiH[nxt][ps] = (T)psi;
            return fmat(-(R)g.ch, dE + psi, Ho);
        }
    }
    return h_update<R>(Ho, El, Er, (R)g.ch);
}

// H^{n+1/2} of every node, written to buffer nxt.
template <typename T>
__global__ void k_step_h(Grids g, State<T> s, int cur, int64_t total)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= total) return;
    const int b = grid_of(g, i);
    const int64_t off = g.off[b], n = g.n[b], k = i - off;
    if (k > n - 2) return;
    T Hn;
    if (sizeof(T) == 4 && g.jdelta)
        Hn = (T)step_h_val<T, float>(g, s, cur, b, off, n, k);
    else
        Hn = (T)step_h_val<T, double>(g, s, cur, b, off, n, k);
    s.H[cur ^ 1][off + k] = Hn;
}

// E^{n+1} (and J^{n+1}, psiE) of interior node k of grid b; H already at
// n+1/2 in buffer nxt.  Returns the new E; writes J and psi when asked.
template <typename T, typename R>
__device__ __forceinline__ R step_interior(const Grids &g, const State<T> &s, int cur, int b,
                                           int64_t off, int64_t n, int64_t k, int64_t m,
                                           bool write)
{
    const int nxt = cur ^ 1;
    const T *H = s.H[nxt] + off;
    R curl = (R)H[k] - (R)H[k - 1];
    if (g.bc == 1) {
        int tab;
        const int slot = cpml_e_slot(g.cpmlP, n, k, tab);
        if (slot >= 0) {
            const int64_t ps = (int64_t)b * 2 * g.cpmlP + slot;
            const R bE = (R)g.cpml[tab], aE = (R)g.cpml[g.cpmlP + tab];
            const R psi = fmat(aE, curl, bE * (R)s.psiE[cur][ps]);
            if (write) s.psiE[nxt][ps] = (T)psi;
            curl = curl + psi;
        }
    }
    const R Eo = (R)s.E[cur][off + k];
    const double wp2 = g.wp2[off + k];
    // the J arrays hold Q^{n-1} = CJ (J^n - b2 E^n) (the FP32 ablation: J^n itself)
    const double Po = s.J[cur][off + k];
    R En;
    NodeCoef<R> c;
    if (wp2 != 0.0) {
        c = node_coef_t<R>(wp2, g.nu[off + k], g.dt, g.dz, g.scheme);
        En = g.jdelta ? e_update_plasma(Eo, Po, curl, c) : e_update_plasma_q(Eo, Po, curl, c);
    } else {
        En = e_update_vac<R>(Eo, curl, (R)g.ce);
    }
    if (k == g.src[b])
        En = add_source<R>(En, source_value((double)m * g.dt, g.src_tau, g.src_t0, g.src_amp));
    if (write) {
        double Pn = 0.0;
        if (wp2 != 0.0) {
            if constexpr (sizeof(R) == 4) {
                Pn = (double)j_update_delta((float)Po, Eo, En, c.a, c.b1, c.b2);
            } else {
                Pn = q_update<R>(Po, (double)Eo, c);
            }
        }
        s.J[nxt][off + k] = Pn;
    }
    return En;
}

// E^{n+1}, J^{n+1}, ends and probe samples of node k, in registers of type R.
template <typename T, typename R>
__device__ __forceinline__ R step_e_val(const Grids &g, const State<T> &s, int cur, int b, int64_t off, int64_t n,
                                        int64_t k, int64_t m)
{
    if (k == 0 || k == n - 1) {
        s.J[cur ^ 1][off + k] = 0.0;
        if (g.bc == 0) {  // first-order Mur: E0' = E1 + cm (E1' - E0)
            const int64_t kn = (k == 0) ? 1 : n - 2;
            const R Enb = step_interior<T, R>(g, s, cur, b, off, n, kn, m, false);
            const T *E = s.E[cur] + off;
            return (R)E[kn] + (R)g.cm * (Enb - (R)E[k]);
        }
        return (R)0;
    }
    return step_interior<T, R>(g, s, cur, b, off, n, k, m, true);
}

// E^{n+1}, J^{n+1}, ends and probe samples; reads buffer cur, writes nxt.
template <typename T>
__global__ void k_step_e(Grids g, State<T> s, int cur, int64_t total, int64_t m, int slot)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= total) return;
    const int b = grid_of(g, i);
    const int64_t off = g.off[b], n = g.n[b], k = i - off;
    if (k >= n) return;
    double Ed;   // E^{n+1} as the step computed it (before its rounding to T)
    if (sizeof(T) == 4 && g.jdelta)
        Ed = (double)step_e_val<T, float>(g, s, cur, b, off, n, k, m);
    else
        Ed = step_e_val<T, double>(g, s, cur, b, off, n, k, m);
    const T En = (T)Ed;
    s.E[cur ^ 1][off + k] = En;
    for (int p = 0; p < g.P; ++p)
        if (g.probe[(int64_t)b * g.P + p] == k)
            g.samp[((int64_t)b * g.P + p) * g.SB + slot] = (double)En;
}

template <typename T>
void launch_step(const Grids &g, State<T> &s, int cur, int64_t total, int64_t m, int slot,
                 hipStream_t st)
{
    const int bs = 256;
    const unsigned nb = (unsigned)((total + bs - 1) / bs);
    hipLaunchKernelGGL(k_step_h<T>, dim3(nb), dim3(bs), 0, st, g, s, cur, total);
    hipLaunchKernelGGL(k_step_e<T>, dim3(nb), dim3(bs), 0, st, g, s, cur, total, m, slot);
}

template void launch_step<float>(const Grids &, State<float> &, int, int64_t, int64_t, int,
                                 hipStream_t);
template void launch_step<double>(const Grids &, State<double> &, int, int64_t, int64_t, int,
                                  hipStream_t);

// ------------------------------------------------------------------- DFT

// tw[i][f] = dt e^{-j 2 pi f (m_first + i) dt} for i < count.
__global__ void k_dft_twiddle(const double *freqs, int F, int64_t m_first, int count, double dt,
                              double2 *tw)
{
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= (int64_t)count * F) return;
    const int i = (int)(t / F), f = (int)(t % F);
    double re, im;
    twiddle(freqs[f] * dt, dt, m_first + i, re, im);
    tw[t] = make_double2(re, im);
}

// X[row][f] += sum_i samp[row][i] tw[i][f] over the window's samples, each
// sum in sample order (deterministic: step(a) + step(b) folds the same
// windows as step(a + b)).  A 1024-thread workgroup takes kDftRows rows and a
// group of 64 frequencies: the twiddles of kDftSamp samples at a time are
// staged in LDS once for all its rows, wave w owns row w of the block, lane l
// frequency l of the group (coalesced twiddle reads, the sample a scalar load
// shared by the wave).
constexpr int kDftRows = 16, kDftSamp = 64;

__global__ __launch_bounds__(1024) void k_dft_accum(const double *samp, int SB, int64_t rows, int F, int count,
                                                    const double2 *tw, double2 *X)
{
    __shared__ double2 ltw[kDftSamp][64];
    const int lane = threadIdx.x & 63;
    const int w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int ngroups = (F + 63) / 64;
    const int64_t rb = blockIdx.x / ngroups;
    const int fg = blockIdx.x % ngroups;
    const int64_t row = rb * kDftRows + w;
    const int f = fg * 64 + lane;
    const bool active = row < rows && f < F;
    const double *sp = samp + (row < rows ? row : 0) * (int64_t)SB;
    double ar = 0.0, ai = 0.0;
    for (int c0 = 0; c0 < count; c0 += kDftSamp) {
        const int cn = count - c0 < kDftSamp ? count - c0 : kDftSamp;
        __syncthreads();   // the previous chunk's reads are done
        for (int e = threadIdx.x; e < cn * 64; e += 1024) {
            const int i = e >> 6, ff = fg * 64 + (e & 63);
            ltw[i][e & 63] = ff < F ? tw[(int64_t)(c0 + i) * F + ff] : make_double2(0.0, 0.0);
        }
        __syncthreads();
        if (row < rows) {
            for (int i = 0; i < cn; ++i) {
                const double v = sp[c0 + i];
                const double2 t = ltw[i][lane];
                ar = fmat(v, t.x, ar);
                ai = fmat(v, t.y, ai);
            }
        }
    }
    if (active) {
        double2 x = X[row * F + f];
        x.x += ar;
        x.y += ai;
        X[row * F + f] = x;
    }
}

void launch_dft(const Grids &g, const double *freqs, int F, int64_t m_first, int count,
                double2 *tw, double2 *X, int64_t rows, hipStream_t st)
{
    // twiddles for at most kTwiddleChunk samples at a time
    const int64_t blocks = (rows + kDftRows - 1) / kDftRows * ((F + 63) / 64);
    for (int c0 = 0; c0 < count; c0 += kTwiddleChunk) {
        const int cnt = count - c0 < kTwiddleChunk ? count - c0 : kTwiddleChunk;
        const int64_t tot = (int64_t)cnt * F;
        hipLaunchKernelGGL(k_dft_twiddle, dim3((unsigned)((tot + 255) / 256)), dim3(256), 0, st,
                           freqs, F, m_first + c0, cnt, g.dt, tw);
        hipLaunchKernelGGL(k_dft_accum, dim3((unsigned)blocks), dim3(1024), 0, st, (const double *)(g.samp + c0),
                           g.SB, rows, F, cnt, (const double2 *)tw, X);
    }
}

// ----------------------------------------------------------------- setup

__global__ void k_fill(uint4 *p, int64_t n16)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t j = i; j < n16; j += stride) p[j] = make_uint4(0, 0, 0, 0);
}

// Zero fill with a kernel (a graph-safe replacement for memset); bytes is a
// multiple of 16 and p 16-byte aligned.
void launch_fill(void *p, int64_t bytes, hipStream_t st)
{
    const int64_t n16 = bytes / 16;
    if (n16 <= 0) return;
    int64_t nb = (n16 + 255) / 256;
    if (nb > 65536) nb = 65536;
    hipLaunchKernelGGL(k_fill, dim3((unsigned)nb), dim3(256), 0, st, (uint4 *)p, n16);
}

__global__ void k_src_table(Grids g, int64_t m_first, int count, double *srcv)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= count) return;
    srcv[i] = source_value((double)(m_first + i) * g.dt, g.src_tau, g.src_t0, g.src_amp);
}

void launch_src_table(const Grids &g, int64_t m_first, int count, double *srcv, hipStream_t st)
{
    if (count <= 0) return;
    hipLaunchKernelGGL(k_src_table, dim3((unsigned)((count + 255) / 256)), dim3(256), 0, st, g, m_first, count,
                       srcv);
}

__global__ void k_cpml_table(double *tab, int P, double m, double smax, double dt)
{
    const int j = blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= P) return;
    double b, a;
    cpml_ab((double)(j + 1), P, m, smax, dt, b, a);   // E node at depth j+1
    tab[j] = b;
    tab[P + j] = a;
    cpml_ab((double)j + 0.5, P, m, smax, dt, b, a);   // H node at depth j+1/2
    tab[2 * P + j] = b;
    tab[3 * P + j] = a;
}

void launch_cpml_table(double *tab, int P, double m, double smax, double dt, hipStream_t st)
{
    hipLaunchKernelGGL(k_cpml_table, dim3((P + 63) / 64), dim3(64), 0, st, tab, P, m, smax, dt);
}

// The step coefficients every register tile of a plasma class loads instead of
// rebuilding them from wp2 and nu at each launch (node_coef_t<double>, the
// values the tiles computed themselves, so every executor keeps its bits):
// SoA [4][total] of eP, -CH (held negated, as the tiles use it), a, qc.
__global__ void k_coef1d(Grids g, int64_t total, double *coef)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= total) return;
    const NodeCoef<double> c = node_coef_t<double>(g.wp2[i], g.nu[i], g.dt, g.dz, g.scheme);
    coef[i] = c.eP;
    coef[total + i] = -c.eH;
    coef[2 * total + i] = c.a;
    coef[3 * total + i] = c.qc;
}

void launch_coef1d(const Grids &g, int64_t total, double *coef, hipStream_t st)
{
    if (total > 0)
        hipLaunchKernelGGL(k_coef1d, dim3((unsigned)((total + 255) / 256)), dim3(256), 0, st, g, total, coef);
}

}  // namespace fdtdp
