// 2D Yee-RKETD kernels for gfx950 (TM: Ez, Hx, Hy; TE: Ex, Ey, Hz), one thread
// a cell, fields updated in place: an H pass (reads E only) then an E/J pass
// (reads H only, each cell its own E and J), so no pass reads a value another
// thread of the same pass writes.  Workgroups of 64 (j, the contiguous axis)
// x 4 (i) cells, dealt so that each XCD takes a contiguous band of rows.
// Arithmetic in FP64 registers at either storage precision; the per-node
// coefficients of eqs.(11)+(12) come from the 1D library (physics.h).
#include <hip/hip_runtime.h>

#include "internal2d.h"
#include "tile1d.h"

namespace fdtdp {

template <typename T>
__device__ __forceinline__ double ld(const T *a, const Grid2 &g, int64_t i, int64_t j)
{
    // field at (i, j): wrapped on a periodic axis, zero outside a walled one
    if (i < 0 || i >= g.nx) {
        if (!g.px) return 0.0;
        i = i < 0 ? i + g.nx : i - g.nx;
    }
    if (j < 0 || j >= g.ny) {
        if (!g.py) return 0.0;
        j = j < 0 ? j + g.ny : j - g.ny;
    }
    return (double)a[i * g.ny + j];
}

__device__ __forceinline__ bool cell_of(const Grid2 &g, int64_t &i, int64_t &j)
{
    const int64_t bj_n = (g.ny + 63) / 64, bi_n = (g.nx + 3) / 4;
    const int64_t b = xcd_block((int64_t)blockIdx.x, bj_n * bi_n);
    i = (b / bj_n) * 4 + (threadIdx.x >> 6);
    j = (b % bj_n) * 64 + (threadIdx.x & 63);
    return i < g.nx && j < g.ny;
}

// H^{n+1/2} from E^n (eq.(14)).
template <typename T, int MODE>
__global__ __launch_bounds__(256) void k2_h(Grid2 g, Fields2<T> f)
{
    int64_t i, j;
    if (!cell_of(g, i, j)) return;
    const int64_t k = i * g.ny + j;
    const double ch = g.ch;
    if constexpr (MODE == 0) {
        const T *Ez = f.E[0];
        const double e = (double)Ez[k];
        f.H[0][k] = (T)__builtin_fma(-ch, ld(Ez, g, i, j + 1) - e, (double)f.H[0][k]);
        f.H[1][k] = (T)__builtin_fma(ch, ld(Ez, g, i + 1, j) - e, (double)f.H[1][k]);
    } else {
        const T *Ex = f.E[0], *Ey = f.E[1];
        const double curl = (ld(Ey, g, i + 1, j) - (double)Ey[k]) - (ld(Ex, g, i, j + 1) - (double)Ex[k]);
        f.H[0][k] = (T)__builtin_fma(-ch, curl, (double)f.H[0][k]);
    }
}

// One E component of a cell: eqs.(11)+(12) solved, the source, the wall, then
// eq.(11); the current and the plasma parameters live on the compact support.
template <typename T>
__device__ __forceinline__ void e_cell(const Grid2 &g, int c, T *Ep, int64_t k, double curl_signed, bool src,
                                       double sv, bool wall, int64_t pidx)
{
    const double Eo = (double)Ep[k];
    double En, J = 0.0;
    Coef cf;
    const bool plasma = pidx >= 0 && g.wp2[c][pidx] != 0.0;
    if (plasma) {
        cf = node_coef(g.wp2[c][pidx], g.nu[c][pidx], g.dt, g.d, 0);
        J = g.J[c][pidx];
        En = __builtin_fma(cf.CH, curl_signed, __builtin_fma(-cf.CJ, J, cf.CA * Eo));
    } else {
        En = __builtin_fma(g.ce, curl_signed, Eo);
    }
    if (src) En = En + sv;
    if (wall) En = 0.0;
    if (plasma) g.J[c][pidx] = __builtin_fma(cf.b2, En, __builtin_fma(cf.b1, Eo, cf.a * J));
    Ep[k] = (T)En;
}

// E^{n+1} and J^{n+1} from H^{n+1/2}; m = n + 1 (the source time).
template <typename T, int MODE>
__global__ __launch_bounds__(256) void k2_e(Grid2 g, Fields2<T> f, int64_t m)
{
    int64_t i, j;
    if (!cell_of(g, i, j)) return;
    const int64_t k = i * g.ny + j;
    const int2 sp = g.span[i];
    const int64_t pidx = (j >= sp.x && j < sp.y) ? g.rowoff[i] + (j - sp.x) : -1;
    const bool src = g.has_src && i == g.si && j == g.sj;
    const double sv = src ? source_value((double)m * g.dt, g.src_tau, g.src_t0, g.src_amp) : 0.0;
    if constexpr (MODE == 0) {
        const T *Hx = f.H[0], *Hy = f.H[1];
        const double curl = ((double)Hy[k] - ld(Hy, g, i - 1, j)) - ((double)Hx[k] - ld(Hx, g, i, j - 1));
        const bool wall = (!g.px && i == 0) || (!g.py && j == 0);
        e_cell<T>(g, 0, f.E[0], k, curl, src, sv, wall, pidx);
    } else {
        const T *Hz = f.H[0];
        const double hz = (double)Hz[k];
        e_cell<T>(g, 0, f.E[0], k, hz - ld(Hz, g, i, j - 1), false, 0.0, !g.py && j == 0, pidx);
        e_cell<T>(g, 1, f.E[1], k, -(hz - ld(Hz, g, i - 1, j)), src, sv, !g.px && i == 0, pidx);
    }
}

// Probe samples of the step just taken into slot `slot` of the window.
template <typename T>
__global__ void k2_sample(Grid2 g, Fields2<T> f, int slot)
{
    const int p = threadIdx.x + blockIdx.x * blockDim.x;
    if (p >= g.P) return;
    const int64_t *q = g.probes + 3 * p;
    g.samp[(int64_t)p * g.SB + slot] = (double)f.E[q[0]][q[1] * g.ny + q[2]];
}

template <typename T>
void launch_step2d(const Grid2 &g, const Fields2<T> &f, int64_t m, int slot, hipStream_t st)
{
    const int64_t blocks = ((g.ny + 63) / 64) * ((g.nx + 3) / 4);
    if (g.mode == 0) {
        hipLaunchKernelGGL((k2_h<T, 0>), dim3((unsigned)blocks), dim3(256), 0, st, g, f);
        hipLaunchKernelGGL((k2_e<T, 0>), dim3((unsigned)blocks), dim3(256), 0, st, g, f, m);
    } else {
        hipLaunchKernelGGL((k2_h<T, 1>), dim3((unsigned)blocks), dim3(256), 0, st, g, f);
        hipLaunchKernelGGL((k2_e<T, 1>), dim3((unsigned)blocks), dim3(256), 0, st, g, f, m);
    }
    if (g.P > 0)
        hipLaunchKernelGGL((k2_sample<T>), dim3((unsigned)((g.P + 63) / 64)), dim3(64), 0, st, g, f, slot);
}

template void launch_step2d<float>(const Grid2 &, const Fields2<float> &, int64_t, int, hipStream_t);
template void launch_step2d<double>(const Grid2 &, const Fields2<double> &, int64_t, int, hipStream_t);

}  // namespace fdtdp
