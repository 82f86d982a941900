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

// A neighbour of cell k = i ny + j one step along an axis: its index (wrapped
// on a periodic axis) and whether it exists (false beyond a wall, where the
// field reads as zero).  The index is always one to load from (the cell itself
// where the neighbour is absent), so every neighbour load is issued
// unconditionally, beside the others, and no load waits on a branch.
struct Nb {
    int64_t k;
    bool ok;
};
__device__ __forceinline__ Nb nb_jp(const Grid2 &g, int64_t k, int64_t j)
{
    const bool in = j + 1 < g.ny;
    return {in ? k + 1 : (g.py ? k - (g.ny - 1) : k), in || g.py};
}
__device__ __forceinline__ Nb nb_jm(const Grid2 &g, int64_t k, int64_t j)
{
    const bool in = j > 0;
    return {in ? k - 1 : (g.py ? k + (g.ny - 1) : k), in || g.py};
}
__device__ __forceinline__ Nb nb_ip(const Grid2 &g, int64_t k, int64_t i)
{
    const bool in = i + 1 < g.nx;
    return {in ? k + g.ny : (g.px ? k - (g.nx - 1) * g.ny : k), in || g.px};
}
__device__ __forceinline__ Nb nb_im(const Grid2 &g, int64_t k, int64_t i)
{
    const bool in = i > 0;
    return {in ? k - g.ny : (g.px ? k + (g.nx - 1) * g.ny : k), in || g.px};
}
template <typename T>
__device__ __forceinline__ double ldn(const T *a, const Nb &n)
{
    const double v = (double)a[n.k];
    return n.ok ? v : 0.0;
}

// The cell of this thread; i is the same for the whole wave (one row).
__device__ __forceinline__ bool cell_of(const Grid2 &g, int64_t &i, int64_t &j)
{
    const int64_t bj_n = (g.ny + 63) / 64, bi_n = (g.nx + 3) / 4;
    const int64_t b = xcd_block((int64_t)blockIdx.x, bj_n * bi_n);
    i = (b / bj_n) * 4 + __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
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
    const Nb jp = nb_jp(g, k, j), ip = nb_ip(g, k, i);
    if constexpr (MODE == 0) {
        const T *Ez = f.E[0];
        const double e = (double)Ez[k], ej = ldn(Ez, jp), ei = ldn(Ez, ip);
        const double hx = (double)f.H[0][k], hy = (double)f.H[1][k];
        f.H[0][k] = (T)__builtin_fma(-ch, ej - e, hx);
        f.H[1][k] = (T)__builtin_fma(ch, ei - e, hy);
    } else {
        const T *Ex = f.E[0], *Ey = f.E[1];
        const double eyi = ldn(Ey, ip), exj = ldn(Ex, jp), hz = (double)f.H[0][k];
        const double curl = (eyi - (double)Ey[k]) - (exj - (double)Ex[k]);
        f.H[0][k] = (T)__builtin_fma(-ch, curl, hz);
    }
}

// One E component of a cell: eqs.(11)+(12) solved, the source, the wall, then
// eq.(11); the current and the plasma parameters live on the compact support
// (index pidx, or -1 off it) and come in already read (w, v, J: wp2, nu, J^n).
template <typename T>
__device__ __forceinline__ void e_cell(const Grid2 &g, int c, T *Ep, int64_t k, double Eo, double curl_signed,
                                       bool src, double sv, bool wall, int64_t pidx, double w, double v, double J)
{
    double En;
    Coef cf;
    const bool plasma = pidx >= 0 && w != 0.0;
    if (plasma) {
        cf = node_coef(w, v, g.dt, g.d, 0);
        En = __builtin_fma(cf.CH, curl_signed, __builtin_fma(-cf.CJ, J, cf.CA * Eo));
    } else {
        En = __builtin_fma(g.ce, curl_signed, Eo);
    }
    if (src) En = En + sv;
    if (wall) En = 0.0;
    if (plasma) g.J[c][pidx] = __builtin_fma(cf.b2, En, __builtin_fma(cf.b1, Eo, cf.a * J));
    Ep[k] = (T)En;
}

// E^{n+1} and J^{n+1} from H^{n+1/2}; m = n + 1 (the source time).  Every load
// a cell needs (H and its neighbours, E, and on the support wp2, nu and J) is
// issued before any arithmetic, so a wave waits on one round of loads.
template <typename T, int MODE>
__global__ __launch_bounds__(256) void k2_e(Grid2 g, Fields2<T> f, int64_t m)
{
    constexpr int NC = MODE == 0 ? 1 : 2;
    int64_t i, j;
    if (!cell_of(g, i, j)) return;
    const int64_t k = i * g.ny + j;
    const int2 sp = g.span[i];                      // the row's support (i is wave-uniform)
    const int64_t ro = g.rowoff[i];
    const int64_t pidx = (j >= sp.x && j < sp.y) ? ro + (j - sp.x) : -1;
    const Nb jm = nb_jm(g, k, j), im = nb_im(g, k, i);
    double Eo[NC], w[NC], v[NC], J[NC];
#pragma unroll
    for (int c = 0; c < NC; ++c) {
        Eo[c] = (double)f.E[c][k];
        w[c] = v[c] = J[c] = 0.0;
    }
    double curl[NC];
    if constexpr (MODE == 0) {
        const T *Hx = f.H[0], *Hy = f.H[1];
        const double hy = (double)Hy[k], hyi = ldn(Hy, im), hx = (double)Hx[k], hxj = ldn(Hx, jm);
        curl[0] = (hy - hyi) - (hx - hxj);
    } else {
        const T *Hz = f.H[0];
        const double hz = (double)Hz[k], hzj = ldn(Hz, jm), hzi = ldn(Hz, im);
        curl[0] = hz - hzj;
        curl[1] = -(hz - hzi);
    }
    if (pidx >= 0) {
#pragma unroll
        for (int c = 0; c < NC; ++c) {
            w[c] = g.wp2[c][pidx];
            v[c] = g.nu[c][pidx];
            J[c] = g.J[c][pidx];
        }
    }
    const bool src = g.has_src && i == g.si && j == g.sj;
    const double sv = src ? source_value((double)m * g.dt, g.src_tau, g.src_t0, g.src_amp) : 0.0;
    if constexpr (MODE == 0) {
        const bool wall = (!g.px && i == 0) || (!g.py && j == 0);
        e_cell<T>(g, 0, f.E[0], k, Eo[0], curl[0], src, sv, wall, pidx, w[0], v[0], J[0]);
    } else {
        e_cell<T>(g, 0, f.E[0], k, Eo[0], curl[0], false, 0.0, !g.py && j == 0, pidx, w[0], v[0], J[0]);
        e_cell<T>(g, 1, f.E[1], k, Eo[1], curl[1], src, sv, !g.px && i == 0, pidx, w[1], v[1], J[1]);
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
