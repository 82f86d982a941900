// 3D Yee-RKETD kernels.  One time step is either
//   k_h3d   H^{n+1/2} from E^n (CPML auxiliaries, TF/SF H corrections fused)
//   k_aux3d the incident 1D grid (TF/SF only): H^{n+1/2}, E^{n+1}, source, Mur
//   k_e3d   E^{n+1} (CPML, TF/SF E corrections or the planar source, PEC walls)
//           and J^{n+1} on the plasma support, fused
// (two passes over the grid, in place), or k_aux3d + k_fused3d (one pass,
// E/H/CPML ping-pong); both call the same per-cell h_cell / e_cell and give
// identical bits.  Then
//   k_sample3d  the sample points into the current slot of the sample buffer
// and every `slots` steps k_tw3d + k_flush3d fold the buffered samples into the
// FP64 DFT accumulators.
//
// The update formulas are the 1D library's per-node physics (physics.h): H by
// one FMA per component, E in vacuum by one FMA, plasma E by the solved
// eqs.(11)+(12) (FP32: delta form around CA - 1), J by eq.(11) in FP64.
#include <hip/hip_runtime.h>

#include "internal3d.h"

namespace fdtdp {

namespace {

// Consecutive logical blocks on one XCD: the hardware deals workgroups to the
// 8 XCDs round-robin, so hardware block b runs on XCD b % 8; give that XCD the
// b / 8-th block of its own contiguous chunk.  Neighbouring i-planes then share
// an L2.
__device__ __forceinline__ int64_t xcd_chunk(int64_t bid, int64_t nblk)
{
    const int64_t q = nblk / 8, r = nblk % 8;
    const int64_t x = bid % 8, j = bid / 8;
    return x * q + (x < r ? x : r) + j;
}

// Cells of a split-kernel workgroup: 64 consecutive k (one wave) x 4 rows j
// x a run of g.np planes i that each thread walks.  i and j are the
// same for the whole wave (kept in scalar registers).
struct Col {
    int64_t i0, i1, j, k;
    bool ok;
};

__device__ __forceinline__ Col col_of(const Geo3 &g)
{
    Col c;
    const int64_t bid = xcd_chunk(blockIdx.x, gridDim.x);
    const int64_t kq = bid % g.kb, r = bid / g.kb;
    const int w = __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
    c.j = (r % g.jb) * 4 + w;
    c.i0 = (r / g.jb) * g.np;
    c.i1 = c.i0 + g.np < g.nx ? c.i0 + g.np : g.nx;
    c.k = kq * 64 + (threadIdx.x & 63);
    c.ok = c.j < g.ny && c.k < g.nz;
    return c;
}

// slab index of node n on an axis of `len` nodes with P-node layers, or -1
__device__ __forceinline__ int64_t slab(int64_t n, int64_t len, int P)
{
    if (n < P) return n;
    if (n >= len - P) return n - (len - 2 * P);
    return -1;
}

// psi' = b psi + a dF (separately rounded, as written), stored only by the
// cell's owner; returns dF + psi'
template <typename T>
__device__ __forceinline__ T cpml_term(const T *pin, T *pout, int64_t idx, T b, T a, T dF, bool store)
{
    const T v = b * pin[idx] + a * dF;
    if (store) pout[idx] = v;
    return dF + v;
}

}  // namespace

// H^{n+1/2} of cell (i, j, k) from its E^n and the E^n of its +1 neighbours
// (zero beyond a wall); hx, hy, hz hold H^{n-1/2} on entry.  CPML auxiliaries
// and the TF/SF correction (Einc^n) included.  Shared by both executors.
template <typename T>
__device__ __forceinline__ void h_cell(const Geo3 &g, const Cpml3<T> &c, const double *Einc, int64_t i,
                                       int64_t j, int64_t k, T ex, T ey, T ez, T ex_j, T ex_k, T ey_i,
                                       T ey_k, T ez_i, T ez_j, T &hx, T &hy, T &hz, bool store)
{
    T dEz_y = ez_j - ez;
    T dEy_z = ey_k - ey;
    T dEx_z = ex_k - ex;
    T dEz_x = ez_i - ez;
    T dEy_x = ey_i - ey;
    T dEx_y = ex_j - ex;
    if (g.P > 0) {
        const int P = g.P, P2 = 2 * g.P;
        if (!g.px) {
            const int64_t s = slab(i, g.nx, P);
            if (s >= 0) {
                const int64_t id = (s * g.ny + j) * g.nz + k;
                const T b = c.tab[(0 * 4 + 2) * P2 + s], a = c.tab[(0 * 4 + 3) * P2 + s];
                dEz_x = cpml_term(c.inH[0][0], c.outH[0][0], id, b, a, dEz_x, store);
                dEy_x = cpml_term(c.inH[0][1], c.outH[0][1], id, b, a, dEy_x, store);
            }
        }
        if (!g.py) {
            const int64_t s = slab(j, g.ny, P);
            if (s >= 0) {
                const int64_t id = (i * P2 + s) * g.nz + k;
                const T b = c.tab[(1 * 4 + 2) * P2 + s], a = c.tab[(1 * 4 + 3) * P2 + s];
                dEz_y = cpml_term(c.inH[1][0], c.outH[1][0], id, b, a, dEz_y, store);
                dEx_y = cpml_term(c.inH[1][1], c.outH[1][1], id, b, a, dEx_y, store);
            }
        }
        const int64_t s = slab(k, g.nz, P);
        if (s >= 0) {
            const int64_t id = (i * g.ny + j) * P2 + s;
            const T b = c.tab[(2 * 4 + 2) * P2 + s], a = c.tab[(2 * 4 + 3) * P2 + s];
            dEy_z = cpml_term(c.inH[2][0], c.outH[2][0], id, b, a, dEy_z, store);
            dEx_z = cpml_term(c.inH[2][1], c.outH[2][1], id, b, a, dEx_z, store);
        }
    }
    const T ch = (T)g.chd;
    hx = fmat(-ch, dEz_y - dEy_z, hx);
    hy = fmat(-ch, dEx_z - dEz_x, hy);
    hz = fmat(-ch, dEy_x - dEx_y, hz);
    if (g.src == 2) {
        // scattered H beside the box reads total Ex across a face: remove the
        // incident part (Einc^n).  Hy(k+1/2) at k = b0-1 and b1; Hz(j+1/2) at
        // j = b0-1 and b1 (walled y), with the minus sign of dEx/dy in curl_z.
        const bool inx = i >= g.xlo && i < g.xhi;
        if (inx && j >= g.ylo && j < g.yhi) {
            if (k == g.b0 - 1) hy = hy + (T)(g.chd * Einc[g.b0 + g.ao]);
            else if (k == g.b1) hy = hy - (T)(g.chd * Einc[g.b1 + g.ao]);
        }
        if (!g.py && inx && k >= g.b0 && k <= g.b1) {
            if (j == g.b0 - 1) hz = hz - (T)(g.chd * Einc[k + g.ao]);
            else if (j == g.b1) hz = hz + (T)(g.chd * Einc[k + g.ao]);
        }
    }
}

template <typename T>
__device__ __forceinline__ NodeCoef<T> coef_at(const Plasma3<T> &pl, int c, int64_t q)
{
    NodeCoef<T> r;
    r.eA = pl.eA[c][q];
    r.eJ = pl.eJ[c][q];
    r.eH = pl.eH[c][q];
    r.a = sizeof(T) == 8 ? (double)pl.ca[c][q] : 1.0 + (double)pl.ca[c][q];
    r.b1 = (double)pl.cb1[c][q];
    r.b2 = (double)pl.cb2[c][q];
    return r;
}

// Coefficient tables of the plasma support (once per create): node_coef of
// physics.h per node and component.
template <typename T>
__global__ void k_coef3d(const double *w0, const double *w1, const double *w2, const double *n0,
                         const double *n1, const double *n2, int64_t S, double dt, double d, T *eA0, T *eA1,
                         T *eA2, T *eJ0, T *eJ1, T *eJ2, T *eH0, T *eH1, T *eH2, T *a0, T *a1, T *a2,
                         T *b10, T *b11, T *b12, T *b20, T *b21, T *b22)
{
    const int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (q >= S) return;
    const double *w[3] = {w0, w1, w2}, *n[3] = {n0, n1, n2};
    T *eA[3] = {eA0, eA1, eA2}, *eJ[3] = {eJ0, eJ1, eJ2}, *eH[3] = {eH0, eH1, eH2};
    T *a[3] = {a0, a1, a2}, *b1[3] = {b10, b11, b12}, *b2[3] = {b20, b21, b22};
#pragma unroll
    for (int c = 0; c < 3; ++c) {
        const NodeCoef<T> r = node_coef_t<T>(w[c][q], n[c][q], dt, d, 0);
        eA[c][q] = r.eA;
        eJ[c][q] = r.eJ;
        eH[c][q] = r.eH;
        a[c][q] = sizeof(T) == 8 ? (T)r.a : (T)(r.a - 1.0);   // a in [1/2, 1]: a - 1 exact
        b1[c][q] = (T)r.b1;
        b2[c][q] = (T)r.b2;
    }
}

// The plasma terms of one cell, read before its E update (with its field
// values, so that no load waits on another): whether the cell is on the
// support, its compact index, J^n and the stored coefficients of the three
// components.  sp, off: the span and offset of the cell's row.
template <typename T>
struct PNode {
    bool on;
    int64_t cq;
    T J[3];
    NodeCoef<T> cf[3];
};

template <typename T>
__device__ __forceinline__ PNode<T> pnode_load(const Plasma3<T> &pl, int2 sp, int64_t off, int64_t k)
{
    PNode<T> n;
    n.on = k >= sp.x && k < sp.y;
    n.cq = off + (k - sp.x);
    if (n.on) {
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            n.J[c] = pl.J[c][n.cq];
            n.cf[c] = coef_at(pl, c, n.cq);
        }
    }
    return n;
}

// E update with the 3D curl sign: E_new = CA E - CJ J + CH curl.
__device__ __forceinline__ double e_plasma3(double E, double J, double curl, const NodeCoef<double> &c)
{
    return fmat(c.eH, curl, fmat(-c.eJ, J, c.eA * E));
}
__device__ __forceinline__ float e_plasma3(float E, float J, float curl, const NodeCoef<float> &c)
{
    return fmat(c.eH, curl, fmat(-c.eJ, J, fmat(c.eA, E, E)));
}

// The corrections of E component C after its update: TF/SF (the total E on
// a box face reads scattered H outside it, so it gains the incident part
// Hinc^{n+1/2} times its CH; Ex at k = b0, b1, Ez at i = b0, b1 of a walled
// x) or the planar source, then PEC (tangential E on the index-0 faces of the
// walled axes).
template <int C, typename T>
__device__ __forceinline__ T e_fix(const Geo3 &g, const double *Hinc, double sval, int64_t i, int64_t j,
                                   int64_t k, double CH, T e)
{
    if (g.src == 2) {
        if constexpr (C == 0) {
            if (i >= g.xlo && i < g.xhi && j >= g.ylo && j < g.yhi) {
                if (k == g.b0) e = e + (T)(CH * Hinc[g.b0 - 1 + g.ao]);
                else if (k == g.b1) e = e - (T)(CH * Hinc[g.b1 + g.ao]);
            }
        }
        if constexpr (C == 2) {
            if (!g.px && j >= g.ylo && j < g.yhi && k >= g.b0 && k < g.b1) {
                if (i == g.b0) e = e - (T)(CH * Hinc[k + g.ao]);
                else if (i == g.b1) e = e + (T)(CH * Hinc[k + g.ao]);
            }
        }
    } else if (g.src == 1 && k == g.src_k && g.src_comp == C) {
        e = add_source(e, sval);
    }
    const bool wx = !g.px && i == 0, wy = !g.py && j == 0, wz = k == 0;
    if ((C == 0 && (wy || wz)) || (C == 1 && (wx || wz)) || (C == 2 && (wx || wy))) e = (T)0;
    return e;
}

// E component C of a plasma node: the E update with its coefficients, the
// corrections, then J^{n+1} in place.
template <int C, typename T>
__device__ __forceinline__ T e_plasma_comp(const Geo3 &g, const Plasma3<T> &pl, const PNode<T> &pn,
                                           const double *Hinc, double sval, int64_t i, int64_t j, int64_t k,
                                           T curl, T eo)
{
    const NodeCoef<T> &cf = pn.cf[C];
    const T J = pn.J[C];
    const T e = e_fix<C>(g, Hinc, sval, i, j, k, (double)cf.eH, e_plasma3(eo, J, curl, cf));
    pl.J[C][pn.cq] = (T)j_update<T>((double)J, (double)eo, (double)e, cf);
    return e;
}

// E^{n+1} of cell (i, j, k) from its H^{n+1/2} and the H^{n+1/2} of its -1
// neighbours (zero beyond a wall); e0..e2 hold E^n on entry.  CPML, TF/SF (or
// the planar source), PEC walls and, on the plasma support (pn, read by the
// caller), J^{n+1} (written in place).  Shared by both executors.
template <typename T>
__device__ __forceinline__ void e_cell(const Geo3 &g, const Plasma3<T> &pl, const PNode<T> &pn,
                                       const Cpml3<T> &c, const double *Hinc, double sval, int64_t i, int64_t j, int64_t k,
                                       T hx, T hy, T hz, T hx_j, T hx_k, T hy_i, T hy_k, T hz_i, T hz_j,
                                       T &e0, T &e1, T &e2)
{
    T dHz_y = hz - hz_j;
    T dHy_z = hy - hy_k;
    T dHx_z = hx - hx_k;
    T dHz_x = hz - hz_i;
    T dHy_x = hy - hy_i;
    T dHx_y = hx - hx_j;
    if (g.P > 0) {
        const int P = g.P, P2 = 2 * g.P;
        if (!g.px) {
            const int64_t s = slab(i, g.nx, P);
            if (s >= 0) {
                const int64_t id = (s * g.ny + j) * g.nz + k;
                const T b = c.tab[(0 * 4 + 0) * P2 + s], a = c.tab[(0 * 4 + 1) * P2 + s];
                dHz_x = cpml_term(c.inE[0][0], c.outE[0][0], id, b, a, dHz_x, true);
                dHy_x = cpml_term(c.inE[0][1], c.outE[0][1], id, b, a, dHy_x, true);
            }
        }
        if (!g.py) {
            const int64_t s = slab(j, g.ny, P);
            if (s >= 0) {
                const int64_t id = (i * P2 + s) * g.nz + k;
                const T b = c.tab[(1 * 4 + 0) * P2 + s], a = c.tab[(1 * 4 + 1) * P2 + s];
                dHz_y = cpml_term(c.inE[1][0], c.outE[1][0], id, b, a, dHz_y, true);
                dHx_y = cpml_term(c.inE[1][1], c.outE[1][1], id, b, a, dHx_y, true);
            }
        }
        const int64_t s = slab(k, g.nz, P);
        if (s >= 0) {
            const int64_t id = (i * g.ny + j) * P2 + s;
            const T b = c.tab[(2 * 4 + 0) * P2 + s], a = c.tab[(2 * 4 + 1) * P2 + s];
            dHy_z = cpml_term(c.inE[2][0], c.outE[2][0], id, b, a, dHy_z, true);
            dHx_z = cpml_term(c.inE[2][1], c.outE[2][1], id, b, a, dHx_z, true);
        }
    }
    const T curl0 = dHz_y - dHy_z, curl1 = dHx_z - dHz_x, curl2 = dHy_x - dHx_y;
    if (!pn.on) {
        const T ce = (T)g.ced;
        e0 = e_fix<0>(g, Hinc, sval, i, j, k, g.ced, fmat(ce, curl0, e0));
        e1 = e_fix<1>(g, Hinc, sval, i, j, k, g.ced, fmat(ce, curl1, e1));
        e2 = e_fix<2>(g, Hinc, sval, i, j, k, g.ced, fmat(ce, curl2, e2));
    } else {
        e0 = e_plasma_comp<0>(g, pl, pn, Hinc, sval, i, j, k, curl0, e0);
        e1 = e_plasma_comp<1>(g, pl, pn, Hinc, sval, i, j, k, curl1, e1);
        e2 = e_plasma_comp<2>(g, pl, pn, Hinc, sval, i, j, k, curl2, e2);
    }
}

// ---- two-kernel step (in place) --------------------------------------------
//
// Each thread walks g.np planes along x for one (j, k): the x
// neighbour it loads for plane i is its own value at plane i+1 (H kernel) or
// was its own value at plane i-1 (E kernel), so it is read once.

template <typename T>
__global__ __launch_bounds__(256) void k_h3d(Geo3 g, Fields3<T> f, Cpml3<T> c, const double *Einc)
{
    const Col q = col_of(g);
    if (!q.ok) return;
    const int64_t j = q.j, k = q.k;
    const int64_t sI = g.ny * g.nz, sJ = g.nz;
    const T *Ex = f.E[0], *Ey = f.E[1], *Ez = f.E[2];
    const bool hasj = g.py || j + 1 < g.ny, hask = k + 1 < g.nz;
    const int64_t dj = j + 1 < g.ny ? sJ : -j * sJ;       // +1 row, periodic wrap
    const int64_t dk = hask ? 1 : 0;
    const T zero = (T)0;
    int64_t p = (q.i0 * g.ny + j) * g.nz + k;
    T ex = Ex[p], ey = Ey[p], ez = Ez[p];
    for (int64_t i = q.i0; i < q.i1; ++i, p += sI) {
        // plane i+1: periodic wrap to plane 0, or zero beyond the wall
        const bool hasi = g.px || i + 1 < g.nx;
        const int64_t pn = i + 1 < g.nx ? p + sI : p - i * sI;
        const T ex1 = Ex[pn], ey1 = Ey[pn], ez1 = Ez[pn];
        const T ez_j = Ez[p + dj], ex_j = Ex[p + dj], ey_k = Ey[p + dk], ex_k = Ex[p + dk];
        T hx = f.H[0][p], hy = f.H[1][p], hz = f.H[2][p];
        h_cell<T>(g, c, Einc, i, j, k, ex, ey, ez, hasj ? ex_j : zero, hask ? ex_k : zero,
                  hasi ? ey1 : zero, hask ? ey_k : zero, hasi ? ez1 : zero, hasj ? ez_j : zero, hx, hy, hz, true);
        f.H[0][p] = hx;
        f.H[1][p] = hy;
        f.H[2][p] = hz;
        ex = ex1;
        ey = ey1;
        ez = ez1;
    }
}

template <typename T>
__global__ __launch_bounds__(256) void k_e3d(Geo3 g, Fields3<T> f, Plasma3<T> pl, Cpml3<T> c,
                                             const double *Hinc, double sval)
{
    const Col q = col_of(g);
    if (!q.ok) return;
    const int64_t j = q.j, k = q.k;
    const int64_t sI = g.ny * g.nz, sJ = g.nz;
    const T *Hx = f.H[0], *Hy = f.H[1], *Hz = f.H[2];
    const bool hasj = g.py || j > 0, hask = k > 0;
    const int64_t dj = j > 0 ? -sJ : (g.ny - 1) * sJ;       // -1 row, periodic wrap
    const int64_t dk = hask ? -1 : 0;
    const T zero = (T)0;
    int64_t p = (q.i0 * g.ny + j) * g.nz + k;
    // plane i0-1: periodic wrap to plane nx-1, or zero beyond the wall
    T hy_i = zero, hz_i = zero;
    if (q.i0 > 0 || g.px) {
        const int64_t pm = q.i0 > 0 ? p - sI : p + (g.nx - 1) * sI;
        hy_i = Hy[pm];
        hz_i = Hz[pm];
    }
    // the support span of the row, read one plane ahead
    int64_t row = q.i0 * g.ny + j;
    int2 sp = pl.span[row];
    int64_t of = pl.off[row];
    for (int64_t i = q.i0; i < q.i1; ++i, p += sI, row += g.ny) {
        int2 spn = sp;
        int64_t ofn = of;
        if (i + 1 < q.i1) {
            spn = pl.span[row + g.ny];
            ofn = pl.off[row + g.ny];
        }
        const T hx = Hx[p], hy = Hy[p], hz = Hz[p];
        const T hz_j = Hz[p + dj], hx_j = Hx[p + dj], hy_k = Hy[p + dk], hx_k = Hx[p + dk];
        T e0 = f.E[0][p], e1 = f.E[1][p], e2 = f.E[2][p];
        const PNode<T> pn = pnode_load(pl, sp, of, k);
        e_cell<T>(g, pl, pn, c, Hinc, sval, i, j, k, hx, hy, hz, hasj ? hx_j : zero, hask ? hx_k : zero, hy_i,
                  hask ? hy_k : zero, hz_i, hasj ? hz_j : zero, e0, e1, e2);
        f.E[0][p] = e0;
        f.E[1][p] = e1;
        f.E[2][p] = e2;
        hy_i = hy;
        hz_i = hz;
        sp = spn;
        of = ofn;
    }
}

// ---- fused step ---------------------------------------------------------------
//
// One wave owns 63 cells of a row, k0 .. k0+62 of row j, over a chunk of
// planes [i0, i1), and marches along x; its 64 lanes hold the cells
// k0-1 .. k0+62.  Per plane every lane computes H^{n+1/2} of its cell and,
// for the E update of its own cell, the Hx and Hz of the cell at j-1 (both
// from E^n and H^{n-1/2} read from the input copy, exactly as the owners of
// those cells compute them); the H at k-1 is the lane below's (a cross-lane
// move), which is why lane 0 holds the cell k0-1 and updates no E.  Then
// E^{n+1} and J^{n+1} of cells k0 .. k0+62 from that H and the H of the
// previous plane, kept in registers; the chunk starts one plane early (i0-1)
// for the H its first E plane needs.  E, H and the CPML auxiliaries are read
// from one copy and written to the other, so no wave reads a value another
// has already advanced and no wave waits on another (no barrier, no LDS).
// The loads of plane i+1 are issued before the arithmetic of plane i.  HBM
// traffic per cell: E and H read once and written once; the rim reads (rows
// j +- 1, the lane-0 column, the lead-in plane) are re-reads that hit L2.

__device__ __forceinline__ float lane_up1(float x)
{
    // lane l receives lane l-1's value, lane 0 receives 0 (DPP wave_shr:1,
    // zero written by the move itself)
    return __builtin_bit_cast(float, __builtin_amdgcn_mov_dpp(__builtin_bit_cast(int, x), 0x138, 0xF, 0xF, true));
}
__device__ __forceinline__ double lane_up1(double x)
{
    const int2 v = __builtin_bit_cast(int2, x);
    return __builtin_bit_cast(double, make_int2(__builtin_amdgcn_mov_dpp(v.x, 0x138, 0xF, 0xF, true),
                                                __builtin_amdgcn_mov_dpp(v.y, 0x138, 0xF, 0xF, true)));
}

// What one plane of a fused-kernel lane reads from the input copy.
template <typename T>
struct Plane3 {
    T e[3];        // E^n(i, j, k)
    T eyi, ezi;    // Ey, Ez at (i+1, j, k)
    T exj, ezj;    // Ex, Ez at (i, j+1, k)
    T exk, eyk;    // Ex, Ey at (i, j, k+1)
    T m[3];        // E^n(i, j-1, k)
    T myk, myi;    // Ey at (i, j-1, k+1) and (i+1, j-1, k)
    T h[3];        // H^{n-1/2}(i, j, k)
    T hmx, hmz;    // Hx, Hz at (i, j-1, k)
};

template <typename T>
__device__ __forceinline__ T ld_if(const T *a, int64_t p, bool ok)
{
    return ok ? a[p] : (T)0;
}

template <typename T>
__global__ __launch_bounds__(256) void k_fused3d(Geo3 g, Fields3<T> fin, Fields3<T> fout, Plasma3<T> pl,
                                                 Cpml3<T> c, const double *Einc, const double *Hinc,
                                                 double sval, int ni)
{
    const int lane = threadIdx.x & 63;
    const int64_t kbf = (g.nz + 62) / 63;
    const int64_t bid = xcd_chunk(blockIdx.x, gridDim.x);
    const int64_t kq = bid % kbf, r = bid / kbf;
    const int w = __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
    const int64_t j = (r % g.jb) * 4 + w;
    if (j >= g.ny) return;                           // the whole wave; no wave waits on another
    const int64_t i0 = (r / g.jb) * ni;
    const int64_t i1 = i0 + ni < g.nx ? i0 + ni : g.nx;
    const int64_t k = kq * 63 - 1 + lane;
    const bool vk = k >= 0 && k < g.nz;             // the lane's cell exists
    const bool own = vk && lane > 0;                 // and is this wave's
    const bool hasj = g.py || j + 1 < g.ny;          // row j+1 exists (wrapped if periodic)
    const bool hasjm = g.py || j > 0;                // row j-1 exists
    const int64_t jp = j + 1 < g.ny ? j + 1 : 0, jm = j > 0 ? j - 1 : g.ny - 1;
    const bool hask = k + 1 < g.nz;
    const T zero = (T)0;

    auto load = [&](int64_t gi, Plane3<T> &q) {
        const bool hasi = g.px || gi + 1 < g.nx;     // plane i+1 exists (wrapped if periodic)
        const int64_t gi1 = gi + 1 < g.nx ? gi + 1 : 0;
        const int64_t p = (gi * g.ny + j) * g.nz + k, p1 = (gi1 * g.ny + j) * g.nz + k;
        const int64_t pj = (gi * g.ny + jp) * g.nz + k, pm = (gi * g.ny + jm) * g.nz + k;
        const int64_t pm1 = (gi1 * g.ny + jm) * g.nz + k;
        const bool hm = vk && hasjm;
#pragma unroll
        for (int a = 0; a < 3; ++a) {
            q.e[a] = ld_if(fin.E[a], p, vk);
            q.m[a] = ld_if(fin.E[a], pm, hm);
            q.h[a] = ld_if(fin.H[a], p, vk);
        }
        q.eyi = ld_if(fin.E[1], p1, vk && hasi);
        q.ezi = ld_if(fin.E[2], p1, vk && hasi);
        q.exj = ld_if(fin.E[0], pj, vk && hasj);
        q.ezj = ld_if(fin.E[2], pj, vk && hasj);
        q.exk = ld_if(fin.E[0], p + 1, vk && hask);
        q.eyk = ld_if(fin.E[1], p + 1, vk && hask);
        q.myk = ld_if(fin.E[1], pm + 1, hm && hask);
        q.myi = ld_if(fin.E[1], pm1, hm && hasi);
        q.hmx = ld_if(fin.H[0], pm, hm);
        q.hmz = ld_if(fin.H[2], pm, hm);
    };
    auto wrap = [&](int64_t i) { return i < 0 ? i + g.nx : i; };

    // the lead-in plane i0-1: wrapped to nx-1 on a periodic x, absent at a wall
    int64_t i = (i0 > 0 || g.px) ? i0 - 1 : i0;
    T hy_i = zero, hz_i = zero;                      // H^{n+1/2} of the previous plane
    Plane3<T> cur, nxt;
    load(wrap(i), cur);
    int2 sp = pl.span[i0 * g.ny + j];                // support span of the next E plane's row
    int64_t of = pl.off[i0 * g.ny + j];
    for (; i < i1; ++i) {
        const int64_t gi = wrap(i);
        const bool lead = i < i0;
        // this plane's plasma terms first, then the next plane's fields: the
        // E update waits on neither the next plane's loads nor a chain of its own
        PNode<T> pn;
        pn.on = false;
        int2 spn = sp;
        int64_t ofn = of;
        if (!lead) {
            pn = pnode_load(pl, sp, of, k);
            if (i + 1 < i1) {
                spn = pl.span[(i + 1) * g.ny + j];
                ofn = pl.off[(i + 1) * g.ny + j];
            }
        }
        if (i + 1 < i1) load(i + 1, nxt);
        T hx = cur.h[0], hy = cur.h[1], hz = cur.h[2];
        if (vk)
            h_cell<T>(g, c, Einc, gi, j, k, cur.e[0], cur.e[1], cur.e[2], cur.exj, cur.exk, cur.eyi, cur.eyk,
                      cur.ezi, cur.ezj, hx, hy, hz, own && !lead);
        const T hxk = lane_up1(hx), hyk = lane_up1(hy);   // H at k-1
        if (own && !lead) {
            T mx = cur.hmx, my = zero, mz = cur.hmz;
            if (hasjm)
                h_cell<T>(g, c, Einc, gi, jm, k, cur.m[0], cur.m[1], cur.m[2], cur.e[0], zero, cur.myi, cur.myk,
                          zero, cur.e[2], mx, my, mz, false);
            T e0 = cur.e[0], e1 = cur.e[1], e2 = cur.e[2];
            const bool kin = k > 0;
            e_cell<T>(g, pl, pn, c, Hinc, sval, gi, j, k, hx, hy, hz, hasjm ? mx : zero, kin ? hxk : zero, hy_i,
                      kin ? hyk : zero, hz_i, hasjm ? mz : zero, e0, e1, e2);
            const int64_t p = (gi * g.ny + j) * g.nz + k;
            fout.H[0][p] = hx;
            fout.H[1][p] = hy;
            fout.H[2][p] = hz;
            fout.E[0][p] = e0;
            fout.E[1][p] = e1;
            fout.E[2][p] = e2;
        }
        hy_i = hy;
        hz_i = hz;
        cur = nxt;
        sp = spn;
        of = ofn;
    }
}

// Incident 1D vacuum grid, one workgroup: Hi from Ei_in, then Ei_out with the
// source and first-order Mur ends (which read the old end values).
__global__ __launch_bounds__(256) void k_aux3d(const double *Ei, double *Eo, double *Hi, int64_t na,
                                               int64_t src, double chd, double ced, double cm, double s)
{
    for (int64_t q = threadIdx.x; q < na - 1; q += blockDim.x) Hi[q] = Hi[q] - chd * (Ei[q + 1] - Ei[q]);
    __syncthreads();
    for (int64_t q = threadIdx.x + 1; q < na - 1; q += blockDim.x) Eo[q] = Ei[q] - ced * (Hi[q] - Hi[q - 1]);
    __syncthreads();
    if (threadIdx.x == 0) {
        Eo[src] = Eo[src] + s;
        Eo[0] = Ei[1] + cm * (Eo[1] - Ei[0]);
        Eo[na - 1] = Ei[na - 2] + cm * (Eo[na - 2] - Ei[na - 1]);
    }
}

// Sample point code: component * N + node (component 0..2 E, 3..5 H).
template <typename T>
__global__ __launch_bounds__(256) void k_sample3d(Fields3<T> f, int64_t N, const int64_t *pts,
                                                  int64_t npts, T *buf)
{
    const int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (q >= npts) return;
    const int64_t code = pts[q];
    const int c = (int)(code / N);
    const int64_t p = code - (int64_t)c * N;
    const T *src = c == 0 ? f.E[0] : c == 1 ? f.E[1] : c == 2 ? f.E[2] : c == 3 ? f.H[0] : c == 4 ? f.H[1] : f.H[2];
    buf[q] = src[p];
}

// Twiddles dt e^{-j 2 pi f t} of slots 0..cnt-1 (samples m0+1 .. m0+cnt):
// [0][s][f] for E (t = m dt), [1][s][f] for H (t = (m - 1/2) dt = (2m-1) dt/2).
__global__ void k_tw3d(const double *freqs, int F, double dt, int64_t m0, int cnt, double2 *tw)
{
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= 2LL * cnt * F) return;
    const int kind = (int)(t / ((int64_t)cnt * F));
    const int64_t r = t - (int64_t)kind * cnt * F;
    const int s = (int)(r / F), fi = (int)(r % F);
    const int64_t m = m0 + s + 1;
    double re, im;
    if (kind == 0) twiddle(freqs[fi] * dt, dt, m, re, im);
    else twiddle(freqs[fi] * (0.5 * dt), dt, 2 * m - 1, re, im);
    tw[t] = make_double2(re, im);
}

// X[f][q] += sum_s v_s tw_s,f, slots in order; one thread per point.  The
// twiddle indices are wave-uniform, so both the E and the H twiddle are read
// as scalars and each lane picks its own.
template <typename T>
__global__ __launch_bounds__(256) void k_flush3d(const T *__restrict__ buf, int cnt, int64_t npts,
                                                 const int64_t *__restrict__ pts, int64_t N, int F,
                                                 const double2 *__restrict__ tw, double2 *__restrict__ X)
{
    const int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (q >= npts) return;
    const bool isH = pts[q] >= 3 * N;
    const double2 *tH = tw + (int64_t)cnt * F;
    double v[kSlotsMax];
#pragma unroll
    for (int s = 0; s < kSlotsMax; ++s) v[s] = s < cnt ? (double)buf[(int64_t)s * npts + q] : 0.0;
    for (int fi = 0; fi < F; ++fi) {
        double2 x = X[(int64_t)fi * npts + q];
#pragma unroll
        for (int s = 0; s < kSlotsMax; ++s) {
            if (s < cnt) {
                const double2 we = tw[(int64_t)s * F + fi], wh = tH[(int64_t)s * F + fi];
                const double wr = isH ? wh.x : we.x, wi = isH ? wh.y : we.y;
                x.x = __builtin_fma(v[s], wr, x.x);
                x.y = __builtin_fma(v[s], wi, x.y);
            }
        }
        X[(int64_t)fi * npts + q] = x;
    }
}

__global__ void k_fill3d(uint4 *p, int64_t n16)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t j = i; j < n16; j += stride) p[j] = make_uint4(0, 0, 0, 0);
}

__global__ void k_copy3d(uint4 *dst, const uint4 *src, int64_t n16)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t j = i; j < n16; j += stride) dst[j] = src[j];
}

// ---- launchers ----------------------------------------------------------------

static dim3 grid3(const Geo3 &g)
{
    return dim3((unsigned)(g.kb * g.jb * ((g.nx + g.np - 1) / g.np)));
}

template <typename T>
void launch_coef3d(const double *const w[3], const double *const n[3], int64_t S, double dt, double d,
                   T *const eA[3], T *const eJ[3], T *const eH[3], T *const a[3], T *const b1[3],
                   T *const b2[3], hipStream_t st)
{
    if (S <= 0) return;
    hipLaunchKernelGGL(k_coef3d<T>, dim3((unsigned)((S + 255) / 256)), dim3(256), 0, st, w[0], w[1], w[2], n[0],
                       n[1], n[2], S, dt, d, eA[0], eA[1], eA[2], eJ[0], eJ[1], eJ[2], eH[0], eH[1], eH[2], a[0],
                       a[1], a[2], b1[0], b1[1], b1[2], b2[0], b2[1], b2[2]);
}

template <typename T>
void launch_h3d(const Geo3 &g, const Fields3<T> &f, const Cpml3<T> &c, const double *Einc, hipStream_t st)
{
    hipLaunchKernelGGL(k_h3d<T>, grid3(g), dim3(256), 0, st, g, f, c, Einc);
}

template <typename T>
void launch_e3d(const Geo3 &g, const Fields3<T> &f, const Plasma3<T> &pl, const Cpml3<T> &c,
                const double *Hinc, double sval, hipStream_t st)
{
    hipLaunchKernelGGL(k_e3d<T>, grid3(g), dim3(256), 0, st, g, f, pl, c, Hinc, sval);
}

void launch_aux3d(const double *Ei, double *Eo, double *Hi, int64_t na, int64_t src, double chd, double ced,
                  double cm, double s, hipStream_t st)
{
    hipLaunchKernelGGL(k_aux3d, dim3(1), dim3(256), 0, st, Ei, Eo, Hi, na, src, chd, ced, cm, s);
}

template <typename T>
void launch_fused3d(const Geo3 &g, const Fields3<T> &fin, const Fields3<T> &fout, const Plasma3<T> &pl,
                    const Cpml3<T> &c, const double *Einc, const double *Hinc, double sval, int ni,
                    hipStream_t st)
{
    // 63 cells along k per wave (see k_fused3d)
    const int64_t nb = ((g.nz + 62) / 63) * g.jb * ((g.nx + ni - 1) / ni);
    hipLaunchKernelGGL(k_fused3d<T>, dim3((unsigned)nb), dim3(256), 0, st, g, fin, fout, pl, c, Einc, Hinc,
                       sval, ni);
}

template <typename T>
void launch_sample3d(const Fields3<T> &f, int64_t N, const int64_t *pts, int64_t npts, T *buf, hipStream_t st)
{
    if (npts <= 0) return;
    hipLaunchKernelGGL(k_sample3d<T>, dim3((unsigned)((npts + 255) / 256)), dim3(256), 0, st, f, N, pts,
                       npts, buf);
}

void launch_tw3d(const double *freqs, int F, double dt, int64_t m0, int cnt, double2 *tw, hipStream_t st)
{
    const int64_t n = 2LL * cnt * F;
    if (n <= 0) return;
    hipLaunchKernelGGL(k_tw3d, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, freqs, F, dt, m0, cnt, tw);
}

template <typename T>
void launch_flush3d(const T *buf, int cnt, int64_t npts, const int64_t *pts, int64_t N, int F,
                    const double2 *tw, double2 *X, hipStream_t st)
{
    if (npts <= 0 || F <= 0 || cnt <= 0) return;
    hipLaunchKernelGGL(k_flush3d<T>, dim3((unsigned)((npts + 255) / 256)), dim3(256), 0, st, buf, cnt, npts,
                       pts, N, F, tw, X);
}

void launch_fill3d(void *p, int64_t bytes, hipStream_t st)
{
    const int64_t n16 = bytes / 16;
    if (n16 <= 0) return;
    int64_t nb = (n16 + 255) / 256;
    if (nb > 65536) nb = 65536;
    hipLaunchKernelGGL(k_fill3d, dim3((unsigned)nb), dim3(256), 0, st, (uint4 *)p, n16);
}

void launch_copy3d(void *dst, const void *src, int64_t bytes, hipStream_t st)
{
    const int64_t n16 = bytes / 16;
    if (n16 <= 0) return;
    int64_t nb = (n16 + 255) / 256;
    if (nb > 65536) nb = 65536;
    hipLaunchKernelGGL(k_copy3d, dim3((unsigned)nb), dim3(256), 0, st, (uint4 *)dst, (const uint4 *)src, n16);
}

#define INST3(T)                                                                                          \
    template void launch_h3d<T>(const Geo3 &, const Fields3<T> &, const Cpml3<T> &, const double *,      \
                                hipStream_t);                                                             \
    template void launch_fused3d<T>(const Geo3 &, const Fields3<T> &, const Fields3<T> &,                \
                                    const Plasma3<T> &, const Cpml3<T> &, const double *, const double *, \
                                    double, int, hipStream_t);                                            \
    template void launch_e3d<T>(const Geo3 &, const Fields3<T> &, const Plasma3<T> &, const Cpml3<T> &,  \
                                const double *, double, hipStream_t);                                     \
    template void launch_sample3d<T>(const Fields3<T> &, int64_t, const int64_t *, int64_t, T *,         \
                                     hipStream_t);                                                        \
    template void launch_flush3d<T>(const T *, int, int64_t, const int64_t *, int64_t, int,             \
                                    const double2 *, double2 *, hipStream_t);                             \
    template void launch_coef3d<T>(const double *const[3], const double *const[3], int64_t, double,     \
                                   double, T *const[3], T *const[3], T *const[3], T *const[3],           \
                                   T *const[3], T *const[3], hipStream_t);
INST3(float)
INST3(double)
#undef INST3

}  // namespace fdtdp
