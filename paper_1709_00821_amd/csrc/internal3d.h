// Interfaces between the 3D host library (api3d.hip) and its kernels
// (kernels3d.hip).  Layout: every field array is [i][j][k] with k fastest,
// p = (i*ny + j)*nz + k.  Kernels map 64 consecutive k of one row to a wave and
// 4 rows (j) to a 256-thread workgroup.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "physics.h"

namespace fdtdp {

constexpr int kSlotsMax = 32;     // samples buffered per point between DFT flushes

struct Geo3 {
    int64_t nx, ny, nz;
    int64_t kb, jb;               // 64-node blocks along k, 4-row blocks along j
    int32_t px, py;               // periodic x / y
    int32_t P;                    // CPML cells per walled end (0: none)
    int32_t src;                  // 0 none, 1 planar, 2 TF/SF
    int32_t src_comp;
    int32_t np;                   // x-planes per thread (split kernels)
    int64_t src_k;
    int64_t b0, b1;               // TF box
    int64_t xlo, xhi, ylo, yhi;   // Ex/Hy index ranges of the TF box (i: [xlo,xhi), j: [ylo,yhi))
    int64_t ao;                   // incident-grid node of z = 0
    double chd, ced;              // dt/(mu0 d), dt/(eps0 d)
    double dt, d;
};

template <typename T>
struct Fields3 {
    T *E[3];
    T *H[3];
};

// Plasma support: per row (i, j) the span [k0, k1) of nodes with a current;
// the row's nodes are stored compactly from off[row].  The per-node
// coefficients of each E component are built once per create (k_coef3d)
// into compact tables in the storage precision: the E-update triple (FP64:
// CA, CJ, CH; FP32: CA - 1, CJ, CH) and the exponential-integrator triple of
// the J update (FP64: a, b1, b2; FP32: a - 1, b1, b2, which J, itself stored
// in FP32, carries to no worse than its own rounding).  The J update runs in
// FP64 registers on the widened values.
template <typename T>
struct Plasma3 {
    const int2 *span;             // [nx*ny] (k0, k1); k0 == k1: no plasma in the row
    const int64_t *off;           // [nx*ny]
    T *J[3];                      // compact [S]
    const T *eA[3], *eJ[3], *eH[3];          // compact [S]
    const T *ca[3], *cb1[3], *cb2[3];        // compact [S]
};

// Build the compact coefficient tables from wp2, nu (compact, FP64).
template <typename T>
void launch_coef3d(const double *const wp2[3], const double *const nu[3], int64_t S, double dt, double d,
                   T *const eA[3], T *const eJ[3], T *const eH[3], T *const ca[3], T *const cb1[3],
                   T *const cb2[3], hipStream_t st);



// CPML auxiliaries, one slab pair per walled axis.  Slab index s in [0, 2P):
// s < P is node s, s >= P is node n - 2P + s.  Slab arrays:
//   x: [2P][ny][nz], y: [nx][2P][nz], z: [nx][ny][2P].
// Per axis the H pair is (derivative of the first, of the second component):
//   x: (Hy <- dEz/dx, Hz <- dEy/dx)   y: (Hx <- dEz/dy, Hz <- dEx/dy)   z: (Hx <- dEy/dz, Hy <- dEx/dz)
// and the E pair
//   x: (Ey <- dHz/dx, Ez <- dHy/dx)   y: (Ex <- dHz/dy, Ez <- dHx/dy)   z: (Ex <- dHy/dz, Ey <- dHx/dz)
// in: the auxiliaries read; out: where updated ones are written (the same
// arrays for the in-place two-kernel step, the other copy for the fused one).
template <typename T>
struct Cpml3 {
    const T *inH[3][2];
    T *outH[3][2];
    const T *inE[3][2];
    T *outE[3][2];
    const T *tab;                 // [3 axes][4: bE, aE, bH, aH][2P]
};


template <typename T>
void launch_h3d(const Geo3 &g, const Fields3<T> &f, const Cpml3<T> &c, const double *Einc,
                hipStream_t st);
// One whole step (H, then E and J) reading fin and writing fout; tiles march
// along i in chunks of ni planes.
template <typename T>
void launch_fused3d(const Geo3 &g, const Fields3<T> &fin, const Fields3<T> &fout, const Plasma3<T> &pl,
                    const Cpml3<T> &c, const double *Einc, const double *Hinc, double src_value, int ni,
                    hipStream_t st);
template <typename T>
void launch_e3d(const Geo3 &g, const Fields3<T> &f, const Plasma3<T> &pl, const Cpml3<T> &c,
                const double *Hinc, double src_value, hipStream_t st);
// Incident grid step: Hi from Ei_in, then Ei_out (source, Mur ends).
void launch_aux3d(const double *Ei_in, double *Ei_out, double *Hi, int64_t na, int64_t src, double chd,
                  double ced, double cm, double s, hipStream_t st);
template <typename T>
void launch_sample3d(const Fields3<T> &f, int64_t N, const int64_t *pts, int64_t npts, T *buf,
                     hipStream_t st);
void launch_tw3d(const double *freqs, int F, double dt, int64_t m0, int cnt, double2 *tw,
                 hipStream_t st);
template <typename T>
void launch_flush3d(const T *buf, int cnt, int64_t npts, const int64_t *pts, int64_t N, int F,
                    const double2 *tw, double2 *X, hipStream_t st);
void launch_fill3d(void *p, int64_t bytes, hipStream_t st);
void launch_copy3d(void *dst, const void *src, int64_t bytes, hipStream_t st);

}  // namespace fdtdp
