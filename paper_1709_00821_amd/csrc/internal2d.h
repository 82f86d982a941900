// Internal interfaces of the 2D library (api2d.hip) and its kernels.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "physics.h"

namespace fdtdp {

// Device view of a 2D grid (passed by value to kernels).  The plasma lives on
// a compact support: row i holds it on j in [span[i].x, span[i].y), at compact
// index rowoff[i] + j - span[i].x of the per-component arrays (the union of
// the components' supports; wp2 = 0 where one component has none).
struct Grid2 {
    int64_t nx, ny;
    int mode, px, py;          // mode 0 TM, 1 TE; periodic x, y
    double dt, d;
    double ch;                 // dt/(mu0 d)
    double ce;                 // dt/(eps0 d), the vacuum E coefficient
    const int2 *span;          // [nx]
    const int64_t *rowoff;     // [nx]
    const double *wp2[2], *nu[2];   // [S] per E component
    double *J[2];              // [S] per E component, FP64
    int has_src;
    int64_t si, sj;
    double src_tau, src_t0, src_amp;
    int P, SB;                 // probes, sample window length
    const int64_t *probes;     // [P][3]
    double *samp;              // [P][SB]
};

template <typename T>
struct Fields2 {
    T *E[2];                   // TM: Ez; TE: Ex, Ey
    T *H[2];                   // TM: Hx, Hy; TE: Hz
};

// One time step: H pass, E/J pass (source time m dt), probe samples into slot.
template <typename T>
void launch_step2d(const Grid2 &g, const Fields2<T> &f, int64_t m, int slot, hipStream_t st);

}  // namespace fdtdp
