/*
 * Oracle interface (test infrastructure only; see rketd1d.c).
 */
#ifndef FDTD_ORACLE_H
#define FDTD_ORACLE_H
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum { OR_BC_MUR1 = 0, OR_BC_CPML = 1, OR_BC_PEC = 2, OR_BC_PERIODIC = 3 };

typedef struct {
    int64_t n;                 /* E nodes 0..n-1; H nodes at k+1/2, k = 0..n-2 */
    double dz, dt;             /* m, s */
    const double *wp2;         /* [n] plasma frequency squared, rad^2/s^2 */
    const double *nu;          /* [n] collision frequency, 1/s */
    int32_t bc;
    int32_t scheme;            /* 0 consistent eq.(11)+(12), 1 printed eq.(13), 2 eq.(9) */
    int64_t cpml_cells;
    double cpml_m;             /* grading order; <= 0 means 3 */
    double cpml_sigma_max;     /* <= 0 means 0.8 (m+1)/(eta0 dz) */
    int64_t src_cell;          /* < 0: no source */
    double src_tau, src_t0, src_amp;
    int32_t n_probes;
    int32_t n_freqs;
    const int64_t *probe_cells;
    const double *freqs;       /* Hz */
} or1d_problem;

typedef struct {
    double *E;                 /* [n] */
    double *H;                 /* [n] (entry n-1 only for periodic) */
    double *J;                 /* [n] */
    double *psiE, *psiH;       /* [n] CPML auxiliaries (may be NULL unless CPML) */
    double *Xre, *Xim;         /* [n_probes][n_freqs] running DFT */
    int64_t step;              /* time index of E on entry / exit */
} or1d_state;

double or_c0(void);
double or_eps0(void);
double or_mu0(void);
void or_phi(double x, double *a, double *phi1, double *phi2);
void or_coeffs(int64_t n, const double *wp2, const double *nu, double dt,
               double dz, int scheme, double *out);
double or_source(double t, double tau, double t0, double amp);
void or_twiddle(double f, double dt, int64_t m, double *c, double *s);
void or_dft_accumulate(int64_t count, const double *samples, int64_t m0,
                       int n_freqs, const double *freqs, double dt,
                       double *Xre, double *Xim);
int or1d_check(const or1d_problem *pb);
int or1d_step(const or1d_problem *pb, or1d_state *st, int64_t nsteps);
int or1d_adjoint_step(const or1d_problem *pb, double *lE, double *lH, double *lJ);
int or1d_adjoint_r2(const or1d_problem *pb, int64_t nsteps, int32_t probe,
                    const double *xv_re, const double *xv_im, double *loss,
                    double *grad, double *X);

/* ---- 3D (see rketd3d.c) ---- */
typedef struct {
    int64_t nx, ny, nz;        /* cells per axis */
    double d, dt;              /* cubic cell side (m), time step (s) */
    const double *wp2[3];      /* [nx*ny*nz] per E component, at its own position */
    const double *nu[3];       /* [nx*ny*nz] per E component */
    int32_t periodic_x, periodic_y;
    int64_t cpml;              /* CPML cells per walled end (0: bare PEC walls) */
    int32_t source;            /* 0 none, 1 planar soft source, 2 TF/SF plane wave */
    int32_t src_comp;          /* planar source: 0 Ex, 1 Ey */
    int64_t src_k;             /* planar source plane */
    double src_tau, src_t0, src_amp;
    int64_t b0, b1;            /* TF box [b0, b1] on walled axes and z */
    int64_t naux, aux_off, aux_src;   /* incident 1D grid */
    int32_t n_points, n_freqs;
    const int32_t *points;     /* [n_points][4]: component (0..2 Ex..Ez, 3..5 Hx..Hz), i, j, k */
    const double *freqs;       /* Hz */
} or3d_problem;

typedef struct {
    double *E[3], *H[3], *J[3];   /* [nx*ny*nz] each */
    double *psi;                  /* [12][nx*ny*nz] CPML auxiliaries (NULL if cpml == 0) */
    double *Einc, *Hinc;          /* [naux] incident grid (NULL unless source == 2) */
    double *Xre, *Xim;            /* [n_points][n_freqs] */
    int64_t step;
} or3d_state;

int or3d_check(const or3d_problem *pb);
int or3d_step(const or3d_problem *pb, or3d_state *st, int64_t nsteps);

/* ---- 2D (see rketd2d.c) ---- */
typedef struct {
    int32_t mode;              /* 0 TM (Ez, Hx, Hy), 1 TE (Ex, Ey, Hz) */
    int64_t nx, ny;            /* cells per axis */
    double d, dt;              /* square cell side (m), time step (s) */
    const double *wp2[2];      /* [nx*ny] per E component of the mode (TM: [0] only) */
    const double *nu[2];
    int32_t periodic_x, periodic_y;
    int32_t has_src;           /* soft point source on Ez (TM) or Ey (TE) */
    int64_t src_i, src_j;
    double src_tau, src_t0, src_amp;
    int32_t n_probes, n_freqs;
    const int64_t *probes;     /* [n_probes][3]: E component of the mode, i, j */
    const double *freqs;       /* Hz */
} or2d_problem;

typedef struct {
    double *E[2], *H[2], *J[2];   /* TM: E[0] Ez, H[0] Hx, H[1] Hy, J[0] Jz;
                                     TE: E[0] Ex, E[1] Ey, H[0] Hz, J[0] Jx, J[1] Jy; [nx*ny] */
    double *Xre, *Xim;            /* [n_probes][n_freqs] */
    int64_t step;
} or2d_state;

int or2d_check(const or2d_problem *pb);
int or2d_step(const or2d_problem *pb, or2d_state *st, int64_t nsteps);

#ifdef __cplusplus
}
#endif
#endif
