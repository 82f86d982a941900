/*
 * fdtd_plasma3d — the 3D Yee form of the RKETD-FDTD Drude-plasma step on one
 * AMD Instinct MI355X (gfx950).  The paper works the method out in 1D and names
 * 2D/3D as its next step (section V); this is the method of section II applied
 * per field component:
 *
 *   Maxwell-Drude system eqs.(1)-(3) on a Yee lattice of cubic cells (side d):
 *     Ex(i+1/2, j, k)  Ey(i, j+1/2, k)  Ez(i, j, k+1/2)
 *     Hx(i, j+1/2, k+1/2)  Hy(i+1/2, j, k+1/2)  Hz(i+1/2, j+1/2, k)
 *   every array [i][j][k] with k fastest, i < nx, j < ny, k < nz, and a current
 *   J with each E component on the plasma support;
 *   H^{n+1/2} = H^{n-1/2} - dt/(mu0 d) curl E^n                     (eq.(14) per component)
 *   E^{n+1}   = CA E^n - CJ J^n + CH curl H^{n+1/2}                  (eqs.(11)+(12) solved)
 *   J^{n+1}   = e^{-nu dt} J^n + b1 E^n + b2 E^{n+1}                 (eq.(11), FP64 coefficients)
 *   with CA, CJ, CH, b1, b2 of the 1D library (fdtd_plasma.h) per component
 *   node (CH carrying 1/d).
 *
 * Boundaries: x and y each periodic or walled, z walled.  A wall is PEC
 * (tangential E zero on the index-0 face; the index-n face lies outside the
 * arrays and reads as zero), optionally lined with a CPML of cpml_cells per end
 * (kappa = 1, alpha = 0, sigma = 0.8 (m+1)/(eta0 d) (depth/cpml_cells)^m, m = 3).
 *
 * Sources: a planar soft source (eq.(15) added to Ex or Ey on the plane
 * k = src_k after the E update), or a total-field/scattered-field plane wave:
 * Ex-polarised, travelling +z, taken from a vacuum 1D Yee grid (same d, dt;
 * eq.(15) soft source; first-order Mur ends) spanning z in [tf_lo - 8, tf_hi + 8]
 * with its source at z = tf_lo - 5, and injected on the faces of the
 * total-field box [tf_lo, tf_hi] (along z and every walled axis).
 *
 * Sampling: every sample point (component, i, j, k) accumulates the FP64 DFT
 *   X(f) = sum_{m >= 1} v_m dt exp(-j 2 pi f t_m),
 * t_m = m dt for E components (value after step m), (m - 1/2) dt for H.
 *
 * Status codes, precisions and error reporting are those of fdtd_plasma.h
 * (FDTD_OK, FDTD_E_*, FDTD_F64 / FDTD_F32); the message of the last failure on
 * this thread is fdtd3d_last_error().  A handle is used by one host thread at a
 * time.
 */
#ifndef FDTD_PLASMA3D_H
#define FDTD_PLASMA3D_H

#include <stddef.h>
#include <stdint.h>

#include "fdtd_plasma.h"

#ifdef __cplusplus
extern "C" {
#endif

typedef struct fdtd3d fdtd3d;      /* opaque handle */

enum { FDTD3D_SRC_NONE = 0, FDTD3D_SRC_PLANAR = 1, FDTD3D_SRC_TFSF = 2 };

/* How a time step is executed (identical bits either way):
 * SPLIT: an H pass and an E/J pass over the grid, fields updated in place;
 * FUSED: one pass (waves marching along x, each recomputing the H of its
 *        j-1 and k-1 rim from E^n), E, H and the CPML auxiliaries ping-ponged
 *        between two copies.  AUTO = SPLIT (the faster of the two on MI355X
 *        at present). */
enum { FDTD3D_EXEC_AUTO = 0, FDTD3D_EXEC_SPLIT = 1, FDTD3D_EXEC_FUSED = 2 };

/* Field selectors of get/set_fields: E, H components, then the currents. */
enum {
    FDTD3D_EX = 0, FDTD3D_EY, FDTD3D_EZ, FDTD3D_HX, FDTD3D_HY, FDTD3D_HZ,
    FDTD3D_JX, FDTD3D_JY, FDTD3D_JZ
};

typedef struct {
    int32_t struct_size;       /* sizeof(fdtd3d_desc) */
    int32_t precision;         /* FDTD_F64 | FDTD_F32: E, H, J, CPML storage and curl arithmetic */
    int64_t nx, ny, nz;        /* cells per axis, each >= 2 (nz >= 4) */
    double d, dt;              /* m, s; c dt / d <= 1/sqrt(3) */
    const double *wp2[3];      /* host [nx*ny*nz] per E component (x, y, z) sampled at that
                                * component's position, rad^2/s^2 >= 0; read during create
                                * only.  The per-row span of nonzero entries (union of the
                                * three components) is the plasma support kept on the GPU. */
    const double *nu[3];       /* host [nx*ny*nz] collision frequency, 1/s >= 0; may alias */
    int32_t periodic_x, periodic_y;   /* 1: periodic axis, 0: walled */
    int32_t cpml_cells;        /* CPML cells per walled end, 0 <= 2 cpml_cells < n */
    int32_t source;            /* FDTD3D_SRC_* */
    int32_t src_comp;          /* planar source: 0 Ex, 1 Ey */
    int64_t src_k;             /* planar source plane, 0 <= src_k < nz */
    double src_tau, src_t0, src_amp;  /* eq.(15): s(t) = amp (t - t0) exp(-(t - t0)^2 / (2 tau^2)) */
    int64_t tf_lo, tf_hi;      /* TF/SF: 1 <= tf_lo < tf_hi <= n - 1 on z and walled axes */
    int32_t n_points, n_freqs; /* sample points (>= 0), DFT frequencies (>= 0) */
    const int32_t *points;     /* host [n_points][4]: component 0..5 (Ex..Hz), i, j, k */
    const double *freqs_hz;    /* host [n_freqs] */
    int32_t sample_slots;      /* samples buffered per point between DFT flushes;
                                * 0 = 32, else 1..32 */
    int32_t exec;              /* FDTD3D_EXEC_* */
    int32_t x_planes;          /* x-planes each thread of the split kernels walks (1..16,
                                * default 4), or each fused-kernel wave (2..128,
                                * default 32); 0 = default */
    int32_t reserved;
    void *stream;              /* hipStream_t to launch on (NULL: the legacy null stream,
                                * which also disables graph capture in fdtd3d_run) */
} fdtd3d_desc;

/* Device workspace the handle needs (bytes, 256-byte aligned regions). */
int fdtd3d_workspace_bytes(const fdtd3d_desc *desc, size_t *bytes);

/* Validate desc, lay out the workspace (caller-owned device memory of at least
 * workspace_bytes, 256-byte aligned; NULL: the library allocates and frees it),
 * copy the plasma support, CPML tables, sample points and frequencies to the
 * device, build the per-node coefficients of eqs.(11)+(12) (and the eq.(11)
 * current fractions) from wp2 and nu, and zero the state (step 0).  The host arrays are not kept. */
int fdtd3d_create(const fdtd3d_desc *desc, void *workspace, size_t bytes, fdtd3d **out);

/* Advance nsteps on the handle's stream (asynchronous); a step is the
 * section II step on the lattice: eq.(14) for H, eqs.(11)+(12) for E, the
 * eq.(15) source, eq.(11) for J, then the sample points.  step(a); step(b)
 * gives the same bits as step(a + b). */
int fdtd3d_step(fdtd3d *h, int64_t nsteps);

/* Reset to the zero state at step 0 and advance nsteps; the launches for a
 * given nsteps are captured into a hipGraph once and replayed afterwards. */
int fdtd3d_run(fdtd3d *h, int64_t nsteps);

/* Spectra of every sample point, host [n_points][n_freqs] each (re, im), the
 * running DFT standing in for section IV-B's FFT; synchronizes the stream.  Buffered samples are included without changing
 * the accumulation order of later steps.  FDTD_E_NONFINITE if any entry is
 * NaN or Inf (the arrays are still written). */
int fdtd3d_spectra(fdtd3d *h, double *re, double *im);

/* Copy one field (FDTD3D_EX .. FDTD3D_JZ) of the current state to/from host
 * memory: [nx*ny*nz] values of the storage precision (double or float).  J is
 * zero off the plasma support and set_fields rejects nonzero J there.
 * Both synchronize the stream. */
int fdtd3d_get_fields(fdtd3d *h, int32_t which, void *host);
int fdtd3d_set_fields(fdtd3d *h, int32_t which, const void *host);

/* Time index of the state (number of steps taken since create / run). */
int fdtd3d_steps_done(fdtd3d *h, int64_t *steps);

/* Per-launch GPU time over the last advance of the handle, measured with HIP
 * events when profiling is on: names[i] (static strings), ms[i] total time,
 * calls[i] launches, cells[i] cell-updates those launches covered.  Enable with
 * on = 1 (adds an event pair per launch and turns graph capture off), read
 * with fdtd3d_profile_read. */
int fdtd3d_profile(fdtd3d *h, int32_t on);
int fdtd3d_profile_read(fdtd3d *h, int32_t max, const char **names, double *ms, int64_t *calls,
                        double *cells, int32_t *count);

/* Release the handle (synchronizes its stream first). */
int fdtd3d_destroy(fdtd3d *h);

const char *fdtd3d_last_error(void);

#ifdef __cplusplus
}
#endif
#endif
