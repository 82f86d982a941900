/*
 * fdtd_plasma2d — the 2D Yee form of the RKETD-FDTD Drude-plasma step on one
 * AMD Instinct MI355X (gfx950).  The paper works the method out in 1D and names
 * 2D and 3D as its next step (section V); this is the method of section II on a
 * 2D lattice of square cells (side d), fields uniform along z, in either mode:
 *
 *   TM: Ez(i, j), Hx(i, j+1/2), Hy(i+1/2, j); a current Jz with Ez;
 *   TE: Ex(i+1/2, j), Ey(i, j+1/2), Hz(i+1/2, j+1/2); Jx with Ex, Jy with Ey;
 *   arrays [i][j] with j fastest, i < nx, j < ny.
 *
 *   TM: Hx -= ch (Ez(i, j+1) - Ez(i, j));   Hy += ch (Ez(i+1, j) - Ez(i, j))
 *       Ez  = CA Ez - CJ Jz + CH [(Hy(i, j) - Hy(i-1, j)) - (Hx(i, j) - Hx(i, j-1))]
 *   TE: Hz -= ch [(Ey(i+1, j) - Ey(i, j)) - (Ex(i, j+1) - Ex(i, j))]
 *       Ex  = CA Ex - CJ Jx + CH (Hz(i, j) - Hz(i, j-1))
 *       Ey  = CA Ey - CJ Jy - CH (Hz(i, j) - Hz(i-1, j))
 *   (eq.(14) for H with ch = dt/(mu0 d); eqs.(11)+(12) solved for E with the
 *   per-node CA, CJ, CH of the 1D library, CH carrying the 1/d), then the soft
 *   point source of eq.(15) on Ez (TM) or Ey (TE) at t = (n+1) dt, the walls,
 *   and eq.(11), J = e^{-nu dt} J + b1 E^n + b2 E^{n+1}, in FP64.
 *
 * Each axis is periodic or walled.  A wall is PEC: the E component tangential
 * to it is held at zero on the index-0 line (TM: Ez at i = 0 and at j = 0;
 * TE: Ey at i = 0, Ex at j = 0); the line at index n lies outside the arrays
 * and reads as zero.
 *
 * Probes: E components (component of the mode, i, j); every probe accumulates
 * the FP64 DFT  X(f) = sum_{m >= 1} E^m dt exp(-j 2 pi f m dt).
 *
 * Status codes, precisions and error reporting follow fdtd_plasma.h
 * (FDTD_OK, FDTD_E_*; FDTD_F64, FDTD_F32 = FP32 storage with every update in
 * FP64 registers, rounded to FP32 where the step stores the fields); the
 * message of the last failure on this thread is fdtd2d_last_error().  A handle
 * is used by one host thread at a time.
 */
#ifndef FDTD_PLASMA2D_H
#define FDTD_PLASMA2D_H

#include <stddef.h>
#include <stdint.h>

#include "fdtd_plasma.h"

#ifdef __cplusplus
extern "C" {
#endif

typedef struct fdtd2d fdtd2d;      /* opaque handle */

enum { FDTD2D_TM = 0, FDTD2D_TE = 1 };

typedef struct {
    uint32_t struct_size;        /* sizeof(fdtd2d_desc) */
    int32_t mode;                /* FDTD2D_TM | FDTD2D_TE */
    int32_t precision;           /* FDTD_F64 | FDTD_F32 */
    int32_t periodic_x, periodic_y;   /* 1: periodic axis, 0: PEC walls */
    int64_t nx, ny;              /* cells, each >= 2 */
    double d;                    /* m, > 0 */
    double dt;                   /* s, > 0, c dt / d <= 1/sqrt(2) */
    const double *wp2;           /* host [ncomp][nx][ny], ncomp = 1 (TM) or 2 (TE: Ex, Ey):
                                    plasma frequency^2 at each E component's position, >= 0 */
    const double *nu;            /* host [ncomp][nx][ny]: collision frequency, 1/s, >= 0 */
    int32_t has_src;             /* soft point source of eq.(15) on Ez (TM) or Ey (TE) */
    int32_t n_probes;            /* >= 0 */
    int64_t src_i, src_j;        /* the source node, inside the grid */
    double src_tau, src_t0, src_amp;   /* s(t) = amp (t-t0) exp(-(t-t0)^2/(2 tau^2)) */
    int32_t n_freqs;             /* >= 1 */
    int32_t reserved;
    const int64_t *probes;       /* host [n_probes][3]: E component of the mode, i, j */
    const double *freqs_hz;      /* host [n_freqs] */
    void *stream;                /* hipStream_t for every launch and copy; NULL = null stream */
} fdtd2d_desc;

/* Device bytes the handle needs (fields, plasma support, samples, spectra);
 * the descriptor is validated as for create. */
int fdtd2d_workspace_bytes(const fdtd2d_desc *desc, size_t *bytes);

/* Validate, lay out the workspace, copy the host arrays (borrowed for the call
 * only) and zero the state; the per-cell coefficients of eqs.(11)+(12) are
 * formed in the E pass from wp2 and nu.  workspace: 256-byte aligned device memory of at
 * least fdtd2d_workspace_bytes, owned by the caller and outliving the handle,
 * or NULL (the library allocates and owns it).  On failure *out is NULL.
 * Errors: FDTD_E_INVALID (a field out of range, a NaN or negative wp2/nu,
 * a source or probe outside the grid), FDTD_E_UNSTABLE (Courant number above
 * 1/sqrt(2)), FDTD_E_WORKSPACE, FDTD_E_DEVICE. */
int fdtd2d_create(const fdtd2d_desc *desc, void *workspace, size_t bytes, fdtd2d **out);

/* Advance nsteps (>= 0), asynchronously on the handle's stream: per step the
 * eq.(14) H pass, then the E/J pass (eqs.(11)+(12), the eq.(15) source, the
 * walls, eq.(11)), then the probe samples.  step(a)
 * followed by step(b) gives the state and spectra of step(a + b) bit for bit. */
int fdtd2d_step(fdtd2d *h, int64_t nsteps);

/* Reset to zero at step 0, then advance nsteps, replaying a HIP graph captured
 * on the first call with this nsteps (the last partial sample window is folded
 * into the spectra inside the run). */
int fdtd2d_run(fdtd2d *h, int64_t nsteps);

/* Probe spectra to host re, im [n_probes][n_freqs] (the running DFT standing
 * in for section IV-B's FFT of the probe record); waits for the stream.
 * FDTD_E_STATE before any step or with no probes. */
int fdtd2d_spectra(fdtd2d *h, double *re, double *im);

/* One field to a host array of nx*ny doubles, waiting for the stream.  which:
 * 0 .. ncomp-1 the E components of the mode (TM: Ez; TE: Ex, Ey), ncomp ..
 * ncomp+nh-1 the H components (TM: Hx, Hy; TE: Hz), then the currents J of
 * the E components (A/m^2). */
int fdtd2d_get_fields(fdtd2d *h, int32_t which, double *out);

/* Steps taken since create or the last run(). */
int fdtd2d_steps_done(fdtd2d *h, int64_t *steps);

/* Release the handle (NULL accepted); waits for the stream, does not free a
 * caller-owned workspace. */
int fdtd2d_destroy(fdtd2d *h);

/* Message of the last failing call on this host thread ("" if none). */
const char *fdtd2d_last_error(void);

#ifdef __cplusplus
}
#endif
#endif /* FDTD_PLASMA2D_H */
