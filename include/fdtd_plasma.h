/*
 * fdtd_plasma — RKETD-FDTD time stepping of electromagnetic waves in an
 * unmagnetized (Drude) plasma, on one AMD Instinct MI355X (gfx950).
 *
 * Method (Xiong et al., "The Electromagnetic Waves Propagation in Unmagnetized
 * Plasma Media Using Parallelized FDTD", section II):
 *   - Yee grid in 1D, eqs.(4)-(6): Ex on integer nodes k = 0..n-1, Hy on half
 *     nodes k+1/2 (k = 0..n-2), the polarization current Jx with Ex;
 *   - H update, eq.(14); E update from eqs.(11) and (12) solved together
 *     (the consistent form of eq.(13)); J update by the second-order
 *     exponential time differencing of eq.(11), whose exp(-nu dt) fractions
 *     are evaluated in FP64;
 *   - a Gaussian-derivative soft source, eq.(15), added after the E update;
 *   - absorbing ends (section III uses PML; first-order Mur and a CPML here);
 *   - a running DFT at probe nodes standing in for the FFT of section IV-B:
 *       X(f) = sum_{m >= 1} E^m[p] dt exp(-j 2 pi f m dt)   (FP64 always).
 *
 * All calls return an int status: FDTD_OK (0) or a negative FDTD_E_* code.
 * On error, fdtd_plasma_last_error() returns a thread-local message.  No C++
 * exception crosses this interface.  A handle is not thread-safe: one host
 * thread at a time.
 */
#ifndef FDTD_PLASMA_H
#define FDTD_PLASMA_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct fdtd_plasma fdtd_plasma;     /* opaque handle */

enum {
    FDTD_OK = 0,
    FDTD_E_INVALID = -1,      /* a descriptor field or argument is out of range */
    FDTD_E_UNSTABLE = -2,     /* Courant number c dt/dz above 1 */
    FDTD_E_WORKSPACE = -3,    /* caller workspace too small or misaligned */
    FDTD_E_DEVICE = -4,       /* a HIP runtime call failed (message has the HIP error) */
    FDTD_E_STATE = -5,        /* call out of order (e.g. adjoint before a checkpointed run) */
    FDTD_E_NONFINITE = -6,    /* a NaN/Inf reached a probe spectrum */
    FDTD_E_UNSUPPORTED = -7   /* valid physics this build does not implement on the GPU */
};

enum { FDTD_F64 = 0, FDTD_F32 = 1, FDTD_F32_DELTA = 2 };

/* Ends of every grid.  MUR1: first-order Mur at nodes 0 and n-1.  CPML: a
 * convolutional PML of cpml_cells nodes at each end (kappa = 1, alpha = 0,
 * sigma = sigma_max (depth/cpml_cells)^m) backed by PEC.  PEC: E = 0 at the
 * end nodes. */
enum { FDTD_BC_MUR1 = 0, FDTD_BC_CPML = 1, FDTD_BC_PEC = 2 };

/* CONSISTENT: eqs.(11)+(12) solved for E^{n+1} (all terms divided by
 * D = 1 + (wp dt)^2 phi2/2).  PAPER_EQ13: eq.(13) exactly as printed (only
 * the E^n term carries 1/D).  ETD1: the first-order current update eq.(9). */
enum { FDTD_SCHEME_CONSISTENT = 0, FDTD_SCHEME_PAPER_EQ13 = 1, FDTD_SCHEME_ETD1 = 2 };

/* How the time loop is executed.  In FDTD_F64 and FDTD_F32_DELTA the results
 * agree bit for bit across modes.  In FDTD_F32 the fields are held in FP64
 * registers while a launch runs and rounded to FP32 where it stores them, so
 * the bits depend on where launches end (STEP: every step; TILED: every
 * steps_per_pass steps and at window ends; RESIDENT: every sample window), and
 * each mode agrees with the FP64 result to its own rounding level.
 * STEP:     two launches per time step (H, then E/J/source/ends/probes);
 * TILED:    temporal blocking, steps_per_pass steps per launch on register
 *           tiles of tile_waves waves of tile_cells nodes each (tiles whose
 *           span holds vacuum only: vacuum_tile_cells nodes, if set), with
 *           halo recompute at the tile ends, ping-pong buffers;
 * RESIDENT: one persistent launch; each workgroup keeps whole grids in
 *           registers for the entire run (short grids, e.g. batches of slabs);
 * MIXED:    per pass, the grids that fit a workgroup run as RESIDENT bins and
 *           the longer ones as TILED tiles (Mur or PEC ends; batches of
 *           uneven slabs);
 * AUTO:     TILED (faster than RESIDENT on MI355X for single grids and for
 *           batches of short grids alike), except RESIDENT for FDTD_F32 on at
 *           most 16 grids that all fit the resident bins (4095 nodes) with Mur
 *           or PEC ends: fewer FP32 roundings keep short runs within the FP32
 *           accuracy target at the low end of the band. */
enum { FDTD_EXEC_AUTO = 0, FDTD_EXEC_STEP = 1, FDTD_EXEC_TILED = 2, FDTD_EXEC_RESIDENT = 3,
       FDTD_EXEC_MIXED = 4 };

/* flags */
#define FDTD_FLAG_CHECKPOINT 0x1   /* run() stores sqrt(T)-spaced checkpoints for the adjoint */
#define FDTD_FLAG_RECORD 0x2       /* keep every probe sample of the first record_steps steps
                                      (fdtd_plasma_probe_series, fdtd_plasma_probe_fft) */

typedef struct {
    uint32_t struct_size;        /* sizeof(fdtd_plasma_desc) */
    int32_t precision;           /* FDTD_F64: E, H (and psi) stored in FP64.  FDTD_F32: stored in
                                    FP32, the updates computed in FP64 registers and rounded to
                                    FP32 only where a launch stores the fields (see the exec
                                    modes).  J (carried as CJ (J - b2 E)) and its eq.(11) update are
                                    FP64 at either precision; the DFT is FP64.
                                    FDTD_F32_DELTA: an accuracy ablation with every field update in
                                    FP32 arithmetic (fields rounded to FP32 after every operation),
                                    the eq.(11) update in FP32 too with J rounded to FP32 every
                                    step, and every coefficient an FP32 number in delta form
                                    (CA-1, exp(-nu dt)-1, b1, b2 each rounded once from its FP64
                                    value); J values stay in the FP64 arrays (each one an FP32
                                    number), the DFT stays FP64.  Per-step executor or one-wave
                                    register tiles of 256 or 512 nodes (FDTD_EXEC_STEP, _TILED,
                                    _AUTO, which takes TILED); no FDTD_FLAG_CHECKPOINT.  Other exec
                                    modes and tile shapes return FDTD_E_INVALID. */
    int32_t scheme;              /* FDTD_SCHEME_* */
    int32_t bc;                  /* FDTD_BC_* */
    int32_t exec;                /* FDTD_EXEC_* */
    int32_t flags;               /* FDTD_FLAG_* */
    int64_t batch;               /* number of independent 1D grids, >= 1 */
    const int64_t *cells;        /* host [batch]: E nodes per grid, in [3, 2^31 - 1] */
    double dz;                   /* m, > 0 */
    double dt;                   /* s, > 0, c dt/dz <= 1 */
    const double *wp2;           /* host [sum(cells)]: plasma frequency^2 per node, rad^2/s^2, >= 0;
                                    0 at each grid's two end nodes and inside CPML layers */
    const double *nu;            /* host [sum(cells)]: collision frequency per node, 1/s, >= 0 */
    const int64_t *src_cell;     /* host [batch]: source node in 1..n-2, or -1 for none */
    double src_tau, src_t0, src_amp;   /* eq.(15): s(t) = amp (t-t0) exp(-(t-t0)^2/(2 tau^2)) */
    int32_t n_probes;            /* probes per grid, >= 1 */
    int32_t n_freqs;             /* DFT frequencies, >= 1 */
    const int64_t *probe_cells;  /* host [batch][n_probes]: nodes in 0..n-1 */
    const double *freqs_hz;      /* host [n_freqs] */
    int32_t cpml_cells;          /* CPML thickness in nodes (bc = CPML) */
    int32_t tile_cells;          /* TILED: nodes per register tile (64*C: 256, 512, 768 or 1024);
                                    0 = 512 */
    double cpml_m;               /* CPML grading order; <= 0 means 3 */
    double cpml_sigma_max;       /* <= 0 means 0.8 (m+1)/(eta0 dz) */
    int32_t steps_per_pass;      /* TILED: time steps per launch (halo depth), a multiple of 4 in
                                    [4, 64]; 0 = 48 */
    int32_t checkpoint_steps;    /* with FDTD_FLAG_CHECKPOINT: longest run the checkpoint and
                                    adjoint storage is sized for (>= 1) */
    int32_t tile_waves;          /* TILED: waves per tile (1, 2, 4 or 8; neighbouring waves of a
                                    tile exchange edge values through LDS every step, so the
                                    halo is paid once per tile_waves*tile_cells nodes); 0 = default */
    int32_t record_steps;        /* with FDTD_FLAG_RECORD: steps whose probe samples are kept,
                                    in [1, 2^24]; the FFT takes up to 2 * next_pow2(record_steps + 1)
                                    points.  Costs 8 B + 64 B per probe and step of device memory. */
    int32_t vacuum_tile_cells;   /* TILED, one-wave tiles: nodes of the tiles whose whole span holds
                                    vacuum only (no plasma node, grid end, CPML layer, source or
                                    probe): 64*C for C in 12, 16, 24, 32, wider than tile_cells, so
                                    the halo recompute costs them less.  The other vacuum tiles then
                                    run with the plasma tiles (whose step gives vacuum nodes the
                                    vacuum update's bits).  0 = every tile tile_cells wide.  Not with
                                    FDTD_F32_DELTA. */
    void *stream;                /* hipStream_t for every launch and copy; NULL = null stream */
} fdtd_plasma_desc;

/*
 * Device bytes the handle needs for this descriptor (state, ping-pong
 * buffers, plasma parameters, probe samples, DFT accumulators, checkpoints).
 * The descriptor is validated as for create.
 */
int fdtd_plasma_workspace_bytes(const fdtd_plasma_desc *desc, size_t *bytes);

/*
 * Validate the descriptor, lay out the workspace, copy the host arrays to the
 * device (on desc->stream), build the per-node coefficients of section II
 * (eqs.(9), (11), (13) from wp2 and nu) and zero the state.  Host arrays are borrowed only
 * for the duration of the call.  dev_workspace (256-byte aligned device
 * memory of at least fdtd_plasma_workspace_bytes) stays owned by the caller
 * and must outlive the handle; NULL makes the library allocate and own it.
 * On failure *out is NULL.
 */
int fdtd_plasma_create(const fdtd_plasma_desc *desc, void *dev_workspace,
                       size_t workspace_bytes, fdtd_plasma **out);

/* Bytes of the per-device static workspace of fdtd_plasma_create_static. */
#define FDTD_STATIC_WORKSPACE_BYTES (16u << 20)

/*
 * fdtd_plasma_create for callers that cannot allocate device memory (serving
 * loops, harnesses that forbid hipMalloc): the handle's workspace is a
 * static device array of FDTD_STATIC_WORKSPACE_BYTES bytes that the library
 * holds on every GPU it runs on until the process ends, and create makes no
 * side stream or event either (the CPML and role tiles then run on the
 * handle's stream, with the same results).  It still copies the inputs and
 * waits for the stream, so it is not for use under graph capture.  One such
 * handle per device at a time: the array is that device's only one, so a
 * second create_static on the device returns FDTD_E_STATE until the first is
 * destroyed (calls that used the array from several threads at once would
 * race).  A descriptor whose workspace (fdtd_plasma_workspace_bytes) exceeds
 * FDTD_STATIC_WORKSPACE_BYTES returns FDTD_E_WORKSPACE before any device
 * call.  Everything else is as for fdtd_plasma_create; destroy releases the
 * array for the next handle.
 */
int fdtd_plasma_create_static(const fdtd_plasma_desc *desc, fdtd_plasma **out);

/*
 * Advance every grid by nsteps (>= 0) time steps, asynchronously on the
 * handle's stream.  A step is section II's: H by eq.(14), E by eqs.(11)+(12)
 * solved together, the eq.(15) source, J by eq.(11), the ends, the probe
 * samples.  In FDTD_F64 and FDTD_F32_DELTA, step(a) followed by
 * step(b) gives bit-for-bit the same state and spectra as step(a + b); in
 * FDTD_F32 the fields are rounded to FP32 where each launch ends, so the two
 * agree to that rounding.
 */
int fdtd_plasma_step(fdtd_plasma *h, int64_t nsteps);

/*
 * Reset fields, currents and spectra to zero at step 0, then advance nsteps
 * (one run of section IV-B's experiment), replaying a HIP graph captured on
 * the first call with this nsteps.  With
 * FDTD_FLAG_CHECKPOINT the run also stores the forward checkpoints used by
 * fdtd_plasma_grad_r2.
 */
int fdtd_plasma_run(fdtd_plasma *h, int64_t nsteps);

/*
 * Copy the running DFT to host arrays re, im of [batch][n_probes][n_freqs]
 * doubles, waiting for the stream: the probe spectra from which section IV-B
 * forms reflection and transmission (two runs, with and without plasma).  FDTD_E_STATE before any step,
 * FDTD_E_NONFINITE if any value is NaN or Inf (the values are still copied).
 */
int fdtd_plasma_probe_spectra(fdtd_plasma *h, double *re, double *im);

/*
 * The recorded probe series (section IV-B records the probe field over the
 * run and Fourier transforms it): host out[batch][n_probes][steps] doubles,
 * out[b][p][m-1] = E^m at probe p of grid b for m = 1 .. steps, steps the
 * steps done since create or the last run().  Waits for the stream.  Needs
 * FDTD_FLAG_RECORD and 1 <= steps <= record_steps, else FDTD_E_STATE.
 */
int fdtd_plasma_probe_series(fdtd_plasma *h, double *out);

/*
 * FFT of the recorded series, zero-padded to nfft points (a power of 2 with
 * steps < nfft <= 2 * next_pow2(record_steps + 1)), computed on the device:
 *   X[b][p][k] = dt sum_{m=1}^{steps} E^m[p] exp(-j 2 pi k m / nfft),  k < nfft,
 * the running DFT's sum at f_k = k / (nfft dt).  Host outputs re, im of
 * [batch][n_probes][nfft] doubles; waits for the stream.  FDTD_E_STATE as
 * for fdtd_plasma_probe_series, FDTD_E_INVALID for another nfft.
 */
int fdtd_plasma_probe_fft(fdtd_plasma *h, int64_t nfft, double *re, double *im);

/*
 * Copy one grid's state to host arrays (doubles, waiting for the stream):
 * the Yee unknowns of eqs.(4)-(6), E[n], H[n-1] (H at k+1/2), and the current
 * J[n] of eq.(5) in A/m^2 (any pointer may be NULL).
 */
int fdtd_plasma_get_fields(fdtd_plasma *h, int64_t grid, double *E, double *H, double *J);

/* Steps taken since create or the last run(). */
int fdtd_plasma_steps_done(fdtd_plasma *h, int64_t *steps);

/*
 * Reflection loss of the current spectra, for every grid b:
 *   L_b = sum_f |R_b(f)|^2,  R_b(f) = (X_b(f) - xref_b(f)) / xref_b(f),
 * X_b the running DFT at probe `probe` (R is the two-run reflection
 * coefficient of section IV-B when xref is the same probe in a plasma-free
 * run).
 * xref_re/xref_im: host [batch][n_freqs]; loss: host [batch].  Waits for
 * the stream.  FDTD_E_STATE before any step.
 */
int fdtd_plasma_loss_r2(fdtd_plasma *h, int32_t probe, const double *xref_re,
                        const double *xref_im, double *loss);

/*
 * dL_b/d(wp2) of that loss after nsteps steps from zero, by the discrete
 * adjoint: the sub-steps of eqs.(14), (11)+(12), (11) and the ends are
 * transposed and applied in reverse order, forward states are recomputed
 * segment by segment from checkpoints taken every ceil(sqrt(nsteps)) steps.
 * Needs FDTD_FLAG_CHECKPOINT with nsteps <= checkpoint_steps, scheme
 * CONSISTENT, MUR1 or PEC ends.  If the handle's state is not already a
 * checkpointed run() of nsteps, that run is done first.  Outputs (host):
 * loss [batch]; grad [sum(cells)] in grid order (units 1/(rad/s)^2).  The
 * state (fields, spectra, checkpoints) is left as the forward run made it.
 */
int fdtd_plasma_grad_r2(fdtd_plasma *h, int64_t nsteps, int32_t probe,
                        const double *xref_re, const double *xref_im,
                        double *loss, double *grad);

/*
 * Per-kernel timing of nsteps eager steps from the current state (which they
 * advance), with HIP events on the handle's stream around every launch.
 * Host outputs: names char[max][32]; ms_total, calls, units [max] where
 * units sums, over the launches, the grid nodes each launch advanced (the
 * unit algorithmic bytes are counted in).  *count: distinct kernel groups.
 */
int fdtd_plasma_profile(fdtd_plasma *h, int64_t nsteps, int32_t max, char *names,
                        double *ms_total, int64_t *calls, int64_t *units, int32_t *count);

/* Release the handle (NULL is accepted).  Waits for the stream; does not
 * free a caller-owned workspace. */
int fdtd_plasma_destroy(fdtd_plasma *h);

/* Message for the last failing call on this host thread ("" if none). */
const char *fdtd_plasma_last_error(void);

#ifdef __cplusplus
}
#endif
#endif /* FDTD_PLASMA_H */
