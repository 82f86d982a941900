/*
 * Oracle: plain, serial, FP64 2D RKETD-FDTD (TEST INFRASTRUCTURE ONLY; only the
 * test suite, the smoke check and the benchmark's CPU-baseline leg load it).
 *
 * The paper's section II scheme on a 2D Yee lattice of square cells of side d,
 * nx x ny cells, fields uniform along z (the paper names 2D and 3D as the
 * next step, section V).  Two independent modes:
 *   TM: Ez(i, j), Hx(i, j+1/2), Hy(i+1/2, j); plasma current Jz with Ez.
 *   TE: Ex(i+1/2, j), Ey(i, j+1/2), Hz(i+1/2, j+1/2); Jx with Ex, Jy with Ey.
 * Arrays [i][j] with j fastest, i < nx, j < ny.  From Maxwell's curl equations
 * with the 1D scheme's per-node coefficients (or_coeffs, consistent eq.(13),
 * CH carrying the 1/d of the curl, ch = dt/(mu0 d)):
 *   TM: Hx -= ch (Ez(i, j+1) - Ez(i, j))
 *       Hy += ch (Ez(i+1, j) - Ez(i, j))
 *       Ez  = CA Ez - CJ Jz + CH [(Hy(i, j) - Hy(i-1, j)) - (Hx(i, j) - Hx(i, j-1))]
 *   TE: Hz -= ch [(Ey(i+1, j) - Ey(i, j)) - (Ex(i, j+1) - Ex(i, j))]
 *       Ex  = CA Ex - CJ Jx + CH (Hz(i, j) - Hz(i, j-1))
 *       Ey  = CA Ey - CJ Jy - CH (Hz(i, j) - Hz(i-1, j))
 * then the soft point source of eq.(15) (added to Ez, TM, or Ey, TE, at
 * t = (n+1) dt), the walls, and eq.(11) for every current:
 *   J = a J + b1 E^n + b2 E^{n+1}.
 *
 * Each axis is periodic (indices wrap) or walled.  A wall is PEC: the E
 * component tangential to it is held at zero on the index-0 line (TM: Ez at
 * i = 0 and at j = 0; TE: Ey at i = 0, Ex at j = 0), and the line at index n
 * lies outside the arrays and reads as zero, as do H values before index 0.
 *
 * Probes: E components (component index within the mode, i, j), sampled after
 * each step, X(f) += E dt exp(-j 2 pi f m dt) at step m (or_dft_accumulate).
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#include "oracle.h"

int or2d_check(const or2d_problem *pb)
{
    if (!pb || (pb->mode != 0 && pb->mode != 1)) return -1;
    if (pb->nx < 2 || pb->ny < 2 || !(pb->d > 0.0) || !(pb->dt > 0.0)) return -1;
    /* 2D Courant limit */
    if (or_c0() * pb->dt / pb->d > 1.0 / sqrt(2.0)) return -2;
    const int nc = pb->mode == 0 ? 1 : 2;
    for (int c = 0; c < nc; ++c)
        if (!pb->wp2[c] || !pb->nu[c]) return -1;
    if (pb->has_src && (pb->src_i < 0 || pb->src_i >= pb->nx || pb->src_j < 0 || pb->src_j >= pb->ny)) return -1;
    for (int p = 0; p < pb->n_probes; ++p) {
        const int64_t *q = pb->probes + 3 * p;
        if (q[0] < 0 || q[0] >= nc || q[1] < 0 || q[1] >= pb->nx || q[2] < 0 || q[2] >= pb->ny) return -1;
    }
    return 0;
}

/* value of a field at (i, j) with the axis rules: wrap if periodic, zero
   outside [0, n) if walled */
static double at(const double *a, const or2d_problem *pb, int64_t i, int64_t j)
{
    if (i < 0 || i >= pb->nx) {
        if (!pb->periodic_x) return 0.0;
        i = (i + pb->nx) % pb->nx;
    }
    if (j < 0 || j >= pb->ny) {
        if (!pb->periodic_y) return 0.0;
        j = (j + pb->ny) % pb->ny;
    }
    return a[i * pb->ny + j];
}

int or2d_step(const or2d_problem *pb, or2d_state *st, int64_t nsteps)
{
    int rc = or2d_check(pb);
    if (rc) return rc;
    const int64_t nx = pb->nx, ny = pb->ny, N = nx * ny;
    const double dt = pb->dt, d = pb->d;
    const double ch = dt / (or_mu0() * d);
    const int nc = pb->mode == 0 ? 1 : 2;
    double *cf[2] = {NULL, NULL}, *Eold[2] = {NULL, NULL};
    double *Hn = (double *)malloc(sizeof(double) * (size_t)N * 2);
    int ok = Hn != NULL;
    for (int c = 0; c < nc; ++c) {
        cf[c] = (double *)malloc(sizeof(double) * 9 * (size_t)N);
        Eold[c] = (double *)malloc(sizeof(double) * (size_t)N);
        ok = ok && cf[c] && Eold[c];
        if (cf[c]) or_coeffs(N, pb->wp2[c], pb->nu[c], dt, d, 0, cf[c]);
    }
    if (!ok) {
        for (int c = 0; c < 2; ++c) { free(cf[c]); free(Eold[c]); }
        free(Hn);
        return -4;
    }

    for (int64_t it = 0; it < nsteps; ++it) {
        /* H^{n+1/2} from E^n (new values into Hn, then copied: every H update
           reads only E) */
#pragma omp parallel for schedule(static)
        for (int64_t i = 0; i < nx; ++i)
            for (int64_t j = 0; j < ny; ++j) {
                const int64_t k = i * ny + j;
                if (pb->mode == 0) {
                    const double *Ez = st->E[0];
                    Hn[k] = st->H[0][k] - ch * (at(Ez, pb, i, j + 1) - Ez[k]);
                    Hn[N + k] = st->H[1][k] + ch * (at(Ez, pb, i + 1, j) - Ez[k]);
                } else {
                    const double *Ex = st->E[0], *Ey = st->E[1];
                    const double curl = (at(Ey, pb, i + 1, j) - Ey[k]) - (at(Ex, pb, i, j + 1) - Ex[k]);
                    Hn[k] = st->H[0][k] - ch * curl;
                }
            }
        memcpy(st->H[0], Hn, sizeof(double) * (size_t)N);
        if (pb->mode == 0) memcpy(st->H[1], Hn + N, sizeof(double) * (size_t)N);

        /* E^{n+1} from E^n, J^n, H^{n+1/2}: eqs.(11)+(12) solved together */
        for (int c = 0; c < nc; ++c) memcpy(Eold[c], st->E[c], sizeof(double) * (size_t)N);
#pragma omp parallel for schedule(static)
        for (int64_t i = 0; i < nx; ++i)
            for (int64_t j = 0; j < ny; ++j) {
                const int64_t k = i * ny + j;
                if (pb->mode == 0) {
                    const double *Hx = st->H[0], *Hy = st->H[1];
                    const double curl = (Hy[k] - at(Hy, pb, i - 1, j)) - (Hx[k] - at(Hx, pb, i, j - 1));
                    const double *q = cf[0] + 9 * k;
                    st->E[0][k] = q[4] * Eold[0][k] - q[5] * st->J[0][k] + q[6] * curl;
                } else {
                    const double *Hz = st->H[0];
                    const double *qx = cf[0] + 9 * k, *qy = cf[1] + 9 * k;
                    st->E[0][k] = qx[4] * Eold[0][k] - qx[5] * st->J[0][k] + qx[6] * (Hz[k] - at(Hz, pb, i, j - 1));
                    st->E[1][k] = qy[4] * Eold[1][k] - qy[5] * st->J[1][k] - qy[6] * (Hz[k] - at(Hz, pb, i - 1, j));
                }
            }
        /* soft source, eq.(15), at t = (n+1) dt */
        if (pb->has_src) {
            const int c = pb->mode == 0 ? 0 : 1;
            st->E[c][pb->src_i * ny + pb->src_j] +=
                or_source((double)(st->step + 1) * dt, pb->src_tau, pb->src_t0, pb->src_amp);
        }
        /* PEC walls: the tangential E on the index-0 lines */
        if (pb->mode == 0) {
            if (!pb->periodic_x) for (int64_t j = 0; j < ny; ++j) st->E[0][j] = 0.0;
            if (!pb->periodic_y) for (int64_t i = 0; i < nx; ++i) st->E[0][i * ny] = 0.0;
        } else {
            if (!pb->periodic_x) for (int64_t j = 0; j < ny; ++j) st->E[1][j] = 0.0;
            if (!pb->periodic_y) for (int64_t i = 0; i < nx; ++i) st->E[0][i * ny] = 0.0;
        }
        /* J^{n+1}, eq.(11) */
        for (int c = 0; c < nc; ++c)
#pragma omp parallel for schedule(static)
            for (int64_t k = 0; k < N; ++k) {
                const double *q = cf[c] + 9 * k;
                st->J[c][k] = q[0] * st->J[c][k] + q[7] * Eold[c][k] + q[8] * st->E[c][k];
            }
        st->step += 1;
        /* running DFT of the probes */
        for (int p = 0; p < pb->n_probes; ++p) {
            const int64_t *q = pb->probes + 3 * p;
            double v = st->E[q[0]][q[1] * ny + q[2]];
            or_dft_accumulate(1, &v, st->step, pb->n_freqs, pb->freqs, dt,
                              st->Xre + (size_t)p * pb->n_freqs, st->Xim + (size_t)p * pb->n_freqs);
        }
    }
    for (int c = 0; c < 2; ++c) { free(cf[c]); free(Eold[c]); }
    free(Hn);
    return 0;
}
