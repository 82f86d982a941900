/*
 * Oracle: plain, serial, FP64 3D RKETD-FDTD (TEST INFRASTRUCTURE ONLY; only the
 * test suite, the smoke check and the benchmark's CPU-baseline leg load it).
 *
 * The paper's section II system, eqs.(1)-(3), on a Yee lattice of cubic cells
 * of side d with nx x ny x nz cells.  Components and their positions:
 *   Ex(i+1/2, j, k)  Ey(i, j+1/2, k)  Ez(i, j, k+1/2)
 *   Hx(i, j+1/2, k+1/2)  Hy(i+1/2, j, k+1/2)  Hz(i+1/2, j+1/2, k)
 * all stored [i][j][k] (k fastest), i < nx, j < ny, k < nz, and a plasma
 * current J co-located with each E component.  The 1D scheme of section II
 * (eqs.(11)-(14)) is applied per component:
 *   H^{n+1/2} = H^{n-1/2} - dt/(mu0 d) curl E^n
 *   E^{n+1}   = CA E^n - CJ J^n + CH curl H^{n+1/2}     (eqs.(11)+(12) solved)
 *   source, walls, then J^{n+1} = a J^n + b1 E^n + b2 E^{n+1}   (eq.(11))
 * with the 1D oracle's per-node coefficients (or_coeffs, consistent scheme;
 * CH carries the 1/d of the curl).
 *
 * Boundaries.  x and y are each periodic or walled; z is walled.  A wall is
 * PEC: the tangential E on the face at index 0 is held at zero and the face at
 * index n lies outside the arrays and reads as zero.  A wall may be lined with
 * a CPML of P cells per end exactly as in the 1D oracle (kappa = 1, alpha = 0,
 * sigma = 0.8 (m+1)/(eta0 d) (depth/P)^m with m = 3, b = exp(-sigma dt/eps0),
 * a = b - 1), here in "difference" units: psi = b psi + a dF, dF += psi for
 * each derivative taken across the layer.
 *
 * Sources (one of):
 *  1: planar soft source of eq.(15): Ex (or Ey) += s((n+1) dt) on every node of
 *     the plane k = src_k (with periodic x and y this is the 1D problem
 *     repeated over x and y);
 *  2: total-field/scattered-field plane wave, Ex-polarised, travelling +z.  The
 *     incident field comes from a vacuum 1D Yee grid of the same d and dt with
 *     the eq.(15) soft source at node aux_src and first-order Mur ends; aux
 *     node q holds Ex at z = q - aux_off and Hy at z = q - aux_off + 1/2.  It is
 *     advanced in step with the 3D grid (its H after the 3D H update, its E
 *     after the 3D E update), so the 3D H update sees Einc^n and the E update
 *     Hinc^{n+1/2}.  The total-field region is the box of positions in
 *     [b0, b1] along each walled axis (all of a periodic axis).  Every curl
 *     difference that straddles the box surface has the incident value of
 *     its far-side term added (total field read from the scattered side) or
 *     removed (scattered field read from the total side).
 *
 * Sampling.  Each sample point (component, i, j, k) feeds a running DFT,
 *   X(f) += v dt exp(-j 2 pi f t),
 * with t = m dt for E components after step m and t = (m - 1/2) dt for H.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#include "oracle.h"

typedef struct {
    double b, a;
} ab_t;

/* CPML depth (in cells) of a position on an axis of n cells, walls at 0 and n */
static double depth3(int64_t n, int64_t P, double pos)
{
    if (P <= 0) return 0.0;
    if (pos < (double)P) return (double)P - pos;
    if (pos > (double)(n - P)) return pos - (double)(n - P);
    return 0.0;
}

static ab_t cpml3(const or3d_problem *pb, double depth)
{
    ab_t r = {1.0, 0.0};
    if (pb->cpml <= 0 || depth <= 0.0) return r;
    const double m = 3.0;
    const double eta0 = sqrt(or_mu0() / or_eps0());
    const double smax = 0.8 * (m + 1.0) / (eta0 * pb->d);
    const double sigma = smax * pow(depth / (double)pb->cpml, m);
    r.b = exp(-sigma * pb->dt / or_eps0());
    r.a = r.b - 1.0;
    return r;
}

int or3d_check(const or3d_problem *pb)
{
    if (pb->nx < 2 || pb->ny < 2 || pb->nz < 4 || !(pb->d > 0.0) || !(pb->dt > 0.0)) return -1;
    if (or_c0() * pb->dt / pb->d > 1.0 / sqrt(3.0)) return -2;
    if (pb->cpml < 0 || 2 * pb->cpml >= pb->nz) return -1;
    if (pb->cpml > 0 && ((!pb->periodic_x && 2 * pb->cpml >= pb->nx) ||
                         (!pb->periodic_y && 2 * pb->cpml >= pb->ny)))
        return -1;
    if (pb->source == 1 && (pb->src_k < 0 || pb->src_k >= pb->nz || pb->src_comp < 0 || pb->src_comp > 1))
        return -1;
    if (pb->source == 2) {
        if (pb->b0 < 1 || pb->b1 > pb->nz - 1 || pb->b1 <= pb->b0) return -1;
        if (!pb->periodic_x && (pb->b0 < 1 || pb->b1 > pb->nx - 1)) return -1;
        if (!pb->periodic_y && (pb->b0 < 1 || pb->b1 > pb->ny - 1)) return -1;
        if (pb->naux < 3 || pb->aux_src < 1 || pb->aux_src >= pb->naux - 1) return -1;
        if (pb->b0 - 1 + pb->aux_off < 0 || pb->b1 + pb->aux_off > pb->naux - 2) return -1;
        if (pb->aux_src >= pb->b0 + pb->aux_off) return -1;   /* source outside the box */
    }
    const int64_t N = pb->nx * pb->ny * pb->nz;
    for (int c = 0; c < 3; ++c)
        for (int64_t p = 0; p < N; ++p)
            if (!(pb->wp2[c][p] >= 0.0) || !(pb->nu[c][p] >= 0.0)) return -1;
    for (int q = 0; q < pb->n_points; ++q) {
        const int32_t *s = pb->points + 4 * q;
        if (s[0] < 0 || s[0] > 5 || s[1] < 0 || s[1] >= pb->nx || s[2] < 0 || s[2] >= pb->ny ||
            s[3] < 0 || s[3] >= pb->nz)
            return -1;
    }
    return 0;
}

int or3d_step(const or3d_problem *pb, or3d_state *st, int64_t nsteps)
{
    int rc = or3d_check(pb);
    if (rc) return rc;
    const int64_t nx = pb->nx, ny = pb->ny, nz = pb->nz, N = nx * ny * nz;
    const double dt = pb->dt, d = pb->d;
    const double chd = dt / (or_mu0() * d), ced = dt / (or_eps0() * d);
    const int px = pb->periodic_x, py = pb->periodic_y;
    const int64_t P = pb->cpml;
#define IX(i, j, k) ((((int64_t)(i)) * ny + (j)) * nz + (k))
    double *cf = (double *)malloc(sizeof(double) * 9 * (size_t)N * 3);
    double *Eold = (double *)malloc(sizeof(double) * 3 * (size_t)N);
    if (!cf || !Eold) { free(cf); free(Eold); return -4; }
    for (int c = 0; c < 3; ++c) or_coeffs(N, pb->wp2[c], pb->nu[c], dt, d, 0, cf + (size_t)9 * N * c);
    double *Ex = st->E[0], *Ey = st->E[1], *Ez = st->E[2];
    double *Hx = st->H[0], *Hy = st->H[1], *Hz = st->H[2];
    const int64_t na = pb->naux, ao = pb->aux_off, b0 = pb->b0, b1 = pb->b1;
    double *Ei = st->Einc, *Hi = st->Hinc;
    /* TF box in index ranges of the Ex / Hy nodes (i: [b0, b1), j: [b0, b1]) */
    const int64_t xlo = px ? 0 : b0, xhi = px ? nx : b1;
    const int64_t ylo = py ? 0 : b0, yhi = py ? ny : b1 + 1;
    const double S = or_c0() * dt / d, cm = (S - 1.0) / (S + 1.0);

    for (int64_t it = 0; it < nsteps; ++it) {
        const double tnew = (double)(st->step + 1) * dt;
        /* ---- H^{n+1/2} (eq.(2)) ---- */
        for (int64_t i = 0; i < nx; ++i)
            for (int64_t j = 0; j < ny; ++j)
                for (int64_t k = 0; k < nz; ++k) {
                    const int64_t p = IX(i, j, k);
                    /* +1 neighbours; a wall's far face reads as zero */
                    const int hasi = px || i + 1 < nx, hasj = py || j + 1 < ny, hask = k + 1 < nz;
                    const int64_t ip = IX((i + 1) % nx, j, k), jp = IX(i, (j + 1) % ny, k), kp = p + 1;
                    double dEz_y = (hasj ? Ez[jp] : 0.0) - Ez[p];
                    double dEy_z = (hask ? Ey[kp] : 0.0) - Ey[p];
                    double dEx_z = (hask ? Ex[kp] : 0.0) - Ex[p];
                    double dEz_x = (hasi ? Ez[ip] : 0.0) - Ez[p];
                    double dEy_x = (hasi ? Ey[ip] : 0.0) - Ey[p];
                    double dEx_y = (hasj ? Ex[jp] : 0.0) - Ex[p];
                    if (P > 0) {
                        const ab_t cx = cpml3(pb, px ? 0.0 : depth3(nx, P, (double)i + 0.5));
                        const ab_t cy = cpml3(pb, py ? 0.0 : depth3(ny, P, (double)j + 0.5));
                        const ab_t cz = cpml3(pb, depth3(nz, P, (double)k + 0.5));
                        double *ps = st->psi;    /* Hx_y Hx_z Hy_z Hy_x Hz_x Hz_y */
                        ps[0 * N + p] = cy.b * ps[0 * N + p] + cy.a * dEz_y; dEz_y += ps[0 * N + p];
                        ps[1 * N + p] = cz.b * ps[1 * N + p] + cz.a * dEy_z; dEy_z += ps[1 * N + p];
                        ps[2 * N + p] = cz.b * ps[2 * N + p] + cz.a * dEx_z; dEx_z += ps[2 * N + p];
                        ps[3 * N + p] = cx.b * ps[3 * N + p] + cx.a * dEz_x; dEz_x += ps[3 * N + p];
                        ps[4 * N + p] = cx.b * ps[4 * N + p] + cx.a * dEy_x; dEy_x += ps[4 * N + p];
                        ps[5 * N + p] = cy.b * ps[5 * N + p] + cy.a * dEx_y; dEx_y += ps[5 * N + p];
                    }
                    Hx[p] = Hx[p] - chd * (dEz_y - dEy_z);
                    Hy[p] = Hy[p] - chd * (dEx_z - dEz_x);
                    Hz[p] = Hz[p] - chd * (dEy_x - dEx_y);
                }
        if (pb->source == 2) {
            /* Hy(k+1/2) reads Ex(k) and Ex(k+1): at k = b0-1 the scattered Hy
             * reads total Ex(b0); at k = b1 the scattered Hy reads total Ex(b1). */
            for (int64_t i = xlo; i < xhi; ++i)
                for (int64_t j = ylo; j < yhi; ++j) {
                    Hy[IX(i, j, b0 - 1)] += chd * Ei[b0 + ao];
                    Hy[IX(i, j, b1)] -= chd * Ei[b1 + ao];
                }
            /* Hz(j+1/2) reads Ex(j) and Ex(j+1), with a minus sign in the curl */
            if (!py)
                for (int64_t i = xlo; i < xhi; ++i)
                    for (int64_t k = b0; k <= b1; ++k) {
                        Hz[IX(i, b0 - 1, k)] -= chd * Ei[k + ao];
                        Hz[IX(i, b1, k)] += chd * Ei[k + ao];
                    }
            /* incident H^{n+1/2} */
            for (int64_t q = 0; q < na - 1; ++q) Hi[q] = Hi[q] - chd * (Ei[q + 1] - Ei[q]);
        }
        /* ---- E^{n+1} (eqs.(1),(3): (11)+(12) solved) ---- */
        for (int c = 0; c < 3; ++c) memcpy(Eold + (size_t)c * N, st->E[c], sizeof(double) * N);
        for (int64_t i = 0; i < nx; ++i)
            for (int64_t j = 0; j < ny; ++j)
                for (int64_t k = 0; k < nz; ++k) {
                    const int64_t p = IX(i, j, k);
                    const int hasi = px || i > 0, hasj = py || j > 0, hask = k > 0;
                    const int64_t im = IX((i + nx - 1) % nx, j, k), jm = IX(i, (j + ny - 1) % ny, k), km = p - 1;
                    double dHz_y = Hz[p] - (hasj ? Hz[jm] : 0.0);
                    double dHy_z = Hy[p] - (hask ? Hy[km] : 0.0);
                    double dHx_z = Hx[p] - (hask ? Hx[km] : 0.0);
                    double dHz_x = Hz[p] - (hasi ? Hz[im] : 0.0);
                    double dHy_x = Hy[p] - (hasi ? Hy[im] : 0.0);
                    double dHx_y = Hx[p] - (hasj ? Hx[jm] : 0.0);
                    if (P > 0) {
                        const ab_t cx = cpml3(pb, px ? 0.0 : depth3(nx, P, (double)i));
                        const ab_t cy = cpml3(pb, py ? 0.0 : depth3(ny, P, (double)j));
                        const ab_t cz = cpml3(pb, depth3(nz, P, (double)k));
                        double *ps = st->psi + 6 * N;   /* Ex_y Ex_z Ey_z Ey_x Ez_x Ez_y */
                        ps[0 * N + p] = cy.b * ps[0 * N + p] + cy.a * dHz_y; dHz_y += ps[0 * N + p];
                        ps[1 * N + p] = cz.b * ps[1 * N + p] + cz.a * dHy_z; dHy_z += ps[1 * N + p];
                        ps[2 * N + p] = cz.b * ps[2 * N + p] + cz.a * dHx_z; dHx_z += ps[2 * N + p];
                        ps[3 * N + p] = cx.b * ps[3 * N + p] + cx.a * dHz_x; dHz_x += ps[3 * N + p];
                        ps[4 * N + p] = cx.b * ps[4 * N + p] + cx.a * dHy_x; dHy_x += ps[4 * N + p];
                        ps[5 * N + p] = cy.b * ps[5 * N + p] + cy.a * dHx_y; dHx_y += ps[5 * N + p];
                    }
                    const double curl[3] = {dHz_y - dHy_z, dHx_z - dHz_x, dHy_x - dHx_y};
                    for (int c = 0; c < 3; ++c) {
                        const double *q = cf + (size_t)9 * N * c + 9 * p;
                        st->E[c][p] = q[4] * st->E[c][p] - q[5] * st->J[c][p] + q[6] * curl[c];
                    }
                }
        if (pb->source == 2) {
            /* Ex(k) reads Hy(k-1/2) and Hy(k+1/2), with a minus sign in the curl */
            for (int64_t i = xlo; i < xhi; ++i)
                for (int64_t j = ylo; j < yhi; ++j) {
                    Ex[IX(i, j, b0)] += cf[9 * IX(i, j, b0) + 6] * Hi[b0 - 1 + ao];
                    Ex[IX(i, j, b1)] -= cf[9 * IX(i, j, b1) + 6] * Hi[b1 + ao];
                }
            /* Ez(i) reads Hy(i-1/2) and Hy(i+1/2) */
            if (!px)
                for (int64_t j = ylo; j < yhi; ++j)
                    for (int64_t k = b0; k < b1; ++k) {
                        const double *q0 = cf + (size_t)9 * N * 2 + 9 * IX(b0, j, k);
                        const double *q1 = cf + (size_t)9 * N * 2 + 9 * IX(b1, j, k);
                        Ez[IX(b0, j, k)] -= q0[6] * Hi[k + ao];
                        Ez[IX(b1, j, k)] += q1[6] * Hi[k + ao];
                    }
        } else if (pb->source == 1) {
            const double s = or_source(tnew, pb->src_tau, pb->src_t0, pb->src_amp);
            for (int64_t i = 0; i < nx; ++i)
                for (int64_t j = 0; j < ny; ++j) st->E[pb->src_comp][IX(i, j, pb->src_k)] += s;
        }
        /* PEC: tangential E on the index-0 faces of walled axes */
        if (!px)
            for (int64_t j = 0; j < ny; ++j)
                for (int64_t k = 0; k < nz; ++k) { Ey[IX(0, j, k)] = 0.0; Ez[IX(0, j, k)] = 0.0; }
        if (!py)
            for (int64_t i = 0; i < nx; ++i)
                for (int64_t k = 0; k < nz; ++k) { Ex[IX(i, 0, k)] = 0.0; Ez[IX(i, 0, k)] = 0.0; }
        for (int64_t i = 0; i < nx; ++i)
            for (int64_t j = 0; j < ny; ++j) { Ex[IX(i, j, 0)] = 0.0; Ey[IX(i, j, 0)] = 0.0; }
        /* ---- J^{n+1}, eq.(11) ---- */
        for (int c = 0; c < 3; ++c)
            for (int64_t p = 0; p < N; ++p) {
                const double *q = cf + (size_t)9 * N * c + 9 * p;
                st->J[c][p] = q[0] * st->J[c][p] + q[7] * Eold[(size_t)c * N + p] + q[8] * st->E[c][p];
            }
        /* ---- incident E^{n+1}: vacuum, soft source, first-order Mur ends ---- */
        if (pb->source == 2) {
            const double e0 = Ei[0], e1 = Ei[1], f0 = Ei[na - 1], f1 = Ei[na - 2];
            for (int64_t q = 1; q < na - 1; ++q) Ei[q] = Ei[q] - ced * (Hi[q] - Hi[q - 1]);
            Ei[pb->aux_src] += or_source(tnew, pb->src_tau, pb->src_t0, pb->src_amp);
            Ei[0] = e1 + cm * (Ei[1] - e0);
            Ei[na - 1] = f1 + cm * (Ei[na - 2] - f0);
        }
        st->step += 1;
        /* ---- running DFT of the sample points ---- */
        for (int q = 0; q < pb->n_points; ++q) {
            const int32_t *s = pb->points + 4 * q;
            const int c = s[0];
            const double v = c < 3 ? st->E[c][IX(s[1], s[2], s[3])] : st->H[c - 3][IX(s[1], s[2], s[3])];
            double *xr = st->Xre + (size_t)q * pb->n_freqs, *xi = st->Xim + (size_t)q * pb->n_freqs;
            for (int f = 0; f < pb->n_freqs; ++f) {
                double cs, sn;
                if (c < 3)
                    or_twiddle(pb->freqs[f], dt, st->step, &cs, &sn);
                else     /* (m - 1/2) dt = (2m - 1) (dt/2) */
                    or_twiddle(pb->freqs[f], 0.5 * dt, 2 * st->step - 1, &cs, &sn);
                xr[f] += v * dt * cs;
                xi[f] -= v * dt * sn;
            }
        }
    }
#undef IX
    free(cf);
    free(Eold);
    return 0;
}
