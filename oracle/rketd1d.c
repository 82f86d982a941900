/*
 * Oracle: plain, serial, FP64 RKETD-FDTD for a 1D unmagnetized (Drude) plasma.
 *
 * TEST INFRASTRUCTURE ONLY.  This file is the slow, obviously-correct reference
 * the HIP path is checked against.  Only the test suite, the smoke check and the
 * benchmark's CPU-baseline leg may load it.  It shares no code, header, constant
 * or table with the GPU library, and the GPU library never calls it.
 *
 * What it computes (paper section II):
 *   - Maxwell-Drude system in 1D, eqs.(4)-(6): Ex at integer nodes k, Hy at
 *     half nodes k+1/2 (stored as H[k]), Jx co-located with Ex.
 *   - H update, eq.(14) (the printed "dx" read as dz).
 *   - J update, eq.(11): ETD with F = eps0*wp^2*E interpolated linearly between
 *     E^n and E^{n+1} (eq.(11) is followed where it disagrees with eq.(10)).
 *   - E update: eqs.(11) and (12) solved together for E^{n+1}.  The printed
 *     eq.(13) divides only the E^n term by D; the consistent solution divides
 *     all three terms.  scheme = 0 is the consistent solution, scheme = 1 the
 *     printed eq.(13) literally, scheme = 2 the first-order ETD of eq.(9).
 *   - Source, eq.(15): a Gaussian-derivative soft source added to E at one node
 *     after the E update and before the J update, at time (n+1)*dt.
 *   - Probes: a running DFT  X(f) = sum_{n>=1} E^n dt exp(-j 2 pi f n dt)  in
 *     place of the FFT of section IV-B.
 *   - Boundaries: first-order Mur, CPML (kappa = 1, alpha = 0, polynomial
 *     grading), PEC, or periodic (periodic exists for the tiny-grid pins only).
 *
 * The per-cell fractions of eq.(11) are written through the phi-functions of
 * the exponential integrator, x = nu*dt:
 *   a = exp(-x),  phi1 = (1 - exp(-x))/x,  phi2 = (exp(-x) - 1 + x)/x^2,
 * so (1-e^{-nu dt})/nu = dt*phi1 and (e^{-nu dt}-1+nu dt)/(nu^2 dt) = dt*phi2.
 * For x <= 0.5 phi1 and phi2 are summed from their Taylor series (the closed
 * forms cancel catastrophically for small x and divide by zero at nu = 0).
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#include "oracle.h"

#define OR_C0   299792458.0
#define OR_EPS0 8.8541878128e-12
#define OR_PI   3.14159265358979323846

double or_c0(void) { return OR_C0; }
double or_eps0(void) { return OR_EPS0; }
double or_mu0(void) { return 1.0 / (OR_EPS0 * OR_C0 * OR_C0); }

/* ---- exponential-integrator coefficients (eqs.(9), (11)) ---------------- */

void or_phi(double x, double *a, double *phi1, double *phi2)
{
    *a = exp(-x);
    if (x <= 0.5) {
        /* phi1 = sum_k (-x)^k/(k+1)!,  phi2 = sum_k (-x)^k/(k+2)! */
        double t1 = 1.0, t2 = 0.5, s1 = 0.0, s2 = 0.0;
        for (int k = 0; k < 24; ++k) {
            s1 += t1;
            s2 += t2;
            t1 *= -x / (double)(k + 2);
            t2 *= -x / (double)(k + 3);
        }
        *phi1 = s1;
        *phi2 = s2;
    } else {
        *phi1 = (1.0 - exp(-x)) / x;
        *phi2 = (exp(-x) - 1.0 + x) / (x * x);
    }
}

/*
 * Per-cell update coefficients for the E and J updates:
 *   E^{n+1} = CA E^n - CJ J^n - CH (H(k+1/2) - H(k-1/2))
 *   J^{n+1} = a J^n + b1 E^n + b2 E^{n+1}
 * out[9*i .. 9*i+8] = {a, phi1, phi2, D, CA, CJ, CH, b1, b2}.
 */
void or_coeffs(int64_t n, const double *wp2, const double *nu, double dt,
               double dz, int scheme, double *out)
{
    const double eps0 = OR_EPS0;
    for (int64_t i = 0; i < n; ++i) {
        double a, p1, p2;
        or_phi(nu[i] * dt, &a, &p1, &p2);
        double w = wp2[i] * dt * dt;            /* (wp dt)^2 */
        double D, CA, CJ, CH, b1, b2;
        if (scheme == 2) {
            /* eq.(9): F held at F_n over the step (first order) */
            b1 = eps0 * wp2[i] * dt * p1;
            b2 = 0.0;
            D = 1.0;
            CA = 1.0 - w * p1 / 2.0;
            CJ = dt * (1.0 + a) / (2.0 * eps0);
            CH = dt / (eps0 * dz);
        } else {
            /* eq.(11): J^{n+1} = a J^n + eps0 wp^2 dt [phi1 E^n + phi2 (E^{n+1}-E^n)] */
            b1 = eps0 * wp2[i] * dt * (p1 - p2);
            b2 = eps0 * wp2[i] * dt * p2;
            /* eq.(12) with eq.(11) substituted: E^{n+1} (1 + dt b2/(2 eps0)) = ... */
            D = 1.0 + w * p2 / 2.0;
            CA = 1.0 - w * p1 / (2.0 * D);
            if (scheme == 1) {               /* eq.(13) as printed */
                CJ = dt * (1.0 + a) / (2.0 * eps0);
                CH = dt / (eps0 * dz);
            } else {                         /* consistent solution */
                CJ = dt * (1.0 + a) / (2.0 * eps0 * D);
                CH = dt / (eps0 * dz * D);
            }
        }
        double *o = out + 9 * i;
        o[0] = a; o[1] = p1; o[2] = p2; o[3] = D; o[4] = CA;
        o[5] = CJ; o[6] = CH; o[7] = b1; o[8] = b2;
    }
}

/* ---- source, eq.(15) ----------------------------------------------------- */

double or_source(double t, double tau, double t0, double amp)
{
    double u = t - t0;
    return amp * u * exp(-(u * u) / (2.0 * tau * tau));
}

/* ---- running DFT --------------------------------------------------------- */

/*
 * One DFT term for sample index m (time m*dt): the phase in cycles is
 * (f*dt)*m, reduced by its nearest integer (exactly), then times 2*pi.
 */
void or_twiddle(double f, double dt, int64_t m, double *c, double *s)
{
    double cyc = (f * dt) * (double)m;
    cyc = cyc - nearbyint(cyc);
    double th = 2.0 * OR_PI * cyc;
    *c = cos(th);
    *s = sin(th);
}

void or_dft_accumulate(int64_t count, const double *samples, int64_t m0,
                       int n_freqs, const double *freqs, double dt,
                       double *Xre, double *Xim)
{
    for (int64_t i = 0; i < count; ++i) {
        for (int f = 0; f < n_freqs; ++f) {
            double c, s;
            or_twiddle(freqs[f], dt, m0 + i, &c, &s);
            Xre[f] += samples[i] * dt * c;
            Xim[f] -= samples[i] * dt * s;
        }
    }
}

/* ---- CPML profiles -------------------------------------------------------- */

/* Depth (in cells) of E node k / H node k (at k+1/2) inside a CPML of P cells
 * at each end of an n-node grid; 0 outside. */
static double cpml_depth(int64_t n, int64_t P, double pos)
{
    double left = (double)P - pos;
    double right = pos - (double)(n - 1 - P);
    if (left > 0.0) return left;
    if (right > 0.0) return right;
    return 0.0;
}

static void cpml_coeff(const or1d_problem *pb, double depth, double *b, double *a)
{
    const double eta0 = sqrt(or_mu0() / OR_EPS0);
    double m = pb->cpml_m > 0.0 ? pb->cpml_m : 3.0;
    double smax = pb->cpml_sigma_max > 0.0 ? pb->cpml_sigma_max
                                           : 0.8 * (m + 1.0) / (eta0 * pb->dz);
    double sigma = smax * pow(depth / (double)pb->cpml_cells, m);
    *b = exp(-sigma * pb->dt / OR_EPS0);
    *a = *b - 1.0;                  /* kappa = 1, alpha = 0 */
}

/* ---- validation ---------------------------------------------------------- */

int or1d_check(const or1d_problem *pb)
{
    if (pb->n < 3 || !(pb->dz > 0.0) || !(pb->dt > 0.0)) return -1;
    double S = OR_C0 * pb->dt / pb->dz;
    if (S > 1.0) return -2;
    for (int64_t k = 0; k < pb->n; ++k) {
        if (!(pb->wp2[k] >= 0.0) || !(pb->nu[k] >= 0.0)) return -1;
        if (pb->bc != OR_BC_PERIODIC && (k == 0 || k == pb->n - 1) && pb->wp2[k] != 0.0)
            return -1;
    }
    if (pb->bc == OR_BC_CPML && (pb->cpml_cells < 1 || 2 * pb->cpml_cells >= pb->n)) return -1;
    if (pb->src_cell >= pb->n) return -1;
    for (int p = 0; p < pb->n_probes; ++p)
        if (pb->probe_cells[p] < 0 || pb->probe_cells[p] >= pb->n) return -1;
    return 0;
}

/* ---- time stepping ------------------------------------------------------- */

/*
 * Advance st by nsteps.  st->step is the time index of the E field held in
 * st->E on entry (0 for the zero initial state).  H has n entries; entry n-1
 * is used only by the periodic boundary.
 */
int or1d_step(const or1d_problem *pb, or1d_state *st, int64_t nsteps)
{
    int rc = or1d_check(pb);
    if (rc) return rc;
    const int64_t n = pb->n;
    const double dt = pb->dt, dz = pb->dz;
    const double mu0 = or_mu0();
    const double ch = dt / (mu0 * dz);                 /* eq.(14) */
    const double S = OR_C0 * dt / dz;
    const double cm = (S - 1.0) / (S + 1.0);           /* first-order Mur */
    const int periodic = pb->bc == OR_BC_PERIODIC;
    const int cpml = pb->bc == OR_BC_CPML;

    double *cf = (double *)malloc(sizeof(double) * 9 * (size_t)n);
    double *Eold = (double *)malloc(sizeof(double) * (size_t)n);
    double *bE = NULL, *aE = NULL, *bH = NULL, *aH = NULL;
    if (!cf || !Eold) { free(cf); free(Eold); return -4; }
    or_coeffs(n, pb->wp2, pb->nu, dt, dz, pb->scheme, cf);
    if (cpml) {
        bE = (double *)calloc((size_t)n, sizeof(double));
        aE = (double *)calloc((size_t)n, sizeof(double));
        bH = (double *)calloc((size_t)n, sizeof(double));
        aH = (double *)calloc((size_t)n, sizeof(double));
        for (int64_t k = 0; k < n; ++k) {
            double de = cpml_depth(n, pb->cpml_cells, (double)k);
            double dh = cpml_depth(n, pb->cpml_cells, (double)k + 0.5);
            cpml_coeff(pb, de, &bE[k], &aE[k]);
            cpml_coeff(pb, dh, &bH[k], &aH[k]);
        }
    }

    const int64_t nH = periodic ? n : n - 1;
    const int64_t e_lo = periodic ? 0 : 1, e_hi = periodic ? n : n - 1;

    for (int64_t it = 0; it < nsteps; ++it) {
        double *E = st->E, *H = st->H, *J = st->J;
        const double E0 = E[0], E1 = E[1], Em2 = E[n - 2], Em1 = E[n - 1];

        /* H^{n+1/2} from E^n, eq.(14) (every node independent: the OpenMP
           pragmas only matter in the context-timing build, -fopenmp) */
#pragma omp parallel for schedule(static)
        for (int64_t k = 0; k < nH; ++k) {
            double dE = E[(k + 1) % n] - E[k];
            if (cpml) {
                st->psiH[k] = bH[k] * st->psiH[k] + aH[k] * dE / dz;
                H[k] = H[k] - ch * dE - (dt / mu0) * st->psiH[k];
            } else {
                H[k] = H[k] - ch * dE;
            }
        }
        /* E^{n+1} from E^n, J^n, H^{n+1/2}: eqs.(11)+(12) solved together */
#pragma omp parallel for schedule(static)
        for (int64_t k = e_lo; k < e_hi; ++k) {
            const double *c = cf + 9 * k;
            double curl = H[k] - H[(k - 1 + n) % n];
            if (cpml) {
                st->psiE[k] = bE[k] * st->psiE[k] + aE[k] * curl / dz;
                curl = curl + dz * st->psiE[k];
            }
            Eold[k] = E[k];
            E[k] = c[4] * E[k] - c[5] * J[k] - c[6] * curl;
        }
        /* soft source, eq.(15), at t = (n+1) dt */
        if (pb->src_cell >= 0) {
            double t = (double)(st->step + 1) * dt;
            E[pb->src_cell] += or_source(t, pb->src_tau, pb->src_t0, pb->src_amp);
        }
        /* J^{n+1}, eq.(11); in vacuum b1 = b2 = 0 and J stays at zero */
#pragma omp parallel for schedule(static)
        for (int64_t k = e_lo; k < e_hi; ++k) {
            const double *c = cf + 9 * k;
            J[k] = c[0] * J[k] + c[7] * Eold[k] + c[8] * E[k];
        }
        /* boundaries */
        if (pb->bc == OR_BC_MUR1) {
            E[0] = E1 + cm * (E[1] - E0);
            E[n - 1] = Em2 + cm * (E[n - 2] - Em1);
        } else if (!periodic) {
            E[0] = 0.0;                          /* PEC (also behind a CPML) */
            E[n - 1] = 0.0;
        }
        st->step += 1;
        /* running DFT of the probes */
        for (int p = 0; p < pb->n_probes; ++p) {
            double v = E[pb->probe_cells[p]];
            or_dft_accumulate(1, &v, st->step, pb->n_freqs, pb->freqs, dt,
                              st->Xre + (size_t)p * pb->n_freqs,
                              st->Xim + (size_t)p * pb->n_freqs);
        }
    }
    free(cf); free(Eold); free(bE); free(aE); free(bH); free(aH);
    return 0;
}
