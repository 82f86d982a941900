/*
 * Oracle: discrete adjoint of the 1D RKETD-FDTD step (TEST INFRASTRUCTURE ONLY).
 *
 * The forward step (see rketd1d.c) maps u^n = (E^n, H^{n-1/2}, J^n) to u^{n+1}
 * in this order of sub-steps:
 *   1. H^{n+1/2} = H^{n-1/2} - ch (E^n[k+1] - E^n[k])                  eq.(14)
 *   2. E*[k] = CA E^n[k] - CJ J^n[k] - CH (H^{n+1/2}[k] - H^{n+1/2}[k-1])
 *                                                   eqs.(11)+(12) solved
 *   3. E*[ks] += s((n+1) dt)                                            eq.(15)
 *   4. J^{n+1} = a J^n + b1 E^n + b2 E*                                 eq.(11)
 *   5. Mur (or PEC) at the two end nodes; E^{n+1} = E* elsewhere
 *   6. X(f) += E^{n+1}[p] dt exp(-j 2 pi f (n+1) dt)
 * The adjoint applies the transposes of 5, 4, 2, 1 in that (reverse) order;
 * the source does not depend on the plasma and drops out.  The whole forward
 * trajectory is stored (no checkpointing): plain and slow on purpose.
 *
 * Loss: L = sum_f |R_f|^2 with R_f = (X_f - Xv_f)/Xv_f, X the running DFT at
 * the reflection probe and Xv the same probe in a plasma-free reference run.
 * Gradient: dL/d(wp^2[k]) for every node k.  Only the consistent scheme and
 * Mur or PEC ends are supported.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#include "oracle.h"

/* One transposed step: lambda^{n+1} (in lE, lH, lJ) -> lambda^n, in place.
 * cf: per-node coefficients from or_coeffs. */
static void adjoint_step(const or1d_problem *pb, const double *cf, double cm,
                         double ch, double *lE, double *lH, double *lJ,
                         double *lEs, double *lEo)
{
    const int64_t n = pb->n;
    /* 5^T: end nodes */
    for (int64_t k = 0; k < n; ++k) { lEs[k] = 0.0; lEo[k] = 0.0; }
    for (int64_t k = 1; k < n - 1; ++k) lEs[k] = lE[k];
    if (pb->bc == OR_BC_MUR1) {
        /* E^{n+1}[0] = E^n[1] + cm (E*[1] - E^n[0]) */
        lEs[1] += cm * lE[0];
        lEo[1] += lE[0];
        lEo[0] += -cm * lE[0];
        lEs[n - 2] += cm * lE[n - 1];
        lEo[n - 2] += lE[n - 1];
        lEo[n - 1] += -cm * lE[n - 1];
    }
    /* 4^T: J^{n+1} = a J^n + b1 E^n + b2 E*  (interior nodes) */
    for (int64_t k = 1; k < n - 1; ++k) {
        const double *c = cf + 9 * k;
        lEs[k] += c[8] * lJ[k];
        lEo[k] += c[7] * lJ[k];
        lJ[k] = c[0] * lJ[k];
    }
    /* 2^T: E* = CA E^n - CJ J^n - CH (H[k] - H[k-1]) */
    for (int64_t k = 1; k < n - 1; ++k) {
        const double *c = cf + 9 * k;
        lEo[k] += c[4] * lEs[k];
        lJ[k] += -c[5] * lEs[k];
        lH[k] += -c[6] * lEs[k];
        lH[k - 1] += c[6] * lEs[k];
    }
    /* 1^T: H^{n+1/2}[k] = H^{n-1/2}[k] - ch (E^n[k+1] - E^n[k]) */
    for (int64_t k = 0; k < n - 1; ++k) {
        lEo[k] += ch * lH[k];
        lEo[k + 1] += -ch * lH[k];
    }
    for (int64_t k = 0; k < n; ++k) lE[k] = lEo[k];
    if (pb->bc == OR_BC_PEC) { lE[0] = 0.0; lE[n - 1] = 0.0; }
}

static int adjoint_supported(const or1d_problem *pb)
{
    if (pb->scheme != 0) return 0;
    return pb->bc == OR_BC_MUR1 || pb->bc == OR_BC_PEC;
}

/* lambda^{n+1} -> lambda^n for the plasma-parameterised linear step (no
 * source, no DFT, no gradient).  Arrays have n entries (lH: n-1 used). */
int or1d_adjoint_step(const or1d_problem *pb, double *lE, double *lH, double *lJ)
{
    int rc = or1d_check(pb);
    if (rc) return rc;
    if (!adjoint_supported(pb)) return -1;
    const int64_t n = pb->n;
    const double S = or_c0() * pb->dt / pb->dz;
    const double cm = (S - 1.0) / (S + 1.0);
    const double ch = pb->dt / (or_mu0() * pb->dz);
    double *cf = (double *)malloc(sizeof(double) * 9 * (size_t)n);
    double *t1 = (double *)malloc(sizeof(double) * (size_t)n);
    double *t2 = (double *)malloc(sizeof(double) * (size_t)n);
    if (!cf || !t1 || !t2) { free(cf); free(t1); free(t2); return -4; }
    or_coeffs(n, pb->wp2, pb->nu, pb->dt, pb->dz, pb->scheme, cf);
    adjoint_step(pb, cf, cm, ch, lE, lH, lJ, t1, t2);
    free(cf); free(t1); free(t2);
    return 0;
}

/*
 * Forward run of nsteps from zero storing the trajectory, then the reverse
 * sweep.  Outputs: *loss, grad[n] = dL/d wp2[k], and (if X != NULL) the
 * probe's spectrum as X[0..F-1] real parts, X[F..2F-1] imaginary parts.
 */
int or1d_adjoint_r2(const or1d_problem *pb, int64_t nsteps, int32_t probe,
                    const double *xv_re, const double *xv_im, double *loss,
                    double *grad, double *X)
{
    int rc = or1d_check(pb);
    if (rc) return rc;
    if (!adjoint_supported(pb) || probe < 0 || probe >= pb->n_probes || nsteps < 1) return -1;
    const int64_t n = pb->n;
    const int F = pb->n_freqs;
    const double dt = pb->dt, eps0 = or_eps0();
    const double S = or_c0() * dt / pb->dz;
    const double cm = (S - 1.0) / (S + 1.0);
    const double ch = dt / (or_mu0() * pb->dz);
    const size_t N = (size_t)n, T = (size_t)nsteps;

    /* trajectory: E^m, J^m for m = 0..T; H^{m+1/2} for m = 0..T-1 */
    double *Et = (double *)calloc((T + 1) * N, sizeof(double));
    double *Jt = (double *)calloc((T + 1) * N, sizeof(double));
    double *Ht = (double *)calloc(T * N, sizeof(double));
    double *cf = (double *)malloc(sizeof(double) * 9 * N);
    double *lE = (double *)calloc(N, sizeof(double));
    double *lH = (double *)calloc(N, sizeof(double));
    double *lJ = (double *)calloc(N, sizeof(double));
    double *t1 = (double *)malloc(sizeof(double) * N);
    double *t2 = (double *)malloc(sizeof(double) * N);
    double *Rre = (double *)calloc((size_t)F, sizeof(double));
    double *Rim = (double *)calloc((size_t)F, sizeof(double));
    or1d_state st;
    memset(&st, 0, sizeof st);
    st.E = (double *)calloc(N, sizeof(double));
    st.H = (double *)calloc(N, sizeof(double));
    st.J = (double *)calloc(N, sizeof(double));
    st.Xre = (double *)calloc((size_t)pb->n_probes * F, sizeof(double));
    st.Xim = (double *)calloc((size_t)pb->n_probes * F, sizeof(double));
    if (!Et || !Jt || !Ht || !cf || !lE || !lH || !lJ || !t1 || !t2 || !Rre || !Rim ||
        !st.E || !st.H || !st.J || !st.Xre || !st.Xim) {
        rc = -4;
        goto done;
    }
    or_coeffs(n, pb->wp2, pb->nu, dt, pb->dz, pb->scheme, cf);

    for (size_t m = 0; m < T; ++m) {
        rc = or1d_step(pb, &st, 1);
        if (rc) goto done;
        memcpy(Et + (m + 1) * N, st.E, N * sizeof(double));
        memcpy(Jt + (m + 1) * N, st.J, N * sizeof(double));
        memcpy(Ht + m * N, st.H, N * sizeof(double));
    }
    /* R_f and the loss */
    {
        const double *Xr = st.Xre + (size_t)probe * F, *Xi = st.Xim + (size_t)probe * F;
        double L = 0.0;
        for (int f = 0; f < F; ++f) {
            /* R = (X - Xv)/Xv */
            double nr = Xr[f] - xv_re[f], ni = Xi[f] - xv_im[f];
            double den = xv_re[f] * xv_re[f] + xv_im[f] * xv_im[f];
            Rre[f] = (nr * xv_re[f] + ni * xv_im[f]) / den;
            Rim[f] = (ni * xv_re[f] - nr * xv_im[f]) / den;
            L += Rre[f] * Rre[f] + Rim[f] * Rim[f];
            if (X) { X[f] = Xr[f]; X[F + f] = Xi[f]; }
        }
        *loss = L;
    }
    for (size_t k = 0; k < N; ++k) grad[k] = 0.0;

    const int64_t pc = pb->probe_cells[probe];
    for (int64_t m = (int64_t)T - 1; m >= 0; --m) {
        /* the DFT sample E^{m+1}[p]: dL/dE = sum_f 2 Re(conj(R_f) dt e^{-j th}/Xv_f) */
        double g = 0.0;
        for (int f = 0; f < F; ++f) {
            double c, s;
            or_twiddle(pb->freqs[f], dt, m + 1, &c, &s);
            /* w = dt (c - j s) / Xv */
            double den = xv_re[f] * xv_re[f] + xv_im[f] * xv_im[f];
            double wr = dt * (c * xv_re[f] - s * xv_im[f]) / den;
            double wi = dt * (-s * xv_re[f] - c * xv_im[f]) / den;
            g += 2.0 * (Rre[f] * wr + Rim[f] * wi);
        }
        lE[pc] += g;

        /* gradient of step m -> m+1, using lambda^{m+1} before it is transposed */
        const double *En = Et + (size_t)m * N, *En1 = Et + (size_t)(m + 1) * N;
        const double *Jn = Jt + (size_t)m * N, *Hh = Ht + (size_t)m * N;
        /* adjoint of E*: lE on interior plus the Mur terms plus b2 lJ */
        for (int64_t k = 0; k < n; ++k) t1[k] = 0.0;
        for (int64_t k = 1; k < n - 1; ++k) t1[k] = lE[k];
        if (pb->bc == OR_BC_MUR1) {
            t1[1] += cm * lE[0];
            t1[n - 2] += cm * lE[n - 1];
        }
        for (int64_t k = 1; k < n - 1; ++k) {
            const double *c = cf + 9 * k;
            double lEs = t1[k] + c[8] * lJ[k];
            double dD = dt * dt * c[2] / 2.0;
            double dCA = -(dt * dt * c[1] / 2.0) / (c[3] * c[3]);
            double dCJ = -c[5] * dD / c[3];
            double dCH = -c[6] * dD / c[3];
            double curl = Hh[k] - Hh[k - 1];
            double db1 = eps0 * dt * (c[1] - c[2]);
            double db2 = eps0 * dt * c[2];
            grad[k] += lEs * (dCA * En[k] - dCJ * Jn[k] - dCH * curl);
            grad[k] += lJ[k] * (db1 * En[k] + db2 * En1[k]);
        }
        adjoint_step(pb, cf, cm, ch, lE, lH, lJ, t1, t2);
    }
    rc = 0;
done:
    free(Et); free(Jt); free(Ht); free(cf); free(lE); free(lH); free(lJ);
    free(t1); free(t2); free(Rre); free(Rim);
    free(st.E); free(st.H); free(st.J); free(st.Xre); free(st.Xim);
    return rc;
}
