// Per-node physics of the 1D RKETD-FDTD plasma step, shared by every kernel of
// the library so that all execution modes (per-step, temporally blocked,
// resident) produce bit-identical results.  Host code uses the same inline
// functions for setup tables.
//
// Paper, section II:
//   eq.(14)  H^{n+1/2}(k+1/2) = H^{n-1/2}(k+1/2) - dt/(mu0 dz) [E^n(k+1) - E^n(k)]
//   eq.(11)  J^{n+1} = e^{-nu dt} J^n + (1-e^{-nu dt})/nu eps0 wp^2 E^n
//                     + (e^{-nu dt}-1+nu dt)/(nu^2 dt) eps0 wp^2 (E^{n+1} - E^n)
//   eq.(12)  E^{n+1} = E^n - dt/(eps0 dz) [H(k+1/2) - H(k-1/2)] - dt/(2 eps0) (J^{n+1} + J^n)
// Solving (11) and (12) together for E^{n+1} gives, with x = nu dt,
//   a = e^{-x}, phi1 = (1-e^{-x})/x, phi2 = (e^{-x}-1+x)/x^2, w = (wp dt)^2,
//   D = 1 + w phi2/2, CA = 1 - w phi1/(2D), CJ = dt (1+a)/(2 eps0 D),
//   CH = dt/(eps0 dz D), b1 = eps0 wp^2 dt (phi1-phi2), b2 = eps0 wp^2 dt phi2:
//   E^{n+1} = CA E^n - CJ J^n - CH curl H,   J^{n+1} = a J^n + b1 E^n + b2 E^{n+1}.
// The printed eq.(13) keeps 1/D on the E^n term only (scheme PAPER_EQ13);
// eq.(9) is the first-order variant (scheme ETD1: b1 = eps0 wp^2 dt phi1, b2 = 0).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace fdtdp {

// SI constants (CODATA 2018 eps0; c exact); mu0 = 1/(eps0 c^2).
constexpr double kC0 = 299792458.0;
constexpr double kEps0 = 8.8541878128e-12;
constexpr double kPi = 3.14159265358979323846;

__host__ __device__ inline double mu0() { return 1.0 / (kEps0 * kC0 * kC0); }

struct Coef {
    double CA, CJ, CH, a, b1, b2;
    double CAm1;   // CA - 1, formed directly (no cancellation); +0 in vacuum
};

// phi-functions of the exponential integrator.  For x <= 0.5 the closed forms
// cancel catastrophically (and divide by zero at nu = 0), so phi2 is summed
// from its Taylor series sum_k (-x)^k/(k+2)! in Horner form; then
// phi1 = 1 - x phi2 and a = 1 - x phi1 are exact identities with no
// cancellation at small x.  Above 0.5 the closed forms are well conditioned.
__host__ __device__ inline void phi_funcs(double x, double &a, double &p1, double &p2)
{
    if (x <= 0.5) {
        // 1/(k+2)! for k = 16 .. 0 (truncation below 2.4e-21 at x = 0.5)
        constexpr double inv[17] = {
            1.0 / 6402373705728000.0,  // 1/18!
            1.0 / 355687428096000.0,   // 1/17!
            1.0 / 20922789888000.0,    // 1/16!
            1.0 / 1307674368000.0,     // 1/15!
            1.0 / 87178291200.0,       // 1/14!
            1.0 / 6227020800.0,        // 1/13!
            1.0 / 479001600.0,         // 1/12!
            1.0 / 39916800.0,          // 1/11!
            1.0 / 3628800.0,           // 1/10!
            1.0 / 362880.0,            // 1/9!
            1.0 / 40320.0,             // 1/8!
            1.0 / 5040.0,              // 1/7!
            1.0 / 720.0,               // 1/6!
            1.0 / 120.0,               // 1/5!
            1.0 / 24.0,                // 1/4!
            1.0 / 6.0,                 // 1/3!
            1.0 / 2.0};                // 1/2!
        // below x = 2^-7 the terms from x^8/10! on fall under 4e-24 of phi2,
        // so the sum starts at 1/9! (every workload here: x <= 1e-2 only above
        // nu = 8e10 s^-1)
        double s;
        if (x <= 0.0078125) {
            s = inv[9];
            for (int k = 10; k < 17; ++k) s = __builtin_fma(s, -x, inv[k]);
        } else {
            s = inv[0];
            for (int k = 1; k < 17; ++k) s = __builtin_fma(s, -x, inv[k]);
        }
        p2 = s;
        p1 = __builtin_fma(-x, p2, 1.0);
        a = __builtin_fma(-x, p1, 1.0);
    } else {
        a = exp(-x);
        p1 = (1.0 - a) / x;
        p2 = (a - 1.0 + x) / (x * x);
    }
}

// Coefficients of one node.  In vacuum (wp2 = 0) this yields CA = 1, CJ = dt
// (1+a)/(2 eps0), CH = dt/(eps0 dz), b1 = b2 = 0.
__host__ __device__ inline Coef node_coef(double wp2, double nu, double dt, double dz, int scheme)
{
    double a, p1, p2;
    phi_funcs(nu * dt, a, p1, p2);
    const double w = wp2 * dt * dt;
    Coef c;
    c.a = a;
    if (scheme == 2) {  // ETD1, eq.(9)
        c.b1 = kEps0 * wp2 * dt * p1;
        c.b2 = 0.0;
        c.CAm1 = 0.0 - 0.5 * w * p1;
        c.CA = 1.0 - 0.5 * w * p1;
        c.CJ = dt * (1.0 + a) / (2.0 * kEps0);
        c.CH = dt / (kEps0 * dz);
        return c;
    }
    c.b1 = kEps0 * wp2 * dt * (p1 - p2);
    c.b2 = kEps0 * wp2 * dt * p2;
    const double D = 1.0 + 0.5 * w * p2;
    const double rD = 1.0 / D;   // one division; the three quotients by D multiply by it
    c.CAm1 = 0.0 - 0.5 * w * p1 * rD;
    c.CA = 1.0 - 0.5 * w * p1 * rD;
    if (scheme == 1) {  // eq.(13) as printed
        c.CJ = dt * (1.0 + a) / (2.0 * kEps0);
        c.CH = dt / (kEps0 * dz);
    } else {
        c.CJ = dt * (1.0 + a) * (0.5 / kEps0) * rD;
        // in vacuum rD = 1 exactly, so CH keeps the bits of dt/(eps0 dz) that
        // the vacuum update uses
        c.CH = (dt / (kEps0 * dz)) * rD;
    }
    return c;
}

// d(coefficient)/d(wp2) for the consistent scheme (adjoint gradients).
struct DCoef {
    double dCA, dCJ, dCH, db1, db2;
};

__host__ __device__ inline DCoef node_dcoef(double wp2, double nu, double dt, double dz)
{
    double a, p1, p2;
    phi_funcs(nu * dt, a, p1, p2);
    const double D = 1.0 + 0.5 * wp2 * dt * dt * p2;
    const double dD = 0.5 * dt * dt * p2;
    const Coef c = node_coef(wp2, nu, dt, dz, 0);
    DCoef d;
    d.dCA = -(0.5 * dt * dt * p1) / (D * D);
    d.dCJ = -c.CJ * dD / D;
    d.dCH = -c.CH * dD / D;
    d.db1 = kEps0 * dt * (p1 - p2);
    d.db2 = kEps0 * dt * p2;
    return d;
}

// eq.(15) soft source value at time t.
__host__ __device__ inline double source_value(double t, double tau, double t0, double amp)
{
    const double u = t - t0;
    return amp * u * exp(-(u * u) / (2.0 * tau * tau));
}

// DFT phase of sample m at frequency f: (f dt) m cycles, reduced exactly by the
// nearest integer, times 2 pi.  The twiddle is dt e^{-j theta}.
__host__ __device__ inline void twiddle(double fdt, double dt, int64_t m, double &re, double &im)
{
    double cyc = fdt * (double)m;
    cyc = cyc - rint(cyc);
    const double th = (2.0 * kPi) * cyc;
    double s, c;
    sincos(th, &s, &c);
    re = dt * c;
    im = -dt * s;
}

// CPML grading at a depth (in nodes, measured from the inner interface):
// sigma = smax (depth/P)^m, b = exp(-sigma dt/eps0), a = b - 1 (kappa = 1, alpha = 0).
__host__ __device__ inline void cpml_ab(double depth, int P, double m, double smax, double dt,
                                        double &b, double &a)
{
    const double sigma = smax * pow(depth / (double)P, m);
    b = exp(-sigma * dt / kEps0);
    a = b - 1.0;
}

// ---- per-node updates (storage type T; plasma nodes computed in FP64) ----

// Fused multiply-add in the precision of T (__builtin_fma alone would promote
// float operands to double).
__host__ __device__ __forceinline__ float fmat(float a, float b, float c)
{
    return __builtin_fmaf(a, b, c);
}
__host__ __device__ __forceinline__ double fmat(double a, double b, double c)
{
    return __builtin_fma(a, b, c);
}

// Soft source: E + s, rounded once to the storage type.
template <typename T>
__device__ __forceinline__ T add_source(T E, double s)
{
    return (T)((double)E + s);
}

template <typename T>
__device__ __forceinline__ T h_update(T H, T Eleft, T Eright, T ch)
{
    return fmat(-ch, Eright - Eleft, H);
}

// Vacuum node: CA = 1, J = 0, CH = dt/(eps0 dz).
template <typename T>
__device__ __forceinline__ T e_update_vac(T E, T curl, T ce)
{
    return fmat(-ce, curl, E);
}

// Coefficients as the kernels hold them: the E-update triple in the storage
// precision (FP64: CA, CJ, CH; FP32: CA-1, CJ, CH, each rounded once from
// FP64), the exponential-integrator triple of the J update always in FP64.
template <typename T>
struct NodeCoef {
    T eA, eJ, eH;
    double a, b1, b2;
    // the 1D steps carry Q^n = CJ (J^{n+1} - b2 E^{n+1}) = CJ (a J^n + b1 E^n)
    // in place of J (eq.(11) rearranged): Q^n = a Q^{n-1} + qc E^n with
    // qc = CJ (a b2 + b1), and E^{n+1} = (CA - CJ b2) E^n - Q^{n-1} - CH curl,
    // the first coefficient held like eA (FP64: itself; FP32: minus 1).  The
    // E update is then two FMAs and the node holds no CJ.
    T eP;
    double qc;
};

template <typename T>
__host__ __device__ inline NodeCoef<T> node_coef_t(double wp2, double nu, double dt, double dz,
                                                   int scheme)
{
    const Coef c = node_coef(wp2, nu, dt, dz, scheme);
    NodeCoef<T> r;
    r.eA = sizeof(T) == 8 ? (T)c.CA : (T)c.CAm1;
    r.eJ = (T)c.CJ;
    r.eH = (T)c.CH;
    r.a = c.a;
    r.b1 = c.b1;
    r.b2 = c.b2;
    r.eP = sizeof(T) == 8 ? (T)(c.CA - c.CJ * c.b2) : (T)(c.CAm1 - c.CJ * c.b2);
    r.qc = c.CJ * (c.a * c.b2 + c.b1);
    return r;
}

// The E update on the carried Q (the algebra above; J^n = Q^{n-1} / CJ +
// b2 E^n), and the Q update, which reads E^n before the E update overwrites
// it.  At a vacuum node (eP as eA = 1, Q = +0, qc = 0) these give the bits of
// the vacuum update, signed zeros included, and keep Q at +0.
__device__ __forceinline__ double e_update_plasma_q(double E, double Q, double curl, const NodeCoef<double> &c)
{
    return fmat(-c.eH, curl, fmat(c.eP, E, -Q));
}
__device__ __forceinline__ float e_update_plasma_q(float E, double Q, float curl, const NodeCoef<float> &c)
{
    return fmat(-c.eH, curl, fmat(c.eP, E, E) - (float)Q);
}
// The same with CH supplied negated (nH = -CH; bit for bit, negation is exact).
__device__ __forceinline__ double e_update_plasma_qneg(double E, double Q, double curl, double nH, double eP)
{
    return fmat(nH, curl, fmat(eP, E, -Q));
}
template <typename T>
__device__ __forceinline__ double q_update(double Q, double Eold, const NodeCoef<T> &c)
{
    return __builtin_fma(c.qc, Eold, c.a * Q);
}

// Plasma node E update.  FP64: CA E - CJ J - CH curl.  FP32: the same in
// delta form, E + (CA-1) E - CJ J - CH curl, so that CA = 1 - 2.5e-4 is not
// rounded to FP32 (which would perturb the plasma term by ~2e-4).  At a vacuum
// node (CA-1 = +0, CA = 1, J = +0, CH = dt/(eps0 dz)) both forms give exactly
// the bits of e_update_vac, signed zeros included.
__device__ __forceinline__ double e_update_plasma(double E, double J, double curl,
                                                  const NodeCoef<double> &c)
{
    return fmat(-c.eH, curl, fmat(-c.eJ, J, c.eA * E));
}
__device__ __forceinline__ float e_update_plasma(float E, double J, float curl,
                                                 const NodeCoef<float> &c)
{
    return fmat(-c.eH, curl, fmat(-c.eJ, (float)J, fmat(c.eA, E, E)));
}

// The same two updates with CJ and CH supplied negated (nJ = -CJ, nH = -CH):
// bit for bit the values above, since negation is exact.  The register tiles
// hold the coefficients this way so that every FMA is an accumulate with
// plain register operands (no negation modifier to fold into the
// instruction).
__device__ __forceinline__ double e_update_plasma_neg(double E, double J, double curl, double nJ, double nH,
                                                      double eA)
{
    return fmat(nH, curl, fmat(nJ, J, eA * E));
}
__device__ __forceinline__ float e_update_plasma_neg(float E, double J, float curl, float nJ, float nH, float eA)
{
    return fmat(nH, curl, fmat(nJ, (float)J, fmat(eA, E, E)));
}

// The FP32 ablation of eq.(11): J_new = J + (a-1) J + b1 E_old + b2 E_new in
// FP32 arithmetic, every coefficient rounded once to FP32 from its FP64 value
// (a-1 formed in FP64 first, so exp(-nu dt) keeps its digits near 1).
__device__ __forceinline__ float j_update_delta(float J, float Eold, float Enew, double a, double b1,
                                                double b2)
{
    return fmat((float)b2, Enew, fmat((float)b1, Eold, fmat((float)(a - 1.0), J, J)));
}

// J_new = a J + b1 E_old + b2 E_new in FP64 for both field precisions (the 3D
// steps; the 1D steps carry Q instead, see NodeCoef): eq.(11)'s exp(-nu dt)
// fractions keep their FP64 accuracy; the E values enter already widened.
template <typename T>
__device__ __forceinline__ double j_update(double J, double Eold, double Enew, const NodeCoef<T> &c)
{
    return __builtin_fma(c.b2, Enew, __builtin_fma(c.b1, Eold, c.a * J));
}

}  // namespace fdtdp
