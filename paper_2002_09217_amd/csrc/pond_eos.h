// pond_eos.h -- caloric equation of state of the Dieterici fluid, for the device
// kernels and for the host code that builds inflow states.
//
// The Supplement's thermodynamics gives de = C_v dT + [T (dp/dT)_v - p] dv with C_v
// constant (polytropic).  Taking C_v as the ideal-gas heat capacity, reached as v -> oo,
// and integrating the volume part along the isotherm from there gives
//   e(rho, T) = C_v T + e_dep,  e_dep = -a int_0^rho exp(-a r / (R T)) / (1 - b r) dr
// for p = rho R T / (1 - b rho) exp(-a rho / (R T)), whose T (dp/dT)_rho - p is
// p a rho / (R T).  With beta = a / (R T b) and q = 1 - b rho the integral is a
// difference of exponential integrals:
//   e_dep = -(a / b) e^-beta [Ei(beta) - Ei(q beta)],
//   Ei(beta) - Ei(q beta) = ln(1 / q) + sum_n>=1 beta^n (1 - q^n) / (n n!),
// the series of Ei about 0 (the Euler constants cancel).  1 - q^n is accumulated as
// c_n = c_n-1 + b rho q^(n-1), which loses nothing when b rho is small.  The heat
// capacity of the state follows by differentiating in T (d beta / dT = -beta / T):
//   (de/dT)_rho = C_v + (a / (b T)) (1 - e^(-beta b rho) - beta e^-beta D).
// The series converges for every beta; the loop stops once a term no longer changes
// the sum (after about beta + 30 terms), and kDietMaxTerms bounds it, which covers
// beta < 150 (T above T_cr / 37 for the critical point T_cr = a / (4 R b)).
//
// The routines stay out of line in device code: inlined into the closure stages of the
// streaming kernels, the Newton loop raised their register pressure into spills.
#pragma once

#include <hip/hip_runtime.h>

#include <cmath>

namespace pond {

constexpr int kDietMaxTerms = 256;

// e(rho, T) of the Dieterici fluid; *cv receives (de/dT)_rho
__host__ __device__ inline __noinline__ double diet_energy(double a, double b, double R, double Cv, double rho, double T,
                                              double *cv)
{
    const double br = b * rho, q = 1.0 - br;
    const double beta = a / (R * T * b);
    double D = -log1p(-br);
    double t = 1.0, qn = 1.0, c = 0.0; // t = beta^n / n!, qn = q^(n-1), c = 1 - q^n
    for (int n = 1; n <= kDietMaxTerms; ++n) {
        t *= beta / n;
        c += br * qn;
        qn *= q;
        const double term = t * c / n;
        const double Dn = D + term;
        if (Dn == D && n > beta) break;
        D = Dn;
    }
    const double eb = exp(-beta);
    if (cv) *cv = Cv + (a / (b * T)) * (-expm1(-beta * br) - beta * eb * D);
    return Cv * T - (a / b) * eb * D;
}

// T with e(rho, T) = e: Newton's method from the van der Waals-like estimate
// (e + a rho) / C_v, each step kept above half the previous T, until the step is below
// 1e-15 T (at most 40 steps)
__host__ __device__ inline __noinline__ double diet_T_of_e(double a, double b, double R, double Cv, double rho, double e)
{
    double T = (e + a * rho) / Cv;
    if (!(T > 0.0)) T = a / (4.0 * R * b); // the critical temperature, for a start
    for (int it = 0; it < 40; ++it) {
        double cv;
        const double f = diet_energy(a, b, R, Cv, rho, T, &cv) - e;
        double Tn = T - f / cv;
        if (!(Tn > 0.5 * T)) Tn = 0.5 * T;
        const bool done = fabs(Tn - T) <= 1e-15 * Tn;
        T = Tn;
        if (done) break;
    }
    return T;
}

// T with p(rho, T) = p: Newton's method on ln p, which increases in T with slope
// 1/T + a rho / (R T^2), from the ideal-gas estimate p (1 - b rho) / (rho R)
__host__ __device__ inline __noinline__ double diet_T_of_p(double a, double b, double R, double rho, double p)
{
    const double lhs = log(p * (1.0 - b * rho) / (rho * R));
    double T = p * (1.0 - b * rho) / (rho * R);
    for (int it = 0; it < 60; ++it) {
        const double g = log(T) - a * rho / (R * T) - lhs;
        double Tn = T - g / (1.0 / T + a * rho / (R * T * T));
        if (!(Tn > 0.5 * T)) Tn = 0.5 * T;
        const bool done = fabs(Tn - T) <= 1e-15 * Tn;
        T = Tn;
        if (done) break;
    }
    return T;
}

} // namespace pond
