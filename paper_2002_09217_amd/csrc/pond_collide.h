// pond_collide.h -- per-node pieces of the non-local closure and the collision of the
// two-population Particles-on-Demand step (eqs. 9, 16-22; App. F), shared by the
// collision kernel (k_force_collide) and the fused step kernel (k_step), so that both
// compute the same arithmetic.  The stencil helpers read LDS regions laid out row by row
// (x fastest) with a given row stride.
#pragma once

#include "pond_device.h"

namespace pond {

// fields of the thermodynamic region of a tile
enum { kThFx = 0, kThFy, kThT, kThH, kThMu, kThKc, kThP, kThFields };

// ---------------------------------------------------------------------------
// Streamed-state moment planes (pond_internal.h, "mom") in FP64, or in the mixed form of
// the FP32 storage precisions: rho, u and the g moment (0,0) = 2 rho E stay FP64 (planes
// of the conserved quantities and the gauge), the other central moments are FP32.
// Memory: the FP64 planes in layout order, then the FP32 planes in layout order.
// ---------------------------------------------------------------------------
template <int DIM, bool MIXED> struct MomIO {
    using L = Layout<DIM>;
    static constexpr int NP = L::kMomPlanes;
    static constexpr int ND = MIXED ? DIM + 2 : NP; // FP64 planes
    static constexpr bool dbl(int i) { return !MIXED || i <= DIM || i == L::kG; }
    // index of plane i among the planes of its type
    static constexpr int slot(int i) { return !MIXED ? i : (i <= DIM ? i : (i == L::kG ? DIM + 1 : (i < L::kG ? i - DIM - 1 : i - DIM - 2))); }
    // bytes per node
    static constexpr int bytes() { return ND * 8 + (NP - ND) * 4; }
    __device__ static __forceinline__ double load(const void *base, size_t N, size_t node, int i)
    {
        if (dbl(i)) return ((const POND_GLOBAL double *)base)[(size_t)slot(i) * N + node];
        return (double)((const POND_GLOBAL float *)((const POND_GLOBAL double *)base + (size_t)ND * N))[(size_t)slot(i) * N + node];
    }
    __device__ static __forceinline__ void store(void *base, size_t N, size_t node, int i, double v)
    {
        if (dbl(i))
            ((POND_GLOBAL double *)base)[(size_t)slot(i) * N + node] = v;
        else
            ((POND_GLOBAL float *)((POND_GLOBAL double *)base + (size_t)ND * N))[(size_t)slot(i) * N + node] = (float)v;
    }
};

// Korteweg stress K = -kappa (rho lap rho + |grad rho|^2/2) I + kappa grad rho grad rho
// (eq. 18) at the position `rb` of an LDS rho region of row stride RX, with the isotropic
// stencils grad = (1/T_L) sum W c, lap = (2/T_L) sum W (. - .0).  K = (xx, xy, yy).
template <int DIM>
__device__ __forceinline__ void korteweg_stress(const double *s_rho, int rb, int RX, double kappa, double K[3])
{
    constexpr int Q = Layout<DIM>::Q;
    const double r0 = s_rho[rb];
    double gx = 0.0, gy = 0.0, lap = 0.0;
#pragma unroll
    for (int q = 0; q < Q; ++q) {
        const int ex = DIM == 2 ? q / 3 - 1 : q - 1;
        const int ey = DIM == 2 ? q % 3 - 1 : 0;
        const double w = DIM == 2 ? kW1[q / 3] * kW1[q % 3] : kW1[q];
        const double rq = s_rho[rb + ex + ey * RX];
        gx += w * (double)ex * rq;
        gy += w * (double)ey * rq;
        lap += w * (rq - r0);
    }
    gx *= kInvTL;
    gy *= kInvTL;
    lap *= 2.0 * kInvTL;
    const double iso = -kappa * (r0 * lap + 0.5 * (gx * gx + gy * gy));
    K[0] = iso + kappa * gx * gx;
    K[1] = kappa * gx * gy;
    K[2] = DIM == 2 ? iso + kappa * gy * gy : 0.0;
}

// F = -div K (App. F) at the position `kb` of an LDS K region of row stride KX
template <int DIM>
__device__ __forceinline__ void korteweg_force(const double *Kxx, const double *Kxy, const double *Kyy, int kb,
                                               int KX, double &Fx, double &Fy)
{
    constexpr int Q = Layout<DIM>::Q;
    double dvx = 0.0, dvy = 0.0;
#pragma unroll
    for (int q = 0; q < Q; ++q) {
        const int ex = DIM == 2 ? q / 3 - 1 : q - 1;
        const int ey = DIM == 2 ? q % 3 - 1 : 0;
        const double w = DIM == 2 ? kW1[q / 3] * kW1[q % 3] : kW1[q];
        const int k = kb + ex + ey * KX;
        dvx += w * (Kxx[k] * (double)ex + Kxy[k] * (double)ey);
        dvy += w * (Kxy[k] * (double)ex + Kyy[k] * (double)ey);
    }
    Fx = -dvx * kInvTL;
    Fy = DIM == 2 ? -dvy * kInvTL : 0.0;
}

// Thermodynamic state of a node from its streamed density, gauge velocity, g sum
// (2 rho E) and force: u-hat = u + F dt/(2 rho), e = E - |u-hat|^2/2, T and p from the
// EoS, h = e + p/rho, mu = (1/omega - 1/2) p dt, k = k_scale mu C_p^ig.  Writes the
// fields of an LDS thermodynamic region (field stride `stride`) at index li; returns the
// admissibility bits.  GEN = false: the van der Waals fluid with its energy equation only
// (the lean variant of the streaming kernels).
template <int DIM, bool GEN = true, typename PT>
__device__ __forceinline__ int thermo_state(const PT &P, double rho, double ux, double uy, double G0, double Fx,
                                            double Fy, double visc, double *th, int stride, int li)
{
    const double dt = P.dt;
    // van der Waals without the generic laws: one division gives 1 / rho and 1 / (1 - b rho)
    const double q = 1.0 - P.b * rho;
    const double i_rq = GEN ? 0.0 : 1.0 / (rho * q);
    const double h_r = GEN ? 0.5 / rho : 0.5 * q * i_rq;
    const double E = G0 * h_r;
    const double uhx = ux + Fx * dt * h_r;
    const double uhy = DIM == 2 ? uy + Fy * dt * h_r : 0.0;
    const double e = E - 0.5 * (uhx * uhx + uhy * uhy);
    const double T = eos_T_of_e<GEN>(P, rho, e);
    const double p = GEN ? eos_p<GEN>(P, rho, T) : vdw_p_lean(P, rho, T, i_rq);
    const int err = eos_bad<GEN>(P, rho, p);
    const double mu = visc * p;
    th[kThFx * stride + li] = Fx;
    th[kThFy * stride + li] = Fy;
    th[kThT * stride + li] = T;
    th[kThH * stride + li] = e + 2.0 * p * h_r;
    th[kThMu * stride + li] = mu;
    th[kThKc * stride + li] = P.k_scale * mu * P.Cp_ig;
    th[kThP * stride + li] = p;
    return err;
}

// Populations of one set in the collision gauge (u, theta = s^2) from its streamed
// central moments about u: f moments with (0,0) = rho and the first moments zero (the
// stored f moments are (1,1), (2,0), (0,2), (2,1), (1,2), (2,2) in 2D, (2) in 1D), or all
// nine g moments (App. C through the moments: the quadratic Lagrange basis of the gauge).
template <int DIM>
__device__ __forceinline__ void pops_from_central(int set, double rho, const double *oset, double s, double *pop)
{
    constexpr int NF = Layout<DIM>::NF;
    double mc[NF];
    if (set == 0) {
        if (DIM == 2) {
            mc[0] = rho;
            mc[1] = 0.0; // (0,1): zero about u
            mc[3] = 0.0; // (1,0)
            mc[4] = oset[0];
            mc[6] = oset[1];
            mc[2] = oset[2];
            mc[7] = oset[3];
            mc[5] = oset[4];
            mc[8] = oset[5];
        } else {
            mc[0] = rho;
            mc[1] = 0.0;
            mc[2] = oset[0];
        }
    } else {
#pragma unroll
        for (int i = 0; i < NF; ++i) mc[i] = oset[i];
    }
    double A[3][3];
    lagrange_coeffs(0.0, s, A);
    if (DIM == 2) {
        // separable: first along y (index n -> l), then along x (m -> k)
        double tt[3][3];
#pragma unroll
        for (int m = 0; m < 3; ++m)
#pragma unroll
            for (int l = 0; l < 3; ++l)
                tt[m][l] = A[l][0] * mc[3 * m] + A[l][1] * mc[3 * m + 1] + A[l][2] * mc[3 * m + 2];
#pragma unroll
        for (int k = 0; k < 3; ++k)
#pragma unroll
            for (int l = 0; l < 3; ++l) pop[3 * k + l] = A[k][0] * tt[0][l] + A[k][1] * tt[1][l] + A[k][2] * tt[2][l];
    } else {
#pragma unroll
        for (int k = 0; k < 3; ++k) pop[k] = A[k][0] * mc[0] + A[k][1] * mc[1] + A[k][2] * mc[2];
    }
}

// f: BGK towards rho W plus the force source S = G^{u}_{u+du}[rho W] - rho W (eqs. 16-17)
template <int DIM, typename PT>
__device__ __forceinline__ void collide_f(const PT &P, double rho, double i_rho, const double *F, double theta,
                                          double s, const double *pop, double *post)
{
    constexpr int Q = Layout<DIM>::Q;
    const double dt = P.dt;
    const double i_theta = 1.0 / theta;
    const double i_s = s * i_theta;
    double sx[3], sy[3] = {0.0, 0.0, 0.0};
    source_axis(F[0] * dt * i_rho, i_theta, i_s, sx);
    if (DIM == 2) source_axis(F[1] * dt * i_rho, i_theta, i_s, sy);
#pragma unroll
    for (int q = 0; q < Q; ++q) {
        const int k = DIM == 2 ? q / 3 : q;
        const int l = DIM == 2 ? q % 3 : 1;
        const double wk = kW1[k], wl = DIM == 2 ? kW1[l] : 1.0;
        const double Sq = DIM == 2 ? rho * (wk * sy[l] + sx[k] * wl + sx[k] * sy[l]) : rho * sx[k];
        const double feq = rho * (wk * wl);
        post[q] = pop[q] + P.omega * (feq - pop[q]) + Sq;
    }
}

// heat-flux correction M0 = 2 div(-mu grad h + k grad T) in flux form (eq. 9), at the
// position hb of an LDS thermodynamic region of row stride HX and field stride HS
template <int DIM, typename PT>
__device__ __forceinline__ double heat_correction(const PT &P, const double *th, int HS, int hb, int HX)
{
    constexpr int Q = Layout<DIM>::Q;
    if (!(P.k_scale >= 0.0)) return 0.0;
    const double T0 = th[kThT * HS + hb], h0 = th[kThH * HS + hb];
    const double m0 = th[kThMu * HS + hb], k0 = th[kThKc * HS + hb];
    double acc = 0.0;
#pragma unroll
    for (int q = 0; q < Q; ++q) {
        const int ex = DIM == 2 ? q / 3 - 1 : q - 1;
        const int ey = DIM == 2 ? q % 3 - 1 : 0;
        const double w = DIM == 2 ? kW1[q / 3] * kW1[q % 3] : kW1[q];
        const int k = hb + ex + ey * HX;
        const double kmid = 0.5 * (th[kThKc * HS + k] + k0);
        const double mmid = 0.5 * (th[kThMu * HS + k] + m0);
        acc += w * (kmid * (th[kThT * HS + k] - T0) - mmid * (th[kThH * HS + k] - h0));
    }
    return 2.0 * (2.0 * kInvTL) * acc;
}

// g: BGK towards the force-extended equilibrium plus (g~ + phi) dt (eqs. 19-22); G0 is
// the streamed g sum 2 rho E
template <int DIM, typename PT>
__device__ __forceinline__ void collide_g(const PT &P, double rho, double i_rho, const double *u, const double *F,
                                          double p, double s, double G0, double M0, const double *pop, double *post)
{
    constexpr int Q = Layout<DIM>::Q;
    const double dt = P.dt;
    const double i_p = 1.0 / p;
    const double E = 0.5 * G0 * i_rho;
    const double uh[2] = {u[0] + 0.5 * F[0] * dt * i_rho, DIM == 2 ? u[1] + 0.5 * F[1] * dt * i_rho : 0.0};
    const double Pr = p * i_rho;
    const double H = E + Pr;
    const double dt_Pr = dt * rho * i_p;                   // dt / Pr
    double X[2][2], M[2], Nm[2][2];
#pragma unroll
    for (int a = 0; a < DIM; ++a)
#pragma unroll
        for (int b = 0; b < DIM; ++b)
            X[a][b] = uh[a] * F[b] + F[a] * uh[b] + 0.5 * dt * F[a] * F[b] * E * i_p;
#pragma unroll
    for (int a = 0; a < DIM; ++a) {
        double xu = 0.0;
#pragma unroll
        for (int b = 0; b < DIM; ++b) xu += X[a][b] * u[b];
        M[a] = dt_Pr * (F[a] * H - xu);
    }
#pragma unroll
    for (int a = 0; a < DIM; ++a)
#pragma unroll
        for (int b = 0; b < DIM; ++b) Nm[a][b] = (a == b ? rho : 0.0) + 0.5 * dt_Pr * X[a][b];
    double work = 0.0;
#pragma unroll
    for (int a = 0; a < DIM; ++a) work += 2.0 * uh[a] * F[a];
    const double c_uc = 0.5 * kInvTL * rho * i_p;          // rho / (2 p T_L)
    const double c_v2 = 0.5 * rho * i_p;                   // rho / (2 p)
#pragma unroll
    for (int q = 0; q < Q; ++q) {
        const double c[2] = {DIM == 2 ? (double)(q / 3 - 1) : (double)(q - 1),
                             DIM == 2 ? (double)(q % 3 - 1) : 0.0};
        const double wq = DIM == 2 ? kW1[q / 3] * kW1[q % 3] : kW1[q];
        double v[2], t1 = 0.0, t2 = 0.0, uc = 0.0, v2 = 0.0;
#pragma unroll
        for (int a = 0; a < DIM; ++a) {
            v[a] = u[a] + s * c[a];
            uc += u[a] * c[a];
            v2 += v[a] * v[a];
        }
#pragma unroll
        for (int a = 0; a < DIM; ++a) t1 += M[a] * (v[a] - u[a]);
#pragma unroll
        for (int a = 0; a < DIM; ++a)
#pragma unroll
            for (int b = 0; b < DIM; ++b) t2 += Nm[a][b] * (v[a] * v[b] - (a == b ? Pr : 0.0) - u[a] * u[b]);
        const double geq = wq * (2.0 * rho * E + t1 + t2);
        const double psi = wq * (1.0 + c_uc * uc * uc - c_v2 * v2 + 0.5 * (double)DIM);
        post[q] = pop[q] + P.omega * (geq - pop[q]) + (M0 + work) * psi * dt;
    }
}

// ---------------------------------------------------------------------------
// The collision in moment space.  The populations of a set in the collision gauge
// (u, theta = s^2) sit on the velocities u + xi, xi = s c, and are fixed by their nine
// central moments about u (the transfer of App. C is exact for them).  The collision is
// linear in the populations, and its equilibria and sources are given in closed form, so
// the central moments of the collided populations follow directly from the streamed
// ones: with the lattice moments of the weights per axis, sum_c W_c xi^k = 1, 0, theta/3,
// 0, theta^2/3 for k = 0..4,
//   f: BGK towards rho W, whose central moments are rho a_m a_n (a = 1, 0, theta/3), plus
//      the force source S = G^{u}_{u+du}[rho W] - rho W, whose moments are
//      rho (e_m(du_x) e_n(du_y) - a_m a_n), e = 1, du, du^2 + theta/3 (eqs. 16-17);
//   g: BGK towards the force-extended equilibrium w_q P(xi) and the source (M0 + 2 u^.F)
//      dt Psi_q, Psi_q = w_q Q(xi), both quadratic polynomials in xi (eqs. 9, 19-22), whose
//      moments are sums of products of the per-axis lattice moments.
// The result is returned as the moments about a reference velocity r (shift d = u - r),
// out[3 m + n] = sum_q f*_q (d_x + xi_x)^m (d_y + xi_y)^n, as moments_about would take
// them from the collided populations.  `oset` holds the streamed central moments of the
// set as stored (f: (1,1), (2,0), (0,2), (2,1), (1,2), (2,2); g: all nine).
// ---------------------------------------------------------------------------
template <int DIM, typename PT>
__device__ __forceinline__ void collide_moments(const PT &P, int set, double rho, double i_rho, double i_p,
                                                const double *u, const double *F, double p, double theta, double G0,
                                                double M0, const double *oset, double dx, double dy, double *out)
{
    constexpr int NF = Layout<DIM>::NF;
    const double dt = P.dt, om = P.omega;
    const double t3 = theta * kTL;                         // theta / 3 = p / rho
    const double mu[5] = {1.0, 0.0, t3, 0.0, theta * t3}; // per-axis lattice moments of xi
    double c[NF];                                          // collided central moments
    if (set == 0) {
        double mc[NF];
        if (DIM == 2) {
            mc[0] = rho;
            mc[1] = 0.0;
            mc[3] = 0.0;
            mc[4] = oset[0];
            mc[6] = oset[1];
            mc[2] = oset[2];
            mc[7] = oset[3];
            mc[5] = oset[4];
            mc[8] = oset[5];
        } else {
            mc[0] = rho;
            mc[1] = 0.0;
            mc[2] = oset[0];
        }
        const double dux = F[0] * dt * i_rho, duy = DIM == 2 ? F[1] * dt * i_rho : 0.0;
        const double a[3] = {1.0, 0.0, t3};
        const double ex[3] = {1.0, dux, dux * dux + t3};
        const double ey[3] = {1.0, duy, duy * duy + t3};
#pragma unroll
        for (int m = 0; m < 3; ++m) {
            if (DIM == 2) {
#pragma unroll
                for (int n = 0; n < 3; ++n) {
                    const double eq = rho * (a[m] * a[n]);
                    const double src = rho * (ex[m] * ey[n] - a[m] * a[n]);
                    c[3 * m + n] = mc[3 * m + n] + om * (eq - mc[3 * m + n]) + src;
                }
            } else {
                const double eq = rho * a[m];
                c[m] = mc[m] + om * (eq - mc[m]) + rho * (ex[m] - a[m]);
            }
        }
    } else {
        const double E = 0.5 * G0 * i_rho;
        const double uh[2] = {u[0] + 0.5 * F[0] * dt * i_rho, DIM == 2 ? u[1] + 0.5 * F[1] * dt * i_rho : 0.0};
        const double Pr = p * i_rho;
        const double H = E + Pr;
        const double dt_Pr = dt * rho * i_p;
        double X[2][2], M[2], Nm[2][2];
#pragma unroll
        for (int a = 0; a < DIM; ++a)
#pragma unroll
            for (int b = 0; b < DIM; ++b)
                X[a][b] = uh[a] * F[b] + F[a] * uh[b] + 0.5 * dt * F[a] * F[b] * E * i_p;
#pragma unroll
        for (int a = 0; a < DIM; ++a) {
            double xu = 0.0;
#pragma unroll
            for (int b = 0; b < DIM; ++b) xu += X[a][b] * u[b];
            M[a] = dt_Pr * (F[a] * H - xu);
        }
#pragma unroll
        for (int a = 0; a < DIM; ++a)
#pragma unroll
            for (int b = 0; b < DIM; ++b) Nm[a][b] = (a == b ? rho : 0.0) + 0.5 * dt_Pr * X[a][b];
        double work = 0.0;
#pragma unroll
        for (int a = 0; a < DIM; ++a) work += 2.0 * uh[a] * F[a];
        const double c_uc = 0.5 * kInvTL * rho * i_p;      // rho / (2 p T_L)
        const double c_v2 = 0.5 * rho * i_p;               // rho / (2 p)
        const double i_th = rho * kTL * i_p; // 1 / theta = rho T_L / p
        const double src = (M0 + work) * dt;
        // equilibrium 2 rho E + M.xi + sum_ab N_ab (xi_a xi_b + u_a xi_b + xi_a u_b - d_ab Pr)
        // and kernel 1 + D/2 + c_uc (u.xi)^2 / theta - c_v2 |u + xi|^2, as coefficients of
        // 1, xi_x, xi_y, xi_x^2, xi_y^2, xi_x xi_y
        double q[6], k[6];
        if (DIM == 2) {
            q[0] = 2.0 * rho * E - Pr * (Nm[0][0] + Nm[1][1]);
            q[1] = M[0] + 2.0 * (Nm[0][0] * u[0] + Nm[0][1] * u[1]);
            q[2] = M[1] + 2.0 * (Nm[1][1] * u[1] + Nm[0][1] * u[0]);
            q[3] = Nm[0][0];
            q[4] = Nm[1][1];
            q[5] = 2.0 * Nm[0][1];
            k[0] = 1.0 + 0.5 * (double)DIM - c_v2 * (u[0] * u[0] + u[1] * u[1]);
            k[1] = -2.0 * c_v2 * u[0];
            k[2] = -2.0 * c_v2 * u[1];
            k[3] = c_uc * u[0] * u[0] * i_th - c_v2;
            k[4] = c_uc * u[1] * u[1] * i_th - c_v2;
            k[5] = 2.0 * c_uc * u[0] * u[1] * i_th;
        } else {
            q[0] = 2.0 * rho * E - Pr * Nm[0][0];
            q[1] = M[0] + 2.0 * Nm[0][0] * u[0];
            q[3] = Nm[0][0];
            q[2] = q[4] = q[5] = 0.0;
            k[0] = 1.0 + 0.5 * (double)DIM - c_v2 * u[0] * u[0];
            k[1] = -2.0 * c_v2 * u[0];
            k[3] = c_uc * u[0] * u[0] * i_th - c_v2;
            k[2] = k[4] = k[5] = 0.0;
        }
        // moments of w_q (combined polynomial): the equilibrium weighted by omega plus the
        // source kernel weighted by src
        double w[6];
#pragma unroll
        for (int i = 0; i < 6; ++i) w[i] = om * q[i] + src * k[i];
#pragma unroll
        for (int m = 0; m < 3; ++m) {
            if (DIM == 2) {
#pragma unroll
                for (int n = 0; n < 3; ++n) {
                    const double pm = w[0] * mu[m] * mu[n] + w[1] * mu[m + 1] * mu[n] + w[2] * mu[m] * mu[n + 1] +
                                      w[3] * mu[m + 2] * mu[n] + w[4] * mu[m] * mu[n + 2] +
                                      w[5] * mu[m + 1] * mu[n + 1];
                    c[3 * m + n] = (1.0 - om) * oset[3 * m + n] + pm;
                }
            } else {
                const double pm = w[0] * mu[m] + w[1] * mu[m + 1] + w[3] * mu[m + 2];
                c[m] = (1.0 - om) * oset[m] + pm;
            }
        }
    }
    // central moments about u -> moments about r: binomial shift by d per axis
    if (DIM == 2) {
        double t[3][3];
#pragma unroll
        for (int n = 0; n < 3; ++n) {
            t[0][n] = c[n];
            t[1][n] = c[3 + n] + dx * c[n];
            t[2][n] = c[6 + n] + 2.0 * dx * c[3 + n] + dx * dx * c[n];
        }
#pragma unroll
        for (int m = 0; m < 3; ++m) {
            out[3 * m] = t[m][0];
            out[3 * m + 1] = t[m][1] + dy * t[m][0];
            out[3 * m + 2] = t[m][2] + 2.0 * dy * t[m][1] + dy * dy * t[m][0];
        }
    } else {
        out[0] = c[0];
        out[1] = c[1] + dx * c[0];
        out[2] = c[2] + 2.0 * dx * c[1] + dx * dx * c[0];
    }
}

} // namespace pond
