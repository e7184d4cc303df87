// pond_device.h -- device-side algebra of the two-population Particles-on-Demand step
// (Reyhanian, Dorschner & Karlin, arXiv:2002.09217) for gfx950.
//
// Everything here is per node and FP64 unless the caller instantiates it with float.
// The lattice is D1Q3 or D2Q9 = C1 x C1 with C1 = {-1, 0, 1}, W = (1/6, 2/3, 1/6),
// T_L = 1/3 (App. B).  Population index q = 3 (cx + 1) + (cy + 1) in 2D (x factor
// outer), q = cx + 1 in 1D.  Moment index mn = 3 m + n for sum_i f_i wx^m wy^n.
#pragma once

#include <hip/hip_runtime.h>

#include "pond_eos.h"
#include "pond_internal.h"

namespace pond {

constexpr double kTL = 1.0 / 3.0;
constexpr double kInvTL = 3.0;
constexpr double kW1[3] = {1.0 / 6.0, 2.0 / 3.0, 1.0 / 6.0};

// Weight of direction q (tensor product of W in 2D).
template <int DIM>
__device__ __forceinline__ double weight_q(int q)
{
    return DIM == 3 ? kW1[q / 9] * kW1[(q / 3) % 3] * kW1[q % 3] : DIM == 2 ? kW1[q / 3] * kW1[q % 3] : kW1[q];
}

// FP32 storage of the populations: each set is kept as its FP64 sum (one plane after
// the 2Q population planes, f then g) and the FP32 deviations f_q - W_q sum.  The
// conserved sums (rho and 2 rho E) keep FP64 precision; FP32 rounding only touches
// the departure from W_q sum, which is small near equilibrium.
template <typename PopT>
constexpr bool kDeviationStore = sizeof(PopT) == 4;

// Device buffers reached through a descriptor are generic pointers to the compiler;
// casting them to the global address space gives global (not flat) loads and stores.
#define POND_GLOBAL __attribute__((address_space(1)))

// ---------------------------------------------------------------------------
// Equations of state (main text; App. A; Supplement).  The van der Waals fluid (e =
// C_v T - a rho) and the Dieterici fluid (e = C_v T plus its departure integral, see
// pond_eos.h) run with the energy equation or isothermally; the double-well pressure
// runs isothermally.  Isothermal runs take T = T0 wherever a temperature is needed, and
// the energy population is passive, carrying e(rho, T0) of the law (C_v T for the
// double well).  The kind is uniform over a launch, so the branches are scalar.  GEN =
// false compiles the van der Waals fluid with the energy equation only: the streaming
// kernels are instantiated both ways, so that the common case carries none of the
// other laws' code and registers.
// ---------------------------------------------------------------------------
enum { kEosVdw = 0, kEosDieterici = 1, kEosWell = 2 };
template <bool GEN = true, typename PT>
__device__ __forceinline__ double eos_p(const PT &P, double rho, double T)
{
    if (GEN && P.eos == kEosDieterici) return rho * P.R * T / (1.0 - P.b * rho) * exp(-P.a * rho / (P.R * T));
    if (GEN && P.eos == kEosWell) {
        // p0 + rho E0' - E0 = p0 + beta dl dv (2 rho (dl + dv) - dl dv), dl = rho - rho_l,
        // dv = rho - rho_v, for E0 = beta dl^2 dv^2
        const double dl = rho - P.eos_c[1], dv = rho - P.eos_c[2];
        return P.eos_c[3] + P.eos_c[0] * dl * dv * (2.0 * rho * (dl + dv) - dl * dv);
    }
    return rho * P.R * T / (1.0 - P.b * rho) - P.a * rho * rho;
}
// van der Waals pressure given i_rq = 1 / (rho (1 - b rho)): the lean closures take one
// division for both 1 / rho and 1 / (1 - b rho)
template <typename PT>
__device__ __forceinline__ double vdw_p_lean(const PT &P, double rho, double T, double i_rq)
{
    return rho * rho * P.R * T * i_rq - P.a * rho * rho;
}
// temperature of a streamed state from its internal energy
template <bool GEN = true, typename PT>
__device__ __forceinline__ double eos_T_of_e(const PT &P, double rho, double e)
{
    if (GEN && P.isothermal) return P.T0;
    if (GEN && P.eos == kEosDieterici) return diet_T_of_e(P.a, P.b, P.R, P.Cv, rho, e);
    return (e + P.a * rho) * P.inv_Cv;
}
// temperature of an initial or inflow state given T
template <typename PT>
__device__ __forceinline__ double eos_state_T(const PT &P, double T)
{
    return P.isothermal ? P.T0 : T;
}
// temperature from the pressure (read-back): the inversion of the law's pressure, or T0
template <typename PT>
__device__ __forceinline__ double eos_T_of_p(const PT &P, double rho, double p)
{
    if (P.isothermal) return P.T0;
    if (P.eos == kEosDieterici) return diet_T_of_p(P.a, P.b, P.R, rho, p);
    return (p + P.a * rho * rho) * (1.0 - P.b * rho) / (rho * P.R);
}
template <typename PT>
__device__ __forceinline__ double eos_e(const PT &P, double rho, double T)
{
    if (P.eos == kEosDieterici) return diet_energy(P.a, P.b, P.R, P.Cv, rho, T, nullptr);
    return P.Cv * T - (P.eos == kEosVdw ? P.a * rho : 0.0);
}
// bit set of the admissibility violations of a state (pressure domain, finiteness)
template <bool GEN = true, typename PT>
__device__ __forceinline__ int eos_bad(const PT &P, double rho, double p)
{
    if (!isfinite(rho) || !isfinite(p)) return kErrNonfinite;
    if (!(p > 0.0) || !(rho > 0.0) || !((GEN && P.eos == kEosWell) || 1.0 - P.b * rho > 0.0)) return kErrPressure;
    return 0;
}

// ---------------------------------------------------------------------------
// Workgroups are dispatched to the 8 XCDs of the MI355X round-robin (workgroup b
// runs on XCD b mod 8), and each XCD has its own L2.  Renumber so that every XCD
// owns one contiguous run of tiles (row-major): neighbouring tiles, and the halos
// they share, then go through the same L2, and consecutive kernels that use the
// same tiling find their inputs where the previous kernel wrote them.  The map is
// a bijection of [0, nb).
// ---------------------------------------------------------------------------
constexpr int kXcds = 8;
constexpr int kCUs = 256; // compute units of the device (MI355X)
__device__ __forceinline__ int xcd_tile(int b, int nb)
{
    const int xcd = b % kXcds, local = b / kXcds;
    const int per = nb / kXcds, rem = nb % kXcds;
    return xcd < rem ? xcd * (per + 1) + local : rem * (per + 1) + (xcd - rem) * per + local;
}

// slot of a global tile: the last slot whose first tile is <= tile (binary search)
template <bool STREAM>
__device__ __forceinline__ int find_slot(const SlotDesc *slots, int nslots, int tile)
{
    int lo = 0, hi = nslots - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        const int b = STREAM ? slots[mid].st_begin : slots[mid].fc_begin;
        if (b <= tile)
            lo = mid;
        else
            hi = mid - 1;
    }
    return lo;
}

// ---------------------------------------------------------------------------
// Lattice extent and face types, held in registers.  The boundary rules below select
// between these values; indexing the parameter block with a per-lane face would be a
// vector load with a wait in front of every neighbour load that depends on it.
// ---------------------------------------------------------------------------
struct Geo {
    int nx, ny;
    int bc00, bc01, bc10, bc11; // bc[axis][side]
    __device__ __forceinline__ int bc(int axis, int side) const
    {
        return axis == 0 ? (side ? bc01 : bc00) : (side ? bc11 : bc10);
    }
};
template <typename PT>
__device__ __forceinline__ Geo make_geo(const PT &P)
{
    return Geo{P.nx, P.ny, P.bc[0][0], P.bc[0][1], P.bc[1][0], P.bc[1][1]};
}

// ---------------------------------------------------------------------------
// boundary mapping: node index >= 0, or -(1 + face) for an inflow ghost,
// face = 2 axis + side.  Periodic faces wrap, outflow faces clamp.
// ---------------------------------------------------------------------------
template <int DIM>
__device__ __forceinline__ int map_node(const Geo &g, int x, int y)
{
    if (x < 0 || x >= g.nx) {
        const int side = x < 0 ? 0 : 1;
        const int bc = g.bc(0, side);
        if (bc == kPeriodic) {
            x = x < 0 ? x + g.nx : x - g.nx;
            if (x < 0 || x >= g.nx) x = ((x % g.nx) + g.nx) % g.nx; // narrower than the halo
        } else if (bc == kOutflow)
            x = x < 0 ? 0 : g.nx - 1;
        else
            return -(1 + side);
    }
    if (DIM == 2) {
        if (y < 0 || y >= g.ny) {
            const int side = y < 0 ? 0 : 1;
            const int bc = g.bc(1, side);
            if (bc == kPeriodic) {
                y = y < 0 ? y + g.ny : y - g.ny;
                if (y < 0 || y >= g.ny) y = ((y % g.ny) + g.ny) % g.ny; // narrower than the halo
            } else if (bc == kOutflow)
                y = y < 0 ? 0 : g.ny - 1;
            else
                return -(1 + 2 + side);
        }
        return x + g.nx * y;
    }
    return x;
}

// ---------------------------------------------------------------------------
// How a derived field is read at lattice position (x, y) (same rule as map_node):
//   kSelf   the position is a node, or wraps onto one (periodic): evaluate there;
//   kCopy   an outflow face clamps it: take the value of the clamped node (cx, cy);
//   kGhost  an inflow face: the ghost state's value (face in *face).
// ---------------------------------------------------------------------------
enum { kSelf = 0, kCopy = 1, kGhost = 2 };
template <int DIM>
__device__ __forceinline__ int classify(const Geo &g, int x, int y, int &cx, int &cy, int &face)
{
    int cls = kSelf;
    cx = x;
    cy = y;
    if (x < 0 || x >= g.nx) {
        const int side = x < 0 ? 0 : 1;
        const int bc = g.bc(0, side);
        if (bc == kInflow) {
            face = side;
            return kGhost;
        }
        if (bc == kOutflow) {
            cx = x < 0 ? 0 : g.nx - 1;
            cls = kCopy;
        }
    }
    if (DIM == 2 && (y < 0 || y >= g.ny)) {
        const int side = y < 0 ? 0 : 1;
        const int bc = g.bc(1, side);
        if (bc == kInflow) {
            face = 2 + side;
            return kGhost;
        }
        if (bc == kOutflow) {
            cy = y < 0 ? 0 : g.ny - 1;
            cls = kCopy;
        }
    }
    return cls;
}

// error bits of a step, with the parity of the state it read if it is the first error
__device__ __forceinline__ void raise_error(int *flags, int bits, int parity)
{
    atomicOr(&flags[kFlagErr], bits);
    atomicCAS(&flags[kFlagErrParity], 0, parity + 1);
}

// ---------------------------------------------------------------------------
// moments of one population set about a reference velocity (rx, ry):
// out[3m+n] = sum_{a,b} f_ab (ux - rx + s (a-1))^m (uy - ry + s (b-1))^n  (2D)
// out[m]    = sum_a f_a (ux - rx + s (a-1))^m                              (1D)
// These are the moments of App. C taken about (rx, ry) instead of 0; the
// shift keeps them well scaled for any flow speed.
// ---------------------------------------------------------------------------
template <int DIM, typename T>
__device__ __forceinline__ void moments_about(const T *f, double dux, double duy, double s,
                                              double *out)
{
    if (DIM == 2) {
        double cy[3] = {duy - s, duy, duy + s};
        double cx[3] = {dux - s, dux, dux + s};
        double col[3][3]; // col[a][n] = sum_b f_ab cy_b^n
#pragma unroll
        for (int a = 0; a < 3; ++a) {
            double s0 = 0.0, s1 = 0.0, s2 = 0.0;
#pragma unroll
            for (int b = 0; b < 3; ++b) {
                const double fv = (double)f[3 * a + b];
                s0 += fv;
                s1 += fv * cy[b];
                s2 += fv * cy[b] * cy[b];
            }
            col[a][0] = s0;
            col[a][1] = s1;
            col[a][2] = s2;
        }
#pragma unroll
        for (int n = 0; n < 3; ++n) {
            out[0 + n] = col[0][n] + col[1][n] + col[2][n];
            out[3 + n] = col[0][n] * cx[0] + col[1][n] * cx[1] + col[2][n] * cx[2];
            out[6 + n] = col[0][n] * cx[0] * cx[0] + col[1][n] * cx[1] * cx[1] +
                         col[2][n] * cx[2] * cx[2];
        }
    } else {
        double cx[3] = {dux - s, dux, dux + s};
        out[0] = (double)f[0] + (double)f[1] + (double)f[2];
        out[1] = (double)f[0] * cx[0] + (double)f[1] * cx[1] + (double)f[2] * cx[2];
        out[2] = (double)f[0] * cx[0] * cx[0] + (double)f[1] * cx[1] * cx[1] +
                 (double)f[2] * cx[2] * cx[2];
    }
}

// ---------------------------------------------------------------------------
// Coefficients of the quadratic Lagrange basis on the three velocities
// du + s c, c = -1, 0, 1 (relative to the same reference as the moments):
// L_k(w) = A[k][0] + A[k][1] w + A[k][2] w^2.  Re-expressing populations given
// by their moments into this gauge is f_k = sum_m A[k][m] M_m per axis; this is
// the transfer matrix M'^{-1} M of App. C written through the moments.
// ---------------------------------------------------------------------------
__device__ __forceinline__ void lagrange_coeffs(double du, double s, double A[3][3])
{
    const double inv = 1.0 / (s * s);
    const double h = 0.5 * inv;
    A[0][0] = (du * du + s * du) * h;
    A[0][1] = -(2.0 * du + s) * h;
    A[0][2] = h;
    A[1][0] = 1.0 - du * du * inv;
    A[1][1] = 2.0 * du * inv;
    A[1][2] = -inv;
    A[2][0] = (du * du - s * du) * h;
    A[2][1] = (s - 2.0 * du) * h;
    A[2][2] = h;
}

// ---------------------------------------------------------------------------
// Cubic Lagrange reconstruction (App. D) for the three departure points of one
// axis, x - (u + s c) dt, c = -1, 0, 1, written into a five-wide window centred on
// the receiver (window column j <-> lattice offset j - 2).  Returns a nonzero
// halo flag when a stencil would leave the window.
// ---------------------------------------------------------------------------
template <typename T>
__device__ __forceinline__ int window_weights(double u, double s, double dt, T w[3][5])
{
    int bad = 0;
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        const double v = u + s * (double)(k - 1);
        const double d = -v * dt;            // displacement of the departure point
        const double fl = floor(d);
        const double t = d - fl + 1.0;       // coordinate inside the 4-node stencil
        int i0 = (int)fl;                    // stencil nodes i0-1 .. i0+2
        const double w0 = -(t - 1.0) * (t - 2.0) * (t - 3.0) * (1.0 / 6.0);
        const double w1 = t * (t - 2.0) * (t - 3.0) * 0.5;
        const double w2 = -t * (t - 1.0) * (t - 3.0) * 0.5;
        const double w3 = t * (t - 1.0) * (t - 2.0) * (1.0 / 6.0);
        if (i0 < -1 || i0 > 0) {
            bad = kErrHalo;
            i0 = i0 < -1 ? -1 : 0;
        }
        const int o = i0 + 1; // first window column of the stencil: 0 or 1
#pragma unroll
        for (int j = 0; j < 5; ++j) w[k][j] = (T)0;
        if (o == 0) {
            w[k][0] = (T)w0; w[k][1] = (T)w1; w[k][2] = (T)w2; w[k][3] = (T)w3;
        } else {
            w[k][1] = (T)w0; w[k][2] = (T)w1; w[k][3] = (T)w2; w[k][4] = (T)w3;
        }
    }
    return bad;
}

// ---------------------------------------------------------------------------
// collision pieces (eqs. 9, 16-22; App. F)
// ---------------------------------------------------------------------------
// Force source S = G^{u}_{u+du}[rho W] - rho W per axis: the equilibrium of the gauge
// (u + du, theta) in the gauge (u, theta) is rho prod_axes (W_c + sig_c(du)) with
// sig_0 = -du^2/theta, sig_pm = du^2/(2 theta) pm du/(2 sqrt(theta)).
__device__ __forceinline__ void source_axis(double du, double inv_theta, double inv_s, double sig[3])
{
    const double q = du * du * inv_theta;
    const double l = 0.5 * du * inv_s;
    sig[0] = 0.5 * q - l;
    sig[1] = -q;
    sig[2] = 0.5 * q + l;
}

// write the post-collision populations of one set (0 = f, 1 = g) of a node: as they
// are, or (FP32 storage) as the FP64 sum and the FP32 deviations from W_q sum
template <int DIM, typename PopT>
__device__ __forceinline__ void store_set(POND_GLOBAL PopT *pop, size_t N, int node, int set,
                                          const double *post)
{
    constexpr int Q = Layout<DIM>::Q;
    POND_GLOBAL PopT *out = pop + (size_t)set * Q * N;
    if constexpr (kDeviationStore<PopT>) {
        double sum = 0.0;
#pragma unroll
        for (int q = 0; q < Q; ++q) sum += post[q];
        POND_GLOBAL double *sums = (POND_GLOBAL double *)(pop + (size_t)2 * Q * N);
        sums[(size_t)set * N + node] = sum;
#pragma unroll
        for (int q = 0; q < Q; ++q) out[(size_t)q * N + node] = (PopT)(post[q] - weight_q<DIM>(q) * sum);
    } else {
#pragma unroll
        for (int q = 0; q < Q; ++q) out[(size_t)q * N + node] = (PopT)post[q];
    }
}

// ---------------------------------------------------------------------------
// conservation monitors: words per block partial and threads per block, and the
// wavefront reductions they use
// ---------------------------------------------------------------------------
constexpr int kMonWords = 8;
constexpr int kMonThreads = 256;

__device__ __forceinline__ double wave_sum(double v)
{
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}
__device__ __forceinline__ double wave_min(double v)
{
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v = fmin(v, __shfl_xor(v, o, 64));
    return v;
}
__device__ __forceinline__ double wave_max(double v)
{
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v = fmax(v, __shfl_xor(v, o, 64));
    return v;
}

} // namespace pond
