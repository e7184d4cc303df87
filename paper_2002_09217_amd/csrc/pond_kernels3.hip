// pond_kernels3.hip -- D3Q27 time step of the two-population Particles-on-Demand model
// (Reyhanian, Dorschner & Karlin, arXiv:2002.09217) on a periodic box, for gfx950.
//
// Same method as the 1D/2D kernels (eqs. 1-4, 9, 16-22; App. B-D, F), laid out for the
// 5 x 5 x 5 donor window of three dimensions, which does not fit in LDS as a tile plus
// halo:
//   k3_stream         one workgroup per x-y tile of one z plane; every predictor-corrector
//                     pass stages the five donor planes z-2 .. z+2 through LDS, one z
//                     power of one plane at a time, and accumulates for each the x-y
//                     contraction of the D2Q9 kernel followed by the z contraction;
//   k3_korteweg, k3_thermo, k3_collide
//                     Korteweg stress, force and thermodynamics, heat-flux correction and
//                     the collisions of f and g (separate waves), 27-point stencils; the
//                     collision stores the populations and each node's 27 + 27 moments
//                     about a common reference velocity (zero), gauge free, into a scratch
//                     buffer: the donor moments the next step's streaming reads;
//   k3_donor_moments  the same moments from stored populations (after a checkpoint load;
//                     an initialisation ends with a collision).
// Index conventions: direction q = 9 (cx+1) + 3 (cy+1) + (cz+1); moment 9 m + 3 n + o
// for sum f wx^m wy^n wz^o.
#include <hip/hip_runtime.h>

#include <type_traits>

#include "pond_device.h"
#include "pond_internal.h"

namespace pond {

using L3 = Layout<3>;

namespace {

struct Box {
    int nx, ny, nz;
    size_t N;
    __device__ __forceinline__ int wrap(int i, int n) const
    {
        i = i < 0 ? i + n : (i >= n ? i - n : i);
        if (i < 0 || i >= n) i = ((i % n) + n) % n; // narrower than the stencil
        return i;
    }
    __device__ __forceinline__ int node(int x, int y, int z) const
    {
        return wrap(x, nx) + nx * (wrap(y, ny) + ny * wrap(z, nz));
    }
};

// the 27 neighbours x + c of a node, c in {-1, 0, 1}^3 in direction order q: three
// wrapped offsets per axis, node index (< 2^29) as a 32-bit integer
struct Nbr27 {
    unsigned xo[3], yo[3], zo[3];
    __device__ __forceinline__ Nbr27(const Box &b, int x, int y, int z)
    {
#pragma unroll
        for (int d = 0; d < 3; ++d) {
            xo[d] = (unsigned)b.wrap(x + d - 1, b.nx);
            yo[d] = (unsigned)b.nx * (unsigned)b.wrap(y + d - 1, b.ny);
            zo[d] = (unsigned)b.nx * (unsigned)b.ny * (unsigned)b.wrap(z + d - 1, b.nz);
        }
    }
    __device__ __forceinline__ unsigned at(int q) const { return xo[q / 9] + yo[(q / 3) % 3] + zo[q % 3]; }
};

template <typename PT>
__device__ __forceinline__ Box make_box(const PT &P)
{
    return Box{P.nx, P.ny, P.nz, (size_t)P.N};
}

__device__ __forceinline__ double w27(int q) { return kW1[q / 9] * kW1[(q / 3) % 3] * kW1[q % 3]; }

// moments out[9m+3n+o] = sum_ijk f_ijk (dx + s(i-1))^m (dy + s(j-1))^n (dz + s(k-1))^o
__device__ __forceinline__ void moments27(const double *f, double dx, double dy, double dz, double s, double *out)
{
    double a1[3][3][3]; // [i][j][o]
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
        for (int j = 0; j < 3; ++j) {
            double s0 = 0.0, s1 = 0.0, s2 = 0.0;
#pragma unroll
            for (int k = 0; k < 3; ++k) {
                const double c = dz + s * (double)(k - 1);
                const double fv = f[9 * i + 3 * j + k];
                s0 += fv;
                s1 += fv * c;
                s2 += fv * c * c;
            }
            a1[i][j][0] = s0;
            a1[i][j][1] = s1;
            a1[i][j][2] = s2;
        }
    double a2[3][3][3]; // [i][n][o]
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
        for (int o = 0; o < 3; ++o) {
            double s0 = 0.0, s1 = 0.0, s2 = 0.0;
#pragma unroll
            for (int j = 0; j < 3; ++j) {
                const double c = dy + s * (double)(j - 1);
                s0 += a1[i][j][o];
                s1 += a1[i][j][o] * c;
                s2 += a1[i][j][o] * c * c;
            }
            a2[i][0][o] = s0;
            a2[i][1][o] = s1;
            a2[i][2][o] = s2;
        }
#pragma unroll
    for (int n = 0; n < 3; ++n)
#pragma unroll
        for (int o = 0; o < 3; ++o) {
            double s0 = 0.0, s1 = 0.0, s2 = 0.0;
#pragma unroll
            for (int i = 0; i < 3; ++i) {
                const double c = dx + s * (double)(i - 1);
                s0 += a2[i][n][o];
                s1 += a2[i][n][o] * c;
                s2 += a2[i][n][o] * c * c;
            }
            out[0 + 3 * n + o] = s0;
            out[9 + 3 * n + o] = s1;
            out[18 + 3 * n + o] = s2;
        }
}

// populations pop[9k+3l+m] = sum A[k][a] A[l][b] A[m][c] mc[9a+3b+c] (separable)
__device__ __forceinline__ void from_moments27(const double A[3][3], const double *mc, double *pop)
{
    double t1[3][3][3]; // [a][b][m]
#pragma unroll
    for (int a = 0; a < 3; ++a)
#pragma unroll
        for (int b = 0; b < 3; ++b)
#pragma unroll
            for (int m = 0; m < 3; ++m)
                t1[a][b][m] = A[m][0] * mc[9 * a + 3 * b] + A[m][1] * mc[9 * a + 3 * b + 1] + A[m][2] * mc[9 * a + 3 * b + 2];
    double t2[3][3][3]; // [a][l][m]
#pragma unroll
    for (int a = 0; a < 3; ++a)
#pragma unroll
        for (int l = 0; l < 3; ++l)
#pragma unroll
            for (int m = 0; m < 3; ++m) t2[a][l][m] = A[l][0] * t1[a][0][m] + A[l][1] * t1[a][1][m] + A[l][2] * t1[a][2][m];
#pragma unroll
    for (int k = 0; k < 3; ++k)
#pragma unroll
        for (int l = 0; l < 3; ++l)
#pragma unroll
            for (int m = 0; m < 3; ++m)
                pop[9 * k + 3 * l + m] = A[k][0] * t2[0][l][m] + A[k][1] * t2[1][l][m] + A[k][2] * t2[2][l][m];
}

// index of moment mno among the 23 stored f central moments (-1 for 000, 100, 010, 001)
__device__ __forceinline__ int fstored_index(int mno)
{
    // skipped: 0 (000), 1 (001), 3 (010), 9 (100)
    if (mno == 0 || mno == 1 || mno == 3 || mno == 9) return -1;
    return mno - 2 - (mno > 3) - (mno > 9);
}

__device__ __forceinline__ void raise_error3(int *flags, int bits, int parity)
{
    atomicOr(&flags[kFlagErr], bits);
    atomicCAS(&flags[kFlagErrParity], 0, parity + 1);
}

} // namespace

// ---------------------------------------------------------------------------
// donor moments about zero velocity, gauge free (one thread per node and set)
// ---------------------------------------------------------------------------
template <typename PopT, typename MomT>
__global__ void __launch_bounds__(256) k3_donor_moments(const SlotDesc *__restrict__ slot)
{
    const SlotDesc &S = *slot;
    const POND_GLOBAL DevParams &P = *(const POND_GLOBAL DevParams *)S.P;
    const size_t N = P.N;
    const size_t it = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (it >= 2 * N) return;
    if (S.flags[kFlagErr] != 0) return;
    const int set = it >= N ? 1 : 0;
    const size_t node = it - (size_t)set * N;
    const POND_GLOBAL PopT *pop = (const POND_GLOBAL PopT *)S.pop_src + (size_t)set * 27 * N;
    const POND_GLOBAL double *side = (const POND_GLOBAL double *)S.side_src;
    double f[27];
#pragma unroll
    for (int q = 0; q < 27; ++q) f[q] = (double)pop[(size_t)q * N + node];
    if constexpr (kDeviationStore<PopT>) {
        const double sum = ((const POND_GLOBAL double *)((const POND_GLOBAL PopT *)S.pop_src + (size_t)54 * N))[set * N + node];
#pragma unroll
        for (int q = 0; q < 27; ++q) f[q] += w27(q) * sum;
    }
    const double ux = side[kSideUx * N + node], uy = side[kSideUy * N + node], uz = side[kSideUz * N + node];
    const double s = sqrt(side[kSideTh * N + node]);
    double m[27];
    moments27(f, ux, uy, uz, s, m);
    POND_GLOBAL MomT *out = (POND_GLOBAL MomT *)S.dmom + (size_t)set * 27 * N;
#pragma unroll
    for (int i = 0; i < 27; ++i) out[(size_t)i * N + node] = (MomT)m[i];
}

// The donor moments of a set that the collision has just stored (post in the gauge u, s),
// as k3_donor_moments computes them from the stored populations: in the FP32 storage
// forms from the stored deviations and sum, so that both give the same bits
template <typename PopT, typename MomT>
__device__ __forceinline__ void store_donor_moments(const SlotDesc &S, size_t N, size_t node, int set,
                                                    const double *post, const double u[3], double s)
{
    double f[27];
    if constexpr (kDeviationStore<PopT>) {
        double sum = 0.0;
#pragma unroll
        for (int q = 0; q < 27; ++q) sum += post[q];
#pragma unroll
        for (int q = 0; q < 27; ++q) f[q] = (double)(PopT)(post[q] - weight_q<3>(q) * sum);
#pragma unroll
        for (int q = 0; q < 27; ++q) f[q] += w27(q) * sum;
    } else {
#pragma unroll
        for (int q = 0; q < 27; ++q) f[q] = post[q];
    }
    double m[27];
    moments27(f, u[0], u[1], u[2], s, m);
    POND_GLOBAL MomT *out = (POND_GLOBAL MomT *)S.dmom + (size_t)set * 27 * N;
#pragma unroll
    for (int i = 0; i < 27; ++i) out[(size_t)i * N + node] = (MomT)m[i];
}

// x-y contraction of the nine fields (m, n, o) of one z power o over a staged donor
// plane, into Y[k][l] += sum_n B_ln sum_r wy_l[r] sum_m A_km sum_c wx_k[c] M_mno[r][c].
// Each axis's cubic stencil covers four of the five window columns; for the directions
// c = -1 and +1 the unused column is the first (k = 0) or the last (k = 2) whenever the
// gauge velocity lies in (-s, s].  FAST (chosen per wave when every lane's weights
// there are zero) leaves those zero taps out; the two variants agree to round-off, and
// the choice depends only on the lanes of a wave, which the tile shape fixes.
template <bool FAST, typename T>
__device__ __forceinline__ T taps3(int k, const T w[5], T v0, T v1, T v2, T v3, T v4)
{
    if (FAST && k == 0) return w[1] * v1 + w[2] * v2 + w[3] * v3 + w[4] * v4;
    if (FAST && k == 2) return w[0] * v0 + w[1] * v1 + w[2] * v2 + w[3] * v3;
    return w[0] * v0 + w[1] * v1 + w[2] * v2 + w[3] * v3 + w[4] * v4;
}

// weight of window column j (0..4) in the cubic stencil of departure velocity v: the
// column weights of window_weights, one at a time (its halo check is not repeated)
__device__ __forceinline__ double window_tap(double v, double dt, int j)
{
    const double d = -v * dt;
    const double fl = floor(d);
    const double t = d - fl + 1.0;
    int i0 = (int)fl;
    i0 = i0 < -1 ? -1 : (i0 > 0 ? 0 : i0);
    const int c = j - (i0 + 1); // stencil node of column j
    if (c == 0) return -(t - 1.0) * (t - 2.0) * (t - 3.0) * (1.0 / 6.0);
    if (c == 1) return t * (t - 2.0) * (t - 3.0) * 0.5;
    if (c == 2) return -t * (t - 1.0) * (t - 3.0) * 0.5;
    if (c == 3) return t * (t - 1.0) * (t - 2.0) * (1.0 / 6.0);
    return 0.0;
}

// the LDS holds the nine fields (m, n) of one z power, field (m, n) at slot 3 m + n; each
// row is x-contracted and added straight into Y with its y weights (no five-row buffer:
// the FP64 window must fit two waves per SIMD)
template <bool FAST, typename LdsT, typename AccT, int LN, int LX>
__device__ __forceinline__ void xy_window(const LdsT *sbase, const LdsT (&wx)[3][5], const LdsT (&wy)[3][5],
                                          const LdsT (&A)[3][3], const AccT (&B)[3][3], AccT (&Y)[3][3])
{
#pragma unroll
    for (int n = 0; n < 3; ++n) {
#pragma unroll
        for (int r = 0; r < 5; ++r) {
            LdsT Zr[3];
#pragma unroll
            for (int m = 0; m < 3; ++m) {
                const LdsT *row = sbase + ((3 * m + n) * LN + r * LX) * 2;
                const LdsT v0 = row[0], v1 = row[2], v2 = row[4], v3 = row[6], v4 = row[8];
#pragma unroll
                for (int k = 0; k < 3; ++k) {
                    const LdsT x = taps3<FAST>(k, wx[k], v0, v1, v2, v3, v4);
                    Zr[k] = m == 0 ? A[k][m] * x : Zr[k] + A[k][m] * x;
                }
            }
#pragma unroll
            for (int l = 0; l < 3; ++l) {
                if (FAST && ((l == 0 && r == 0) || (l == 2 && r == 4))) continue; // zero taps
                const AccT c = B[l][n] * (AccT)wy[l][r];
#pragma unroll
                for (int k = 0; k < 3; ++k) Y[k][l] += c * (AccT)Zr[k];
            }
        }
        __builtin_amdgcn_sched_barrier(0);
    }
}

// ---------------------------------------------------------------------------
// streaming passes: x-y tile of TX x TY receivers of one z plane, two lanes per
// receiver (set f / g), the 5 x 5 x 5 window staged plane by plane.
//
// Interpolation and contraction are linear in the donor moments, and every cubic
// Lagrange stencil reproduces a constant exactly.  In the FP32 form the LDS therefore
// holds each donor moment minus a reference value of the tile (the moment of the tile's
// centre node in the receiver plane): the FP32 window arithmetic then carries only the
// variation across the tile, and the reference part, the same for every donor, is
// contracted with the receiver's gauge coefficients in FP64.  A uniform region is so
// streamed exactly, and the FP32 rounding scales with the local variation, not with
// the moment itself.
// ---------------------------------------------------------------------------
template <typename LdsT, int TX, int TY, bool GEN>
__global__ void __launch_bounds__(2 * TX *TY, sizeof(LdsT) == 4 ? 3 : 2) k3_stream(const SlotDesc *__restrict__ slot)
{
    constexpr int LX = TX + 4, LY = TY + 4, LN = LX * LY, NT = 2 * TX * TY;
    constexpr bool kDev = sizeof(LdsT) == 4;
    using AccT = LdsT; // window accumulators: FP64, or FP32 deviations
    // a donor plane is staged in three rounds, the nine fields of one z power per set
    // each (35 KB of LDS in FP64, 17 KB in FP32 instead of 104 and 52 KB for the whole
    // plane), so that two FP64 or three FP32 workgroups share a CU
    constexpr int FPS = 9; // fields per set and round
    __shared__ __align__(16) LdsT lds[2 * FPS * LN];
    __shared__ LdsT ref[kDev ? 54 : 1];
    // z coefficients of the pass, per receiver: the FP32 window keeps the 45 products
    // C_mo wz_m[sz] of its rounds, the FP64 window the nine C_mo and fifteen wz_m[sz] whose
    // product each round forms (23 and 25 KB of LDS)
    constexpr int NR = TX * TY;
    constexpr int kCz = kDev ? 45 : 24;
    __shared__ AccT s_cz[kCz * NR];
    __shared__ int s_wfast[NT / 64]; // per wave: its lanes allow the zero-tap-free window
    __shared__ int abort_block;
    const SlotDesc &S = *slot;
    const POND_GLOBAL DevParams &P = *(const POND_GLOBAL DevParams *)S.P;
    const Box box = make_box(P);
    const size_t N = box.N;
    int *flags = S.flags;
    const int tid = threadIdx.x + 2 * TX * threadIdx.y;
    int err_before = 0;
    if (tid == 0) err_before = flags[kFlagErr];

    // Block order: blocks are dealt to the XCDs in turn; xcd_tile gives each XCD a
    // contiguous range of logical blocks, and z runs fastest in that range, so the
    // blocks one XCD runs together are consecutive planes of one tile column and
    // re-read their shared donor planes from that XCD's L2.
    const int tiles_x = (box.nx + TX - 1) / TX;
    const int lb = xcd_tile((int)blockIdx.x, (int)gridDim.x);
    const int tile = lb / box.nz, z = lb - tile * box.nz;
    const int bx0 = (tile % tiles_x) * TX, by0 = (tile / tiles_x) * TY;
    const int lxr = (int)threadIdx.x >> 1, myset = (int)threadIdx.x & 1;
    const int rcv = lxr + TX * (int)threadIdx.y; // receiver index in the tile
    const int gx = bx0 + lxr, gy = by0 + (int)threadIdx.y;
    const bool inside = gx < box.nx && gy < box.ny;
    const int node = min(gx, box.nx - 1) + box.nx * (min(gy, box.ny - 1) + box.ny * z);
    const POND_GLOBAL double *side = (const POND_GLOBAL double *)S.side_src;
    const POND_GLOBAL LdsT *dmom = (const POND_GLOBAL LdsT *)S.dmom;
    if (kDev && tid < 54) {
        const int cnode = min(bx0 + TX / 2, box.nx - 1) + box.nx * (min(by0 + TY / 2, box.ny - 1) + box.ny * z);
        ref[tid] = dmom[(size_t)tid * N + cnode]; // ordered before its readers by the first barrier
    }
    double U[3] = {side[kSideUx * N + node], side[kSideUy * N + node], side[kSideUz * N + node]};
    double th = side[kSideTh * N + node];
    const double Fp[3] = {side[kSideFx * N + node], side[kSideFy * N + node], side[kSideFz * N + node]};
    const double dt = P.dt;
    const int wbase = (int)threadIdx.y * LX + lxr; // window corner (gx-2, gy-2) in the tile plane
    // staging: lane tid < LN owns window node tid of a plane (its x-y node offset is the
    // same in every plane) and moves both sets of the nine moments of that node of the
    // round's z power, each field read from a uniform plane base plus a 32-bit byte offset
    static_assert(LN <= NT, "one staging lane per window node");
    const bool stager = tid < LN;
    const unsigned ndxy = (unsigned)(box.wrap(bx0 - 2 + tid % LX, box.nx) +
                                     box.nx * box.wrap(by0 - 2 + tid / LX, box.ny));
    const unsigned plane = (unsigned)box.nx * (unsigned)box.ny;
    using Pair = typename std::conditional<kDev, float2, double2>::type;

    double acc[27];
    double sU[3] = {U[0], U[1], U[2]}, sS = 1.0, rho = 0.0;
    int err = 0;
    for (int pass = 0; pass < P.n_pass; ++pass) {
        const double s = sqrt(th);
        LdsT wx[3][5], wy[3][5];
        double wz[3][5]; // only its halo check is kept: the z taps go to LDS in the first round
        const int werr = window_weights<LdsT>(U[0], s, dt, wx) | window_weights<LdsT>(U[1], s, dt, wy) |
                         window_weights<double>(U[2], s, dt, wz);
        if (inside) err |= werr; // lanes past the lattice edge only pad the tile
        LdsT A[3][3];
        AccT B[3][3];
        {
            double Ad[3][3], Bd[3][3];
            lagrange_coeffs(U[0], s, Ad);
            lagrange_coeffs(U[1], s, Bd);
#pragma unroll
            for (int k = 0; k < 3; ++k)
#pragma unroll
                for (int m = 0; m < 3; ++m) {
                    A[k][m] = (LdsT)Ad[k][m];
                    B[k][m] = (AccT)Bd[k][m];
                }
        }
        AccT av[27];
#pragma unroll
        for (int q = 0; q < 27; ++q) av[q] = (AccT)0;
        // zero-tap-free window variant when every lane of the wave allows it
        const bool fast = __all(wx[0][0] == (LdsT)0 && wx[2][4] == (LdsT)0 && wy[0][0] == (LdsT)0 &&
                                wy[2][4] == (LdsT)0);

        // the block takes the zero-tap-free window when every wave allows it (a choice
        // uniform over the block: the rounds hold barriers).  The pass's z coefficients are
        // read in the rounds after their second barrier; the barrier here ends every read
        // of the previous pass's, and of the previous pass's votes
        if ((tid & 63) == 0) s_wfast[tid >> 6] = fast ? 1 : 0;
        __syncthreads();
        bool block_fast = true;
#pragma unroll
        for (int w = 0; w < NT / 64; ++w) block_fast = block_fast && s_wfast[w] != 0;
        if (myset == 0) {
            double Cd[3][3];
            lagrange_coeffs(U[2], s, Cd);
#pragma unroll
            for (int m = 0; m < 3; ++m) {
                const double vz = U[2] + s * (double)(m - 1);
#pragma unroll
                for (int j = 0; j < 5; ++j) {
                    const double tap = window_tap(vz, dt, j);
                    if (kDev) {
#pragma unroll
                        for (int o = 0; o < 3; ++o) s_cz[((5 * o + j) * 3 + m) * NR + rcv] = (AccT)(Cd[m][o] * tap);
                    } else {
                        s_cz[(9 + 5 * m + j) * NR + rcv] = (AccT)tap;
                    }
                }
                if (!kDev) {
#pragma unroll
                    for (int o = 0; o < 3; ++o) s_cz[(3 * m + o) * NR + rcv] = (AccT)Cd[m][o];
                }
            }
        }

        auto rounds = [&](auto fast_tag) -> bool {
            constexpr bool FAST = decltype(fast_tag)::value;
#pragma unroll 1
            for (int szo = 0; szo < 15; ++szo) {
                // stage the 18 fields of z power so of the donor plane z + sz - 2 of the tile
                // window (field 9 m + 3 n + so = 3 j + so at slot j = 3 m + n).  The five planes
                // of one power come before the next power: the blocks that run together on an
                // XCD are consecutive z planes, so block z - 1 stages the same plane and power
                // one round after block z, while it is still in the XCD's L2
                const int so = szo / 5, sz = szo - 5 * so;
                __syncthreads();
                const int zz = box.wrap(z + sz - 2, box.nz);
                if (stager) {
                    const unsigned off = (ndxy + plane * (unsigned)zz) * (unsigned)sizeof(LdsT);
                    // loads in batches of MB fields per set before their stores, so that
                    // their latencies overlap
                    constexpr int MB = 9;
                    static_assert(FPS % MB == 0, "whole batches of fields");
#pragma unroll
                    for (int m0 = 0; m0 < FPS; m0 += MB) {
                        LdsT a[MB], b[MB];
#pragma unroll
                        for (int j = 0; j < MB; ++j) {
                            const int f = 3 * (m0 + j) + so;
                            a[j] = *(const POND_GLOBAL LdsT *)((const POND_GLOBAL char *)(dmom + (size_t)f * N) + off);
                            b[j] = *(const POND_GLOBAL LdsT *)((const POND_GLOBAL char *)(dmom + (size_t)(27 + f) * N) + off);
                        }
#pragma unroll
                        for (int j = 0; j < MB; ++j) {
                            const int f = 3 * (m0 + j) + so;
                            Pair v;
                            if (kDev) {
                                v.x = a[j] - ref[f];
                                v.y = b[j] - ref[27 + f];
                            } else {
                                v.x = a[j];
                                v.y = b[j];
                            }
                            *(Pair *)&lds[((m0 + j) * LN + tid) * 2] = v;
                        }
                    }
                }
                if (pass == 0 && szo == 0 && tid == 0) {
                    abort_block = err_before;
                    // one step more has started without an earlier failure
                    if (blockIdx.x == 0 && err_before == 0) atomicAdd(&flags[kFlagSteps], 1);
                }
                __syncthreads();
                if (abort_block != 0) return false;

                const LdsT *sbase = &lds[wbase * 2 + myset];
                AccT Y[3][3];
#pragma unroll
                for (int k = 0; k < 3; ++k)
#pragma unroll
                    for (int l = 0; l < 3; ++l) Y[k][l] = (AccT)0;
                xy_window<FAST, LdsT, AccT, LN, LX>(sbase, wx, wy, A, B, Y);
                // z contraction: departure point m of the receiver takes its z tap of plane sz
                // times its z Lagrange coefficient of power so
#pragma unroll
                for (int m = 0; m < 3; ++m) {
                    const AccT cz = kDev ? s_cz[(3 * szo + m) * NR + rcv]
                                         : s_cz[(3 * m + so) * NR + rcv] * s_cz[(9 + 5 * m + sz) * NR + rcv];
#pragma unroll
                    for (int k = 0; k < 3; ++k)
#pragma unroll
                        for (int l = 0; l < 3; ++l) av[9 * k + 3 * l + m] += cz * Y[k][l];
                }
            }
            return true;
        };
        if (!(block_fast ? rounds(std::true_type{}) : rounds(std::false_type{}))) return;
        if (kDev) {
            // reference part: sum_mno A_km B_ln C_m'o R_mno in FP64 (the window weights of
            // each axis sum to one).  The inputs pass an empty asm so that the coefficients
            // are recomputed here rather than kept live across the window loop.
            double su = s, u0 = U[0], u1 = U[1], u2 = U[2];
            asm volatile("" : "+v"(su), "+v"(u0), "+v"(u1), "+v"(u2));
            double Ad[3][3], Bd[3][3], Cd[3][3];
            lagrange_coeffs(u0, su, Ad);
            lagrange_coeffs(u1, su, Bd);
            lagrange_coeffs(u2, su, Cd);
            const LdsT *R = &ref[27 * myset];
#pragma unroll
            for (int k = 0; k < 3; ++k) {
                double T1[3][3]; // [n][o]
#pragma unroll
                for (int n = 0; n < 3; ++n)
#pragma unroll
                    for (int o = 0; o < 3; ++o)
                        T1[n][o] = Ad[k][0] * (double)R[3 * n + o] + Ad[k][1] * (double)R[9 + 3 * n + o] +
                                   Ad[k][2] * (double)R[18 + 3 * n + o];
#pragma unroll
                for (int l = 0; l < 3; ++l) {
                    double T2[3];
#pragma unroll
                    for (int o = 0; o < 3; ++o) T2[o] = Bd[l][0] * T1[0][o] + Bd[l][1] * T1[1][o] + Bd[l][2] * T1[2][o];
#pragma unroll
                    for (int m = 0; m < 3; ++m)
                        acc[9 * k + 3 * l + m] =
                            (Cd[m][0] * T2[0] + Cd[m][1] * T2[1] + Cd[m][2] * T2[2]) + (double)av[9 * k + 3 * l + m];
                }
            }
        } else {
#pragma unroll
            for (int q = 0; q < 27; ++q) acc[q] = (double)av[q];
        }
        // moments of the streamed populations (eq. 2) and the EoS closure
        double s0 = 0.0, sx = 0.0, sy = 0.0, szm = 0.0;
#pragma unroll
        for (int q = 0; q < 27; ++q) {
            s0 += acc[q];
            sx += acc[q] * (U[0] + s * (double)(q / 9 - 1));
            sy += acc[q] * (U[1] + s * (double)((q / 3) % 3 - 1));
            szm += acc[q] * (U[2] + s * (double)(q % 3 - 1));
        }
        const double o0 = __shfl_xor(s0, 1, 64), ox = __shfl_xor(sx, 1, 64);
        const double oy = __shfl_xor(sy, 1, 64), oz = __shfl_xor(szm, 1, 64);
        rho = myset == 0 ? s0 : o0;
        const double j[3] = {myset == 0 ? sx : ox, myset == 0 ? sy : oy, myset == 0 ? szm : oz};
        const double G2 = myset == 0 ? o0 : s0;
        const double i_rho = 1.0 / rho; // one reciprocal for every quotient by rho
        const double E = 0.5 * G2 * i_rho;
        double uh2 = 0.0, un[3];
#pragma unroll
        for (int a = 0; a < 3; ++a) {
            un[a] = j[a] * i_rho;
            const double uh = un[a] + 0.5 * Fp[a] * dt * i_rho;
            uh2 += uh * uh;
        }
        const double e = E - 0.5 * uh2;
        const double T = eos_T_of_e<GEN>(P, rho, e);
        const double p = eos_p<GEN>(P, rho, T);
        if (inside) err |= eos_bad<GEN>(P, rho, p);
#pragma unroll
        for (int a = 0; a < 3; ++a) {
            sU[a] = U[a];
            U[a] = un[a];
        }
        sS = s;
        th = p * i_rho * kInvTL;
    }

    if (inside) {
        const size_t n = (size_t)node;
        POND_GLOBAL double *mom = (POND_GLOBAL double *)S.mom;
        double mc[27];
        moments27(acc, sU[0] - U[0], sU[1] - U[1], sU[2] - U[2], sS, mc);
        if (myset == 0) {
            mom[(size_t)L3::kRho * N + n] = rho;
            mom[(size_t)L3::kUx * N + n] = U[0];
            mom[(size_t)L3::kUy * N + n] = U[1];
            mom[(size_t)L3::kUz * N + n] = U[2];
#pragma unroll
            for (int i = 0; i < 27; ++i) {
                const int si = fstored_index(i);
                if (si >= 0) mom[(size_t)(L3::kF + si) * N + n] = mc[i];
            }
        } else {
#pragma unroll
            for (int i = 0; i < 27; ++i) mom[(size_t)(L3::kG + i) * N + n] = mc[i];
        }
    }
    if (err) raise_error3(flags, err, S.parity);
}

// ---------------------------------------------------------------------------
// Korteweg stress K = -kappa (rho lap rho + |grad rho|^2/2) I + kappa grad rho grad rho
// from the streamed density (planes xx, xy, xz, yy, yz, zz)
// ---------------------------------------------------------------------------
__global__ void __launch_bounds__(256) k3_korteweg(const SlotDesc *__restrict__ slot)
{
    const SlotDesc &S = *slot;
    const POND_GLOBAL DevParams &P = *(const POND_GLOBAL DevParams *)S.P;
    const Box box = make_box(P);
    const size_t N = box.N;
    const size_t n = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (n >= N || S.flags[kFlagErr] != 0) return;
    const int x = (int)(n % box.nx), y = (int)((n / box.nx) % box.ny), z = (int)(n / ((size_t)box.nx * box.ny));
    const double *rho = S.mom + (size_t)L3::kRho * N;
    const double r0 = rho[n];
    const Nbr27 nb(box, x, y, z);
    double g[3] = {0.0, 0.0, 0.0}, lap = 0.0;
#pragma unroll
    for (int q = 0; q < 27; ++q) {
        const int cx = q / 9 - 1, cy = (q / 3) % 3 - 1, cz = q % 3 - 1;
        const double rq = rho[nb.at(q)];
        const double w = w27(q);
        g[0] += w * (double)cx * rq;
        g[1] += w * (double)cy * rq;
        g[2] += w * (double)cz * rq;
        lap += w * (rq - r0);
    }
#pragma unroll
    for (int a = 0; a < 3; ++a) g[a] *= kInvTL;
    lap *= 2.0 * kInvTL;
    const double iso = -P.kappa * (r0 * lap + 0.5 * (g[0] * g[0] + g[1] * g[1] + g[2] * g[2]));
    double *kor = S.kor;
    kor[0 * N + n] = iso + P.kappa * g[0] * g[0];
    kor[1 * N + n] = P.kappa * g[0] * g[1];
    kor[2 * N + n] = P.kappa * g[0] * g[2];
    kor[3 * N + n] = iso + P.kappa * g[1] * g[1];
    kor[4 * N + n] = P.kappa * g[1] * g[2];
    kor[5 * N + n] = iso + P.kappa * g[2] * g[2];
}

__device__ __forceinline__ void force_at3(const Box &box, const double *kor, int x, int y, int z, double F[3])
{
    const size_t N = box.N;
    const Nbr27 nb(box, x, y, z);
    const double *k0 = kor, *k1 = kor + N, *k2 = kor + 2 * N, *k3 = kor + 3 * N, *k4 = kor + 4 * N, *k5 = kor + 5 * N;
    double dv[3] = {0.0, 0.0, 0.0};
    // the neighbours in three groups of nine (one x offset each): the loads of a group
    // are in flight together, and the next group's wait until this one is summed, which
    // bounds the registers
#pragma unroll
    for (int q0 = 0; q0 < 27; q0 += 9) {
#pragma unroll
        for (int q = q0; q < q0 + 9; ++q) {
            const int c[3] = {q / 9 - 1, (q / 3) % 3 - 1, q % 3 - 1};
            const unsigned m = nb.at(q);
            const double w = w27(q);
            const double kxx = k0[m], kxy = k1[m], kxz = k2[m];
            const double kyy = k3[m], kyz = k4[m], kzz = k5[m];
            dv[0] += w * (kxx * c[0] + kxy * c[1] + kxz * c[2]);
            dv[1] += w * (kxy * c[0] + kyy * c[1] + kyz * c[2]);
            dv[2] += w * (kxz * c[0] + kyz * c[1] + kzz * c[2]);
        }
        __builtin_amdgcn_sched_barrier(0);
    }
#pragma unroll
    for (int a = 0; a < 3; ++a) F[a] = -dv[a] * kInvTL;
}

// ---------------------------------------------------------------------------
// force and thermodynamic state of the step: aux planes F_x, F_y, F_z, T, h, mu, k, p
// ---------------------------------------------------------------------------
__global__ void __launch_bounds__(256) k3_thermo(const SlotDesc *__restrict__ slot)
{
    const SlotDesc &S = *slot;
    const POND_GLOBAL DevParams &P = *(const POND_GLOBAL DevParams *)S.P;
    const Box box = make_box(P);
    const size_t N = box.N;
    const size_t n = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (n >= N || S.flags[kFlagErr] != 0) return;
    const int x = (int)(n % box.nx), y = (int)((n / box.nx) % box.ny), z = (int)(n / ((size_t)box.nx * box.ny));
    const double *mom = S.mom;
    double F[3] = {0.0, 0.0, 0.0};
    if (P.kappa != 0.0) force_at3(box, S.kor, x, y, z, F);
    const double rho = mom[L3::kRho * N + n];
    const double h_r = 0.5 / rho;
    const double E = mom[(size_t)L3::kG * N + n] * h_r;
    double uh2 = 0.0;
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        const double uh = mom[(size_t)(L3::kUx + a) * N + n] + F[a] * P.dt * h_r;
        uh2 += uh * uh;
    }
    const double e = E - 0.5 * uh2;
    const double T = eos_T_of_e(P, rho, e);
    const double p = eos_p(P, rho, T);
    const int bad = eos_bad(P, rho, p);
    if (bad) raise_error3(S.flags, bad, S.parity);
    const double mu = (1.0 / P.omega - 0.5) * p * P.dt;
    double *aux = S.aux;
    aux[0 * N + n] = F[0];
    aux[1 * N + n] = F[1];
    aux[2 * N + n] = F[2];
    aux[3 * N + n] = T;
    aux[4 * N + n] = e + 2.0 * p * h_r;
    aux[5 * N + n] = mu;
    aux[6 * N + n] = P.k_scale * mu * P.Cp_ig;
    aux[7 * N + n] = p;
}

// ---------------------------------------------------------------------------
// collision (eqs. 9, 16-22): blockIdx.y = 0 collides f, 1 collides g
// ---------------------------------------------------------------------------
template <typename PopT, typename MomT>
__global__ void __launch_bounds__(256) k3_collide(const SlotDesc *__restrict__ slot)
{
    const SlotDesc &S = *slot;
    const POND_GLOBAL DevParams &P = *(const POND_GLOBAL DevParams *)S.P;
    const Box box = make_box(P);
    const size_t N = box.N;
    const size_t n = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int set = blockIdx.y;
    if (n >= N || S.flags[kFlagErr] != 0) return;
    const double *mom = S.mom, *aux = S.aux;
    const double dt = P.dt;
    const double rho = mom[L3::kRho * N + n];
    const double i_rho = 1.0 / rho;
    const double u[3] = {mom[L3::kUx * N + n], mom[L3::kUy * N + n], mom[L3::kUz * N + n]};
    const double F[3] = {aux[0 * N + n], aux[1 * N + n], aux[2 * N + n]};
    const double p = aux[7 * N + n];
    const double theta = p * i_rho * kInvTL;
    const double s = sqrt(theta);

    double mc[27];
    if (set == 0) {
#pragma unroll
        for (int i = 0; i < 27; ++i) {
            const int si = fstored_index(i);
            mc[i] = si >= 0 ? mom[(size_t)(L3::kF + si) * N + n] : 0.0;
        }
        mc[0] = rho;
    } else {
#pragma unroll
        for (int i = 0; i < 27; ++i) mc[i] = mom[(size_t)(L3::kG + i) * N + n];
    }
    double A[3][3];
    lagrange_coeffs(0.0, s, A);
    double pop[27], post[27];
    from_moments27(A, mc, pop);
    POND_GLOBAL PopT *pout = (POND_GLOBAL PopT *)S.pop_dst;

    if (set == 0) {
        // f: BGK towards rho W plus the force source, per axis rho prod (W + sigma) - rho W
        const double i_theta = 1.0 / theta, i_s = s * i_theta;
        double sg[3][3];
#pragma unroll
        for (int a = 0; a < 3; ++a) source_axis(F[a] * dt * i_rho, i_theta, i_s, sg[a]);
#pragma unroll
        for (int q = 0; q < 27; ++q) {
            const int k = q / 9, l = (q / 3) % 3, m = q % 3;
            const double Wq = kW1[k] * kW1[l] * kW1[m];
            const double Sq = rho * ((kW1[k] + sg[0][k]) * (kW1[l] + sg[1][l]) * (kW1[m] + sg[2][m]) - Wq);
            post[q] = pop[q] + P.omega * (rho * Wq - pop[q]) + Sq;
        }
        store_set<3, PopT>(pout, N, (int)n, 0, post);
        store_donor_moments<PopT, MomT>(S, N, n, 0, post, u, s);
        POND_GLOBAL double *side = (POND_GLOBAL double *)S.side_dst;
        side[kSideUx * N + n] = u[0];
        side[kSideUy * N + n] = u[1];
        side[kSideUz * N + n] = u[2];
        side[kSideTh * N + n] = theta;
        side[kSideFx * N + n] = F[0];
        side[kSideFy * N + n] = F[1];
        side[kSideFz * N + n] = F[2];
        return;
    }

    // heat-flux correction M0 = 2 div(-mu grad h + k grad T), flux form (eq. 9)
    double M0 = 0.0;
    if (P.k_scale >= 0.0) {
        const int x = (int)(n % box.nx), y = (int)((n / box.nx) % box.ny), z = (int)(n / ((size_t)box.nx * box.ny));
        const double T0 = aux[3 * N + n], h0 = aux[4 * N + n], m0 = aux[5 * N + n], k0 = aux[6 * N + n];
        const Nbr27 nb(box, x, y, z);
        const double *aT = aux + 3 * N, *ah = aux + 4 * N, *amu = aux + 5 * N, *ak = aux + 6 * N;
        double accm = 0.0;
#pragma unroll
        for (int q0 = 0; q0 < 27; q0 += 9) {
#pragma unroll
            for (int q = q0; q < q0 + 9; ++q) {
                const unsigned m = nb.at(q);
                const double kmid = 0.5 * (ak[m] + k0);
                const double mmid = 0.5 * (amu[m] + m0);
                accm += w27(q) * (kmid * (aT[m] - T0) - mmid * (ah[m] - h0));
            }
            __builtin_amdgcn_sched_barrier(0);
        }
        M0 = 2.0 * (2.0 * kInvTL) * accm;
    }
    // g: BGK towards the force-extended equilibrium plus (g~ + phi) dt (eqs. 19-22)
    const double i_p = 1.0 / p;
    const double E = 0.5 * mc[0] * i_rho;
    double uh[3];
#pragma unroll
    for (int a = 0; a < 3; ++a) uh[a] = u[a] + 0.5 * F[a] * dt * i_rho;
    const double Pr = p * i_rho, H = E + Pr, dt_Pr = dt * rho * i_p;
    double X[3][3], M[3], Nm[3][3];
#pragma unroll
    for (int a = 0; a < 3; ++a)
#pragma unroll
        for (int b = 0; b < 3; ++b) X[a][b] = uh[a] * F[b] + F[a] * uh[b] + 0.5 * dt * F[a] * F[b] * E * i_p;
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        const double xu = X[a][0] * u[0] + X[a][1] * u[1] + X[a][2] * u[2];
        M[a] = dt_Pr * (F[a] * H - xu);
#pragma unroll
        for (int b = 0; b < 3; ++b) Nm[a][b] = (a == b ? rho : 0.0) + 0.5 * dt_Pr * X[a][b];
    }
    const double work = 2.0 * (uh[0] * F[0] + uh[1] * F[1] + uh[2] * F[2]);
    const double c_uc = 0.5 * kInvTL * rho * i_p, c_v2 = 0.5 * rho * i_p;
#pragma unroll
    for (int q = 0; q < 27; ++q) {
        const double c[3] = {(double)(q / 9 - 1), (double)((q / 3) % 3 - 1), (double)(q % 3 - 1)};
        double v[3], t1 = 0.0, t2 = 0.0, uc = 0.0, v2 = 0.0;
#pragma unroll
        for (int a = 0; a < 3; ++a) {
            v[a] = u[a] + s * c[a];
            uc += u[a] * c[a];
            v2 += v[a] * v[a];
            t1 += M[a] * (v[a] - u[a]);
        }
#pragma unroll
        for (int a = 0; a < 3; ++a)
#pragma unroll
            for (int b = 0; b < 3; ++b) t2 += Nm[a][b] * (v[a] * v[b] - (a == b ? Pr : 0.0) - u[a] * u[b]);
        const double wq = w27(q);
        const double geq = wq * (2.0 * rho * E + t1 + t2);
        const double psi = wq * (1.0 + c_uc * uc * uc - c_v2 * v2 + 1.5);
        post[q] = pop[q] + P.omega * (geq - pop[q]) + (M0 + work) * psi * dt;
    }
    store_set<3, PopT>(pout, N, (int)n, 1, post);
    store_donor_moments<PopT, MomT>(S, N, n, 1, post, u, s);
}

// ---------------------------------------------------------------------------
// initial state (streamed-state planes of the equilibrium of rho, u_hat, T with the
// force F0 = -div K(rho)); aux planes 0-4 hold rho, u_hat (3), T, mom plane 0 rho and
// kor the stress of rho
// ---------------------------------------------------------------------------
__global__ void __launch_bounds__(256) k3_init_equilibrium(const SlotDesc *__restrict__ slot)
{
    const SlotDesc &S = *slot;
    const POND_GLOBAL DevParams &P = *(const POND_GLOBAL DevParams *)S.P;
    const Box box = make_box(P);
    const size_t N = box.N;
    const size_t n = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (n >= N) return;
    const int x = (int)(n % box.nx), y = (int)((n / box.nx) % box.ny), z = (int)(n / ((size_t)box.nx * box.ny));
    const double *aux = S.aux;
    double *mom = S.mom;
    double F[3] = {0.0, 0.0, 0.0};
    if (P.kappa != 0.0) force_at3(box, S.kor, x, y, z, F);
    const double rho = aux[0 * N + n], T = eos_state_T(P, aux[4 * N + n]);
    const double uh[3] = {aux[1 * N + n], aux[2 * N + n], aux[3 * N + n]};
    double u[3];
#pragma unroll
    for (int a = 0; a < 3; ++a) u[a] = uh[a] - F[a] * P.dt / (2.0 * rho);
    const double p = eos_p(P, rho, T);
    const int bad = eos_bad(P, rho, p);
    if (bad) raise_error3(S.flags, bad, 0);
    const double e = eos_e(P, rho, T);
    const double E = e + 0.5 * (uh[0] * uh[0] + uh[1] * uh[1] + uh[2] * uh[2]);
    const double theta = p / (rho * kTL), s = sqrt(theta);
    // f = rho W: central moments rho prod_axes {1, 0, theta T_L}
    const double mu1[3] = {1.0, 0.0, theta * kTL};
    mom[(size_t)L3::kRho * N + n] = rho;
    mom[(size_t)L3::kUx * N + n] = u[0];
    mom[(size_t)L3::kUy * N + n] = u[1];
    mom[(size_t)L3::kUz * N + n] = u[2];
#pragma unroll
    for (int i = 0; i < 27; ++i) {
        const int si = fstored_index(i);
        if (si >= 0) mom[(size_t)(L3::kF + si) * N + n] = rho * mu1[i / 9] * mu1[(i / 3) % 3] * mu1[i % 3];
    }
    // g = g^eq (eqs. 20-22) in the gauge (u, theta), then its central moments
    const double Pr = p / rho, H = E + Pr;
    double X[3][3], M[3], Nm[3][3];
#pragma unroll
    for (int a = 0; a < 3; ++a)
#pragma unroll
        for (int b = 0; b < 3; ++b) X[a][b] = uh[a] * F[b] + F[a] * uh[b] + P.dt * F[a] * F[b] * E / (2.0 * p);
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        const double xu = X[a][0] * u[0] + X[a][1] * u[1] + X[a][2] * u[2];
        M[a] = P.dt / Pr * (F[a] * H - xu);
#pragma unroll
        for (int b = 0; b < 3; ++b) Nm[a][b] = (a == b ? rho : 0.0) + P.dt / (2.0 * Pr) * X[a][b];
    }
    double g[27];
#pragma unroll
    for (int q = 0; q < 27; ++q) {
        const double c[3] = {(double)(q / 9 - 1), (double)((q / 3) % 3 - 1), (double)(q % 3 - 1)};
        double v[3], t1 = 0.0, t2 = 0.0;
#pragma unroll
        for (int a = 0; a < 3; ++a) {
            v[a] = u[a] + s * c[a];
            t1 += M[a] * (v[a] - u[a]);
        }
#pragma unroll
        for (int a = 0; a < 3; ++a)
#pragma unroll
            for (int b = 0; b < 3; ++b) t2 += Nm[a][b] * (v[a] * v[b] - (a == b ? Pr : 0.0) - u[a] * u[b]);
        g[q] = w27(q) * (2.0 * rho * E + t1 + t2);
    }
    double mg[27];
    moments27(g, 0.0, 0.0, 0.0, s, mg);
#pragma unroll
    for (int i = 0; i < 27; ++i) mom[(size_t)(L3::kG + i) * N + n] = mg[i];
}

// ---------------------------------------------------------------------------
// macroscopic fields: rho, u_hat (3 planes), T, p, E
// ---------------------------------------------------------------------------
template <typename PopT>
__global__ void __launch_bounds__(256) k3_macro(const DevParams *__restrict__ Pp, const PopT *__restrict__ pop,
                                                const double *__restrict__ side, double *__restrict__ out)
{
    const DevParams &P = *Pp;
    const size_t N = P.N;
    const size_t n = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (n >= N) return;
    double r = 0.0;
    for (int q = 0; q < 27; ++q) r += (double)pop[(size_t)q * N + n];
    if (kDeviationStore<PopT>) r += ((const double *)(pop + (size_t)54 * N))[n];
    const int su[3] = {kSideUx, kSideUy, kSideUz}, sf[3] = {kSideFx, kSideFy, kSideFz};
    double h2 = 0.0;
    for (int a = 0; a < 3; ++a) {
        const double v = side[su[a] * N + n] + side[sf[a] * N + n] * P.dt / (2.0 * r);
        out[(1 + a) * N + n] = v;
        h2 += v * v;
    }
    const double pr = r * side[kSideTh * N + n] * kTL;
    const double T = eos_T_of_p(P, r, pr);
    out[0 * N + n] = r;
    out[4 * N + n] = T;
    out[5 * N + n] = pr;
    out[6 * N + n] = eos_e(P, r, T) + 0.5 * h2;
}

__global__ void __launch_bounds__(kMonThreads) k3_monitor_partials(const DevParams *__restrict__ Pp,
                                                                   const double *__restrict__ macro,
                                                                   const double *__restrict__ side,
                                                                   double *__restrict__ partials)
{
    const DevParams &P = *Pp;
    const Box box = make_box(P);
    const size_t N = box.N;
    const size_t n = (size_t)blockIdx.x * kMonThreads + threadIdx.x;
    double v[kMonWords];
    for (int i = 0; i < kMonWords; ++i) v[i] = 0.0;
    v[6] = 1e300; // min p
    if (n < N) {
        const int x = (int)(n % box.nx), y = (int)((n / box.nx) % box.ny), z = (int)(n / ((size_t)box.nx * box.ny));
        const double r = macro[n], E = macro[6 * N + n];
        double g[3] = {0.0, 0.0, 0.0};
        for (int q = 0; q < 27; ++q) {
            const int c[3] = {q / 9 - 1, (q / 3) % 3 - 1, q % 3 - 1};
            const double rq = macro[box.node(x + c[0], y + c[1], z + c[2])];
            for (int a = 0; a < 3; ++a) g[a] += w27(q) * (double)c[a] * rq;
        }
        for (int a = 0; a < 3; ++a) g[a] *= kInvTL;
        v[0] = r;
        for (int a = 0; a < 3; ++a) v[1 + a] = r * macro[(1 + a) * N + n];
        v[4] = r * E;
        v[5] = r * E + 0.5 * P.kappa * (g[0] * g[0] + g[1] * g[1] + g[2] * g[2]);
        v[6] = macro[5 * N + n];
        const double s = sqrt(side[kSideTh * N + n]);
        const double ax = fabs(side[kSideUx * N + n]) + s, ay = fabs(side[kSideUy * N + n]) + s;
        const double az = fabs(side[kSideUz * N + n]) + s;
        v[7] = sqrt(ax * ax + ay * ay + az * az) * P.dt;
    }
    __shared__ double red[kMonThreads / 64][kMonWords];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    for (int i = 0; i < kMonWords; ++i) {
        const double w = i == 6 ? wave_min(v[i]) : i == 7 ? wave_max(v[i]) : wave_sum(v[i]);
        if (lane == 0) red[wave][i] = w;
    }
    __syncthreads();
    if (threadIdx.x < kMonWords) {
        const int i = threadIdx.x;
        double acc = red[0][i];
        for (int wv = 1; wv < kMonThreads / 64; ++wv)
            acc = i == 6 ? fmin(acc, red[wv][i]) : i == 7 ? fmax(acc, red[wv][i]) : acc + red[wv][i];
        partials[(size_t)blockIdx.x * kMonWords + i] = acc;
    }
}

// ---------------------------------------------------------------------------
// launchers
// ---------------------------------------------------------------------------
// streaming tile: 16 x 8 receivers in every precision (16 x 16 was slower in both); a
// staging round of 18 fields takes 17 KB of LDS in FP32 and 35 KB in FP64
void stream3_tile(int fp32, int *tx, int *ty)
{
    (void)fp32;
    *tx = 16;
    *ty = 8;
}

template <typename LdsT, int TX, int TY>
static void launch_stream3_t(const LaunchCtx &c, const SlotDesc *slot)
{
    const int tiles = ((c.nx + TX - 1) / TX) * ((c.ny + TY - 1) / TY);
    if (c.gen_eos)
        hipLaunchKernelGGL((k3_stream<LdsT, TX, TY, true>), dim3(tiles * c.nz), dim3(2 * TX, TY), 0, c.st, slot);
    else
        hipLaunchKernelGGL((k3_stream<LdsT, TX, TY, false>), dim3(tiles * c.nz), dim3(2 * TX, TY), 0, c.st, slot);
}

static inline dim3 grid_nodes(const LaunchCtx &c, int per = 1)
{
    return dim3((unsigned)(((size_t)c.N * per + 255) / 256));
}

// the donor moments of the state the step reads are those the collision before it wrote
// (or, after a checkpoint load, launch_donor_moments3's)
hipError_t launch_stream3(const LaunchCtx &c, const SlotDesc *slot)
{
    if (c.ev_start) (void)hipEventRecord(c.ev_start, c.st);
    if (c.fp32 == 1)
        launch_stream3_t<float, 16, 8>(c, slot);
    else
        launch_stream3_t<double, 16, 8>(c, slot);
    if (c.ev_stop) (void)hipEventRecord(c.ev_stop, c.st);
    return hipGetLastError();
}

hipError_t launch_donor_moments3(const LaunchCtx &c, const SlotDesc *slot)
{
    if (c.fp32 == 1)
        hipLaunchKernelGGL((k3_donor_moments<float, float>), grid_nodes(c, 2), dim3(256), 0, c.st, slot);
    else if (c.fp32 == 2)
        hipLaunchKernelGGL((k3_donor_moments<float, double>), grid_nodes(c, 2), dim3(256), 0, c.st, slot);
    else
        hipLaunchKernelGGL((k3_donor_moments<double, double>), grid_nodes(c, 2), dim3(256), 0, c.st, slot);
    return hipGetLastError();
}

// the Korteweg stress of the streamed density (mom plane 0), the rest of the closure and
// the collision
hipError_t launch_collide3(const LaunchCtx &c, const SlotDesc *slot)
{
    if (c.ev_start) (void)hipEventRecord(c.ev_start, c.st);
    hipLaunchKernelGGL(k3_korteweg, grid_nodes(c), dim3(256), 0, c.st, slot);
    hipLaunchKernelGGL(k3_thermo, grid_nodes(c), dim3(256), 0, c.st, slot);
    dim3 g = grid_nodes(c);
    g.y = 2;
    // the collision also writes the donor moments of the state it stores
    if (c.fp32 == 1)
        hipLaunchKernelGGL((k3_collide<float, float>), g, dim3(256), 0, c.st, slot);
    else if (c.fp32 == 2)
        hipLaunchKernelGGL((k3_collide<float, double>), g, dim3(256), 0, c.st, slot);
    else
        hipLaunchKernelGGL((k3_collide<double, double>), g, dim3(256), 0, c.st, slot);
    if (c.ev_stop) (void)hipEventRecord(c.ev_stop, c.st);
    return hipGetLastError();
}

hipError_t launch_init3(const LaunchCtx &c, const DevState &s, const SlotDesc *slot)
{
    // rho of the initial state into mom plane 0, its stress, then the equilibrium planes
    hipError_t e = hipMemcpyAsync(s.mom, s.aux, sizeof(double) * (size_t)c.N, hipMemcpyDeviceToDevice, c.st);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k3_korteweg, grid_nodes(c), dim3(256), 0, c.st, slot);
    hipLaunchKernelGGL(k3_init_equilibrium, grid_nodes(c), dim3(256), 0, c.st, slot);
    return hipGetLastError();
}

hipError_t launch_macro3(const LaunchCtx &c, const DevState &s, int cur, double *out)
{
    if (c.fp32)
        hipLaunchKernelGGL((k3_macro<float>), grid_nodes(c), dim3(256), 0, c.st, s.params, (const float *)s.pop[cur],
                           s.side[cur], out);
    else
        hipLaunchKernelGGL((k3_macro<double>), grid_nodes(c), dim3(256), 0, c.st, s.params,
                           (const double *)s.pop[cur], s.side[cur], out);
    return hipGetLastError();
}

hipError_t launch_monitors3(const LaunchCtx &c, const DevState &s, int cur, double *partials, int nblocks,
                            double *out)
{
    hipError_t e = launch_macro3(c, s, cur, s.aux);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k3_monitor_partials, dim3(nblocks), dim3(kMonThreads), 0, c.st, s.params, s.aux,
                       s.side[cur], partials);
    return launch_monitor_final(c, partials, nblocks, out);
}

} // namespace pond
