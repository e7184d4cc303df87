// pond_step.hip -- the fused time step of D1Q3 and D2Q9 lattices: one kernel per step.
//
// The state between steps is the streamed state of the last step, gauge free (the moment
// planes rho, u and the central moments of f and g about u; pond_internal.h), before its
// collision.  Each workgroup of k_step
//   1. recomputes the non-local closure and the collision of that state on its tile and a
//      2-node halo: density on a 5-node halo, Korteweg stress K on 4 (eq. 18), force
//      F = -div K and the thermodynamic state on 3 (App. F), the heat-flux correction M0
//      (eq. 9) and the collisions of f and g on 2 (eqs. 16-22);
//   2. collides every donor of the tile and its halo on its central moments (the
//      collision is linear in the populations and its equilibria and sources are
//      polynomials of the peculiar velocity, pond_collide.h) and shifts them to the
//      tile's reference velocity in LDS: the moments the two-kernel step takes of its
//      stored populations;
//   3. streams (the predictor-corrector passes of k_stream, pond_stream.h) and writes the
//      new streamed state.
// So the collided populations never reach HBM: a step reads and writes the 18 moment
// planes once (FP64 144 B per node each way), against populations and side fields in,
// moment planes out, moment planes in, populations and side fields out for two kernels.
// The recomputation costs the collision of the halo ring (a 20 x 20 donor region for a
// 16 x 16 tile) and the closure stages on their wider regions.
#include <hip/hip_ext.h>
#include <hip/hip_runtime.h>

#include <type_traits>

#include "pond_collide.h"
#include "pond_device.h"
#include "pond_internal.h"
#include "pond_stream.h"

namespace pond {

// Two lanes per receiver (lane 2 i + set), as in k_stream; blocks of at most 256 lanes
// are compiled for three waves per SIMD, larger ones for two.
template <int DIM, bool MIXED, typename LdsT, int TX, int TY, bool GEN>
__global__ void __launch_bounds__(2 * TX *TY, 2 * TX *TY <= 256 ? 3 : 2)
    k_step(const SlotDesc *__restrict__ slots, int nslots)
{
    using L = Layout<DIM>;
    using MIO = MomIO<DIM, MIXED>;
    constexpr int Q = L::Q, NF = L::NF;
    constexpr int NT = 2 * TX * TY;
    constexpr int LX = TX + 4, LY = DIM == 2 ? TY + 4 : 1, LN = LX * LY;   // donors: halo 2
    constexpr int HX = TX + 6, HY = DIM == 2 ? TY + 6 : 1, HN = HX * HY;   // closure: halo 3
    constexpr int KX = TX + 8, KY = DIM == 2 ? TY + 8 : 1, KN = KX * KY;   // stress: halo 4
    constexpr int RX = TX + 10, RY = DIM == 2 ? TY + 10 : 1, RN = RX * RY; // density: halo 5
    // The donors' moment fields (written after the closure) share LDS with the density
    // and stress regions (dead once the closure is computed).
    constexpr size_t kFieldBytes = (size_t)2 * NF * LN * sizeof(LdsT);
    constexpr size_t kRKBytes = (size_t)(RN + 3 * KN) * sizeof(double);
    constexpr size_t kUnionWords = ((kFieldBytes > kRKBytes ? kFieldBytes : kRKBytes) + 7) / 8;
    __shared__ __align__(16) double s_union[kUnionWords];
    __shared__ double s_th[kThFields * HN];
    __shared__ int abort_block;
    LdsT *lds = (LdsT *)s_union;
    double *s_rho = s_union;
    double *s_K = s_union + RN; // xx, xy, yy planes of KN

    // lattice and tile of this workgroup
    const int gtile = xcd_tile(blockIdx.x, gridDim.x);
    const SlotDesc &S = slots[find_slot<true>(slots, nslots, gtile)];
    const int tile = gtile - S.st_begin;
    int *__restrict__ flags = S.flags;
    const void *msrc = S.smom_src;
    const int tid = threadIdx.x + 2 * TX * threadIdx.y;
    int err_before = 0;
    if (tid == 0) err_before = flags[kFlagErr];
    const POND_GLOBAL DevParams &P = *(const POND_GLOBAL DevParams *)S.P;
    const Geo geo = make_geo(P);
    const size_t N = P.N;
    const int bx0 = (tile % S.st_tiles_x) * TX;
    const int by0 = DIM == 2 ? (tile / S.st_tiles_x) * TY : 0;
    const double dt = P.dt;
    const bool force = P.kappa != 0.0;
    const double visc = (1.0 / P.omega - 0.5) * dt; // mu = visc p
    // copy stages are needed when the stress region (halo 4, the widest one with copied
    // cells) reaches an outflow face (uniform over the block)
    const bool has_copy = (bx0 - 4 < 0 && geo.bc(0, 0) == kOutflow) || (bx0 + TX + 4 > P.nx && geo.bc(0, 1) == kOutflow) ||
                          (DIM == 2 && ((by0 - 4 < 0 && geo.bc(1, 0) == kOutflow) ||
                                        (by0 + TY + 4 > P.ny && geo.bc(1, 1) == kOutflow)));

    // the tile's reference velocity for the donor moments: the gauge velocity (= the
    // streamed u) at the clamped tile centre
    const int cnode = min(bx0 + TX / 2, P.nx - 1) + P.nx * (DIM == 2 ? min(by0 + TY / 2, P.ny - 1) : 0);
    const double rx = MIO::load(msrc, N, cnode, L::kUx);
    const double ry = DIM == 2 ? MIO::load(msrc, N, cnode, L::kUy) : 0.0;
    const double rho_c = MIO::load(msrc, N, cnode, L::kRho);
    constexpr bool kDevI = sizeof(LdsT) == 4;
    const double refR0 = rho_c;                                   // the f sum (kept by the collision)
    const double refR1 = kDevI ? MIO::load(msrc, N, cnode, L::kG) : 0.0; // the streamed g sum

    // this lane's receiver and its own streamed state
    const int lxr = (int)threadIdx.x >> 1;
    const int myset = (int)threadIdx.x & 1;
    const int gx = bx0 + lxr;
    const int gy = by0 + (DIM == 2 ? threadIdx.y : 0);
    const bool inside = gx < P.nx && (DIM == 1 || gy < P.ny);
    const int node = inside ? gx + P.nx * gy : cnode;
    double Ux = MIO::load(msrc, N, node, L::kUx);
    double Uy = DIM == 2 ? MIO::load(msrc, N, node, L::kUy) : 0.0;
    const double rho_own = MIO::load(msrc, N, node, L::kRho);

    // --- global loads of the whole closure and collision, issued together ---------
    constexpr int RITEMS = (RN + NT - 1) / NT;
    double pre_rho[RITEMS];
    if (force) {
#pragma unroll
        for (int j = 0; j < RITEMS; ++j) {
            const int li = tid + j * NT;
            pre_rho[j] = 0.0;
            if (li < RN) {
                const int nb = map_node<DIM>(geo, bx0 - 5 + li % RX, by0 - 5 + li / RX);
                pre_rho[j] = nb >= 0 ? MIO::load(msrc, N, nb, L::kRho) : P.ghost[-nb - 1].rho;
            }
        }
    }
    constexpr int HITEMS = (HN + NT - 1) / NT;
    double pre_c[HITEMS][4]; // rho, u_x, u_y, g sum of the closure positions
#pragma unroll
    for (int j = 0; j < HITEMS; ++j) {
        const int li = tid + j * NT;
        if (li < HN) {
            int cx, cy, face;
            const int px = bx0 - 3 + li % HX, py = by0 - 3 + li / HX;
            if (classify<DIM>(geo, px, py, cx, cy, face) == kSelf) {
                const int nb = map_node<DIM>(geo, px, DIM == 2 ? py : 0);
                pre_c[j][0] = force ? 0.0 : MIO::load(msrc, N, nb, L::kRho);
                pre_c[j][1] = MIO::load(msrc, N, nb, L::kUx);
                pre_c[j][2] = DIM == 2 ? MIO::load(msrc, N, nb, L::kUy) : 0.0;
                pre_c[j][3] = MIO::load(msrc, N, nb, L::kG);
            }
        }
    }
    // donor nodes (the tile and its 2-node halo), one per lane: rho, u, the stored f
    // moments and the nine g moments; each lane collides both sets of its node
    constexpr int DNODES = (LN + NT - 1) / NT;
    constexpr int NOWN = DIM == 2 ? 3 : 2;
    constexpr int NFS = L::kFStored;
    constexpr int NPRE = NOWN + NFS + NF;
    double pre_d[DNODES][NPRE];
#pragma unroll
    for (int j = 0; j < DNODES; ++j) {
        const int li = tid + j * NT;
        if (li < LN) {
            const int px = bx0 - 2 + li % LX, py = by0 - 2 + li / LX;
            int cx, cy, face;
            if (classify<DIM>(geo, px, py, cx, cy, face) == kSelf) {
                const int nb = map_node<DIM>(geo, px, DIM == 2 ? py : 0);
#pragma unroll
                for (int i = 0; i < NOWN; ++i) pre_d[j][i] = MIO::load(msrc, N, nb, i);
#pragma unroll
                for (int i = 0; i < NFS; ++i) pre_d[j][NOWN + i] = MIO::load(msrc, N, nb, L::kF + i);
#pragma unroll
                for (int i = 0; i < NF; ++i) pre_d[j][NOWN + NFS + i] = MIO::load(msrc, N, nb, L::kG + i);
            }
        }
    }

    // --- stage 1: density ----------------------------------------------------------
    if (force) {
#pragma unroll
        for (int j = 0; j < RITEMS; ++j) {
            const int li = tid + j * NT;
            if (li < RN) s_rho[li] = pre_rho[j];
        }
    }
    if (tid == 0) {
        abort_block = err_before;
        // one step more has started without an earlier failure
        if (tile == 0 && err_before == 0) atomicAdd(&flags[kFlagSteps], 1);
    }
    __syncthreads();
    // leave the state alone after an earlier failure
    if (abort_block != 0) return;

    // --- stage 2: Korteweg stress --------------------------------------------------
    if (force) {
        for (int li = tid; li < KN; li += NT) {
            const int kx = li % KX, ky = li / KX;
            int cx, cy, face;
            const int cls = classify<DIM>(geo, bx0 - 4 + kx, by0 - 4 + ky, cx, cy, face);
            if (cls == kSelf) {
                double K[3];
                korteweg_stress<DIM>(s_rho, (DIM == 2 ? (ky + 1) * RX : 0) + kx + 1, RX, P.kappa, K);
                s_K[li] = K[0];
                s_K[KN + li] = K[1];
                s_K[2 * KN + li] = K[2];
            } else if (cls == kGhost) {
                s_K[li] = s_K[KN + li] = s_K[2 * KN + li] = 0.0; // uniform inflow state
            }
        }
        __syncthreads();
        if (has_copy) {
            for (int li = tid; li < KN; li += NT) {
                const int kx = li % KX, ky = li / KX;
                int cx, cy, face;
                if (classify<DIM>(geo, bx0 - 4 + kx, by0 - 4 + ky, cx, cy, face) == kCopy) {
                    const int src = (cx - (bx0 - 4)) + (DIM == 2 ? (cy - (by0 - 4)) * KX : 0);
                    s_K[li] = s_K[src];
                    s_K[KN + li] = s_K[KN + src];
                    s_K[2 * KN + li] = s_K[2 * KN + src];
                }
            }
            __syncthreads();
        }
    }

    // --- stage 3: force and thermodynamic state of the collision -------------------
    int err_c = 0;
#pragma unroll
    for (int j = 0; j < HITEMS; ++j) {
        const int li = tid + j * NT;
        if (li >= HN) break;
        const int hx = li % HX, hy = li / HX;
        int cx, cy, face;
        const int cls = classify<DIM>(geo, bx0 - 3 + hx, by0 - 3 + hy, cx, cy, face);
        if (cls == kSelf) {
            double Fx = 0.0, Fy = 0.0;
            if (force) korteweg_force<DIM>(s_K, s_K + KN, s_K + 2 * KN, (DIM == 2 ? (hy + 1) * KX : 0) + hx + 1, KX, Fx, Fy);
            const double rho = force ? s_rho[(DIM == 2 ? (hy + 2) * RX : 0) + hx + 2] : pre_c[j][0];
            err_c |= thermo_state<DIM, GEN>(P, rho, pre_c[j][1], pre_c[j][2], pre_c[j][3], Fx, Fy, visc, s_th, HN, li);
        } else if (cls == kGhost) {
            const POND_GLOBAL GhostFace &G = P.ghost[face];
            s_th[kThT * HN + li] = G.T;
            s_th[kThH * HN + li] = G.h;
            s_th[kThMu * HN + li] = G.mu;
            s_th[kThKc * HN + li] = G.kc;
        }
    }
    __syncthreads();
    if (has_copy) {
        for (int li = tid; li < HN; li += NT) {
            const int hx = li % HX, hy = li / HX;
            int cx, cy, face;
            if (classify<DIM>(geo, bx0 - 3 + hx, by0 - 3 + hy, cx, cy, face) == kCopy) {
                const int src = (cx - (bx0 - 3)) + (DIM == 2 ? (cy - (by0 - 3)) * HX : 0);
#pragma unroll
                for (int f = 0; f < kThFields; ++f) s_th[f * HN + li] = s_th[f * HN + src];
            }
        }
        __syncthreads();
    }
    // an error here makes the state this launch read the first bad one
    if (err_c) raise_error(flags, err_c | kErrCollideStage, S.parity);

    // FP32 windows hold deviations from R (1, v, v, v^2) of the tile centre, with v = p /
    // rho = theta T_L the per-axis second moment of the centre's collision gauge
    const int cb = (DIM == 2 ? (cnode / P.nx - by0 + 3) * HX : 0) + (cnode % P.nx - bx0 + 3);
    const double refT = kDevI ? s_th[kThP * HN + cb] * (1.0 / rho_c) : 0.0;

    // --- stage 4: collision of the donors, reduced to moments about (rx, ry) --------
    // each lane takes both sets of one donor node: they share its closure fields, and
    // the pair of moments goes to LDS in one store
    using LdsT2 = typename std::conditional<sizeof(LdsT) == 4, float2, double2>::type;
#pragma unroll
    for (int j = 0; j < DNODES; ++j) {
        const int li = tid + j * NT;
        const int wx = li % LX, wy = li / LX;
        int cx, cy, face;
        const int cls = li < LN ? classify<DIM>(geo, bx0 - 2 + wx, by0 - 2 + wy, cx, cy, face) : kCopy;
        if (cls != kCopy) {
            double mf[NF], mg[NF];
            if (cls == kSelf) {
                // collision in moment space, straight to the moments about (rx, ry)
                const double rho = pre_d[j][L::kRho];
                const int hb = (DIM == 2 ? (wy + 1) * HX : 0) + wx + 1;
                const double p = s_th[kThP * HN + hb];
                const double i_rp = 1.0 / (rho * p); // one division for 1 / rho and 1 / p
                const double i_rho = p * i_rp, i_p = rho * i_rp;
                const double u[2] = {pre_d[j][L::kUx], DIM == 2 ? pre_d[j][L::kUy] : 0.0};
                const double F[2] = {s_th[kThFx * HN + hb], DIM == 2 ? s_th[kThFy * HN + hb] : 0.0};
                const double theta = p * i_rho * kInvTL;
                const double M0 = heat_correction<DIM>(P, s_th, HN, hb, HX);
                double of[NF], og[NF];
#pragma unroll
                for (int i = 0; i < NF; ++i) {
                    of[i] = i < NFS ? pre_d[j][NOWN + i] : 0.0;
                    og[i] = pre_d[j][NOWN + NFS + i];
                }
                collide_moments<DIM>(P, 0, rho, i_rho, i_p, u, F, p, theta, og[0], 0.0, of, u[0] - rx, u[1] - ry, mf);
                collide_moments<DIM>(P, 1, rho, i_rho, i_p, u, F, p, theta, og[0], M0, og, u[0] - rx, u[1] - ry, mg);
            } else {
                // inflow ghost: the equilibrium of the face state in its own gauge
                const POND_GLOBAL GhostFace &G = P.ghost[face];
                double pf[Q], pg[Q];
#pragma unroll
                for (int q = 0; q < Q; ++q) {
                    pf[q] = G.f[q];
                    pg[q] = G.g[q];
                }
                const double gs = sqrt(G.theta);
                moments_about<DIM>(pf, G.ux - rx, G.uy - ry, gs, mf);
                moments_about<DIM>(pg, G.ux - rx, G.uy - ry, gs, mg);
            }
            if constexpr (kDevI) {
                mf[0] -= refR0;
                mf[2] -= refR0 * refT;
                mg[0] -= refR1;
                mg[2] -= refR1 * refT;
                if (DIM == 2) {
                    mf[6] -= refR0 * refT;
                    mf[8] -= refR0 * refT * refT;
                    mg[6] -= refR1 * refT;
                    mg[8] -= refR1 * refT * refT;
                }
            }
#pragma unroll
            for (int i = 0; i < NF; ++i) {
                LdsT2 v;
                v.x = (LdsT)mf[i];
                v.y = (LdsT)mg[i];
                *(LdsT2 *)&lds[(i * LN + li) * 2] = v;
            }
        }
    }
    __syncthreads();
    if (has_copy) {
        for (int li = tid; li < LN; li += NT) {
            const int wx = li % LX, wy = li / LX;
            int cx, cy, face;
            if (classify<DIM>(geo, bx0 - 2 + wx, by0 - 2 + wy, cx, cy, face) == kCopy) {
                const int src = (cx - (bx0 - 2)) + (DIM == 2 ? (cy - (by0 - 2)) * LX : 0);
#pragma unroll
                for (int i = 0; i < NF; ++i) {
                    lds[(i * LN + li) * 2] = lds[(i * LN + src) * 2];
                    lds[(i * LN + li) * 2 + 1] = lds[(i * LN + src) * 2 + 1];
                }
            }
        }
        __syncthreads();
    }

    // --- streaming --------------------------------------------------------------------
    // both lanes of a receiver leave together, so the exchanges always pair up
    if (!inside) return;
    // the receiver's gauge and force: its collision of the streamed state
    const int hr = (DIM == 2 ? (threadIdx.y + 3) * HX : 0) + lxr + 3;
    double th = s_th[kThP * HN + hr] * (1.0 / rho_own) * kInvTL;
    const double Fpx = s_th[kThFx * HN + hr];
    const double Fpy = DIM == 2 ? s_th[kThFy * HN + hr] : 0.0;
    const int wbase = (DIM == 2 ? threadIdx.y * LX : 0) + lxr; // window (gx-2, gy-2)
    const LdsT *sbase = &lds[wbase * 2 + myset];
    double pq[Q];
    double sUx = Ux, sUy = Uy, sS = 1.0;
    double rho = 0.0;
    const int err = stream_passes<DIM, LdsT, LN, LX, NT, GEN>(P, sbase, tid, myset, rx, ry, refR0, refR1, refT, Ux,
                                                              Uy, th, Fpx, Fpy, pq, rho, sUx, sUy, sS);
    store_streamed<DIM, MIXED>(S.smom_dst, N, node, myset, pq, rho, Ux, Uy, sUx, sUy, sS);
    if (err) raise_error(flags, err, S.parity);
}

template <int DIM, bool MIXED, typename LdsT, int TX, int TY, bool GEN>
static hipError_t launch_step_g(const LaunchCtx &c, const SlotDesc *slots, int nslots, int tiles)
{
    dim3 block(2 * TX, TY);
    if (c.ev_start)
        hipExtLaunchKernelGGL((k_step<DIM, MIXED, LdsT, TX, TY, GEN>), dim3(tiles), block, 0, c.st, c.ev_start,
                              c.ev_stop, 0, slots, nslots);
    else
        hipLaunchKernelGGL((k_step<DIM, MIXED, LdsT, TX, TY, GEN>), dim3(tiles), block, 0, c.st, slots, nslots);
    return hipGetLastError();
}

template <int DIM, bool MIXED, typename LdsT, int TX, int TY>
static hipError_t launch_step_t(const LaunchCtx &c, const SlotDesc *slots, int nslots, int tiles)
{
    return c.gen_eos ? launch_step_g<DIM, MIXED, LdsT, TX, TY, true>(c, slots, nslots, tiles)
                     : launch_step_g<DIM, MIXED, LdsT, TX, TY, false>(c, slots, nslots, tiles);
}

// the tile shapes of k_stream (stream_tile_shape), same indices
template <bool MIXED, typename LdsT>
static hipError_t launch_step_v(const LaunchCtx &c, const SlotDesc *slots, int nslots, int tiles)
{
    if (c.dim == 2) {
        switch (c.stream_tile) {
        case 1: return launch_step_t<2, MIXED, LdsT, 32, 4>(c, slots, nslots, tiles);
        case 2: return launch_step_t<2, MIXED, LdsT, 16, 8>(c, slots, nslots, tiles);
        case 3: return launch_step_t<2, MIXED, LdsT, 64, 4>(c, slots, nslots, tiles);
        case 4: return launch_step_t<2, MIXED, LdsT, 16, 4>(c, slots, nslots, tiles);
        case 5: return launch_step_t<2, MIXED, LdsT, 16, 16>(c, slots, nslots, tiles);
        default: return launch_step_t<2, MIXED, LdsT, 32, 8>(c, slots, nslots, tiles);
        }
    }
    if (c.stream_tile == 1) return launch_step_t<1, MIXED, LdsT, 64, 1>(c, slots, nslots, tiles);
    return launch_step_t<1, MIXED, LdsT, 128, 1>(c, slots, nslots, tiles);
}

// This file is compiled twice (build.py): once for the FP32 windows and the dispatcher,
// once with POND_STEP_DOUBLE_WINDOWS for the FP64 windows, which LLVM's max-ilp scheduling
// makes 1-2.5% faster and the FP32 ones slower.
#ifndef POND_STEP_DOUBLE_WINDOWS
hipError_t launch_step_fused(const LaunchCtx &c, const SlotDesc *slots, int nslots, int tiles)
{
    if (c.fp32 == 1) return launch_step_v<true, float>(c, slots, nslots, tiles);
    return launch_step_double_windows(c, slots, nslots, tiles);
}
#else
hipError_t launch_step_double_windows(const LaunchCtx &c, const SlotDesc *slots, int nslots, int tiles)
{
    if (c.fp32 == 2) return launch_step_v<true, double>(c, slots, nslots, tiles);
    return launch_step_v<false, double>(c, slots, nslots, tiles);
}
#endif

} // namespace pond
