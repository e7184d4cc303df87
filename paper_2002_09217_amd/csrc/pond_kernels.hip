// pond_kernels.hip -- HIP kernels (gfx950) of the two-population Particles-on-Demand
// time step of Reyhanian, Dorschner & Karlin, arXiv:2002.09217.
//
// One time step is two kernels on the device state (see pond_internal.h):
//   k_stream         semi-Lagrangian streaming of f and g at v_i = sqrt(theta) c_i + u
//                    (eqs. 1, 3-4) with donors re-expressed in the receiver gauge
//                    (App. C) and cubic reconstruction (App. D), inside the fixed-count
//                    predictor-corrector on (rho, u, E) through the EoS; writes the
//                    streamed state as gauge-free moments
//   k_force_collide  Korteweg stress K (eq. 18) and force F = -div K, the
//                    thermodynamic state of the step, the heat-flux correction M0
//                    (eq. 9), re-expression of the streamed state in the collision
//                    gauge (u, theta), BGK collision of f with the force source
//                    (eqs. 16-17) and of g with the force-extended equilibrium and the
//                    sources g~ + phi (eqs. 19-22); LDS-staged halos
// The initial state additionally uses k_korteweg and k_init_equilibrium.
//
// The streaming kernel works "moment first": every donor's populations are reduced
// once to their nine moments about a tile reference velocity (LDS), the nine moment
// fields are interpolated at the departure points, and the receiver-gauge
// populations follow from the quadratic Lagrange coefficients of the receiver
// velocities.  Since the transfer matrix is M'^{-1} M and the reconstruction is
// linear, this equals re-gauging every donor first and interpolating afterwards.
#include <hip/hip_ext.h>
#include <hip/hip_runtime.h>

#include "pond_collide.h"
#include "pond_device.h"
#include "pond_internal.h"
#include "pond_stream.h"

namespace pond {

// ---------------------------------------------------------------------------
// flags
// ---------------------------------------------------------------------------
__global__ void k_reset_flags(int *flags)
{
    if (threadIdx.x < kFlagWords) flags[threadIdx.x] = 0;
}

hipError_t launch_reset_flags(const LaunchCtx &c, int *flags)
{
    hipLaunchKernelGGL(k_reset_flags, dim3(1), dim3(64), 0, c.st, flags);
    return hipGetLastError();
}

// flags of every lattice of a descriptor array: clear them, or copy them into one
// array (slot s at out[s kFlagWords ...]) for a single read-back
__global__ void k_reset_slot_flags(const SlotDesc *__restrict__ slots, int nslots)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < nslots * kFlagWords) slots[i / kFlagWords].flags[i % kFlagWords] = 0;
}

__global__ void k_gather_slot_flags(const SlotDesc *__restrict__ slots, int nslots, int *__restrict__ out)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < nslots * kFlagWords) out[i] = slots[i / kFlagWords].flags[i % kFlagWords];
}

hipError_t launch_reset_slot_flags(hipStream_t st, const SlotDesc *slots, int nslots)
{
    const int n = nslots * kFlagWords;
    hipLaunchKernelGGL(k_reset_slot_flags, dim3((n + 255) / 256), dim3(256), 0, st, slots, nslots);
    return hipGetLastError();
}

hipError_t launch_gather_slot_flags(hipStream_t st, const SlotDesc *slots, int nslots, int *out)
{
    const int n = nslots * kFlagWords;
    hipLaunchKernelGGL(k_gather_slot_flags, dim3((n + 255) / 256), dim3(256), 0, st, slots, nslots, out);
    return hipGetLastError();
}


// ---------------------------------------------------------------------------
// streaming with the predictor-corrector
// ---------------------------------------------------------------------------
// Two lanes per receiver: lane 2 i + set works on population set `set` (0 = f, 1 = g)
// of receiver i; the pass moments are exchanged between the two lanes.  Blocks of at
// most 256 lanes are compiled for three waves per SIMD, larger ones for two.
template <int DIM, typename PopT, typename LdsT, int TX, int TY, bool GEN>
__global__ void __launch_bounds__(2 * TX *TY, 2 * TX *TY <= 256 ? 3 : 2)
    k_stream(const SlotDesc *__restrict__ slots, int nslots)
{
    using L = Layout<DIM>;
    constexpr int Q = L::Q, NF = L::NF, H = 2;
    constexpr int LX = TX + 2 * H;
    constexpr int LY = DIM == 2 ? TY + 2 * H : 1;
    constexpr int LN = LX * LY;
    constexpr int NT = 2 * TX * TY;
    // Moment fields of the tile.  The two sets of a node are adjacent (index
    // ((mn LN + node) 2 + set)), so the two lanes of a receiver and neighbouring
    // receivers read one contiguous run of LDS words: no bank conflicts.
    constexpr int CS = 2;                                         // column stride
    __shared__ LdsT lds[2 * NF * LN];
    __shared__ int abort_block;

    // lattice and tile of this workgroup
    const int gtile = xcd_tile(blockIdx.x, gridDim.x);
    const SlotDesc &S = slots[find_slot<true>(slots, nslots, gtile)];
    const int tile = gtile - S.st_begin;
    int *__restrict__ flags = S.flags;
    const POND_GLOBAL PopT *__restrict__ fpop = (const POND_GLOBAL PopT *)S.pop_src;
    const POND_GLOBAL double *__restrict__ side = (const POND_GLOBAL double *)S.side_src;
    POND_GLOBAL double *__restrict__ mom = (POND_GLOBAL double *)S.mom;

    // Error state of earlier steps: read now, acted on after the fill (which only reads),
    // so that its latency overlaps the fill's loads.  The decision is taken once per
    // block, so every wave of the block leaves together.
    const int tid = threadIdx.x + 2 * TX * threadIdx.y;
    int err_before = 0;
    if (tid == 0) err_before = flags[kFlagErr];
    const POND_GLOBAL DevParams &P = *(const POND_GLOBAL DevParams *)S.P;
    const Geo geo = make_geo(P);
    const size_t N = P.N; // plane offsets reach 5 N (side) and 2 Q N (populations)
    const int bx0 = (tile % S.st_tiles_x) * TX;
    const int by0 = DIM == 2 ? (tile / S.st_tiles_x) * TY : 0;

    // reference velocity of the tile: gauge velocity at its (clamped) centre node
    const int cnode = min(bx0 + TX / 2, P.nx - 1) + P.nx * (DIM == 2 ? min(by0 + TY / 2, P.ny - 1) : 0);
    const double rx = side[kSideUx * N + cnode];
    const double ry = DIM == 2 ? side[kSideUy * N + cnode] : 0.0;

    // FP32 streaming: the LDS holds every donor moment minus a reference moment vector of
    // the tile, and the FP32 window arithmetic carries only that variation.  The reference
    // is the equilibrium-shaped vector of the tile's centre node, R (1, v, v, v^2) at the
    // moments (0,0), (0,2), (2,0), (2,2) and zero elsewhere, with R its FP64 set sum (rho
    // for f, 2 rho E for g) and v = theta T_L the per-axis second moment of the weights in
    // the centre's gauge.  Each axis's Lagrange weights reproduce a constant, so the
    // reference streams to sum_mn A_km B_ln Mref_mn = R a_k b_l with a_k = A_k0 + v A_k2,
    // b_l = B_l0 + v B_l2, added in FP64.
    constexpr bool kDevI = sizeof(LdsT) == 4;
    static_assert(!kDevI || kDeviationStore<PopT>, "FP32 streaming comes with the FP32 store");
    const POND_GLOBAL double *__restrict__ fsum = (const POND_GLOBAL double *)(fpop + (size_t)2 * Q * N);
    double refR0 = 0.0, refR1 = 0.0, refT = 0.0;
    if constexpr (kDevI) {
        refR0 = fsum[cnode];
        refR1 = fsum[(size_t)N + cnode];
        refT = side[kSideTh * N + cnode] * kTL;
    }

    // the receiver's own gauge and force, loaded now so that the latency overlaps the fill
    const int lxr = (int)threadIdx.x >> 1;
    const int myset = (int)threadIdx.x & 1;
    const int gx = bx0 + lxr;
    const int gy = by0 + (DIM == 2 ? threadIdx.y : 0);
    const bool inside = gx < P.nx && (DIM == 1 || gy < P.ny);
    const int node = inside ? gx + P.nx * gy : cnode;
    double Ux = side[kSideUx * N + node];
    double Uy = DIM == 2 ? side[kSideUy * N + node] : 0.0;
    double th = side[kSideTh * N + node];
    const double Fpx = side[kSideFx * N + node];
    const double Fpy = DIM == 2 ? side[kSideFy * N + node] : 0.0;

    // donors of the tile and its halo: moments about (rx, ry) into LDS, one work item
    // per (node, set).  Each thread takes its items two at a time and issues the global
    // loads of both before using either, so the memory latency of the fill is paid once
    // per pair.
    constexpr int NITEMS = 2 * LN;
    constexpr bool dev = kDeviationStore<PopT>;
    struct Raw {
        int li, set, node;
        double ux, uy, th;
        PopT p[Q];
        double sum; // FP32 storage: the set's sum
    };
    auto load_raw = [&](int it, Raw &r) {
        r.li = it >> 1;
        r.set = it & 1;
        const int lx = r.li % LX, ly = r.li / LX;
        r.node = map_node<DIM>(geo, bx0 - H + lx, by0 - H + ly);
        if (r.node >= 0) {
            r.ux = side[kSideUx * N + r.node];
            r.uy = DIM == 2 ? side[kSideUy * N + r.node] : 0.0;
            r.th = side[kSideTh * N + r.node];
            const POND_GLOBAL PopT *src = fpop + (size_t)r.set * Q * N;
#pragma unroll
            for (int q = 0; q < Q; ++q) r.p[q] = src[(size_t)q * N + r.node];
            if (dev) r.sum = fsum[(size_t)r.set * N + r.node];
        } else {
            const POND_GLOBAL GhostFace &G = P.ghost[-r.node - 1];
            r.ux = G.ux;
            r.uy = G.uy;
            r.th = G.theta;
            const POND_GLOBAL double *src = r.set == 0 ? G.f : G.g;
            double sum = 0.0;
            if (dev) {
#pragma unroll
                for (int q = 0; q < Q; ++q) sum += src[q];
            }
            r.sum = sum;
#pragma unroll
            for (int q = 0; q < Q; ++q) r.p[q] = (PopT)(src[q] - (dev ? weight_q<DIM>(q) * sum : 0.0));
        }
    };
    auto store_moments = [&](const Raw &r) {
        const double s = sqrt(r.th);
        double fr[Q], m[NF];
#pragma unroll
        for (int q = 0; q < Q; ++q) fr[q] = dev ? weight_q<DIM>(q) * r.sum + (double)r.p[q] : (double)r.p[q];
        moments_about<DIM>(fr, r.ux - rx, r.uy - ry, s, m);
        if constexpr (kDevI) {
            const double R = r.set == 0 ? refR0 : refR1;
            m[0] -= R;
            m[2] -= R * refT;
            if (DIM == 2) {
                m[6] -= R * refT;
                m[8] -= R * refT * refT;
            }
        }
#pragma unroll
        for (int i = 0; i < NF; ++i) lds[(i * LN + r.li) * 2 + r.set] = (LdsT)m[i];
    };
    for (int it = tid; it < NITEMS; it += 2 * NT) {
        Raw ra, rb;
        const bool two = it + NT < NITEMS;
        load_raw(it, ra);
        if (two) load_raw(it + NT, rb);
        store_moments(ra);
        if (two) store_moments(rb);
    }
    if (tid == 0) {
        abort_block = err_before;
        // one step more has started without an earlier failure
        if (tile == 0 && err_before == 0) atomicAdd(&flags[kFlagSteps], 1);
    }
    __syncthreads();
    // leave the state alone after an earlier failure
    if (abort_block != 0) return;

    // both lanes of a receiver leave together, so the exchanges below always pair up
    if (!inside) return;
    const int wbase = (DIM == 2 ? threadIdx.y * LX : 0) + lxr; // window (gx-2, gy-2)
    const double dt = P.dt;

    // this lane's set of the receiver, in the gauge (sUx, sUy, sS) of the last pass
    double pq[Q];
    double sUx = Ux, sUy = Uy, sS = 1.0;
    double rho = 0.0;
    int err = 0;
    const LdsT *sbase = &lds[wbase * 2 + myset];
    err |= stream_passes<DIM, LdsT, LN, LX, NT, GEN>(P, sbase, tid, myset, rx, ry, refR0, refR1, refT, Ux, Uy, th,
                                                     Fpx, Fpy, pq, rho, sUx, sUy, sS);

    store_streamed<DIM, false>(S.mom, N, node, myset, pq, rho, Ux, Uy, sUx, sUy, sS);
    if (err) raise_error(flags, err, S.parity);
}

template <int DIM, typename PopT, typename LdsT, int TX, int TY, bool GEN>
static hipError_t launch_stream_g(const LaunchCtx &c, const SlotDesc *slots, int nslots, int tiles)
{
    dim3 block(2 * TX, TY);
    if (c.ev_start)
        hipExtLaunchKernelGGL((k_stream<DIM, PopT, LdsT, TX, TY, GEN>), dim3(tiles), block, 0, c.st,
                              c.ev_start, c.ev_stop, 0, slots, nslots);
    else
        hipLaunchKernelGGL((k_stream<DIM, PopT, LdsT, TX, TY, GEN>), dim3(tiles), block, 0, c.st, slots,
                           nslots);
    return hipGetLastError();
}
template <int DIM, typename PopT, typename LdsT, int TX, int TY>
static hipError_t launch_stream_t(const LaunchCtx &c, const SlotDesc *slots, int nslots, int tiles)
{
    return c.gen_eos ? launch_stream_g<DIM, PopT, LdsT, TX, TY, true>(c, slots, nslots, tiles)
                     : launch_stream_g<DIM, PopT, LdsT, TX, TY, false>(c, slots, nslots, tiles);
}

// Tile shapes of the streaming kernel (receivers per block, x by y); the library picks
// one per lattice, by measurement or as requested (pond_config.tile).
static const int kTiles2D[][2] = {{32, 8}, {32, 4}, {16, 8}, {64, 4}, {16, 4}, {16, 16}};
static const int kTiles1D[][2] = {{128, 1}, {64, 1}};

int stream_variants(int dim) { return dim == 3 ? 1 : dim == 2 ? 6 : 2; }
void stream_tile_shape(int dim, int v, int *tx, int *ty)
{
    if (dim == 3) {
        stream3_tile(1, tx, ty); // one shape in every precision
        return;
    }
    *tx = dim == 2 ? kTiles2D[v][0] : kTiles1D[v][0];
    *ty = dim == 2 ? kTiles2D[v][1] : kTiles1D[v][1];
}

template <typename PopT, typename LdsT>
static hipError_t launch_stream_v(const LaunchCtx &c, const SlotDesc *slots, int nslots, int tiles)
{
    if (c.dim == 2) {
        switch (c.stream_tile) {
        case 1: return launch_stream_t<2, PopT, LdsT, 32, 4>(c, slots, nslots, tiles);
        case 2: return launch_stream_t<2, PopT, LdsT, 16, 8>(c, slots, nslots, tiles);
        case 3: return launch_stream_t<2, PopT, LdsT, 64, 4>(c, slots, nslots, tiles);
        case 4: return launch_stream_t<2, PopT, LdsT, 16, 4>(c, slots, nslots, tiles);
        case 5: return launch_stream_t<2, PopT, LdsT, 16, 16>(c, slots, nslots, tiles);
        default: return launch_stream_t<2, PopT, LdsT, 32, 8>(c, slots, nslots, tiles);
        }
    }
    if (c.stream_tile == 1) return launch_stream_t<1, PopT, LdsT, 64, 1>(c, slots, nslots, tiles);
    return launch_stream_t<1, PopT, LdsT, 128, 1>(c, slots, nslots, tiles);
}

hipError_t launch_stream(const LaunchCtx &c, const SlotDesc *slots, int nslots, int tiles)
{
    if (c.dim == 3) return launch_stream3(c, slots); // one lattice per launch
    if (c.fp32 == 1) return launch_stream_v<float, float>(c, slots, nslots, tiles);
    if (c.fp32 == 2) return launch_stream_v<float, double>(c, slots, nslots, tiles);
    return launch_stream_v<double, double>(c, slots, nslots, tiles);
}

// ---------------------------------------------------------------------------
// Korteweg stress K = -kappa (rho lap rho + |grad rho|^2/2) I + kappa grad rho grad rho
// with the isotropic lattice stencils grad = (1/T_L) sum W c, lap = (2/T_L) sum W (. - .0)
// ---------------------------------------------------------------------------
template <int DIM>
__global__ void k_korteweg(const DevParams *__restrict__ Pp, const double *__restrict__ rho,
                           double *__restrict__ kor, const int *__restrict__ flags)
{
    if (flags[kFlagErr] != 0) return;
    const DevParams &P = *Pp;
    const Geo geo = make_geo(P);
    const int x = blockIdx.x * blockDim.x + threadIdx.x;
    const int y = DIM == 2 ? blockIdx.y * blockDim.y + threadIdx.y : 0;
    if (x >= P.nx || y >= (DIM == 2 ? P.ny : 1)) return;
    const int node = x + P.nx * y;
    const size_t N = P.N;
    const double r0 = rho[node];
    double gx = 0.0, gy = 0.0, lap = 0.0;
    constexpr int Q = Layout<DIM>::Q;
#pragma unroll
    for (int q = 0; q < Q; ++q) {
        const int cx = DIM == 2 ? q / 3 - 1 : q - 1;
        const int cy = DIM == 2 ? q % 3 - 1 : 0;
        const double w = DIM == 2 ? kW1[q / 3] * kW1[q % 3] : kW1[q];
        const int nb = map_node<DIM>(geo, x + cx, y + cy);
        const double rq = nb >= 0 ? rho[nb] : P.ghost[-nb - 1].rho;
        gx += w * (double)cx * rq;
        gy += w * (double)cy * rq;
        lap += w * (rq - r0);
    }
    gx /= kTL;
    gy /= kTL;
    lap *= 2.0 / kTL;
    const double iso = -P.kappa * (r0 * lap + 0.5 * (gx * gx + gy * gy));
    kor[0 * (size_t)N + node] = iso + P.kappa * gx * gx;
    kor[1 * (size_t)N + node] = P.kappa * gx * gy;
    kor[2 * (size_t)N + node] = DIM == 2 ? iso + P.kappa * gy * gy : 0.0;
}

static inline void grid2(const LaunchCtx &c, dim3 &grid, dim3 &block)
{
    if (c.dim == 2) {
        block = dim3(64, 4);
        grid = dim3((c.nx + 63) / 64, (c.ny + 3) / 4);
    } else {
        block = dim3(256, 1);
        grid = dim3((c.nx + 255) / 256, 1);
    }
}

hipError_t launch_korteweg(const LaunchCtx &c, const DevState &s, const double *rho)
{
    dim3 grid, block;
    grid2(c, grid, block);
    if (c.dim == 2)
        hipLaunchKernelGGL(k_korteweg<2>, grid, block, 0, c.st, s.params, rho, s.kor, s.flags);
    else
        hipLaunchKernelGGL(k_korteweg<1>, grid, block, 0, c.st, s.params, rho, s.kor, s.flags);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// F = -div K at a node from the stress planes (initial state only)
// ---------------------------------------------------------------------------
template <int DIM, typename PT>
__device__ __forceinline__ void korteweg_force_at(const PT &P, const double *__restrict__ kor,
                                                  int x, int y, double &Fx, double &Fy)
{
    const Geo geo = make_geo(P);
    Fx = 0.0;
    Fy = 0.0;
    if (P.kappa == 0.0) return;
    const size_t N = P.N;
    double dvx = 0.0, dvy = 0.0;
    constexpr int Q = Layout<DIM>::Q;
#pragma unroll
    for (int q = 0; q < Q; ++q) {
        const int cx = DIM == 2 ? q / 3 - 1 : q - 1;
        const int cy = DIM == 2 ? q % 3 - 1 : 0;
        const double w = DIM == 2 ? kW1[q / 3] * kW1[q % 3] : kW1[q];
        const int nb = map_node<DIM>(geo, x + cx, y + cy);
        double kxx = 0.0, kxy = 0.0, kyy = 0.0; // inflow ghosts are uniform: K = 0
        if (nb >= 0) {
            kxx = kor[0 * N + nb];
            kxy = kor[1 * N + nb];
            kyy = kor[2 * N + nb];
        }
        dvx += w * (kxx * (double)cx + kxy * (double)cy);
        dvy += w * (kxy * (double)cx + kyy * (double)cy);
    }
    Fx = -dvx / kTL;
    Fy = DIM == 2 ? -dvy / kTL : 0.0;
}


// ---------------------------------------------------------------------------
// Fused non-local closure and collision of one tile (eqs. 9, 16-22; App. F):
//   LDS stage 1  rho on the tile + 3-node halo (from the streamed state)
//   LDS stage 2  Korteweg stress K on the tile + 2-node halo
//   LDS stage 3  F = -div K, actual velocity, T, p, h, mu, k on the tile + 1-node halo
//   per node     heat-flux correction M0, re-expression of the streamed state in the
//                collision gauge (u, theta), BGK collision of f (force source S) and g
//                (force-extended equilibrium, sources g~ + phi); writes the new state.
// Two lanes per node, in separate waves: the first half of the block works on the
// f sets of the tile's nodes, the second half on their g sets (and the heat-flux
// correction, which only g uses); the stencil stages use all lanes of the block.
// ---------------------------------------------------------------------------
template <int DIM> struct CollideTile;
template <> struct CollideTile<2> { static constexpr int TX = 16, TY = 8; };
template <> struct CollideTile<1> { static constexpr int TX = 256, TY = 1; };

// MODE of the closure-and-collision kernel: store the collided state (the second kernel of
// the two-kernel step, or the read-back of a fused-step state), or only evaluate the
// thermodynamic closure of every node and raise its admissibility errors (the check of the
// last state of a run of fused steps)
enum { kCollideStore = 0, kCollideCheck = 1 };

template <int DIM, typename PopT, bool MIXED, int MODE, int TX, int TY>
__global__ void __launch_bounds__(2 * TX *TY)
    k_force_collide(const SlotDesc *__restrict__ slots, int nslots)
{
    using L = Layout<DIM>;
    using MIO = MomIO<DIM, MIXED>;
    constexpr int Q = L::Q, NF = L::NF;
    constexpr int RX = TX + 6, RY = DIM == 2 ? TY + 6 : 1; // rho region (halo 3)
    constexpr int KX = TX + 4, KY = DIM == 2 ? TY + 4 : 1; // K region (halo 2)
    constexpr int HX = TX + 2, HY = DIM == 2 ? TY + 2 : 1; // thermo region (halo 1)
    constexpr int HS = HX * HY;                            // field stride of s_th
    constexpr int NN = TX * TY;                            // nodes of the tile
    constexpr int NT = 2 * NN;
    static_assert(NN % 64 == 0, "each population set must fill whole waves");
    __shared__ double s_rho[RX * RY];
    __shared__ double s_K[3][KX * KY];
    __shared__ double s_th[kThFields * HS];
    __shared__ int abort_block;

    // lattice and tile of this workgroup
    const int gtile = xcd_tile(blockIdx.x, gridDim.x);
    const SlotDesc &S = slots[find_slot<false>(slots, nslots, gtile)];
    const int tile = gtile - S.fc_begin;
    int *__restrict__ flags = S.flags;
    const void *mom = S.mom;
    POND_GLOBAL PopT *__restrict__ fout = (POND_GLOBAL PopT *)S.pop_dst;
    POND_GLOBAL double *__restrict__ side_out = (POND_GLOBAL double *)S.side_dst;

    // error state of earlier steps, acted on once the loads below are under way
    const int tid = threadIdx.x;
    int err_before = 0;
    if (tid == 0) err_before = flags[kFlagErr];

    const POND_GLOBAL DevParams &P = *(const POND_GLOBAL DevParams *)S.P;
    const Geo geo = make_geo(P);
    const size_t N = P.N;
    const int x0 = (tile % S.fc_tiles_x) * TX;
    const int y0 = DIM == 2 ? (tile / S.fc_tiles_x) * TY : 0;
    const double dt = P.dt;
    const bool force = P.kappa != 0.0;
    const double visc = (1.0 / P.omega - 0.5) * dt;   // mu = visc p
    // Whether the K region (halo 2, the widest region with copied cells) reaches an
    // outflow face: only then do the copy stages below have work, and their barriers
    // are skipped otherwise (uniform over the block).
    const bool has_copy = (x0 - 2 < 0 && geo.bc(0, 0) == kOutflow) || (x0 + TX + 2 > P.nx && geo.bc(0, 1) == kOutflow) ||
                          (DIM == 2 && ((y0 - 2 < 0 && geo.bc(1, 0) == kOutflow) ||
                                        (y0 + TY + 2 > P.ny && geo.bc(1, 1) == kOutflow)));

    // this lane's population set (0 = f, 1 = g; uniform per wave) and node
    const int set = tid >= NN ? 1 : 0;
    const int t = tid - set * NN;
    const int lx = t % TX;
    const int ly = t / TX;
    const int x = x0 + lx;
    const int y = y0 + (DIM == 2 ? ly : 0);
    const bool inside = x < P.nx && (DIM == 1 || y < P.ny);
    const int node = inside ? x + P.nx * y : 0;

    // Issue every global load this lane needs before the LDS stages, so that their
    // latencies overlap: rho and u of its node and the moments of its set (used last),
    // and the velocity and energy of its thermo-stage positions (used in stage 3).
    constexpr int NOWN = DIM == 2 ? 3 : 2;           // rho, u
    double own[NOWN], oset[NF];
    if (MODE == kCollideStore && inside) {
#pragma unroll
        for (int i = 0; i < NOWN; ++i) own[i] = MIO::load(mom, N, node, i);
        // NF consecutive planes from the set's first one (the f lanes read the stored f
        // moments and a few g planes they ignore): no branch, so no wait between the sets
        const int base = set == 0 ? L::kF : L::kG;
#pragma unroll
        for (int i = 0; i < NF; ++i) oset[i] = MIO::load(mom, N, node, base + i);
    }
    constexpr int HITEMS = (HX * HY + NT - 1) / NT;
    double pre_u[HITEMS][3];
    int pre_nb[HITEMS];
#pragma unroll
    for (int j = 0; j < HITEMS; ++j) {
        const int li = tid + j * NT;
        pre_nb[j] = -1;
        if (li < HX * HY) {
            const int gx = x0 - 1 + li % HX, gy = y0 - 1 + li / HX;
            int cx, cy, face;
            if (classify<DIM>(geo, gx, gy, cx, cy, face) == kSelf) {
                const int nb = map_node<DIM>(geo, gx, DIM == 2 ? gy : 0);
                pre_nb[j] = nb;
                pre_u[j][0] = MIO::load(mom, N, nb, L::kUx);
                pre_u[j][1] = DIM == 2 ? MIO::load(mom, N, nb, L::kUy) : 0.0;
                pre_u[j][2] = MIO::load(mom, N, nb, L::kG);
            }
        }
    }

    // density of the streamed state on the rho region, loaded with the rest
    constexpr int RITEMS = (RX * RY + NT - 1) / NT;
    double pre_rho[RITEMS];
    if (force) {
#pragma unroll
        for (int j = 0; j < RITEMS; ++j) {
            const int li = tid + j * NT;
            pre_rho[j] = 0.0;
            if (li < RX * RY) {
                const int gx = x0 - 3 + li % RX, gy = y0 - 3 + li / RX;
                const int nb = map_node<DIM>(geo, gx, DIM == 2 ? gy : 0);
                pre_rho[j] = nb >= 0 ? MIO::load(mom, N, nb, L::kRho) : P.ghost[-nb - 1].rho;
            }
        }
    }

    // stage 1: density of the streamed state into LDS
    if (force) {
#pragma unroll
        for (int j = 0; j < RITEMS; ++j) {
            const int li = tid + j * NT;
            if (li < RX * RY) s_rho[li] = pre_rho[j];
        }
        // leave the state alone after an earlier failure (once per block, before any
        // store; the first barrier of either path publishes the decision)
        if (tid == 0) abort_block = err_before;
        __syncthreads();
        if (abort_block != 0) return;
        // stage 2: Korteweg stress on the K region
        for (int li = tid; li < KX * KY; li += NT) {
            const int kx = li % KX, ky = li / KX;
            int cx, cy, face;
            const int cls = classify<DIM>(geo, x0 - 2 + kx, y0 - 2 + ky, cx, cy, face);
            if (cls == kSelf) {
                double K[3];
                korteweg_stress<DIM>(s_rho, (DIM == 2 ? (ky + 1) * RX : 0) + kx + 1, RX, P.kappa, K);
                s_K[0][li] = K[0];
                s_K[1][li] = K[1];
                s_K[2][li] = K[2];
            } else if (cls == kGhost) {
                s_K[0][li] = s_K[1][li] = s_K[2][li] = 0.0; // uniform inflow state
            }
        }
        __syncthreads();
        if (has_copy) {
            for (int li = tid; li < KX * KY; li += NT) {
                const int kx = li % KX, ky = li / KX;
                int cx, cy, face;
                if (classify<DIM>(geo, x0 - 2 + kx, y0 - 2 + ky, cx, cy, face) == kCopy) {
                    const int src = (cx - (x0 - 2)) + (DIM == 2 ? (cy - (y0 - 2)) * KX : 0);
                    s_K[0][li] = s_K[0][src];
                    s_K[1][li] = s_K[1][src];
                    s_K[2][li] = s_K[2][src];
                }
            }
            __syncthreads();
        }
    }

    // stage 3: force and thermodynamic state of the step
    int err = 0;
#pragma unroll
    for (int j = 0; j < HITEMS; ++j) {
        const int li = tid + j * NT;
        if (li >= HX * HY) break;
        const int hx = li % HX, hy = li / HX;
        const int gx = x0 - 1 + hx, gy = y0 - 1 + hy;
        int cx, cy, face;
        const int cls = classify<DIM>(geo, gx, gy, cx, cy, face);
        if (cls == kSelf) {
            double Fx = 0.0, Fy = 0.0;
            if (force)
                korteweg_force<DIM>(s_K[0], s_K[1], s_K[2], (DIM == 2 ? (hy + 1) * KX : 0) + hx + 1, KX, Fx, Fy);
            const int nb = pre_nb[j];
            const double rho = force ? s_rho[(DIM == 2 ? (hy + 2) * RX : 0) + hx + 2] : MIO::load(mom, N, nb, L::kRho);
            err |= thermo_state<DIM>(P, rho, pre_u[j][0], pre_u[j][1], pre_u[j][2], Fx, Fy, visc, s_th, HS, li);
        } else if (cls == kGhost) {
            const POND_GLOBAL GhostFace &G = P.ghost[face];
            s_th[kThT * HS + li] = G.T;
            s_th[kThH * HS + li] = G.h;
            s_th[kThMu * HS + li] = G.mu;
            s_th[kThKc * HS + li] = G.kc;
        }
    }
    if (MODE == kCollideCheck) {
        // the closure of the state is the check: count the launch, report the errors
        if (!force && tid == 0) abort_block = err_before;
        if (!force) __syncthreads();
        if (abort_block != 0) return;
        if (tid == 0 && tile == 0 && err_before == 0) atomicAdd(&flags[kFlagSteps], 1);
        if (err) raise_error(flags, err | kErrCollideStage, S.parity);
        return;
    }
    if (!force && tid == 0) abort_block = err_before;
    __syncthreads();
    if (abort_block != 0) return;
    if (has_copy) {
        for (int li = tid; li < HX * HY; li += NT) {
            const int hx = li % HX, hy = li / HX;
            int cx, cy, face;
            if (classify<DIM>(geo, x0 - 1 + hx, y0 - 1 + hy, cx, cy, face) == kCopy) {
                const int src = (cx - (x0 - 1)) + (DIM == 2 ? (cy - (y0 - 1)) * HX : 0);
#pragma unroll
                for (int f = 0; f < kThFields; ++f) s_th[f * HS + li] = s_th[f * HS + src];
            }
        }
        __syncthreads();
    }
    if (err) raise_error(flags, err, S.parity);

    if (!inside) return;
    const int hb = (DIM == 2 ? (ly + 1) * HX : 0) + lx + 1;

    const double rho = own[L::kRho];
    const double i_rho = 1.0 / rho;
    const double u[2] = {own[L::kUx], DIM == 2 ? own[L::kUy] : 0.0};
    const double F[2] = {s_th[kThFx * HS + hb], DIM == 2 ? s_th[kThFy * HS + hb] : 0.0};
    const double p = s_th[kThP * HS + hb];
    const double theta = p * i_rho * kInvTL;
    const double s = sqrt(theta);

    // this set's streamed populations in the collision gauge (u, theta)
    double pop[Q], post[Q];
    pops_from_central<DIM>(set, rho, oset, s, pop);
    if (set == 0) {
        collide_f<DIM>(P, rho, i_rho, F, theta, s, pop, post);
        store_set<DIM, PopT>(fout, N, node, 0, post);
        side_out[kSideUx * N + node] = u[0];
        side_out[kSideTh * N + node] = theta;
        side_out[kSideFx * N + node] = F[0];
        if (DIM == 2) {
            side_out[kSideUy * N + node] = u[1];
            side_out[kSideFy * N + node] = F[1];
        }
        return;
    }
    const double M0 = heat_correction<DIM>(P, s_th, HS, hb, HX);
    collide_g<DIM>(P, rho, i_rho, u, F, p, s, oset[0], M0, pop, post);
    store_set<DIM, PopT>(fout, N, node, 1, post);
}

template <int DIM, typename PopT, bool MIXED, int MODE>
static hipError_t launch_force_collide_t(const LaunchCtx &c, const SlotDesc *slots, int nslots, int tiles)
{
    constexpr int TX = CollideTile<DIM>::TX, TY = CollideTile<DIM>::TY;
    if (c.ev_start)
        hipExtLaunchKernelGGL((k_force_collide<DIM, PopT, MIXED, MODE, TX, TY>), dim3(tiles), dim3(2 * TX * TY), 0,
                              c.st, c.ev_start, c.ev_stop, 0, slots, nslots);
    else
        hipLaunchKernelGGL((k_force_collide<DIM, PopT, MIXED, MODE, TX, TY>), dim3(tiles), dim3(2 * TX * TY), 0,
                           c.st, slots, nslots);
    return hipGetLastError();
}

template <int DIM, bool MIXED, int MODE>
static hipError_t launch_force_collide_d(const LaunchCtx &c, const SlotDesc *slots, int nslots, int tiles)
{
    return c.fp32 ? launch_force_collide_t<DIM, float, MIXED, MODE>(c, slots, nslots, tiles)
                  : launch_force_collide_t<DIM, double, MIXED, MODE>(c, slots, nslots, tiles);
}

// The two-kernel step reads FP64 moment planes; the fused step's states are read back
// (and checked) from its moment planes, mixed in the FP32 storage precisions.
hipError_t launch_force_collide(const LaunchCtx &c, const SlotDesc *slots, int nslots, int tiles)
{
    if (c.dim == 3) return launch_collide3(c, slots);
    const bool mixed = c.fused && c.fp32;
    if (c.dim == 2)
        return mixed ? launch_force_collide_d<2, true, kCollideStore>(c, slots, nslots, tiles)
                     : launch_force_collide_d<2, false, kCollideStore>(c, slots, nslots, tiles);
    return mixed ? launch_force_collide_d<1, true, kCollideStore>(c, slots, nslots, tiles)
                 : launch_force_collide_d<1, false, kCollideStore>(c, slots, nslots, tiles);
}

hipError_t launch_collide_check(const LaunchCtx &c, const SlotDesc *slots, int nslots, int tiles)
{
    const bool mixed = c.fp32 != 0;
    if (c.dim == 2)
        return mixed ? launch_force_collide_t<2, float, true, kCollideCheck>(c, slots, nslots, tiles)
                     : launch_force_collide_t<2, double, false, kCollideCheck>(c, slots, nslots, tiles);
    return mixed ? launch_force_collide_t<1, float, true, kCollideCheck>(c, slots, nslots, tiles)
                 : launch_force_collide_t<1, double, false, kCollideCheck>(c, slots, nslots, tiles);
}

void tile_counts(const LaunchCtx &c, int *st_tiles_x, int *st_count, int *fc_tiles_x, int *fc_count)
{
    if (c.dim == 3) { // the 3D launchers size their grids themselves
        *st_tiles_x = *st_count = *fc_tiles_x = *fc_count = 1;
        return;
    }
    int tx, ty;
    stream_tile_shape(c.dim, c.stream_tile, &tx, &ty);
    *st_tiles_x = (c.nx + tx - 1) / tx;
    *st_count = *st_tiles_x * (c.dim == 2 ? (c.ny + ty - 1) / ty : 1);
    const int fx = c.dim == 2 ? CollideTile<2>::TX : CollideTile<1>::TX;
    const int fy = c.dim == 2 ? CollideTile<2>::TY : CollideTile<1>::TY;
    *fc_tiles_x = (c.nx + fx - 1) / fx;
    *fc_count = *fc_tiles_x * (c.dim == 2 ? (c.ny + fy - 1) / fy : 1);
}

// ---------------------------------------------------------------------------
// initial state: equilibrium of (rho, u_hat, T) with the force F0 = -div K(rho),
// written as the streamed-state moments so that the regular closure and collision
// kernels turn it into the stored populations
// ---------------------------------------------------------------------------
template <int DIM, bool MIXED>
__global__ void k_init_equilibrium(const DevParams *__restrict__ Pp, const double *__restrict__ rho_in,
                                   const double *__restrict__ u_in, const double *__restrict__ T_in,
                                   const double *__restrict__ kor, void *__restrict__ mom,
                                   int *__restrict__ flags)
{
    using L = Layout<DIM>;
    using MIO = MomIO<DIM, MIXED>;
    constexpr int Q = L::Q, NF = L::NF;
    const DevParams &P = *Pp;
    const int x = blockIdx.x * blockDim.x + threadIdx.x;
    const int y = DIM == 2 ? blockIdx.y * blockDim.y + threadIdx.y : 0;
    if (x >= P.nx || y >= (DIM == 2 ? P.ny : 1)) return;
    const int node = x + P.nx * y;
    const size_t N = P.N;
    const double dt = P.dt;
    double F[2];
    korteweg_force_at<DIM>(P, kor, x, y, F[0], F[1]);
    const double r = rho_in[node];
    const double uh[2] = {u_in[node], DIM == 2 ? u_in[N + node] : 0.0};
    const double u[2] = {uh[0] - F[0] * dt / (2.0 * r), DIM == 2 ? uh[1] - F[1] * dt / (2.0 * r) : 0.0};
    const double T = eos_state_T(P, T_in[node]);
    const double p = eos_p(P, r, T);
    const int bad = eos_bad(P, r, p);
    if (bad) atomicOr(&flags[kFlagErr], bad);
    const double e = eos_e(P, r, T);
    const double E = e + 0.5 * (uh[0] * uh[0] + uh[1] * uh[1]);
    const double theta = p / (r * kTL);
    const double s = sqrt(theta);
    const double Pr = p / r;
    const double H = E + Pr;
    double X[2][2], M[2], Nm[2][2];
    for (int a = 0; a < DIM; ++a)
        for (int b = 0; b < DIM; ++b)
            X[a][b] = uh[a] * F[b] + F[a] * uh[b] + dt * F[a] * F[b] * E / (2.0 * p);
    for (int a = 0; a < DIM; ++a) {
        double xu = 0.0;
        for (int b = 0; b < DIM; ++b) xu += X[a][b] * u[b];
        M[a] = dt / Pr * (F[a] * H - xu);
    }
    for (int a = 0; a < DIM; ++a)
        for (int b = 0; b < DIM; ++b) Nm[a][b] = (a == b ? r : 0.0) + dt / (2.0 * Pr) * X[a][b];
    double f[Q], g[Q];
    for (int q = 0; q < Q; ++q) {
        const double c[2] = {DIM == 2 ? (double)(q / 3 - 1) : (double)(q - 1),
                             DIM == 2 ? (double)(q % 3 - 1) : 0.0};
        const double wq = DIM == 2 ? kW1[q / 3] * kW1[q % 3] : kW1[q];
        double v[2], t1 = 0.0, t2 = 0.0;
        for (int a = 0; a < DIM; ++a) v[a] = u[a] + s * c[a];
        for (int a = 0; a < DIM; ++a) t1 += M[a] * (v[a] - u[a]);
        for (int a = 0; a < DIM; ++a)
            for (int b = 0; b < DIM; ++b) t2 += Nm[a][b] * (v[a] * v[b] - (a == b ? Pr : 0.0) - u[a] * u[b]);
        f[q] = r * wq;
        g[q] = wq * (2.0 * r * E + t1 + t2);
    }
    double mf[NF], mg[NF];
    moments_about<DIM>(f, 0.0, 0.0, s, mf);
    moments_about<DIM>(g, 0.0, 0.0, s, mg);
    MIO::store(mom, N, node, L::kRho, r);
    MIO::store(mom, N, node, L::kUx, u[0]);
    if (DIM == 2) {
        MIO::store(mom, N, node, L::kUy, u[1]);
        MIO::store(mom, N, node, L::kF + 0, mf[4]);
        MIO::store(mom, N, node, L::kF + 1, mf[6]);
        MIO::store(mom, N, node, L::kF + 2, mf[2]);
        MIO::store(mom, N, node, L::kF + 3, mf[7]);
        MIO::store(mom, N, node, L::kF + 4, mf[5]);
        MIO::store(mom, N, node, L::kF + 5, mf[8]);
    } else {
        MIO::store(mom, N, node, L::kF, mf[2]);
    }
    for (int i = 0; i < NF; ++i) MIO::store(mom, N, node, L::kG + i, mg[i]);
}

hipError_t launch_init_equilibrium(const LaunchCtx &c, const DevState &s, const double *rho,
                                   const double *u, const double *T, void *mom)
{
    dim3 grid, block;
    grid2(c, grid, block);
    // the fused step keeps its streamed states mixed FP64/FP32 in the FP32 precisions
    const bool mixed = c.fused && c.fp32;
    if (c.dim == 2) {
        if (mixed)
            hipLaunchKernelGGL((k_init_equilibrium<2, true>), grid, block, 0, c.st, s.params, rho, u, T, s.kor, mom,
                               s.flags);
        else
            hipLaunchKernelGGL((k_init_equilibrium<2, false>), grid, block, 0, c.st, s.params, rho, u, T, s.kor, mom,
                               s.flags);
    } else {
        if (mixed)
            hipLaunchKernelGGL((k_init_equilibrium<1, true>), grid, block, 0, c.st, s.params, rho, u, T, s.kor, mom,
                               s.flags);
        else
            hipLaunchKernelGGL((k_init_equilibrium<1, false>), grid, block, 0, c.st, s.params, rho, u, T, s.kor, mom,
                               s.flags);
    }
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// macroscopic fields of a state: rho, u_hat (dim planes), T, p, E
// ---------------------------------------------------------------------------
template <int DIM, typename PopT>
__global__ void k_macro(const DevParams *__restrict__ Pp, const PopT *__restrict__ fpop,
                        const double *__restrict__ side, double *__restrict__ out)
{
    constexpr int Q = Layout<DIM>::Q;
    const DevParams &P = *Pp;
    const int x = blockIdx.x * blockDim.x + threadIdx.x;
    const int y = DIM == 2 ? blockIdx.y * blockDim.y + threadIdx.y : 0;
    if (x >= P.nx || y >= (DIM == 2 ? P.ny : 1)) return;
    const int n = x + P.nx * y;
    const size_t N = P.N;
    double r = 0.0;
    for (int q = 0; q < Q; ++q) r += (double)fpop[q * N + n];
    if (kDeviationStore<PopT>) r += ((const double *)(fpop + (size_t)2 * Q * N))[n];
    const double hx = side[kSideUx * N + n] + side[kSideFx * N + n] * P.dt / (2.0 * r);
    const double hy = DIM == 2 ? side[kSideUy * N + n] + side[kSideFy * N + n] * P.dt / (2.0 * r) : 0.0;
    const double pr = r * side[kSideTh * N + n] * kTL;
    const double T = eos_T_of_p(P, r, pr);
    const double e = eos_e(P, r, T);
    out[0 * N + n] = r;
    out[1 * N + n] = hx;
    if (DIM == 2) out[2 * N + n] = hy;
    out[(1 + DIM) * N + n] = T;
    out[(2 + DIM) * N + n] = pr;
    out[(3 + DIM) * N + n] = e + 0.5 * (hx * hx + hy * hy);
}

hipError_t launch_macro(const LaunchCtx &c, const DevState &s, int cur, double *out)
{
    if (c.dim == 3) return launch_macro3(c, s, cur, out);
    dim3 grid, block;
    grid2(c, grid, block);
    if (c.dim == 2) {
        if (c.fp32)
            hipLaunchKernelGGL((k_macro<2, float>), grid, block, 0, c.st, s.params,
                               (const float *)s.pop[cur], s.side[cur], out);
        else
            hipLaunchKernelGGL((k_macro<2, double>), grid, block, 0, c.st, s.params,
                               (const double *)s.pop[cur], s.side[cur], out);
    } else {
        if (c.fp32)
            hipLaunchKernelGGL((k_macro<1, float>), grid, block, 0, c.st, s.params,
                               (const float *)s.pop[cur], s.side[cur], out);
        else
            hipLaunchKernelGGL((k_macro<1, double>), grid, block, 0, c.st, s.params,
                               (const double *)s.pop[cur], s.side[cur], out);
    }
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// conservation monitors: per-block partial sums (wavefront shuffles, then LDS),
// reduced in a fixed order by one block.  Inputs are the macroscopic planes
// written by k_macro (rho, u_hat, T, p, E).
//   0 sum rho, 1..DIM sum rho u_hat, DIM+1 sum rho E,
//   DIM+2 sum (rho E + kappa |grad rho|^2 / 2), DIM+3 min p, DIM+4 max |v_i| dt
// ---------------------------------------------------------------------------

template <int DIM>
__global__ void __launch_bounds__(kMonThreads)
    k_monitor_partials(const DevParams *__restrict__ Pp, const double *__restrict__ macro,
                       const double *__restrict__ side, double *__restrict__ partials)
{
    const DevParams &P = *Pp;
    const Geo geo = make_geo(P);
    const size_t N = P.N;
    const int n = blockIdx.x * kMonThreads + threadIdx.x;
    double v[kMonWords];
    for (int i = 0; i < kMonWords; ++i) v[i] = 0.0;
    v[DIM + 3] = 1e300;  // min p
    v[DIM + 4] = 0.0;    // max |v| dt
    if (n < P.N) {
        const int x = n % P.nx, y = n / P.nx;
        const double r = macro[n];
        const double E = macro[(3 + DIM) * N + n];
        double gx = 0.0, gy = 0.0;
        constexpr int Q = Layout<DIM>::Q;
        for (int q = 0; q < Q; ++q) {
            const int cx = DIM == 2 ? q / 3 - 1 : q - 1;
            const int cy = DIM == 2 ? q % 3 - 1 : 0;
            const double w = DIM == 2 ? kW1[q / 3] * kW1[q % 3] : kW1[q];
            const int nb = map_node<DIM>(geo, x + cx, y + cy);
            const double rq = nb >= 0 ? macro[nb] : P.ghost[-nb - 1].rho;
            gx += w * (double)cx * rq;
            gy += w * (double)cy * rq;
        }
        gx /= kTL;
        gy /= kTL;
        v[0] = r;
        v[1] = r * macro[1 * N + n];
        if (DIM == 2) v[2] = r * macro[2 * N + n];
        v[DIM + 1] = r * E;
        v[DIM + 2] = r * E + 0.5 * P.kappa * (gx * gx + gy * gy);
        v[DIM + 3] = macro[(2 + DIM) * N + n];
        const double s = sqrt(side[kSideTh * N + n]);
        const double ax = fabs(side[kSideUx * N + n]) + s;
        const double ay = DIM == 2 ? fabs(side[kSideUy * N + n]) + s : 0.0;
        v[DIM + 4] = sqrt(ax * ax + ay * ay) * P.dt;
    }
    __shared__ double red[kMonThreads / 64][kMonWords];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    for (int i = 0; i < kMonWords; ++i) {
        double w;
        if (i == DIM + 3)
            w = wave_min(v[i]);
        else if (i == DIM + 4)
            w = wave_max(v[i]);
        else
            w = wave_sum(v[i]);
        if (lane == 0) red[wave][i] = w;
    }
    __syncthreads();
    if (threadIdx.x < kMonWords) {
        const int i = threadIdx.x;
        double acc = red[0][i];
        for (int wv = 1; wv < kMonThreads / 64; ++wv) {
            if (i == DIM + 3)
                acc = fmin(acc, red[wv][i]);
            else if (i == DIM + 4)
                acc = fmax(acc, red[wv][i]);
            else
                acc += red[wv][i];
        }
        partials[(size_t)blockIdx.x * kMonWords + i] = acc;
    }
}

// One block of kMonFinalThreads: thread t combines word t % kMonWords over the partial
// blocks t / kMonWords, t / kMonWords + kMonLanes, ... in that order; the kMonLanes
// results of a word are then combined pairwise in a fixed order, so the sums do not
// depend on timing.  Word dim + 3 is a minimum, word dim + 4 a maximum, the rest sums.
constexpr int kMonFinalThreads = 256;
constexpr int kMonLanes = kMonFinalThreads / kMonWords;
static_assert(kMonFinalThreads % kMonWords == 0, "whole lanes per word");

__global__ void __launch_bounds__(kMonFinalThreads)
    k_monitor_final(const double *__restrict__ partials, int nblocks, int dim, double *__restrict__ out)
{
    __shared__ double s[kMonFinalThreads];
    const int t = threadIdx.x, i = t % kMonWords, j = t / kMonWords;
    const int kind = i == dim + 3 ? 1 : (i == dim + 4 ? 2 : 0);
    auto combine = [kind](double a, double x) { return kind == 1 ? fmin(a, x) : (kind == 2 ? fmax(a, x) : a + x); };
    double acc = kind == 1 ? INFINITY : (kind == 2 ? -INFINITY : 0.0);
    for (int b = j; b < nblocks; b += kMonLanes) acc = combine(acc, partials[(size_t)b * kMonWords + i]);
    s[t] = acc;
    __syncthreads();
    for (int w = kMonLanes / 2; w >= 1; w >>= 1) {
        if (j < w) s[t] = combine(s[t], s[t + w * kMonWords]);
        __syncthreads();
    }
    if (t < kMonWords) out[t] = s[t];
}

int monitor_blocks(const LaunchCtx &c) { return (c.N + kMonThreads - 1) / kMonThreads; }

hipError_t launch_monitor_final(const LaunchCtx &c, const double *partials, int nblocks, double *out)
{
    hipLaunchKernelGGL(k_monitor_final, dim3(1), dim3(kMonFinalThreads), 0, c.st, partials, nblocks, c.dim, out);
    return hipGetLastError();
}

hipError_t launch_monitors(const LaunchCtx &c, const DevState &s, int cur, double *partials,
                           int nblocks, double *out)
{
    if (c.dim == 3) return launch_monitors3(c, s, cur, partials, nblocks, out);
    hipError_t e = launch_macro(c, s, cur, s.aux);
    if (e != hipSuccess) return e;
    if (c.dim == 2)
        hipLaunchKernelGGL(k_monitor_partials<2>, dim3(nblocks), dim3(kMonThreads), 0, c.st,
                           s.params, s.aux, s.side[cur], partials);
    else
        hipLaunchKernelGGL(k_monitor_partials<1>, dim3(nblocks), dim3(kMonThreads), 0, c.st,
                           s.params, s.aux, s.side[cur], partials);
    hipLaunchKernelGGL(k_monitor_final, dim3(1), dim3(kMonFinalThreads), 0, c.st, partials, nblocks, c.dim, out);
    return hipGetLastError();
}

} // namespace pond
