// pond_internal.h -- data layout and launcher declarations shared by the HIP
// kernels and the C-ABI layer of libpond.  Not part of the public ABI.
#pragma once

#include <hip/hip_runtime.h>

namespace pond {

// Steps are replayed from captured HIP graphs: runs of 2 kRunPairs steps, and pairs
// for what is left.  Every graph has an even step count, so it ends on the buffer
// parity it starts from.  A graph launch costs a few microseconds more than a kernel
// boundary inside a graph, which longer runs amortise.
constexpr int kRunPairs = 8;
enum { kPeriodic = 0, kOutflow = 1, kInflow = 2 };

// error bits written by the kernels into flags[0]; kErrCollideStage marks an error of
// the closure that precedes a state's collision (fused step and its check), which makes
// that state, not the next one, the first bad one
enum { kErrPressure = 1, kErrNonfinite = 2, kErrHalo = 4, kErrCollideStage = 8 };

// The fused step keeps the streamed states of three consecutive steps (a ring), so that
// after an error found in the closure of a state the state before it is still intact.
// Its graphs replay runs of kFusedRun and of kFusedRing steps, which return to the ring
// slot they start from.
constexpr int kFusedRing = 3;
constexpr int kFusedRun = 45;

// Inflow ghost state of one face: the equilibrium of (rho, u, T) with F = 0, as
// populations in its own gauge plus the scalar fields the gradient stencils read.
struct GhostFace {
    double f[9], g[9];     // populations, same index convention as the lattice
    double ux, uy, theta;  // gauge
    double rho, T, h, mu, kc;
};

// Per-lattice parameters, resident in device memory and read through a pointer.
struct DevParams {
    int dim, nx, ny, N;    // N = nx * ny * nz nodes, index = x + nx * (y + ny * z)
    int bc[2][2];
    int n_pass, nz;
    double a, b, R, delta, omega, kappa, k_scale, dt;
    double Cv, Cp_ig;      // R/delta and R(1 + delta)/delta
    double inv_Cv;         // delta/R: T = (e + a rho) / C_v as a product
    int eos, isothermal;   // pond_config: equation of state, T = T0 switch
    double T0, eos_c[4];
    GhostFace ghost[4];    // face 2 axis + side
};

// ---------------------------------------------------------------------------
// Plane layout (structure of arrays, one plane of N values per entry).
//   state:  f[Q], g[Q]       populations, PopT (double or float), node's own gauge;
//                            with float: deviations f_q - W_q sum_f, g_q - W_q sum_g,
//                            followed by the two sum planes in double
//           side[5]          u_x, u_y, theta (gauge), F_x, F_y  (double)
//   mom:    the streamed state after the predictor-corrector, gauge free:
//           rho, u_x, u_y, then the central moments about u of f (those not fixed
//           by rho and u) and of g.  2D: 3 + 6 + 9 = 18 planes; 1D: 2 + 1 + 3 = 6.
//   kor:    Korteweg stress K_xx, K_xy, K_yy (initial state only)
//   aux:    staging of the initial fields and of the macroscopic read-back
// ---------------------------------------------------------------------------
template <int DIM> struct Layout;
template <> struct Layout<2> {
    static constexpr int Q = 9, NF = 9;
    static constexpr int kRho = 0, kUx = 1, kUy = 2, kF = 3, kG = 9, kMomPlanes = 18;
    // central f moments stored: (m,n) = (1,1), (2,0), (0,2), (2,1), (1,2), (2,2)
    static constexpr int kFStored = 6;
};
template <> struct Layout<1> {
    static constexpr int Q = 3, NF = 3;
    static constexpr int kRho = 0, kUx = 1, kUy = 1, kF = 2, kG = 3, kMomPlanes = 6;
    static constexpr int kFStored = 1; // m = 2
};
// D3Q27 (periodic box): moment index 9 m + 3 n + o for sum_i f_i wx^m wy^n wz^o; the f
// moments stored are the 23 that rho and u do not fix (all but 000, 100, 010, 001)
template <> struct Layout<3> {
    static constexpr int Q = 27, NF = 27;
    static constexpr int kRho = 0, kUx = 1, kUy = 2, kUz = 3, kF = 4, kG = 27, kMomPlanes = 54;
    static constexpr int kFStored = 23;
};
// side planes: 5 in 1D/2D, 7 in 3D (u_z and F_z appended)
enum { kSideUx = 0, kSideUy = 1, kSideTh = 2, kSideFx = 3, kSideFy = 4, kSidePlanes = 5,
       kSideUz = 5, kSideFz = 6, kSidePlanes3 = 7 };
enum { kAuxPlanes = 7, kAuxPlanes3 = 9 };
enum { kKorPlanes = 3, kKorPlanes3 = 6 };
inline int side_planes(int dim) { return dim == 3 ? kSidePlanes3 : kSidePlanes; }
inline int mom_planes(int dim) { return dim == 3 ? Layout<3>::kMomPlanes : dim == 2 ? Layout<2>::kMomPlanes : Layout<1>::kMomPlanes; }
inline int aux_planes(int dim) { return dim == 3 ? kAuxPlanes3 : kAuxPlanes; }
inline int kor_planes(int dim) { return dim == 3 ? kKorPlanes3 : kKorPlanes; }

// flags[0]: error bits.  flags[1]: streaming launches of the current batch of steps
// whose first tile found no error (the failing step itself may or may not count: its
// first tile can run before or after another tile raises the error).  flags[2]: 1 +
// the parity of the state buffer read by the step that raised the first error, which
// settles that ambiguity (the state it read is the last complete one).
enum { kFlagErr = 0, kFlagSteps = 1, kFlagErrParity = 2, kFlagWords = 4 };

// One lattice of a launch of the step kernels: where the step reads and writes and
// which workgroups of the launch are its tiles.  A single lattice is a launch of one
// slot; a batch launches the tiles of all its lattices together.
struct SlotDesc {
    const DevParams *P;
    const void *pop_src;     // state read by the streaming kernel
    const double *side_src;
    void *pop_dst;           // state written by the collision kernel
    double *side_dst;
    double *mom;             // streamed-state scratch of this lattice
    int *flags;              // error bits and step counter of this lattice
    int st_tiles_x, st_begin, st_count; // streaming-kernel tiles: per row, first, number
    int fc_tiles_x, fc_begin, fc_count; // collision-kernel tiles
    int parity;              // index of the state buffer pop_src belongs to (0 or 1)
    // 3D only: donor moments, Korteweg stress and thermodynamic scratch
    void *dmom;
    double *kor, *aux;
    // fused step: streamed state read (the collision recomputed on the fly) and written;
    // `parity` is then the ring slot of smom_src
    const void *smom_src;
    void *smom_dst;
};

// device buffers of one lattice
struct DevState {
    void *pop[2];       // 2 Q planes each: f then g
    double *side[2];    // kSidePlanes planes each
    double *mom;        // kMomPlanes planes
    double *kor;        // kKorPlanes planes
    double *aux;        // kAuxPlanes planes
    int *flags;         // kFlagWords ints
    DevParams *params;  // device copy
    void *dmom;         // 3D: donor moments, 54 planes (float with FP32 streaming)
    // fused step: the streamed states of three consecutive steps; pop[0] and side[0]
    // then receive the collided state for read-back (pop[1], side[1] and mom unused)
    void *ring[kFusedRing];
};

// ---------------------------------------------------------------------------
// launchers (pond_kernels.hip); all enqueue on `st` and return hipError_t
// ---------------------------------------------------------------------------
struct LaunchCtx {
    int dim, nx, ny, N;
    int fp32;           // 0: FP64; 1: populations stored as float, streamed in float;
                        // 2: stored as float, all arithmetic in double
    hipStream_t st;
    int stream_tile;    // tile-shape variant of the streaming kernel
    // when set, the step kernels are launched with these start/stop events, which the
    // runtime records at the kernel's own start and end (measurement only)
    hipEvent_t ev_start = nullptr, ev_stop = nullptr;
    int nz = 1;
    // streaming kernels with the general equation of state (isothermal runs or a
    // non-van-der-Waals pressure); false: the van der Waals fluid with its energy
    bool gen_eos = false;
    // fused step (one kernel per step, the state between steps is the streamed moment
    // planes, mixed FP64/FP32 in the FP32 storage precisions); false: two kernels per
    // step with stored populations
    bool fused = false;
};

int stream_variants(int dim);
void stream_tile_shape(int dim, int variant, int *tx, int *ty);

hipError_t launch_reset_flags(const LaunchCtx &c, int *flags);
// clear the flags of every slot of a device descriptor array / copy them into `out`
// (kFlagWords ints per slot, in slot order)
hipError_t launch_reset_slot_flags(hipStream_t st, const SlotDesc *slots, int nslots);
hipError_t launch_gather_slot_flags(hipStream_t st, const SlotDesc *slots, int nslots, int *out);
// step kernels over the tiles of `nslots` lattices (device descriptor array); every
// lattice must share dim and precision with c; `tiles` is the total tile count
hipError_t launch_stream(const LaunchCtx &c, const SlotDesc *slots, int nslots, int tiles);
// closure and collision of the moment planes `mom` into pop_dst/side_dst (the second
// kernel of the two-kernel step; for a fused-step lattice, the read-back of its state)
hipError_t launch_force_collide(const LaunchCtx &c, const SlotDesc *slots, int nslots, int tiles);
// fused step: collision of smom_src recomputed on each tile and its halo, then the
// streaming into smom_dst; `tiles` as for launch_stream
hipError_t launch_step_fused(const LaunchCtx &c, const SlotDesc *slots, int nslots, int tiles);
// the same for the FP64 windows (FP64 and FP32 storage with FP64 arithmetic)
hipError_t launch_step_double_windows(const LaunchCtx &c, const SlotDesc *slots, int nslots, int tiles);
// fused step: closure of the state in `mom` (every node), raising its errors with
// kErrCollideStage and counting as a launch; `tiles` as for launch_force_collide
hipError_t launch_collide_check(const LaunchCtx &c, const SlotDesc *slots, int nslots, int tiles);
// tile counts of one lattice for the current tile shapes
void tile_counts(const LaunchCtx &c, int *st_tiles_x, int *st_count, int *fc_tiles_x, int *fc_count);
hipError_t launch_korteweg(const LaunchCtx &c, const DevState &s, const double *rho);
// the streamed-state planes of the equilibrium of (rho, u_hat, T) into `mom` (FP64, or
// mixed for a fused-step lattice in an FP32 storage precision)
hipError_t launch_init_equilibrium(const LaunchCtx &c, const DevState &s, const double *rho,
                                   const double *u, const double *T, void *mom);
hipError_t launch_macro(const LaunchCtx &c, const DevState &s, int cur, double *out);
hipError_t launch_monitors(const LaunchCtx &c, const DevState &s, int cur, double *partials,
                           int nblocks, double *out);
int monitor_blocks(const LaunchCtx &c);
hipError_t launch_monitor_final(const LaunchCtx &c, const double *partials, int nblocks, double *out);

// D3Q27 (pond_kernels3.hip), one lattice per launch, descriptor in device memory:
// streaming = passes over the donor moments; collision = Korteweg stress +
// thermodynamics + collision (which also writes the next state's donor moments).  With
// start/stop events set, each group is bracketed by them.
hipError_t launch_stream3(const LaunchCtx &c, const SlotDesc *slot);
hipError_t launch_collide3(const LaunchCtx &c, const SlotDesc *slot);
// the donor moments of the state in pop_src/side_src (the collision writes them for the
// state it stores; this recomputes them after the populations were set otherwise)
hipError_t launch_donor_moments3(const LaunchCtx &c, const SlotDesc *slot);
// initial state from rho, u_hat (3 planes), T staged in aux planes 0-4: streamed-state
// planes of the equilibrium (then launch_collide3 stores the collided populations)
hipError_t launch_init3(const LaunchCtx &c, const DevState &s, const SlotDesc *slot);
hipError_t launch_macro3(const LaunchCtx &c, const DevState &s, int cur, double *out);
hipError_t launch_monitors3(const LaunchCtx &c, const DevState &s, int cur, double *partials, int nblocks,
                            double *out);
void stream3_tile(int fp32, int *tx, int *ty);

} // namespace pond
