// pond_stream.h -- the predictor-corrector passes of the semi-Lagrangian streaming
// (eqs. 1-4, App. C-D) and the store of the streamed state, shared by the two-kernel
// streaming kernel (k_stream) and the fused step kernel (k_step).  The moment fields of
// a tile and its 2-node halo sit in LDS as written by the kernels' fill stages: field
// (m, n) of set s at window node li at index ((3 m + n) LN + li) 2 + s.
#pragma once

#include "pond_collide.h"
#include "pond_device.h"

namespace pond {

// The 2D window of one FP64 set without its zero taps: acc[3k+l] += sum_n B_ln sum_r
// wy_l[r] sum_m A_km sum_c wx_k[c] M_mn[r][c], for a wave in which every lane's departure
// stencils of k = 0 and l = 0 start at window column/row 1 and those of k = 2 and l = 2
// end at column/row 3 (the usual case: |u| < sqrt(theta)).  Same group order, one-ahead
// LDS reads and row accumulation as the general window in k_stream.
template <int LN, int LX>
__device__ __forceinline__ void window2_no_zero_taps(const double *sbase, const double (&wx)[3][5],
                                                     const double (&wy)[3][5], const double (&A)[3][3],
                                                     const double (&Bd)[3][3], double (&acc)[9])
{
    constexpr int CS = 2;
#pragma unroll
    for (int n = 0; n < 3; ++n) {
        auto load_group = [&](int g, double v[5]) {
            const double *row = sbase + ((3 * (g % 3) + n) * LN + (g / 3) * LX) * CS;
#pragma unroll
            for (int c = 0; c < 5; ++c) v[c] = row[c * CS];
        };
        double Z[3], cur[5], nxt[5];
        load_group(0, cur);
#pragma unroll
        for (int g = 0; g < 15; ++g) {
            const int r = g / 3, m = g % 3;
            if (g + 1 < 15) load_group(g + 1, nxt);
            const double x0 = wx[0][1] * cur[1] + wx[0][2] * cur[2] + wx[0][3] * cur[3] + wx[0][4] * cur[4];
            const double x1 =
                wx[1][0] * cur[0] + wx[1][1] * cur[1] + wx[1][2] * cur[2] + wx[1][3] * cur[3] + wx[1][4] * cur[4];
            const double x2 = wx[2][0] * cur[0] + wx[2][1] * cur[1] + wx[2][2] * cur[2] + wx[2][3] * cur[3];
            Z[0] = m == 0 ? A[0][0] * x0 : Z[0] + A[0][m] * x0;
            Z[1] = m == 0 ? A[1][0] * x1 : Z[1] + A[1][m] * x1;
            Z[2] = m == 0 ? A[2][0] * x2 : Z[2] + A[2][m] * x2;
            if (m == 2) {
#pragma unroll
                for (int l = 0; l < 3; ++l) {
                    if ((l == 0 && r == 0) || (l == 2 && r == 4)) continue;
                    const double C = Bd[l][n] * wy[l][r];
#pragma unroll
                    for (int k = 0; k < 3; ++k) acc[3 * k + l] += C * Z[k];
                }
            }
#pragma unroll
            for (int c = 0; c < 5; ++c) cur[c] = nxt[c];
        }
        __builtin_amdgcn_sched_barrier(0);
    }
}

// The passes of one receiver lane (lane 2 i + set of receiver i): interpolate this set's
// moment fields at the departure points of the receiver's gauge (Ux, Uy, th), contract
// them into populations in that gauge, take the moments with the partner lane and close
// them through the EoS for the next gauge, n_pass times.  FP32 windows (LdsT = float) hold
// deviations from the tile's reference moment vector R (1, v, v, v^2) (refR0, refR1 and
// refT = v, the per-axis second moment theta T_L of the centre's gauge).  On return pq holds this set's populations in the gauge (sUx, sUy, sS)
// of the last pass, and (Ux, Uy, th) the gauge it produced; returns the error bits.
template <int DIM, typename LdsT, int LN, int LX, int NT, bool GEN>
__device__ __forceinline__ int stream_passes(const POND_GLOBAL DevParams &P, const LdsT *sbase, int tid, int myset, double rx, double ry,
                                             double refR0, double refR1, double refT, double &Ux, double &Uy,
                                             double &th, double Fpx, double Fpy, double (&pq)[Layout<DIM>::Q],
                                             double &rho, double &sUx, double &sUy, double &sS)
{
    constexpr int Q = Layout<DIM>::Q;
    constexpr int CS = 2; // column stride of the LDS fields
    constexpr bool kDevI = sizeof(LdsT) == 4;
    const double dt = P.dt;
    int err = 0;
    // When the grid is one workgroup per CU (512 lanes, two waves per SIMD), the SIMD
    // issues for the older wave first, the younger one falls behind and finishes its
    // last pass alone, with nothing to hide its latencies.  Favouring the younger wave
    // in the first pass lets both finish at about the same time.
    const int young = __builtin_amdgcn_readfirstlane((tid >> 6) >= NT / 128 && NT == 512 && gridDim.x <= kCUs ? 1 : 0);
    for (int pass = 0; pass < P.n_pass; ++pass) {
        if (pass == 0 && young) __builtin_amdgcn_s_setprio(1);
        else __builtin_amdgcn_s_setprio(0);
        const double s = sqrt(th);
        LdsT wx[3][5], wy[3][5];
        err |= window_weights<LdsT>(Ux, s, dt, wx);
        if (DIM == 2) err |= window_weights<LdsT>(Uy, s, dt, wy);
        double Ad[3][3], Bd[3][3];
        lagrange_coeffs(Ux - rx, s, Ad);
        if (DIM == 2) lagrange_coeffs(Uy - ry, s, Bd);
        LdsT A[3][3];
#pragma unroll
        for (int k = 0; k < 3; ++k)
#pragma unroll
            for (int m = 0; m < 3; ++m) A[k][m] = (LdsT)Ad[k][m];

        // populations of this set in the receiver gauge, one per direction:
        //   f_kl = sum_n B_ln sum_r wy_l[r] sum_m A_km sum_c wx_k[c] M_mn[r][c]
        double acc[Q];
        if constexpr (kDevI) {
            // the reference part (see the fill); the window adds the deviations
            const double R = myset == 0 ? refR0 : refR1;
#pragma unroll
            for (int k = 0; k < 3; ++k) {
                const double ak = R * (Ad[k][0] + refT * Ad[k][2]);
                if (DIM == 2) {
#pragma unroll
                    for (int l = 0; l < 3; ++l) acc[3 * k + l] = ak * (Bd[l][0] + refT * Bd[l][2]);
                } else {
                    acc[k] = ak;
                }
            }
        } else {
#pragma unroll
            for (int q = 0; q < Q; ++q) acc[q] = 0.0;
        }
        // FP64 windows in eight-wave workgroups (two waves per SIMD, registers to spare)
        // also carry the variant without zero taps, taken by every wave that can
        bool no_zero_taps = false;
        if constexpr (DIM == 2 && NT == 512 && sizeof(LdsT) == 8) {
            if (__all(wx[0][0] == 0.0 && wx[2][4] == 0.0 && wy[0][0] == 0.0 && wy[2][4] == 0.0)) {
                window2_no_zero_taps<LN, LX>(sbase, wx, wy, A, Bd, acc);
                no_zero_taps = true;
            }
        }
        if (DIM == 2 && !no_zero_taps) {
#pragma unroll
            for (int n = 0; n < 3; ++n) {
                // Row r of field (m, n) is group g = 3 r + m of five window values; each
                // group is read from LDS one group ahead of its use, so that the read
                // latency overlaps the arithmetic of the group before.
                auto load_group = [&](int g, LdsT v[5]) {
                    const LdsT *row = sbase + ((3 * (g % 3) + n) * LN + (g / 3) * LX) * CS;
#pragma unroll
                    for (int c = 0; c < 5; ++c) v[c] = row[c * CS];
                };
                // FP64 windows add each row straight into acc with the weights
                // B_ln wy_l[r] (no I registers); FP32 windows sum the rows in FP32 first
                constexpr bool kRowsToAcc = sizeof(LdsT) == 8;
                LdsT I[3][3]; // sum_r wy_l[r] Z_k[r]
                LdsT Z[3];    // sum_m A_km (x-interpolated M_mn) of the current row
                LdsT cur[5], nxt[5];
                load_group(0, cur);
#pragma unroll
                for (int g = 0; g < 15; ++g) {
                    const int r = g / 3, m = g % 3;
                    if (g + 1 < 15) load_group(g + 1, nxt);
#pragma unroll
                    for (int k = 0; k < 3; ++k) {
                        const LdsT xk = wx[k][0] * cur[0] + wx[k][1] * cur[1] + wx[k][2] * cur[2] +
                                        wx[k][3] * cur[3] + wx[k][4] * cur[4];
                        Z[k] = m == 0 ? A[k][m] * xk : Z[k] + A[k][m] * xk;
                    }
                    if (m == 2 && kRowsToAcc) {
                        double C[3];
#pragma unroll
                        for (int l = 0; l < 3; ++l) C[l] = Bd[l][n] * (double)wy[l][r];
#pragma unroll
                        for (int k = 0; k < 3; ++k)
#pragma unroll
                            for (int l = 0; l < 3; ++l) acc[3 * k + l] += C[l] * (double)Z[k];
                    } else if (m == 2) {
#pragma unroll
                        for (int k = 0; k < 3; ++k)
#pragma unroll
                            for (int l = 0; l < 3; ++l) I[k][l] = r == 0 ? wy[l][r] * Z[k] : I[k][l] + wy[l][r] * Z[k];
                    }
#pragma unroll
                    for (int c = 0; c < 5; ++c) cur[c] = nxt[c];
                }
                if (!kRowsToAcc) {
#pragma unroll
                    for (int k = 0; k < 3; ++k)
#pragma unroll
                        for (int l = 0; l < 3; ++l) acc[3 * k + l] += Bd[l][n] * (double)I[k][l];
                }
                // keep the three n-blocks apart: the scheduler would otherwise hoist the
                // loads of all of them and run out of registers
                __builtin_amdgcn_sched_barrier(0);
            }
        } else if (DIM == 1) {
#pragma unroll
            for (int m = 0; m < 3; ++m) {
                const LdsT *row = sbase + m * LN * CS;
                const LdsT v0 = row[0], v1 = row[CS], v2 = row[2 * CS], v3 = row[3 * CS], v4 = row[4 * CS];
#pragma unroll
                for (int k = 0; k < 3; ++k) {
                    const LdsT xk = wx[k][0] * v0 + wx[k][1] * v1 + wx[k][2] * v2 + wx[k][3] * v3 + wx[k][4] * v4;
                    acc[k] += Ad[k][m] * (double)xk;
                }
            }
        }
#pragma unroll
        for (int q = 0; q < Q; ++q) pq[q] = acc[q];

        // moments of the streamed populations (eq. 2) and the EoS closure: each lane sums
        // its own set; the partner lane supplies the other sums
        double s0 = 0.0, sx = 0.0, sy = 0.0;
#pragma unroll
        for (int q = 0; q < Q; ++q) {
            const double cx = DIM == 2 ? (double)(q / 3 - 1) : (double)(q - 1);
            const double cy = DIM == 2 ? (double)(q % 3 - 1) : 0.0;
            s0 += pq[q];
            sx += pq[q] * (Ux + s * cx);
            if (DIM == 2) sy += pq[q] * (Uy + s * cy);
        }
        const double o0 = __shfl_xor(s0, 1, 64);
        const double ox = __shfl_xor(sx, 1, 64);
        const double oy = DIM == 2 ? __shfl_xor(sy, 1, 64) : 0.0;
        const double r0 = myset == 0 ? s0 : o0;
        const double jx = myset == 0 ? sx : ox;
        const double jy = myset == 0 ? sy : oy;
        const double G2 = myset == 0 ? o0 : s0;
        rho = r0;
        // one reciprocal of rho serves every quotient by it (FP64 division is a
        // long dependent sequence on this hardware); the lean van der Waals closure
        // takes it and 1 / (1 - b rho) from one division
        const double q = 1.0 - P.b * rho;
        const double i_rq = GEN ? 0.0 : 1.0 / (rho * q);
        const double i_rho = GEN ? 1.0 / rho : q * i_rq;
        const double E = 0.5 * G2 * i_rho;
        const double ux = jx * i_rho;
        const double uy = DIM == 2 ? jy * i_rho : 0.0;
        const double uhx = ux + 0.5 * Fpx * dt * i_rho;
        const double uhy = DIM == 2 ? uy + 0.5 * Fpy * dt * i_rho : 0.0;
        const double e = E - 0.5 * (uhx * uhx + uhy * uhy);
        const double T = eos_T_of_e<GEN>(P, rho, e);
        const double p = GEN ? eos_p<GEN>(P, rho, T) : vdw_p_lean(P, rho, T, i_rq);
        err |= eos_bad<GEN>(P, rho, p);
        sUx = Ux;
        sUy = Uy;
        sS = s;
        Ux = ux;
        Uy = uy;
        th = p * i_rho * kInvTL;
    }

    return err;
}

// Store the streamed state of a receiver for the collision, gauge free: rho and u (the f
// lane), and the central moments of the lane's set about u (moment planes of
// pond_internal.h, in FP64 or the mixed FP32 form).
template <int DIM, bool MIXED>
__device__ __forceinline__ void store_streamed(void *mom, size_t N, size_t node, int myset, const double *pq,
                                               double rho, double Ux, double Uy, double sUx, double sUy, double sS)
{
    using L = Layout<DIM>;
    using MIO = MomIO<DIM, MIXED>;
    constexpr int NF = L::NF;
    double mq[NF];
    moments_about<DIM>(pq, sUx - Ux, sUy - Uy, sS, mq);
    if (myset == 0) {
        MIO::store(mom, N, node, L::kRho, rho);
        MIO::store(mom, N, node, L::kUx, Ux);
        if constexpr (DIM == 2) {
            MIO::store(mom, N, node, L::kUy, Uy);
            MIO::store(mom, N, node, (L::kF + 0), mq[4]); // (1,1)
            MIO::store(mom, N, node, (L::kF + 1), mq[6]); // (2,0)
            MIO::store(mom, N, node, (L::kF + 2), mq[2]); // (0,2)
            MIO::store(mom, N, node, (L::kF + 3), mq[7]); // (2,1)
            MIO::store(mom, N, node, (L::kF + 4), mq[5]); // (1,2)
            MIO::store(mom, N, node, (L::kF + 5), mq[8]); // (2,2)
        } else {
            MIO::store(mom, N, node, L::kF, mq[2]);
        }
    } else {
#pragma unroll
        for (int i = 0; i < NF; ++i) MIO::store(mom, N, node, (L::kG + i), mq[i]);
    }
}

} // namespace pond
