"""Algorithmic cost model of one time step (per lattice node), used to express measured
throughput against the MI355X rooflines.

Bytes (compulsory HBM traffic; neighbour reuse through LDS or caches is not counted).
The fused step is one kernel: it reads the streamed-state moment planes of the previous
step (rho, u and the central moments: 18 planes in 2D, 6 in 1D), recomputes the collision
of each tile and its halo on chip, streams, and writes the next streamed state
(fused_step_bytes_per_node: 288 B in FP64 D2Q9, 176 B with the FP32 moment planes).
The two-kernel step stores the collided state in between:
  streaming  reads one state (2 Q populations and the five side fields: gauge u_x, u_y,
             theta and the force F_x, F_y) and writes the moment planes;
  collision  reads those moment planes and writes the next state.
bytes_per_node_step is that two-kernel traffic (656 B in FP64 D2Q9, 544 B with FP32
population storage).  fused_bytes_per_node_step is the floor of a step that kept the
collided populations with their side fields on chip, i.e. one such state read and one
written (368 B and 256 B).

FLOPs of the streaming kernel (the dominant one), per receiver and pass, for the
moment-first reconstruction: every set (f, g) has NF moment fields; each field is
interpolated at the departure points of all Q directions with separable cubic weights
(x: 3 departure abscissae x 5 window rows x 4 taps; y: Q directions x 4 taps) and
contracted into the Q populations (one multiply and one FMA each).  A FMA counts as
two flops.  The weights, Lagrange coefficients, moments and EoS of a pass, the donor
moments of the tile and the output moments are added as fixed terms.
"""
from __future__ import annotations

# MI355X (gfx950) peaks
HBM_PEAK_GBS = 8000.0
# 256 CUs x 4 SIMD x 16 lanes x 2 flop (FMA) x 2.4 GHz; FP64 vector and non-packed FP32
VALU_PEAK_TFLOPS = 256 * 4 * 16 * 2 * 2.4e9 / 1e12


def state_bytes_per_node(dim: int, fp32_store: bool) -> int:
    """One state of a node: 2Q populations (FP32 storage: 2Q FP32 deviations and the
    two FP64 set sums) and the five FP64 side fields."""
    q = 9 if dim == 2 else 3
    pops = 2 * q * 4 + 2 * 8 if fp32_store else 2 * q * 8
    return pops + 5 * 8


def moment_bytes_per_node(dim: int) -> int:
    """The streamed-state moment planes the streaming kernel hands to the collision
    kernel (FP64): rho, u and the central moments, 18 planes in 2D and 6 in 1D."""
    return (18 if dim == 2 else 6) * 8


def bytes_per_node_step(dim: int, fp32_store: bool) -> int:
    """Compulsory traffic of the two-kernel step as built: each kernel reads and writes
    one state or the moment planes once."""
    return 2 * (state_bytes_per_node(dim, fp32_store) + moment_bytes_per_node(dim))


def fused_bytes_per_node_step(dim: int, fp32_store: bool) -> int:
    """Floor of a step whose streamed state never leaves the chip: one state read, one
    written."""
    return 2 * state_bytes_per_node(dim, fp32_store)


def stream_bytes_per_node(dim: int, fp32_store: bool) -> int:
    """Compulsory HBM bytes of the streaming kernel alone per receiver: it reads the
    populations and the five side fields and writes the streamed-state moment planes."""
    return state_bytes_per_node(dim, fp32_store) + moment_bytes_per_node(dim)


def collide_bytes_per_node(dim: int, fp32_store: bool) -> int:
    """Compulsory HBM bytes of the collision kernel per node: the moment planes in, the
    next state out (the halo re-reads of its stencils are not counted)."""
    return moment_bytes_per_node(dim) + state_bytes_per_node(dim, fp32_store)


def fused_state_bytes_per_node(dim: int, fp32_store: bool) -> int:
    """One state of the fused step: the streamed moment planes (FP64, or in the FP32
    storage precisions rho, u and 2 rho E in FP64 and the other moments in FP32)."""
    planes = 18 if dim == 2 else 6
    dbl = dim + 2 if fp32_store else planes
    return dbl * 8 + (planes - dbl) * 4


def fused_step_bytes_per_node(dim: int, fp32_store: bool) -> int:
    """Compulsory traffic of the fused step as built: one state read, one written (288 B in
    FP64 D2Q9, 176 B in the FP32 storage precisions); halo re-reads are not counted."""
    return 2 * fused_state_bytes_per_node(dim, fp32_store)


def collide_flops_per_node(dim: int) -> int:
    """Closure and collision of one node in moment space, as the fused step computes it
    (my count, FMA = 2 flops).  2D: Korteweg stress and its divergence (~90),
    thermodynamic state (~30), the heat-flux correction M0 (~100), f collision on its
    nine central moments with the force source (~80), g collision: the force-extended
    equilibrium and source polynomials (~130) and their nine moments (~190), and both
    sets shifted to the tile velocity (~55).  1D: the same terms on three moments."""
    return 680 if dim == 2 else 230


def stream_flops_per_node(dim: int, n_pass: int) -> int:
    if dim == 3:
        # per z-window plane and z power: the D2Q9 x-y contraction of 9 fields (972 FMA
        # with the zero taps) and 27 FMA of the z contraction; 5 planes x 3 powers per set
        per_set_pass = 5 * 3 * (972 + 27)
        fixed_pass = 3 * 16 + 3 * 20 + 81 + 20           # weights, Lagrange coeffs, moments, EoS
        return n_pass * (2 * per_set_pass * 2 + 2 * fixed_pass) + 2 * 250 + 2 * 250
    if dim == 2:
        per_field = 2 * (3 * 5 * 4 + 9 * 4 + 9) + 9   # 2 x 105 FMA + 9 MUL = 219
        fields = 18
        fixed_pass = 6 * 16 + 2 * 20 + 54 + 20         # weights, Lagrange coeffs, moments, EoS
        donor = 340                                     # tile moments incl. the 2-node halo
        out = 200                                       # central moments of the result
    else:
        per_field = 2 * (3 * 4 + 3) + 3
        fields = 6
        fixed_pass = 3 * 16 + 20 + 18 + 20
        donor = 60
        out = 60
    return n_pass * (fields * per_field + fixed_pass) + donor + out
