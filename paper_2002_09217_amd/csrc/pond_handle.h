// pond_handle.h -- the library-side definition of a lattice handle, shared by the
// C-ABI layer (pond_api.hip) and the batch scheduler (pond_batch.hip).  Not part of
// the public ABI.
#pragma once

#include <hip/hip_runtime.h>

#include "pond.h"
#include "pond_internal.h"

struct pond_handle {
    pond_config cfg;
    pond::LaunchCtx lc;
    pond::DevState ds;
    hipStream_t stream = nullptr;       // where work runs (caller's or owned)
    bool own_stream = false;
    hipStream_t capture_stream = nullptr; // used only to record graphs; created on first use
    // [0]: the short run, [1]: the long run of steps (two-kernel step: 2 and 2 kRunPairs
    // steps; fused step: kFusedRing and kFusedRun), each starting from state buffer or ring
    // slot s; a run returns to the slot it starts from
    hipGraphExec_t step_exec[2][pond::kFusedRing] = {};
    bool graphs_ok = true;
    bool tuned = false;                 // streaming tile shape fixed
    int cur = 0;                        // state buffer (two-kernel step) or ring slot
                                        // (fused step) holding the current state
    long long steps = 0;
    bool initialised = false;
    bool failed = false;
    double *mon_partials = nullptr;
    double *mon_out = nullptr;
    int *flags_host = nullptr;          // pinned host copy of the flags (read-back)
    int mon_blocks = 0;
    char msg[256] = "ok";
    // step-kernel descriptors of this lattice: [p] reads state p and writes state 1 - p
    // (two-kernel step), or reads ring slot p and writes slot p + 1 (fused step)
    pond::SlotDesc desc_h[pond::kFusedRing];
    pond::SlotDesc *desc_d = nullptr;
    int st_tiles = 0, fc_tiles = 0;    // tiles of the two step kernels
    pond_batch *batch = nullptr;       // batch the handle belongs to, if any
    // state buffers or ring slots the steps cycle through
    int states() const { return lc.fused ? pond::kFusedRing : 2; }
};

namespace pond {
int handle_fail(pond_handle *h, int code, const char *fmt, ...);
int handle_update_desc(pond_handle *h);
int handle_finish_batch(pond_handle *h, const int *flags, int nsteps);
// completed steps of a run of nsteps steps that started on state buffer or ring slot
// `cur` of `states` (2: two-kernel step; kFusedRing: fused step, whose run ends with the
// closure check of its last state), given its flags
int completed_steps(const int *flags, int cur, int states, int nsteps);
// graph lengths of the short and long runs of steps
int run_length(const pond_handle *h, int kind);
// pond_create's checks of a configuration (POND_OK or POND_E_INVALID)
int config_valid(const pond_config *cfg);
// bytes of the population part of one state buffer (the side planes follow it)
size_t state_pop_bytes(int dim, long long N, int fp32);
// device parameter block of a valid configuration (POND_E_INVALID: bad inflow state)
int make_params(const pond_config &c, DevParams &P);
int err_code(int bits);
const char *err_name(int bits);
} // namespace pond


