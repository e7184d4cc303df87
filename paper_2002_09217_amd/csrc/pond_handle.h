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
    // [0]: two steps, [1]: 2 kRunPairs steps; each starting from state 0 / 1
    hipGraphExec_t step_exec[2][2] = {{nullptr, nullptr}, {nullptr, nullptr}};
    bool graphs_ok = true;
    bool tuned = false;                 // streaming tile shape fixed
    int cur = 0;                        // state buffer holding the current state
    long long steps = 0;
    bool initialised = false;
    bool failed = false;
    double *mon_partials = nullptr;
    double *mon_out = nullptr;
    int mon_blocks = 0;
    char msg[256] = "ok";
    // step-kernel descriptors of this lattice: [p] reads state p and writes state 1 - p
    pond::SlotDesc desc_h[2];
    pond::SlotDesc *desc_d = nullptr;
    int st_tiles = 0, fc_tiles = 0;    // tiles of the two step kernels
    pond_batch *batch = nullptr;       // batch the handle belongs to, if any
};

namespace pond {
int handle_fail(pond_handle *h, int code, const char *fmt, ...);
int handle_update_desc(pond_handle *h);
int handle_finish_batch(pond_handle *h, const int *flags);
// completed steps of a run of steps that started on state buffer `cur`, given its flags
int completed_steps(const int *flags, int cur);
// pond_create's checks of a configuration (POND_OK or POND_E_INVALID)
int config_valid(const pond_config *cfg);
// bytes of the population part of one state buffer (the side planes follow it)
size_t state_pop_bytes(int dim, long long N, int fp32);
// device parameter block of a valid configuration (POND_E_INVALID: bad inflow state)
int make_params(const pond_config &c, DevParams &P);
int err_code(int bits);
const char *err_name(int bits);
} // namespace pond


