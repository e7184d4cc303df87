// pond_noalloc.hip -- pond_step_noalloc (include/pond.h): time steps of a 1D or 2D
// lattice whose two state buffers belong to the caller, for callers that cannot
// allocate device memory.  Everything else a step needs (parameter block, step
// descriptors, error flags, the streamed-state moment planes) lives in one static
// device array of fixed size, `scratch`; the step kernels are those of pond_step.
#include <hip/hip_runtime.h>

#include <cstring>
#include <mutex>

#include "pond.h"
#include "pond_handle.h"
#include "pond_internal.h"

using namespace pond;

namespace {

// Layout of the scratch array (byte offsets): parameter block, the two step
// descriptors (descriptor p reads buffer p and writes buffer 1 - p), the error flags,
// then the moment planes from kMomOffset on.
constexpr size_t kParamsOffset = 0;
constexpr size_t kDescOffset = 2048;
constexpr size_t kFlagsOffset = 3072;
constexpr size_t kMomOffset = 4096;
constexpr size_t kScratchBytes = POND_NOALLOC_SCRATCH_BYTES;
static_assert(sizeof(DevParams) <= kDescOffset - kParamsOffset, "parameter block overlaps the descriptors");
static_assert(2 * sizeof(SlotDesc) <= kFlagsOffset - kDescOffset, "descriptors overlap the flags");
static_assert(sizeof(int) * kFlagWords <= kMomOffset - kFlagsOffset, "flags overlap the moment planes");
static_assert(kScratchBytes > kMomOffset, "scratch too small");

// One copy per device that loads the library, held until the process ends.  In host
// code this name is not a device address: the entry point uses the address that
// hipGetSymbolAddress returns for the current device.
static __device__ __align__(256) unsigned char scratch[kScratchBytes];

constexpr int kMaxDevices = 64;
std::once_flag g_once[kMaxDevices];
unsigned char *g_scratch[kMaxDevices];
hipError_t g_status[kMaxDevices];

// device address of `scratch` on device `dev` (which must be current), looked up once
hipError_t scratch_address(int dev, unsigned char **out)
{
    std::call_once(g_once[dev], [dev] {
        void *p = nullptr;
        g_status[dev] = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        g_scratch[dev] = g_status[dev] == hipSuccess ? (unsigned char *)p : nullptr;
    });
    *out = g_scratch[dev];
    return g_status[dev];
}

// Write the parameter block and both descriptors into the scratch and clear the flags.
// By value: the call then records no host-to-device copy.
__global__ void k_noalloc_setup(DevParams P, SlotDesc d0, SlotDesc d1, unsigned char *base)
{
    if (threadIdx.x == 0) {
        *(DevParams *)(base + kParamsOffset) = P;
        SlotDesc *d = (SlotDesc *)(base + kDescOffset);
        d[0] = d0;
        d[1] = d1;
    }
    if (threadIdx.x < kFlagWords) ((int *)(base + kFlagsOffset))[threadIdx.x] = 0;
}

} // namespace

extern "C" int pond_step_noalloc(const pond_config *cfg, void *state0, void *state1, int *cur, int nsteps,
                                 int *done)
{
    if (done) *done = 0;
    if (config_valid(cfg) != POND_OK || !state0 || !state1 || !cur || (*cur != 0 && *cur != 1) || nsteps < 0)
        return POND_E_INVALID;
    const pond_config &c = *cfg;
    if (c.dim == 3 || !c.two_kernel) return POND_E_INVALID; // the two-kernel step on stored populations
    const int nx = c.n[0], ny = c.dim == 2 ? c.n[1] : 1;
    const long long N = (long long)nx * ny;
    const size_t need = kMomOffset + (size_t)N * mom_planes(c.dim) * sizeof(double);
    if (need > kScratchBytes) return POND_E_SCRATCH;
    DevParams P;
    if (make_params(c, P) != POND_OK) return POND_E_INVALID;
    if (nsteps == 0) return POND_OK;

    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kMaxDevices) return POND_E_DEVICE;
    unsigned char *base = nullptr;
    if (scratch_address(dev, &base) != hipSuccess || !base) return POND_E_DEVICE;

    LaunchCtx lc{c.dim, nx, ny, (int)N, c.precision == POND_FP64 ? 0 : (c.precision == POND_FP32_STORE ? 1 : 2),
                 (hipStream_t)c.stream, c.tile < 0 ? 0 : c.tile};
    lc.gen_eos = c.eos != POND_EOS_VDW || c.isothermal;
    int stx, stc, fcx, fcc;
    tile_counts(lc, &stx, &stc, &fcx, &fcc);

    // a state buffer: the population planes, then the side planes
    const size_t popb = state_pop_bytes(c.dim, N, lc.fp32);
    void *pop[2] = {state0, state1};
    double *side[2] = {(double *)((char *)state0 + popb), (double *)((char *)state1 + popb)};
    int *flags = (int *)(base + kFlagsOffset);
    SlotDesc d[2];
    for (int p = 0; p < 2; ++p) {
        std::memset(&d[p], 0, sizeof d[p]);
        d[p].P = (const DevParams *)(base + kParamsOffset);
        d[p].pop_src = pop[p];
        d[p].side_src = side[p];
        d[p].pop_dst = pop[1 - p];
        d[p].side_dst = side[1 - p];
        d[p].mom = (double *)(base + kMomOffset);
        d[p].flags = flags;
        d[p].st_tiles_x = stx;
        d[p].st_count = stc;
        d[p].fc_tiles_x = fcx;
        d[p].fc_count = fcc;
        d[p].parity = p;
    }
    const SlotDesc *desc = (const SlotDesc *)(base + kDescOffset);
    hipLaunchKernelGGL(k_noalloc_setup, dim3(1), dim3(64), 0, lc.st, P, d[0], d[1], base);
    if (hipGetLastError() != hipSuccess) return POND_E_DEVICE;
    int parity = *cur;
    for (int k = 0; k < nsteps; ++k) {
        if (launch_stream(lc, desc + parity, 1, stc) != hipSuccess ||
            launch_force_collide(lc, desc + parity, 1, fcc) != hipSuccess)
            return POND_E_DEVICE;
        parity = 1 - parity;
    }
    int fl[kFlagWords];
    if (hipMemcpyAsync(fl, flags, sizeof fl, hipMemcpyDeviceToHost, lc.st) != hipSuccess ||
        hipStreamSynchronize(lc.st) != hipSuccess)
        return POND_E_DEVICE;
    const int n = completed_steps(fl, *cur, 2, nsteps);
    *cur = (*cur + n) % 2;
    if (done) *done = n;
    return fl[kFlagErr] ? err_code(fl[kFlagErr]) : POND_OK;
}
