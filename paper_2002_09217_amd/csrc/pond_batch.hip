// pond_batch.hip -- batches of independent lattices advanced together (C ABI in
// include/pond.h).  Scheduling only: every member keeps its own state, parameters,
// error flags and step counter, and each step kernel reads a member's descriptor
// exactly as it does for a lattice stepped alone, so results are bitwise identical.
//
// Members that share (dim, precision, tile shape, equation-of-state variant) form a
// group; a batch step is one launch of each step kernel per group over the
// concatenated tiles of its members.  The members of a batch share the form of the step (fused, or two
// kernels), which fixes the number of state buffers or ring slots R (3 or 2) they cycle
// through.  R descriptor arrays per batch: array a holds, for every member, the
// descriptor reading the state a steps after the one current when the arrays were built;
// steps cycle through them, so runs of a multiple of R steps replay one captured HIP
// graph.  A run of fused steps ends with the closure check of every member's last state.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <climits>
#include <cstring>
#include <new>
#include <vector>

#include "pond.h"
#include "pond_handle.h"
#include "pond_internal.h"

using namespace pond;

namespace {

// largest tile count of one launch: keeps blocks x threads per block below 2^31
constexpr long long kMaxLaunchTiles = 1LL << 21;

struct Group {
    int dim, fp32, tile;
    bool gen_eos;            // streaming kernels with the general equation of state
    int first, count;        // slot range in the descriptor arrays
    int st_tiles, fc_tiles;  // total tiles of the two step kernels
};

} // namespace

struct pond_batch {
    hipStream_t stream = nullptr;
    bool own_stream = false;
    hipStream_t capture_stream = nullptr;
    std::vector<pond_handle *> members;  // order of addition
    // built from the members on demand
    bool dirty = true;
    std::vector<Group> groups;
    std::vector<int> slot_of;            // member index -> slot
    std::vector<SlotDesc> desc_h;        // [2][slots]
    SlotDesc *desc_d = nullptr;
    int *flags_d = nullptr;
    std::vector<int> flags_h;
    int cap = 0;                         // slots the device arrays hold
    int phase = 0;                       // descriptor array reading the current states
    bool fused = false;                  // form of the step of every member
    // [0]: the short run, [1]: the long run of steps (run_length); each starting from
    // descriptor array a
    hipGraphExec_t step_exec[2][kFusedRing] = {};
    bool graphs_ok = true;
    int states() const { return fused ? kFusedRing : 2; }
    int run(int kind) const { return fused ? (kind ? kFusedRun : kFusedRing) : (kind ? 2 * kRunPairs : 2); }
};

namespace {

void drop_graphs(pond_batch *b)
{
    for (auto &kind : b->step_exec)
        for (auto &g : kind)
            if (g) {
                (void)hipGraphExecDestroy(g);
                g = nullptr;
            }
}

// regroup the members and upload the descriptor arrays
int rebuild(pond_batch *b)
{
    drop_graphs(b);
    const int M = (int)b->members.size();
    b->groups.clear();
    b->slot_of.assign(M, -1);
    std::vector<int> order(M);
    for (int i = 0; i < M; ++i) order[i] = i;
    auto key = [&](int i) {
        const pond_handle *h = b->members[i];
        return ((h->lc.dim * 3 + h->lc.fp32) * 16 + h->lc.stream_tile) * 2 + (h->lc.gen_eos ? 1 : 0);
    };
    std::stable_sort(order.begin(), order.end(), [&](int x, int y) { return key(x) < key(y); });
    if (M > b->cap) {
        if (hipStreamSynchronize(b->stream) != hipSuccess) return POND_E_DEVICE;
        if (b->desc_d) (void)hipFree(b->desc_d);
        if (b->flags_d) (void)hipFree(b->flags_d);
        const int cap = std::max(M, 2 * b->cap);
        b->desc_d = nullptr;
        b->flags_d = nullptr;
        b->cap = 0;
        if (hipMalloc((void **)&b->desc_d, sizeof(SlotDesc) * kFusedRing * cap) != hipSuccess ||
            hipMalloc((void **)&b->flags_d, sizeof(int) * kFlagWords * cap) != hipSuccess)
            return POND_E_NOMEM;
        b->cap = cap;
    }
    const int R = b->states();
    b->desc_h.assign((size_t)R * std::max(M, 1), SlotDesc{});
    b->flags_h.assign((size_t)kFlagWords * std::max(M, 1), 0);
    int gkey = -1;
    for (int s = 0; s < M; ++s) {
        const int i = order[s];
        pond_handle *h = b->members[i];
        if (key(i) != gkey) {
            gkey = key(i);
            b->groups.push_back(Group{h->lc.dim, h->lc.fp32, h->lc.stream_tile, h->lc.gen_eos, s, 0, 0, 0});
        }
        Group &g = b->groups.back();
        b->slot_of[i] = s;
        for (int a = 0; a < R; ++a) {
            SlotDesc d = h->desc_h[(h->cur + a) % R];
            d.st_begin = g.st_tiles;
            d.fc_begin = g.fc_tiles;
            b->desc_h[(size_t)a * M + s] = d;
        }
        g.count += 1;
        g.st_tiles += h->st_tiles;
        g.fc_tiles += h->fc_tiles;
    }
    if (M > 0 && hipMemcpy(b->desc_d, b->desc_h.data(), sizeof(SlotDesc) * R * M, hipMemcpyHostToDevice) != hipSuccess)
        return POND_E_DEVICE;
    b->phase = 0;
    b->dirty = false;
    return POND_OK;
}

hipError_t enqueue_step(pond_batch *b, hipStream_t st, int arr)
{
    const int M = (int)b->members.size();
    for (const Group &g : b->groups) {
        LaunchCtx c{g.dim, 0, 0, 0, g.fp32, st, g.tile};
        c.gen_eos = g.gen_eos;
        c.fused = b->fused;
        const SlotDesc *d = b->desc_d + (size_t)arr * M + g.first;
        hipError_t e;
        if (b->fused) {
            e = launch_step_fused(c, d, g.count, g.st_tiles);
        } else {
            e = launch_stream(c, d, g.count, g.st_tiles);
            if (e == hipSuccess) e = launch_force_collide(c, d, g.count, g.fc_tiles);
        }
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

// fused steps: the closure check of every member's state read by descriptor array `arr`
hipError_t enqueue_check(pond_batch *b, hipStream_t st, int arr)
{
    const int M = (int)b->members.size();
    for (const Group &g : b->groups) {
        LaunchCtx c{g.dim, 0, 0, 0, g.fp32, st, g.tile};
        c.fused = true;
        hipError_t e = launch_collide_check(c, b->desc_d + (size_t)arr * M + g.first, g.count, g.fc_tiles);
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

// record a run of b->run(kind) steps from descriptor array `arr`
bool build_step_graph(pond_batch *b, int kind, int arr)
{
    hipGraphExec_t &exec = b->step_exec[kind][arr];
    if (exec) return true;
    hipGraph_t g = nullptr;
    if (hipStreamBeginCapture(b->capture_stream, hipStreamCaptureModeThreadLocal) != hipSuccess) return false;
    hipError_t e = hipSuccess;
    for (int k = 0; k < b->run(kind) && e == hipSuccess; ++k) e = enqueue_step(b, b->capture_stream, (arr + k) % b->states());
    const hipError_t ec = hipStreamEndCapture(b->capture_stream, &g);
    if (e != hipSuccess || ec != hipSuccess || !g) {
        if (g) (void)hipGraphDestroy(g);
        return false;
    }
    e = hipGraphInstantiate(&exec, g, nullptr, nullptr, 0);
    (void)hipGraphDestroy(g);
    if (e != hipSuccess) {
        exec = nullptr;
        return false;
    }
    return true;
}

int find_member(const pond_batch *b, const pond_handle *h)
{
    for (size_t i = 0; i < b->members.size(); ++i)
        if (b->members[i] == h) return (int)i;
    return -1;
}

} // namespace

extern "C" {

int pond_batch_create(void *stream, pond_batch **out)
{
    if (!out) return POND_E_INVALID;
    *out = nullptr;
    pond_batch *b = new (std::nothrow) pond_batch();
    if (!b) return POND_E_NOMEM;
    int rc = POND_OK;
    if (stream) {
        b->stream = (hipStream_t)stream;
    } else if (hipStreamCreateWithFlags(&b->stream, hipStreamNonBlocking) == hipSuccess) {
        b->own_stream = true;
    } else {
        rc = POND_E_DEVICE;
    }
    if (rc == POND_OK && hipStreamCreateWithFlags(&b->capture_stream, hipStreamNonBlocking) != hipSuccess)
        rc = POND_E_DEVICE;
    if (rc != POND_OK) {
        if (b->own_stream) (void)hipStreamDestroy(b->stream);
        delete b;
        return rc;
    }
    *out = b;
    return POND_OK;
}

int pond_batch_add(pond_batch *b, pond_handle *h)
{
    if (!b || !h || h->batch) return POND_E_INVALID;
    if (h->lc.dim == 3) return handle_fail(h, POND_E_INVALID, "D3Q27 lattices are stepped alone");
    if (!h->initialised || h->failed)
        return handle_fail(h, POND_E_STATE, h->failed ? "handle in error state" : "not initialised");
    if (!b->members.empty() && h->lc.fused != b->fused)
        return handle_fail(h, POND_E_INVALID, "the members of a batch share the form of the step (two_kernel)");
    long long st = h->st_tiles, fc = h->fc_tiles;
    for (const pond_handle *m : b->members)
        if (m->lc.dim == h->lc.dim && m->lc.fp32 == h->lc.fp32 && m->lc.stream_tile == h->lc.stream_tile) {
            st += m->st_tiles;
            fc += m->fc_tiles;
        }
    if (st > kMaxLaunchTiles || fc > kMaxLaunchTiles)
        return handle_fail(h, POND_E_INVALID, "batch group would exceed %lld tiles per launch", kMaxLaunchTiles);
    if (hipStreamSynchronize(h->stream) != hipSuccess) return handle_fail(h, POND_E_DEVICE, "stream sync");
    try {
        b->members.push_back(h);
    } catch (...) {
        return POND_E_NOMEM;
    }
    h->batch = b;
    if (b->members.size() == 1 && b->fused != h->lc.fused) {
        drop_graphs(b);
        b->fused = h->lc.fused;
    }
    b->dirty = true;
    return POND_OK;
}

int pond_batch_remove(pond_batch *b, pond_handle *h)
{
    if (!b || !h) return POND_E_INVALID;
    const int i = find_member(b, h);
    if (i < 0) return POND_E_INVALID;
    (void)hipStreamSynchronize(b->stream);
    b->members.erase(b->members.begin() + i);
    h->batch = nullptr;
    b->dirty = true;
    return POND_OK;
}

int pond_batch_step(pond_batch *b, int nsteps)
{
    if (!b || nsteps < 0) return POND_E_INVALID;
    if (nsteps == 0 || b->members.empty()) return POND_OK;
    if (b->dirty) {
        const int rc = rebuild(b);
        if (rc != POND_OK) return rc;
    }
    const int M = (int)b->members.size();
    if (launch_reset_slot_flags(b->stream, b->desc_d, M) != hipSuccess) return POND_E_DEVICE;
    int arr = b->phase;
    int left = nsteps;
    // long runs, then short runs; each returns to the descriptor array it starts from
    for (int kind = 1; kind >= 0 && b->graphs_ok; --kind) {
        const int len = b->run(kind);
        if (left < len) continue;
        if (!build_step_graph(b, kind, arr)) {
            b->graphs_ok = false;
            break;
        }
        for (; left >= len; left -= len)
            if (hipGraphLaunch(b->step_exec[kind][arr], b->stream) != hipSuccess) return POND_E_DEVICE;
    }
    for (; left > 0; --left) {
        if (enqueue_step(b, b->stream, arr) != hipSuccess) return POND_E_DEVICE;
        arr = (arr + 1) % b->states();
    }
    if (b->fused && enqueue_check(b, b->stream, arr) != hipSuccess) return POND_E_DEVICE;
    if (launch_gather_slot_flags(b->stream, b->desc_d, M, b->flags_d) != hipSuccess) return POND_E_DEVICE;
    if (hipMemcpyAsync(b->flags_h.data(), b->flags_d, sizeof(int) * kFlagWords * M, hipMemcpyDeviceToHost,
                       b->stream) != hipSuccess ||
        hipStreamSynchronize(b->stream) != hipSuccess)
        return POND_E_DEVICE;
    b->phase = arr;
    // every member moves on by its own count of completed steps; failed ones leave
    int first_err = POND_OK;
    std::vector<pond_handle *> keep;
    keep.reserve(M);
    for (int i = 0; i < M; ++i) {
        pond_handle *h = b->members[i];
        const int rc = handle_finish_batch(h, &b->flags_h[(size_t)kFlagWords * b->slot_of[i]], nsteps);
        if (rc == POND_OK) {
            keep.push_back(h);
        } else {
            h->batch = nullptr;
            if (first_err == POND_OK) first_err = rc;
        }
    }
    if ((int)keep.size() != M) {
        b->members.swap(keep);
        b->dirty = true;
    }
    return first_err;
}

int pond_batch_size(const pond_batch *b, int *out)
{
    if (!b || !out) return POND_E_INVALID;
    *out = (int)b->members.size();
    return POND_OK;
}

int pond_batch_destroy(pond_batch *b)
{
    if (!b) return POND_OK;
    if (b->stream) (void)hipStreamSynchronize(b->stream);
    for (pond_handle *h : b->members) h->batch = nullptr;
    drop_graphs(b);
    if (b->desc_d) (void)hipFree(b->desc_d);
    if (b->flags_d) (void)hipFree(b->flags_d);
    if (b->capture_stream) (void)hipStreamDestroy(b->capture_stream);
    if (b->own_stream && b->stream) (void)hipStreamDestroy(b->stream);
    delete b;
    return POND_OK;
}

} // extern "C"
